"""Continuous-batching server: requests of different shapes, sizes and state
points, admitted as slots and memory free up and swept together, return
exactly the result each gives alone (tolerance 0: the same random streams, the
same arithmetic), and that result is the oracle's: the final state and the
observables are bit-exact, except that an oriented request may differ from the
oracle by near-contact trials and what follows from them (the rule of
parity_util)."""
import numpy as np
import pytest

from paper_1508_07077_amd import workloads as wl
from parity_util import compare_sweeps, make_pair

pytestmark = pytest.mark.gpu

OBS = dict(probes=50000)


def _stream(count=12, seed=3):
    rng = np.random.default_rng(seed)
    shapes = [(wl.SPHERE, (1.0,), 0.10), (wl.HEMISPHERE, (1.0,), 0.15), (wl.DISCOID, (0.5, 0.1), 0.2)]
    out = []
    for i in range(count):
        kind, params, q = shapes[i % 3]
        n = int(rng.integers(150, 900))
        sp = wl.StatePoint(kind, params, n, float(rng.uniform(0.05, 0.3)), q, float(rng.uniform(0.0, 0.4)),
                           d_trans=0.03, a_rot=0.03 if kind else 0.0, p_rot=0.5 if kind else 0.0,
                           seed=1000 + i, replica_id=i)
        out.append(sp)
    return out


def _sweeps(i):
    return 10 + 3 * (i % 4)


def _oracle_observables(o, sp):
    from oracle import pyoracle

    r_max = min(3.0, 0.5 * sp.L)
    g = o.observables(pyoracle.OBS_GR, n_bins=60, r_max=r_max)
    fv = o.observables(pyoracle.OBS_FREE_VOLUME, n_probe=OBS["probes"], obs_seq=1)
    sdf = o.observables(pyoracle.OBS_SDF, n_bins=20, x_max=0.05, n_fit=6, n_probe=OBS["probes"], obs_seq=2, eps=0.01)
    return {"g_r": g, "alpha": fv[0], "phi_p": fv[1], "beta_P": sdf[0], "beta_P_hard": sdf[1], "beta_P_dep": sdf[2]}


def _same_result(a, b):
    if not np.array_equal(a["g_r"], b["g_r"]):
        return "g_r"
    for k in ("alpha", "phi_p", "beta_P", "beta_P_hard", "beta_P_dep"):
        if a[k] != b[k]:
            return k
    return None


def test_results_same_alone_in_the_mix_and_in_the_oracle():
    from paper_1508_07077_amd import serve

    specs = _stream()
    reqs = [serve.Request(sp, _sweeps(i), arrival=0.0, rid=i) for i, sp in enumerate(specs)]
    srv = serve.Server(max_active=5, sweeps_per_tick=2, keep_state=True)  # slots force staggered admission
    done = {r.rid: r for r in srv.run(reqs, realtime=False)}
    assert len(done) == len(specs)
    assert max(r.admitted for r in done.values()) > 0.0  # staggered: some requests waited for a slot
    for i, sp in enumerate(specs):
        mix = done[i].result
        assert "error" not in mix, mix
        alone = serve.Server(max_active=1, sweeps_per_tick=1, keep_state=True)
        res = alone.run([serve.Request(sp, _sweeps(i), arrival=0.0, rid=i)], realtime=False)[0].result
        assert _same_result(res, mix) is None, (i, _same_result(res, mix))
        assert np.array_equal(res["pos"], mix["pos"]) and res["sweep"] == mix["sweep"] == _sweeps(i)
        # the same request against the oracle, sweep by sweep, traced
        pos, quat = sp.initial_state()
        g, o = make_pair(sp, pos, quat)
        _, div = compare_sweeps(g, o, _sweeps(i), allow_near=sp.kind != wl.SPHERE)
        g.close()
        if div == 0:
            po, qo, so = o.get_state()
            assert so == mix["sweep"]
            assert np.array_equal(po, mix["pos"]), i
            if mix["quat"] is not None:
                assert np.array_equal(qo, mix["quat"]), i
            why = _same_result(_oracle_observables(o, sp), mix)
            assert why is None, (i, why)


def test_admission_never_exceeds_the_hbm_budget():
    from paper_1508_07077_amd import serve

    specs = _stream(count=9, seed=11)
    probe = serve.Server(max_active=len(specs) + 1)
    need = [probe._handle(serve.Request(sp, 1, 0.0)) for sp in specs]
    base = probe.batch.workspace.numel()
    budget = base + int(2.2 * max(need))  # room for two or three requests at a time
    big = wl.StatePoint(wl.SPHERE, (1.0,), 60000, 0.3, 0.1, 0.2, d_trans=0.01, seed=9, replica_id=99)
    reqs = [serve.Request(sp, 6, arrival=0.0, rid=i) for i, sp in enumerate(specs)]
    reqs.append(serve.Request(big, 6, arrival=0.0, rid=99))  # can never fit: refused
    srv = serve.Server(hbm_budget=budget, max_active=len(reqs), sweeps_per_tick=1)
    done = {r.rid: r for r in srv.run(reqs, realtime=False)}
    assert "error" in done[99].result and "budget" in done[99].result["error"]
    assert srv.ticks and all(used <= budget for _, used, _ in srv.ticks)
    assert max(n for _, _, n in srv.ticks) < len(specs)  # memory, not slots, made requests wait
    assert srv.used == base
    for i, sp in enumerate(specs):
        assert "error" not in done[i].result
        alone = serve.Server(max_active=1, sweeps_per_tick=1)
        res = alone.run([serve.Request(sp, 6, arrival=0.0, rid=i)], realtime=False)[0].result
        assert _same_result(res, done[i].result) is None, i
