"""Continuous-batching server: requests of different shapes, sizes and state
points admitted as slots free up and swept together return exactly the result
each gives alone (tolerance 0: the same random streams, the same arithmetic)."""
import numpy as np
import pytest

from paper_1508_07077_amd import workloads as wl

pytestmark = pytest.mark.gpu


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


def test_results_same_alone_and_in_the_mix():
    from paper_1508_07077_amd import serve

    specs = _stream()
    sweeps = [10 + 3 * (i % 4) for i in range(len(specs))]
    reqs = [serve.Request(sp, sw, arrival=0.0, rid=i) for i, (sp, sw) in enumerate(zip(specs, sweeps))]
    srv = serve.Server(max_active=5, sweeps_per_tick=2)  # slots force staggered admission
    done = {r.rid: r for r in srv.run(reqs, realtime=False)}
    assert len(done) == len(specs)
    for i, (sp, sw) in enumerate(zip(specs, sweeps)):
        alone = serve.Server(max_active=1, sweeps_per_tick=1)
        res = alone.run([serve.Request(sp, sw, arrival=0.0, rid=i)], realtime=False)[0].result
        mix = done[i].result
        assert np.array_equal(res["g_r"], mix["g_r"]), i
        for k in ("alpha", "phi_p", "beta_P", "beta_P_hard", "beta_P_dep"):
            assert res[k] == mix[k], (i, k)
    # staggered: some requests waited for a slot
    assert max(r.admitted for r in done.values()) > 0.0
