"""Batched replicas (hpmc_sweep_batch): independent boxes of uneven size,
density and fugacity swept in shared launches give every replica exactly the
trajectory it has alone, and that trajectory is the oracle's."""
import numpy as np
import pytest

from paper_1508_07077_amd import workloads as wl
from parity_util import TRACE_FIELDS

pytestmark = pytest.mark.gpu


def _replicas(kind, count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for r in range(count):
        n = int(rng.integers(60, 400))
        phi = float(rng.uniform(0.05, 0.3))
        eta = float(rng.uniform(0.0, 0.4))
        if kind == wl.SPHERE:
            sp = wl.StatePoint(wl.SPHERE, (1.0,), n, phi, 0.2, eta, n_trial=int(r % 3), d_trans=0.05,
                               seed=100 + r, replica_id=r)
        else:
            sp = wl.StatePoint(wl.DISCOID, (0.5, 0.1), n, phi, 0.2, eta, n_trial=int(r % 2), d_trans=0.03,
                               a_rot=0.03, p_rot=0.5, seed=200 + r, replica_id=r)
        out.append(sp)
    return out


def _handle(sp, pos, quat):
    import paper_1508_07077_amd as hp

    g = hp.Sim(sp.n, sp.L, sp.seed, sp.replica_id)
    g.set_shape(sp.kind, sp.params)
    g.set_fugacity(sp.z_p, sp.d_dep, sp.n_trial)
    g.set_moves(sp.d_trans, sp.a_rot, sp.p_rot)
    g.set_state(pos, quat)
    return g


@pytest.mark.parametrize("kind", [wl.SPHERE, wl.DISCOID], ids=["sphere", "discoid"])
def test_batch_equals_alone(kind):
    import paper_1508_07077_amd as hp

    sps = _replicas(kind, 10, 7 if kind == wl.SPHERE else 8)
    states = [sp.initial_state() for sp in sps]
    batch_sims = [_handle(sp, p, q) for sp, (p, q) in zip(sps, states)]
    alone = [_handle(sp, p, q) for sp, (p, q) in zip(sps, states)]
    b = hp.Batch(batch_sims)
    cb = b.sweep(4)
    for g, sp, c in zip(alone, sps, cb):
        ca = g.sweep(4)
        for k in ("trials", "accepts", "depletants_drawn", "depletants_resolved", "rej_overlap", "cb_trials"):
            assert ca[k] == c[k], (sp.name, k)
    for g, h in zip(alone, batch_sims):
        pa, qa, sa = g.get_state()
        pb, qb, sb = h.get_state()
        assert sa == sb == 4
        assert np.array_equal(pa, pb)
        if qa is not None:
            assert np.array_equal(qa, qb)


def test_batch_needs_one_stream():
    """handles on different streams are not batched: both batched entry points
    refuse them before any device work, and every handle still sweeps alone"""
    import torch

    import paper_1508_07077_amd as hp

    sps = _replicas(wl.SPHERE, 2, 5)
    side = torch.cuda.Stream()
    sims = []
    for i, sp in enumerate(sps):
        g = hp.Sim(sp.n, sp.L, sp.seed, sp.replica_id, stream=side if i == 1 else None)
        g.set_shape(sp.kind, sp.params)
        g.set_fugacity(sp.z_p, sp.d_dep, sp.n_trial)
        g.set_moves(sp.d_trans, sp.a_rot, sp.p_rot)
        g.set_state(*sp.initial_state())
        sims.append(g)
    b = hp.Batch(sims)
    for call in (lambda: b.sweep(1), lambda: b.autotune(1)):
        with pytest.raises(hp.HpmcError) as e:
            call()
        assert e.value.code == -1 and "stream" in str(e.value)
    for g, sp in zip(sims, sps):
        assert g.get_state()[2] == 0
        assert g.sweep(1)["trials"] == sp.n


def test_batch_matches_oracle():
    import paper_1508_07077_amd as hp
    from oracle import pyoracle

    sps = _replicas(wl.SPHERE, 6, 11)
    states = [sp.initial_state() for sp in sps]
    sims = [_handle(sp, p, q) for sp, (p, q) in zip(sps, states)]
    hp.Batch(sims).sweep(3)
    for sp, (p, q), g in zip(sps, states, sims):
        o = pyoracle.OracleSim(sp.n, sp.L, sp.seed, sp.replica_id)
        o.set_shape(sp.kind, sp.params)
        o.set_fugacity(sp.z_p, sp.d_dep, sp.n_trial)
        o.set_moves(sp.d_trans, sp.a_rot, sp.p_rot)
        o.set_state(p, q)
        o.sweep(3)
        po, _, _ = o.get_state()
        pg, _, _ = g.get_state()
        assert np.array_equal(po, pg), sp.name


@pytest.mark.parametrize("counters", [True, False])
def test_mixed_kinds_concurrent_groups(counters):
    """Spheres, hemispheres and swept disks in one batch: the three shape
    groups run on separate streams (and, for untimed multi-sweep calls, as
    parallel branches of one graph); every replica still matches its lone run."""
    import paper_1508_07077_amd as hp

    sps = _replicas(wl.SPHERE, 3, 7) + _replicas(wl.DISCOID, 3, 8)
    sps.append(wl.StatePoint(wl.HEMISPHERE, (1.0,), 150, 0.15, 0.15, 0.2, d_trans=0.04, a_rot=0.04, p_rot=0.5,
                             seed=901, replica_id=99))
    states = [sp.initial_state() for sp in sps]
    batch = [_handle(sp, *st) for sp, st in zip(sps, states)]
    alone = [_handle(sp, *st) for sp, st in zip(sps, states)]
    b = hp.Batch(batch)
    for _ in range(3):
        b.sweep(2, counters=counters)
    for a in alone:
        a.sweep(6, counters=True)
    for x, y in zip(batch, alone):
        px, qx, sx = x.get_state()
        py, qy, sy = y.get_state()
        assert sx == sy == 6
        assert np.array_equal(px, py)
        if qx is not None:
            assert np.array_equal(qx, qy)


def test_counter_array_equals_the_records():
    """Batch.sweep(as_array=True) returns the counters the dict form does:
    two identical batches swept side by side"""
    import paper_1508_07077_amd as hp

    sps = _replicas(wl.SPHERE, 5, 41) + _replicas(wl.DISCOID, 4, 42)
    a, b = [], []
    for sp in sps:
        pos, quat = sp.initial_state()
        a.append(_handle(sp, pos, quat))
        b.append(_handle(sp, pos, quat))
    ba, bb = hp.Batch(a), hp.Batch(b)
    for _ in range(3):
        recs = ba.sweep(1, counters=True)
        arr = bb.sweep(1, counters=True, as_array=True)
        assert arr.shape == (len(sps),) and arr.dtype == hp.COUNTER_DTYPE
        for r, x in zip(recs, arr):
            assert all(r[f] == int(x[f]) for f in hp.COUNTERS)
            assert x["sweep_ms"] > 0.0
    for x in a + b:
        x.close()


def test_replicas_past_the_block_cap_equal_alone():
    """A replica that needs more than the 1,024 blocks a batched phase launch
    gives it: 16,384 hemispheres (1,728 active cells) at one wave per
    workgroup, whose waves then take several cells in turn, and 60,000
    spheres (9,261 active cells) at 8 cells per one-wave workgroup,
    whose chunk of cells grows instead.  Both sweep exactly as alone."""
    import paper_1508_07077_amd as hp

    hem = wl.StatePoint(wl.HEMISPHERE, (1.0,), 16384, 0.20, 0.15, 0.3, d_trans=0.05, a_rot=0.05, p_rot=0.5,
                        seed=51, replica_id=1)
    sph = wl.StatePoint(wl.SPHERE, (1.0,), 60000, 0.30, 0.10, 0.3, n_trial=2, d_trans=0.01, seed=52, replica_id=2)
    sps = [hem, sph]
    states = [sp.initial_state() for sp in sps]
    batch_sims = [_handle(sp, p, q) for sp, (p, q) in zip(sps, states)]
    alone = [_handle(sp, p, q) for sp, (p, q) in zip(sps, states)]
    for g in batch_sims + alone:
        g.set_tuning(8 if g.kind == wl.SPHERE else 0, 1, 0)
    cb = hp.Batch(batch_sims).sweep(2)
    for g, sp, c in zip(alone, sps, cb):
        ca = g.sweep(2)
        for k in ("trials", "accepts", "depletants_drawn", "depletants_resolved", "rej_overlap", "cb_trials"):
            assert ca[k] == c[k], (sp.name, k)
    for g, h in zip(alone, batch_sims):
        pa, qa, sa = g.get_state()
        pb, qb, sb = h.get_state()
        assert sa == sb == 2 and np.array_equal(pa, pb)
        if qa is not None:
            assert np.array_equal(qa, qb)
    for g in batch_sims + alone:
        g.close()
