"""Launch shapes never change a result: trajectories under explicit shapes and
after the autotuner equal the default's bit for bit, and the autotuner leaves
the handle's state and sweep index as they were."""
import numpy as np
import pytest

from paper_1508_07077_amd import workloads as wl
from parity_util import cells_per_axis

pytestmark = pytest.mark.gpu


def _sim(sp, pos, quat):
    import paper_1508_07077_amd as hp

    g = hp.Sim(sp.n, sp.L, sp.seed)
    g.set_shape(sp.kind, sp.params)
    g.set_fugacity(sp.z_p, sp.d_dep, sp.n_trial)
    g.set_moves(sp.d_trans, sp.a_rot, sp.p_rot)
    g.set_state(pos, quat)
    return g


SPHERES = wl.StatePoint(wl.SPHERE, (1.0,), 3000, 0.30, 0.10, 0.30, n_trial=4, d_trans=0.01, seed=31)
HEMIS = wl.StatePoint(wl.HEMISPHERE, (1.0,), 2000, 0.20, 0.15, 0.30, d_trans=0.05, a_rot=0.05, p_rot=0.5, seed=32)


@pytest.mark.parametrize("sp,shapes", [
    (SPHERES, [(1, 1, 0), (7, 2, 0), (64, 4, 0), (33, 1, 0)]),
    (HEMIS, [(0, 1, 1), (0, 2, 37), (0, 4, 100000)]),
], ids=["spheres", "hemispheres"])
def test_launch_shape_invariance(sp, shapes):
    pos, quat = sp.initial_state()
    ref = _sim(sp, pos, quat)
    ref.sweep(4, counters=True)
    pr, qr, _ = ref.get_state()
    for c, w, m in shapes:
        g = _sim(sp, pos, quat)
        g.set_tuning(c, w, m)
        cg = g.sweep(4, counters=True)
        pg, qg, _ = g.get_state()
        assert np.array_equal(pg, pr), (c, w, m)
        if qr is not None:
            assert np.array_equal(qg, qr), (c, w, m)
        assert cg["trials"] == 4 * sp.n


@pytest.mark.parametrize("sp", [SPHERES, HEMIS], ids=["spheres", "hemispheres"])
def test_autotune_keeps_state_and_trajectory(sp):
    pos, quat = sp.initial_state()
    ref = _sim(sp, pos, quat)
    g = _sim(sp, pos, quat)
    for s in (ref, g):
        s.sweep(2, counters=False)
    p0, q0, sw0 = g.get_state()
    t = g.autotune(sweeps=1)
    p1, q1, sw1 = g.get_state()
    assert sw1 == sw0 and np.array_equal(p1, p0)
    assert t["candidates"] >= 9 and t["best_ms"] > 0 and t["best_ms"] <= t["default_ms"]
    for s in (ref, g):
        s.sweep(3, counters=False)
    pr, qr, swr = ref.get_state()
    pg, qg, swg = g.get_state()
    assert swr == swg and np.array_equal(pr, pg)
    if qr is not None:
        assert np.array_equal(qr, qg)


def _replicas():
    """a mixed batch: a small sphere box (one workgroup sweeps it), two larger
    sphere boxes, two hemisphere boxes, and swept-disk boxes of two and more
    cells per axis"""
    sps = [wl.StatePoint(wl.SPHERE, (1.0,), 200, 0.30, 0.10, 0.30, n_trial=2, d_trans=0.05, seed=41, replica_id=0),
           wl.StatePoint(wl.SPHERE, (1.0,), 3000, 0.30, 0.10, 0.30, n_trial=4, d_trans=0.01, seed=42, replica_id=1),
           wl.StatePoint(wl.SPHERE, (1.0,), 5000, 0.25, 0.10, 0.20, d_trans=0.02, seed=43, replica_id=2),
           wl.StatePoint(wl.HEMISPHERE, (1.0,), 2000, 0.20, 0.15, 0.30, d_trans=0.05, a_rot=0.05, p_rot=0.5, seed=44,
                         replica_id=3),
           wl.StatePoint(wl.HEMISPHERE, (1.0,), 1200, 0.25, 0.15, 0.10, d_trans=0.05, a_rot=0.05, p_rot=0.5, seed=45,
                         replica_id=4)]
    disks = sorted(wl.c4_discoid_replicas(count=24), key=lambda sp: sp.n)
    return sps + [disks[0], disks[1], disks[12]]


def _make(sp):
    import paper_1508_07077_amd as hp

    pos, quat = sp.initial_state()
    g = hp.Sim(sp.n, sp.L, sp.seed, sp.replica_id)
    g.set_shape(sp.kind, sp.params)
    g.set_fugacity(sp.z_p, sp.d_dep, sp.n_trial)
    g.set_moves(sp.d_trans, sp.a_rot, sp.p_rot)
    g.set_state(pos, quat)
    return g


def test_batch_autotune_per_group_keeps_states_and_trajectories():
    import paper_1508_07077_amd as hp

    sps = _replicas()
    ref = [_make(sp) for sp in sps]
    tun = [_make(sp) for sp in sps]
    assert [cells_per_axis(sp) for sp in sps[5:]][:2] == [2, 2] and cells_per_axis(sps[7]) > 2
    br, bt = hp.Batch(ref), hp.Batch(tun)
    br.sweep(2, counters=False)
    bt.sweep(2, counters=False)
    before = [s.get_state() for s in tun]
    shapes = bt.autotune(sweeps=1)
    for s, (p0, q0, w0) in zip(tun, before):
        p1, q1, w1 = s.get_state()
        assert w1 == w0 and np.array_equal(p1, p0)
        if q0 is not None:
            assert np.array_equal(q1, q0)
    assert shapes[0]["candidates"] == 0  # the small sphere box has no shape to tune
    for sp, t in zip(sps[1:], shapes[1:]):
        assert t["candidates"] >= 9 and 0 < t["best_ms"] <= t["default_ms"], (sp.name, t)
    # members of one launch group share one shape and one timing
    assert shapes[1]["best_ms"] == shapes[2]["best_ms"] and shapes[3]["best_ms"] == shapes[4]["best_ms"]
    assert (shapes[1]["cells_per_wave"], shapes[1]["waves_per_block"]) == \
        (shapes[2]["cells_per_wave"], shapes[2]["waves_per_block"])
    cr = br.sweep(3, counters=True)
    ct = bt.sweep(3, counters=True)
    for a, b, sp in zip(ref, tun, sps):
        pa, qa, wa = a.get_state()
        pb, qb, wb = b.get_state()
        assert wa == wb and np.array_equal(pa, pb), sp.name
        if qa is not None:
            assert np.array_equal(qa, qb), sp.name
    assert [c["accepts"] for c in cr] == [c["accepts"] for c in ct]
    for s in ref + tun:
        s.close()
