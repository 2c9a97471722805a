"""Launch shapes never change a result: trajectories under explicit shapes and
after the autotuner equal the default's bit for bit, and the autotuner leaves
the handle's state and sweep index as they were."""
import numpy as np
import pytest

from paper_1508_07077_amd import workloads as wl

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
