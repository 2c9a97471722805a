"""FP32 geometry with an FP64 guard band (precision HPMC_FP32_GUARDED): the
sphere depletant tests run in FP32 and fall back to FP64 only within 1e-5 sigma
of contact, so every decision equals the FP64 oracle's, bit for bit."""
import pytest

from paper_1508_07077_amd import workloads as wl
from parity_util import compare_sweeps, make_pair
from test_gpu_parity import _melt

pytestmark = pytest.mark.gpu
FP32_GUARDED = 1


@pytest.mark.parametrize("n_trial", [0, 4])
def test_c1_fp32_guarded(n_trial):
    sp = wl.c1_spheres_small(n_trial)
    pos, _ = sp.initial_state()
    g, o = make_pair(sp, pos, precision=FP32_GUARDED)
    tot, div = compare_sweeps(g, o, 40)
    assert div == 0 and tot["accepts"] > 0


@pytest.mark.parametrize("region", [0, 1])
def test_c3_shaped_fp32_guarded(region):
    sp = wl.c3_spheres_large(n=3000, d_trans=0.003)
    pos, _ = _melt(sp, 20)
    g, o = make_pair(sp, pos, precision=FP32_GUARDED, region=region)
    tot, div = compare_sweeps(g, o, 3)
    assert div == 0
    # the band is hit now and then: rarely for points spread over the ball,
    # more often in the thin shell, whose points all lie near the old pose's surface
    rate = 1e-4 if region == 0 else 1e-2
    assert tot["fp64_fallbacks"] < rate * tot["depletants_drawn"] + 10


@pytest.mark.parametrize("kind", [wl.HEMISPHERE, wl.DISCOID])
def test_oriented_fp32_guarded(kind):
    """hemisphere and swept-disk depletant predicates in FP32 with the guard band"""
    if kind == wl.HEMISPHERE:
        sp = wl.StatePoint(kind, (1.0,), 400, 0.20, 0.15, 0.30, n_trial=0, d_trans=0.05, a_rot=0.05, p_rot=0.5,
                           seed=61)
    else:
        sp = wl.StatePoint(kind, (0.5, 0.1), 300, 0.25, 0.2, 0.30, n_trial=2, d_trans=0.04, a_rot=0.04, p_rot=0.5,
                           seed=62)
    pos, quat = _melt(sp, 10)
    g, o = make_pair(sp, pos, quat, precision=FP32_GUARDED)
    tot, div = compare_sweeps(g, o, 6, allow_near=True)
    assert div <= 1 and tot["accepts"] > 0
    assert tot["fp64_fallbacks"] < 1e-3 * tot["depletants_drawn"] + 10
