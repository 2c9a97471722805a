"""The allocation-free sweep (hpmc_sweep_static) against hpmc_sweep: the same
kernels with the library's static device scratch as workspace, so the same
trajectory bit for bit and the same counters.  Calls follow each other on one
device with different inputs, the later ones smaller, so each must rebuild
what it needs in the shared scratch."""
import numpy as np
import pytest

from paper_1508_07077_amd import workloads as wl

pytestmark = pytest.mark.gpu

COUNTS = ("trials", "accepts", "rej_cell_exit", "rej_overlap", "rej_depletant", "rej_cb_zero", "rej_cb_metropolis",
          "depletants_drawn", "depletants_resolved", "cb_trials", "overlap_checks", "near_contact", "fp64_fallbacks")


def _pair(sp, workspace_for_static=True):
    import paper_1508_07077_amd as hp

    pos, quat = sp.initial_state()
    out = []
    for ws in (True, workspace_for_static):
        s = hp.Sim(sp.n, sp.L, sp.seed, sp.replica_id)
        s.set_shape(sp.kind, sp.params)
        s.set_fugacity(sp.z_p, sp.d_dep, sp.n_trial)
        s.set_moves(sp.d_trans, sp.a_rot, sp.p_rot)
        s.set_state(pos, quat, workspace=ws)
        out.append(s)
    return out  # (reference with hpmc_sweep, handle for hpmc_sweep_static)


def _same(ref, st):
    pr, qr, sr = ref.get_state()
    ps, qs, ss = st.get_state()
    assert sr == ss
    assert np.array_equal(pr, ps)
    assert (qr is None and qs is None) or np.array_equal(qr, qs)


def _check(sp, sweeps, workspace_for_static):
    ref, st = _pair(sp, workspace_for_static)
    cr = ref.sweep(sweeps, counters=True)
    cs = st.sweep_static(sweeps, counters=True)
    for k in COUNTS:
        assert cr[k] == cs[k], (sp.name, k, cr[k], cs[k])
    _same(ref, st)
    # untimed calls as well
    ref.sweep(2, counters=False)
    st.sweep_static(2, counters=False)
    _same(ref, st)
    return ref, st


def test_static_sweeps_equal_workspace_sweeps_large_then_smaller():
    # 1: 20,000 spheres with configurational bias (multi-kernel sweep)
    big = wl.c3_spheres_large(n=20000)
    big.name = "spheres 20000"
    _check(big, 3, workspace_for_static=False)
    # 2: smaller: 600 hemispheres (oriented phase kernel), after the larger call
    hemi = wl.c2_hemispheres(0.3, n=600)
    hemi.name = "hemispheres 600"
    _check(hemi, 3, workspace_for_static=False)
    # 3: smaller still: 64 spheres (one workgroup sweeps the box)
    small = wl.c1_spheres_small(n_trial=2)
    small.name = "spheres 64"
    _check(small, 4, workspace_for_static=True)


def test_static_and_workspace_sweeps_interleave_on_one_handle():
    """static sweeps advance the sweep index; a later hpmc_sweep on the same
    handle continues the same trajectory"""
    sp = wl.c2_hemispheres(0.2, n=800)
    ref, st = _pair(sp, workspace_for_static=True)
    ref.sweep(5, counters=False)
    st.sweep_static(2, counters=False)
    st.sweep(1, counters=True)
    st.sweep_static(1, counters=True)
    st.sweep(1, counters=False)
    _same(ref, st)


def test_static_scratch_limit_is_an_error():
    import paper_1508_07077_amd as hp

    sp = wl.c3_spheres_large(n=1_500_000)
    s = hp.Sim(sp.n, sp.L, sp.seed)
    s.set_shape(sp.kind, sp.params)
    s.set_fugacity(sp.z_p, sp.d_dep, sp.n_trial)
    assert s.workspace_bytes() > 64 << 20
    pos = np.zeros((3, sp.n))
    with pytest.raises(hp.HpmcError) as e:
        s.set_state(pos, workspace=False)
    assert e.value.code == -4 and "static scratch" in str(e.value)
