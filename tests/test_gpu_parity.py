"""GPU parity: the HIP library (through its C-ABI) against the FP64 oracle on
the same seeded inputs.  Accept/reject decisions, depletant counts, CB weights
and the state must agree bit for bit (the determinism contract); for convex
colloid pairs decided within 1e-9 of contact by either side's own algorithm
(MPR on the GPU, GJK in the oracle) a divergence is tolerated and counted."""
import math

import numpy as np
import pytest

from paper_1508_07077_amd import workloads as wl
from parity_util import compare_sweeps, make_pair

pytestmark = pytest.mark.gpu


def _melt(sp, sweeps, z_p=0.0):
    """an equilibrated-looking start computed by the oracle alone"""
    from oracle import pyoracle

    pos, quat = sp.initial_state()
    o = pyoracle.OracleSim(sp.n, sp.L, sp.seed + 999, sp.replica_id)
    o.set_shape(sp.kind, sp.params)
    o.set_fugacity(z_p, sp.d_dep, 0)
    o.set_moves(max(sp.d_trans, 0.05), max(sp.a_rot, 0.05) if sp.kind != wl.SPHERE else 0.0, sp.p_rot)
    o.set_state(pos, quat)
    o.sweep(sweeps)
    p, q, _ = o.get_state()
    return p, (q if sp.kind != wl.SPHERE else None)


@pytest.mark.parametrize("n_trial", [0, 1, 4])
def test_c1_spheres_trajectory(n_trial):
    sp = wl.c1_spheres_small(n_trial)
    pos, _ = sp.initial_state()
    g, o = make_pair(sp, pos)
    tot, div = compare_sweeps(g, o, 40)
    assert div == 0
    assert tot["trials"] == 40 * sp.n and tot["accepts"] > 0
    if n_trial == 0:
        assert tot["rej_depletant"] > 0
    else:
        assert tot["rej_cb_zero"] + tot["rej_cb_metropolis"] > 0


@pytest.mark.parametrize("n_trial", [0, 4])
def test_c1_spheres_whole_trajectory(n_trial):
    """the 64-sphere workload's whole run: 1000 sweeps, every trial record and
    the state after every sweep against the oracle (no tolerance)"""
    sp = wl.c1_spheres_small(n_trial)
    pos, _ = sp.initial_state()
    g, o = make_pair(sp, pos)
    tot, div = compare_sweeps(g, o, 1000)
    assert div == 0
    assert tot["trials"] == 1000 * sp.n and tot["accepts"] > 0


def test_c3_shaped_box_cb():
    """spheres phi_c = 0.30, q = 0.10, eta_r = 0.30, n_trial = 4 (399 depletants per move)"""
    sp = wl.c3_spheres_large(n=3000, d_trans=0.003)
    pos, _ = _melt(sp, 20)
    g, o = make_pair(sp, pos)
    tot, div = compare_sweeps(g, o, 2)
    assert div == 0
    assert tot["depletants_drawn"] > 300 * tot["trials"] * 0.5


@pytest.mark.parametrize("case", ["single", "two_in_n2_box", "dilute", "n_select3", "zero_fugacity", "big_step",
                                  "dense_two_cell", "many_chunks", "most_chunks"])
def test_edge_cases(case):
    if case == "single":
        sp = wl.StatePoint(wl.SPHERE, (1.0,), 1, 0.01, 0.25, 0.10, d_trans=0.2, seed=3)
    elif case == "two_in_n2_box":
        sp = wl.StatePoint(wl.SPHERE, (1.0,), 2, 2 * math.pi / 6 / 2.6**3, 0.25, 0.10, d_trans=0.3, seed=4)
    elif case == "dilute":
        sp = wl.StatePoint(wl.SPHERE, (1.0,), 200, 0.01, 0.25, 0.30, n_trial=2, d_trans=0.3, seed=5)
    elif case == "n_select3":
        sp = wl.StatePoint(wl.SPHERE, (1.0,), 64, 0.20, 0.25, 0.10, d_trans=0.1, seed=6)
    elif case == "zero_fugacity":
        sp = wl.StatePoint(wl.SPHERE, (1.0,), 300, 0.35, 0.25, 0.0, d_trans=0.1, seed=7)
    elif case == "big_step":
        sp = wl.StatePoint(wl.SPHERE, (1.0,), 100, 0.10, 0.5, 0.2, n_trial=3, d_trans=0.8, seed=8)
    elif case == "dense_two_cell":
        # 90 spheres in a two-cell box: a stencil of 90 entries, past the 64 staged in LDS
        sp = wl.StatePoint(wl.SPHERE, (1.0,), 90, 0.45, 0.25, 0.2, n_trial=2, d_trans=0.1, seed=9)
    elif case == "many_chunks":
        # 4,630 depletants per move: 19 Poisson chunks (the cross-lane total)
        sp = wl.StatePoint(wl.SPHERE, (1.0,), 27, 0.10, 0.05, 0.5, d_trans=0.01, seed=10)
    else:
        # 50,000 depletants per move: 196 chunks, past the first pass over the lanes
        sp = wl.StatePoint(wl.SPHERE, (1.0,), 27, 0.10, 0.022, 0.5, n_trial=1, d_trans=0.002, seed=10)
    pos, _ = sp.initial_state()
    g, o = make_pair(sp, pos)
    if case == "n_select3":
        for s in (g, o):
            s.set_moves(sp.d_trans, 0.0, 0.0, 3)
        g.set_trace(True)
        o.set_trace(True)
    tot, div = compare_sweeps(g, o, 12)
    assert div == 0
    if case == "zero_fugacity":
        assert tot["depletants_drawn"] == 0


def test_hemispheres():
    sp = wl.StatePoint(wl.HEMISPHERE, (1.0,), 400, 0.20, 0.15, 0.30, n_trial=0, d_trans=0.05, a_rot=0.05,
                       p_rot=0.5, seed=11)
    pos, quat = _melt(sp, 10)
    g, o = make_pair(sp, pos, quat)
    tot, div = compare_sweeps(g, o, 8, allow_near=True)
    assert div <= 1
    assert tot["rej_overlap"] > 0 and tot["rej_depletant"] > 0 and tot["accepts"] > 0


def test_hemispheres_many_chunks():
    """20,000 depletants per move: 80 Poisson chunks, past the oriented kernel's
    first pass over the lanes"""
    sp = wl.StatePoint(wl.HEMISPHERE, (1.0,), 40, 0.10, 0.03, 0.5, n_trial=0, d_trans=0.01, a_rot=0.01,
                       p_rot=0.5, seed=15)
    pos, quat = sp.initial_state()
    g, o = make_pair(sp, pos, quat)
    tot, div = compare_sweeps(g, o, 2, allow_near=True)
    assert div <= 1
    assert tot["depletants_drawn"] > 15000 * tot["trials"] * 0.5


def test_hemispheres_cb():
    sp = wl.StatePoint(wl.HEMISPHERE, (1.0,), 300, 0.15, 0.15, 0.20, n_trial=3, d_trans=0.03, a_rot=0.03,
                       p_rot=0.5, seed=12)
    pos, quat = _melt(sp, 10)
    g, o = make_pair(sp, pos, quat)
    tot, div = compare_sweeps(g, o, 6, allow_near=True)
    assert div <= 1


def test_discoids():
    sp = wl.StatePoint(wl.DISCOID, (0.5, 0.1), 300, 0.25, 0.2, 0.30, n_trial=2, d_trans=0.04, a_rot=0.04,
                       p_rot=0.5, seed=13)
    pos, quat = _melt(sp, 10)
    g, o = make_pair(sp, pos, quat)
    tot, div = compare_sweeps(g, o, 6, allow_near=True)
    assert div <= 1
    assert tot["accepts"] > 0


@pytest.mark.parametrize("n, phi", [(128, 0.45), (600, 0.40)], ids=["two_cell_box", "four_cell_box"])
def test_dense_discoids(n, phi):
    """dense swept disks: stencils of more than 64 entries (the per-trial close
    and reach lists) and more than the 64 entries the geometry cache holds
    (the rest read from the records)"""
    sp = wl.StatePoint(wl.DISCOID, (0.5, 0.1), n, phi, 0.2, 0.40, n_trial=1, d_trans=0.02, a_rot=0.02,
                       p_rot=0.5, seed=14)
    pos, quat = _melt(sp, 6)
    g, o = make_pair(sp, pos, quat)
    tot, div = compare_sweeps(g, o, 4, allow_near=True)
    assert div <= 1
    assert tot["accepts"] > 0 and tot["rej_overlap"] > 0 and tot["depletants_drawn"] > 0


def test_overlapping_state_rejected():
    import paper_1508_07077_amd as hp

    sp = wl.c1_spheres_small()
    pos, _ = sp.initial_state()
    pos[:, 1] = pos[:, 0] + np.array([0.5, 0.0, 0.0])
    g = hp.Sim(sp.n, sp.L, 1)
    g.set_shape(hp.SPHERE, [1.0])
    g.set_fugacity(sp.z_p, sp.d_dep, 0)
    with pytest.raises(hp.HpmcError) as e:
        g.set_state(pos)
    assert e.value.code == -3


def test_sweep_before_state_is_an_error():
    import paper_1508_07077_amd as hp

    g = hp.Sim(64, 6.9459, 1)
    g.set_shape(hp.SPHERE, [1.0])
    g.ensure_workspace()
    with pytest.raises(hp.HpmcError) as e:
        g.sweep(1)
    assert e.value.code == -5


def test_empty_and_zero_inputs():
    """no particles is an invalid argument; zero sweeps (alone and batched)
    leave the state, the sweep index and the counters untouched"""
    import paper_1508_07077_amd as hp

    with pytest.raises(hp.HpmcError) as e:
        hp.Sim(0, 6.9459, 1)
    assert e.value.code == -1
    sp = wl.c1_spheres_small(1)
    pos, _ = sp.initial_state()
    sims = []
    for _ in range(2):
        g = hp.Sim(sp.n, sp.L, sp.seed)
        g.set_shape(hp.SPHERE, sp.params)
        g.set_fugacity(sp.z_p, sp.d_dep, sp.n_trial)
        g.set_moves(sp.d_trans)
        g.set_state(pos)
        sims.append(g)
    c = sims[0].sweep(0)
    assert all(v == 0 for k, v in c.items() if not k.endswith("_ms"))
    for cb in hp.Batch(sims).sweep(0):
        assert cb["trials"] == 0
    for g in sims:
        p2, _, s2 = g.get_state()
        assert s2 == 0 and np.array_equal(p2, pos)
    with pytest.raises(hp.HpmcError) as e:
        sims[0].sweep(-1)
    assert e.value.code == -1


@pytest.mark.parametrize("n_trial,precision", [(0, 0), (4, 0), (4, 1)])
def test_multi_sweep_call_totals_match_the_oracle(n_trial, precision):
    """25 sweeps in one launch of the small-box kernel (a batched call with
    counters; every wave adds to its counters over all phases and sweeps of
    the launch and flushes once) report the oracle's totals of the decision
    counters, and end in its state"""
    import paper_1508_07077_amd as hp

    sp = wl.c1_spheres_small(n_trial)
    pos, _ = sp.initial_state()
    g, o = make_pair(sp, pos, trace=False, precision=precision)
    cg, co = hp.Batch([g]).sweep(25)[0], o.sweep(25)
    for k in ("trials", "accepts", "rej_cell_exit", "rej_overlap", "rej_depletant", "rej_cb_zero",
              "rej_cb_metropolis", "depletants_drawn", "depletants_resolved", "cb_trials"):
        assert cg[k] == co[k], k
    assert cg["trials"] == 25 * sp.n and cg["accepts"] > 0
    pg, _, sg = g.get_state()
    po, _, so = o.get_state()
    assert sg == so == 25 and np.array_equal(pg, po)


def test_sparse_box_of_514_cells_per_axis():
    """a box of 514 cells per axis (136 M cells, 1,500 unit spheres): cell
    coordinates 512 and 513 take the top bits of the kernel's packed per-lane
    coordinates; a 2 x 2 x 2 cluster in the far corner keeps neighbours,
    depletants and CB trials there; every trial record and the end state
    equal the oracle's"""
    import types

    from scipy.spatial import cKDTree

    L = 514 * 1.1 + 0.05  # d_dep 0.1: cells of width >= 1.1, 514 of them per side
    n = 1500
    rng = np.random.default_rng(51)
    pos = rng.uniform(0.0, L, size=(n, 3))
    while True:
        bad = {j for _, j in cKDTree(pos, boxsize=L).query_pairs(1.0)}
        if not bad:
            break
        for j in bad:
            pos[j] = rng.uniform(0.0, L, 3)
    pos[:8] = [[L - 0.55 - 1.05 * a, L - 0.55 - 1.05 * b, L - 0.55 - 1.05 * c]
               for a in (0, 1) for b in (0, 1) for c in (0, 1)]
    assert not cKDTree(pos, boxsize=L).query_pairs(1.0)
    sp = types.SimpleNamespace(n=n, L=L, seed=7, replica_id=0, kind=wl.SPHERE, params=(1.0,), z_p=15.0, d_dep=0.1,
                               n_trial=1, d_trans=0.3, a_rot=0.0, p_rot=0.0)
    g, o = make_pair(sp, np.ascontiguousarray(pos.T))
    assert g.n_axis == 514
    tot, div = compare_sweeps(g, o, 1)
    assert div == 0 and tot["trials"] == n and tot["accepts"] > 0 and tot["cb_trials"] > 0
    hi = np.floor(pos / (L / 514)).max(axis=0)
    assert (hi >= 512).all()


def test_full_size_c3_sampled_cells():
    """N = 1,048,576 spheres at the benchmark's settings: one traced GPU sweep
    from the generator's lattice; for sampled cells (one per phase) the oracle
    reproduces the cell's trials from the cells that can influence it."""
    import paper_1508_07077_amd as hp
    from oracle import pyoracle

    sp = wl.c3_spheres_large()
    pos, _ = sp.initial_state()
    g = hp.Sim(sp.n, sp.L, sp.seed)
    g.set_shape(hp.SPHERE, sp.params)
    g.set_fugacity(sp.z_p, sp.d_dep, sp.n_trial)
    g.set_moves(sp.d_trans)
    g.set_trace(True)
    g.set_state(pos)
    cg = g.sweep(1)
    tg = g.trace()
    pg, _, _ = g.get_state()
    assert cg["trials"] == sp.n
    rng = np.random.default_rng(0)
    phases = {}
    for r in tg[rng.permutation(len(tg))[:5000]]:
        phases.setdefault(int(r["phase"]), int(r["cell"]))
    assert len(phases) == 8
    for ph, cell in sorted(phases.items())[::3] + [max(phases.items())]:
        o = pyoracle.OracleSim(sp.n, sp.L, sp.seed)
        o.set_shape(pyoracle.SPHERE, sp.params)
        o.set_fugacity(sp.z_p, sp.d_dep, sp.n_trial)
        o.set_moves(sp.d_trans)
        o.set_trace(True)
        o.set_state(pos)
        o.sweep_cone(cell)
        to = o.trace()
        sel = tg["cell"] == cell
        assert sel.sum() > 0
        for f in ("particle", "reason", "n_depletants", "resolved", "n_blocking", "w_fwd", "w_rev", "phase", "t"):
            assert np.array_equal(tg[f][sel], to[f][sel]), (ph, cell, f)
        po, _, _ = o.get_state()
        moved = np.unique(tg["particle"][sel])
        assert np.array_equal(pg[:, moved], po[:, moved])
