"""Parity at the benchmark's full sizes, in the launch configurations the
benchmark times: a whole sweep of the 1,048,576 spheres, 16,384 hemispheres
swept by one handle, and the 256 swept-disk replicas swept together in shared
launches, each against the oracle run on the same inputs.  A trial decided within 1e-9 of a colloid
contact by either side's own convex test (MPR on the GPU, GJK in the oracle)
may differ, and so may what follows from it in its light cone (the rule of
parity_util); every other decision, count and coordinate is bit-exact."""
import numpy as np
import pytest

from paper_1508_07077_amd import workloads as wl
from parity_util import compare_sweeps, make_pair, near_contact_explains

pytestmark = pytest.mark.gpu


def test_full_size_spheres_whole_sweep():
    """the 1,048,576-sphere workload: one whole sweep, all 1,048,576 trials
    compared record by record (sphere tests are exact: no tolerance)"""
    sp = wl.c3_spheres_large()
    pos, _ = sp.initial_state()
    g, o = make_pair(sp, pos)
    tot, div = compare_sweeps(g, o, 1)
    assert div == 0
    assert tot["trials"] == sp.n and tot["cb_trials"] > 0


@pytest.mark.parametrize("eta_r", [0.1, 0.4])
def test_full_size_hemispheres(eta_r):
    sp = wl.c2_hemispheres(eta_r)
    pos, quat = sp.initial_state()
    g, o = make_pair(sp, pos, quat)
    tot, div = compare_sweeps(g, o, 2, allow_near=True)
    assert tot["trials"] == 2 * sp.n
    assert div <= 1
    assert tot["accepts"] > 0 and tot["rej_depletant"] > 0


def test_full_size_discoid_replicas_batched():
    import paper_1508_07077_amd as hp
    from oracle import pyoracle

    sps = wl.c4_discoid_replicas()
    sims, oracles = [], []
    for sp in sps:
        pos, quat = sp.initial_state()
        g = hp.Sim(sp.n, sp.L, sp.seed, sp.replica_id)
        o = pyoracle.OracleSim(sp.n, sp.L, sp.seed, sp.replica_id)
        for s in (g, o):
            s.set_shape(sp.kind, sp.params)
            s.set_fugacity(sp.z_p, sp.d_dep, sp.n_trial)
            s.set_moves(sp.d_trans, sp.a_rot, sp.p_rot)
            s.set_state(pos, quat)
        sims.append(g)
        oracles.append(o)
    cb = hp.Batch(sims).sweep(1)
    differing = 0
    for g, o, c, sp in zip(sims, oracles, cb, sps):
        co = o.sweep(1)
        pg, qg, sg = g.get_state()
        po, qo, so = o.get_state()
        assert sg == so == 1
        same = np.array_equal(pg, po) and np.array_equal(qg, qo)
        if same:
            for k in ("trials", "accepts", "rej_overlap", "rej_depletant", "depletants_drawn", "depletants_resolved"):
                assert c[k] == co[k], (sp.name, k)
            continue
        # A differing replica: sweep it again alone, traced, from the same start
        # on both sides.  The lone GPU sweep must end where the batched one did
        # (a replica's trajectory does not depend on the batch), and every
        # difference from the oracle must follow from near-contact trials.
        differing += 1
        pos, quat = sp.initial_state()
        g1, o1 = make_pair(sp, pos, quat)
        g1.sweep(1)
        o1.sweep(1)
        p1, q1, _ = g1.get_state()
        assert np.array_equal(p1, pg) and np.array_equal(q1, qg), sp.name
        po1, qo1, _ = o1.get_state()
        why = near_contact_explains(g1.trace(), o1.trace(), g1.n_axis, np.vstack([p1, q1]), np.vstack([po1, qo1]))
        assert why is None, (sp.name, why)
    assert differing <= 8
    assert sum(c["trials"] for c in cb) == sum(sp.n for sp in sps)
