"""Dense sphere boxes whose cells hold more than the 64 members the phase
kernel stages in LDS: the members past the stage are read and committed in
place in HBM, and every trial still matches the oracle bit for bit.  The
capacity flag (raised only when a stencil exceeds its packing bound, which
overlap-free states cannot reach) stays clear, and the synchronising calls
that report it succeed after untimed sweeps."""
import numpy as np
import pytest

from paper_1508_07077_amd import workloads as wl
from parity_util import compare_sweeps, make_pair

pytestmark = pytest.mark.gpu


# depletants of diameter 3 to 4.2 make cells 4 to 5.2 wide: two cells per
# axis, about 75 and 106 spheres per cell (no depletant fits between the
# colloids, so every one is ignored; the stage-crossing paths are the proposal,
# the hard-overlap test, the survivor tests and the commit)
@pytest.mark.parametrize("n,phi,q,eta_r,n_trial", [(850, 0.30, 3.0, 1.2, 0), (850, 0.15, 4.0, 2.0, 2),
                                                   (600, 0.12, 4.2, 3.0, 1)])
def test_cells_past_the_stage_match_the_oracle(n, phi, q, eta_r, n_trial):
    sp = wl.StatePoint(wl.SPHERE, (1.0,), n, phi, q, eta_r, n_trial=n_trial, d_trans=0.15, seed=77 + n)
    pos, _ = sp.initial_state()
    g, o = make_pair(sp, pos)
    assert g.n_axis == 2 and n / 8 > 64
    tot, div = compare_sweeps(g, o, 4)
    assert div == 0 and tot["trials"] == 4 * n and tot["accepts"] > 0
    # untimed sweeps (no counters, graph replay), then the synchronising calls
    g.set_trace(False)
    o.set_trace(False)
    g.sweep(5, counters=False)
    o.sweep(5)
    pg, _, sg = g.get_state()
    po, _, so = o.get_state()
    assert sg == so and np.array_equal(pg, po)
    import paper_1508_07077_amd as hp

    fv = g.observables(hp.OBS_FREE_VOLUME, n_probe=2000, obs_seq=3)
    assert 0.0 <= fv[0] <= 1.0
