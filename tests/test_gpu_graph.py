"""Untimed multi-sweep calls replay one captured sweep (hipGraph).  The replay
must give, call after call, exactly the eagerly launched trajectory, with the
program's own eager work and synchronisations between the replays."""
import numpy as np
import pytest

from paper_1508_07077_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _pair(sp):
    import paper_1508_07077_amd as hp

    pos, quat = sp.initial_state()
    out = []
    for _ in range(2):
        g = hp.Sim(sp.n, sp.L, sp.seed)
        g.set_shape(sp.kind, sp.params)
        g.set_fugacity(sp.z_p, sp.d_dep, sp.n_trial)
        g.set_moves(sp.d_trans, sp.a_rot, sp.p_rot)
        g.set_state(pos, quat)
        out.append(g)
    return out


@pytest.mark.parametrize("sp", [wl.c1_spheres_small(4),
                                wl.StatePoint(wl.HEMISPHERE, (1.0,), 200, 0.15, 0.15, 0.2, d_trans=0.05, a_rot=0.05,
                                              p_rot=0.5, seed=5)], ids=["spheres", "hemispheres"])
def test_graph_replay_equals_eager(sp):
    graph, eager = _pair(sp)
    for call in range(5):
        graph.sweep(3, counters=False)          # captured once, replayed 3x per call
        for _ in range(3):
            eager.sweep(1, counters=True)       # timed path: eager launches
        pg, qg, sg = graph.get_state()          # synchronises between replays
        pe, qe, se = eager.get_state()
        assert sg == se == 4 * call + 3
        assert np.array_equal(pg, pe), call
        if qg is not None:
            assert np.array_equal(qg, qe), call
        # eager work on the graph's handle between replays
        graph.sweep(1, counters=True)
        eager.sweep(1, counters=True)
