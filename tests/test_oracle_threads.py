"""The oracle with OpenMP threads over the active cells of a phase gives the
single-threaded oracle's result bit for bit: cells of one colour share no
stencil cell and each trial moves only a member of its own cell (Sec. III.E),
so the order in which a phase's cells run cannot matter."""
import numpy as np
import pytest

from paper_1508_07077_amd import workloads as wl


def _run(sp, threads, sweeps):
    from oracle import pyoracle

    pos, quat = sp.initial_state()
    o = pyoracle.OracleSim(sp.n, sp.L, sp.seed, sp.replica_id)
    o.set_shape(sp.kind, sp.params)
    o.set_fugacity(sp.z_p, sp.d_dep, sp.n_trial)
    o.set_moves(sp.d_trans, sp.a_rot, sp.p_rot)
    o.set_threads(threads)
    o.set_trace(True)
    o.set_state(pos, quat)
    out = []
    for _ in range(sweeps):
        c = o.sweep(1)
        p, q, sw = o.get_state()
        out.append((c, o.trace().copy(), p, q, sw))
    return out


@pytest.mark.parametrize("case", ["spheres_cb", "hemispheres"])
def test_threads_give_the_serial_result(case):
    if case == "spheres_cb":
        sp = wl.c3_spheres_large(n=4000, d_trans=0.003)
    else:
        sp = wl.c2_hemispheres(0.3, n=1500)
    one = _run(sp, 1, 2)
    many = _run(sp, 4, 2)
    for (c1, t1, p1, q1, s1), (c4, t4, p4, q4, s4) in zip(one, many):
        assert c1 == c4
        assert s1 == s4
        assert np.array_equal(t1, t4)
        assert np.array_equal(p1, p4) and np.array_equal(q1, q4)
    assert one[-1][0]["accepts"] > 0
