"""The chunk-count table the kernels load is a compact copy of the inverse CDF
(the entries a 52-bit uniform can stop at, and a sentinel for the last
index).  Through hpmc_poisson_draw — the kernels' scan on the table they load,
run on the host — every draw equals the oracle's scan of its full table
(Sec. III.B, step 2): at each table value, its neighbours in the last place,
both ends of the uniform's range and, where the running sum stops below one,
the uniforms above it (no GPU)."""
import ctypes
import math

import numpy as np
import pytest

from oracle import pyoracle

UMIN, UMAX = 2.0 ** -53, 1.0 - 2.0 ** -53
L_BOX, D_DEP = 20.0, 0.1
VOL0 = 4.0 / 3.0 * math.pi * (0.5 + 0.5 * D_DEP) ** 3
# chunk means from 0 to just under 256, and sums of several chunks
Z_P = [0.0, 1.0, 17.9, 143.5, 287.0, 358.8, 365.9, 2869.8, 30000.0]


def _handle(z_p):
    import paper_1508_07077_amd as hp

    lib = hp.lib()
    h = ctypes.c_void_p()
    assert lib.hpmc_create(ctypes.byref(h), 100, L_BOX, 1, 0, 0, None) == 0
    one = np.array([1.0])
    assert lib.hpmc_set_shape(h, 0, one.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 1) == 0
    assert lib.hpmc_set_fugacity(h, z_p, D_DEP, 0) == 0
    return lib, h


def _uniforms(F, rng):
    us = {UMIN, UMAX, 0.5}
    for f in F[:-1]:
        for v in (f, np.nextafter(f, 0.0), np.nextafter(f, 2.0)):
            if UMIN <= v <= UMAX:
                us.add(float(v))
    top = F[-2]  # the running sum where it stops growing
    if top < UMAX:
        us |= {float(np.nextafter(top, 2.0)), UMAX, float((top + UMAX) / 2)}
    us |= set(rng.uniform(UMIN, UMAX, 2000).tolist())
    return sorted(us)


@pytest.mark.parametrize("z_p", Z_P)
def test_compact_table_draws_equal_the_oracle(z_p):
    o = pyoracle.OracleSim(100, L_BOX, 1)
    o.set_shape(pyoracle.SPHERE, (1.0,))
    o.set_fugacity(z_p, D_DEP, 0)
    lam_c = o.derived()["lambda_c"]
    F = pyoracle.poisson_table(lam_c)
    lib, h = _handle(z_p)
    k = ctypes.c_int32(0)
    rng = np.random.default_rng(int(z_p * 10) + 1)
    try:
        for u in _uniforms(F, rng):
            assert lib.hpmc_poisson_draw(h, u, ctypes.byref(k)) == 0
            assert k.value == pyoracle.poisson_draw(F, u), (z_p, lam_c, u)
    finally:
        lib.hpmc_destroy(h)


def test_both_kinds_of_table_end_are_covered():
    """some tables reach 1 - 2^-53, others stop growing below it (then the
    largest uniforms draw the last index)"""
    tops = []
    for z_p in Z_P[1:]:
        o = pyoracle.OracleSim(100, L_BOX, 1)
        o.set_shape(pyoracle.SPHERE, (1.0,))
        o.set_fugacity(z_p, D_DEP, 0)
        tops.append(pyoracle.poisson_table(o.derived()["lambda_c"])[-2])
    assert any(t < UMAX for t in tops) and any(t >= UMAX for t in tops)


def test_draw_argument_checks():
    lib, h = _handle(100.0)
    k = ctypes.c_int32(0)
    try:
        assert lib.hpmc_poisson_draw(h, 0.0, ctypes.byref(k)) == -1
        assert lib.hpmc_poisson_draw(h, 1.0, ctypes.byref(k)) == -1
        assert lib.hpmc_poisson_draw(None, 0.5, ctypes.byref(k)) == -1
    finally:
        lib.hpmc_destroy(h)
