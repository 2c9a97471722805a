"""Pins of the Poisson depletant number (Sec. III.B step 2: N_p ~ Poisson(z_p vol V_0))."""
import math

import numpy as np
from scipy import stats


def test_table_matches_poisson_cdf(oracle):
    for lam in (0.5, 12.5, 45.06, 199.65, 256.0):
        F = oracle.poisson_table(lam)
        assert F[-1] == 2.0
        k = np.arange(len(F) - 1)
        ref = stats.poisson.cdf(k, lam)
        # forward recursion: relative error grows slowly with k
        assert np.max(np.abs(F[:-1] - ref)) < 1e-11
        assert np.all(np.diff(F[:-1]) >= 0)


def test_draw_is_inverse_cdf(oracle):
    F = oracle.poisson_table(12.5)
    assert oracle.poisson_draw(F, F[0] * 0.5) == 0
    assert oracle.poisson_draw(F, F[0]) == 0
    assert oracle.poisson_draw(F, np.nextafter(F[0], 1.0)) == 1
    assert oracle.poisson_draw(F, F[10]) == 10
    assert oracle.poisson_draw(F, 1.0 - 2**-53) <= len(F) - 1


def test_draw_chi_square(oracle):
    lam = 12.5
    F = oracle.poisson_table(lam)
    rng = np.random.default_rng(11)
    us = (rng.integers(0, 2**52, size=50000) + 0.5) / 2**52
    ks = np.array([oracle.poisson_draw(F, u) for u in us])
    assert abs(ks.mean() - lam) < 4 * math.sqrt(lam / len(ks))
    edges = np.arange(0, 30)
    obs = np.array([(ks == k).sum() for k in edges[:-1]] + [(ks >= edges[-1]).sum()])
    exp = np.concatenate([stats.poisson.pmf(edges[:-1], lam), [stats.poisson.sf(edges[-1] - 1, lam)]]) * len(ks)
    chi2, p = stats.chisquare(obs, exp)
    assert p > 1e-4


def test_depletant_number_mean_and_variance(oracle):
    """<N_p> = z_p vol(V_0) and Var = mean, through the full trial (single sphere)."""
    z_p = 0.10 / (math.pi * 0.25**3 / 6)
    s = oracle.OracleSim(1, 6.9459, 7)
    s.set_shape(oracle.SPHERE, [1.0])
    s.set_fugacity(z_p, 0.25, 0)
    s.set_moves(0.1)
    s.set_state(np.array([[1.0], [1.0], [1.0]]))
    reasons, nd = s.try_move_many(0, [1.0, 1.0, 1.0], None, 0, 100000)
    lam = z_p * 4.0 / 3.0 * math.pi * 0.625**3
    assert abs(nd.mean() - lam) < 4 * math.sqrt(lam / len(nd))
    assert abs(nd.var() / lam - 1.0) < 0.03
    # a null move has no blocking depletant: V'_excl minus V_excl is empty
    assert np.all(reasons == oracle.ACCEPT)


def test_chunked_large_lambda(oracle):
    """lambda above the chunk size is split into equal chunks; the sum is Poisson."""
    z_p = 0.30 / (math.pi * 0.1**3 / 6)
    s = oracle.OracleSim(1, 10.0, 5)
    s.set_shape(oracle.SPHERE, [1.0])
    s.set_fugacity(z_p, 0.1, 0)
    s.set_moves(0.0)
    d = s.derived()
    assert d["n_chunks"] == 2 and abs(d["lambda"] - 399.30) < 0.01
    s.set_state(np.array([[1.0], [1.0], [1.0]]))
    _, nd = s.try_move_many(0, [1.0, 1.0, 1.0], None, 0, 20000)
    assert abs(nd.mean() - d["lambda"]) < 4 * math.sqrt(d["lambda"] / len(nd))
    assert abs(nd.var() / d["lambda"] - 1.0) < 0.06
