"""Ensemble averages of independent chains: the GPU chain (one seed) and the
oracle chain (another seed) sample the same semigrand ensemble, so their
averages of the free-volume fraction alpha, the contact value of g(r) and
the SDF pressure agree within statistical error (blocking errors of the
correlated samples; a 3-sigma bound keeps the false-failure rate of the
three comparisons below 1 %)."""
import math

import numpy as np
import pytest

from paper_1508_07077_amd import workloads as wl

pytestmark = pytest.mark.gpu

SP = wl.StatePoint(wl.SPHERE, (1.0,), 216, 0.20, 0.25, 0.15, n_trial=0, d_trans=0.12, seed=41)
NB, RMAX = 30, 2.5


def _series(sim, samples, every):
    from oracle import pyoracle

    a, g1, bp = [], [], []
    for k in range(samples):
        if isinstance(sim, pyoracle.OracleSim):
            sim.sweep(every)
        else:
            sim.sweep(every, counters=False)
        g = sim.observables(pyoracle.OBS_GR, n_bins=NB, r_max=RMAX)
        fv = sim.observables(pyoracle.OBS_FREE_VOLUME, n_probe=8000, obs_seq=100 + k)
        sdf = sim.observables(pyoracle.OBS_SDF, n_bins=20, x_max=0.05, n_fit=6, n_probe=8000, obs_seq=5000 + k,
                              eps=0.01)
        a.append(fv[0])
        g1.append(g[int(1.0 / (RMAX / NB))])  # the bin just outside contact
        bp.append(sdf[0])
    return np.array(a), np.array(g1), np.array(bp)


def _blocked(x, nblk=10):
    b = x[: len(x) // nblk * nblk].reshape(nblk, -1).mean(1)
    return b.mean(), b.std(ddof=1) / math.sqrt(nblk)


def test_gpu_and_oracle_chains_sample_the_same_ensemble():
    import paper_1508_07077_amd as hp
    from oracle import pyoracle

    pos, _ = SP.initial_state()
    g = hp.Sim(SP.n, SP.L, seed=1001)
    o = pyoracle.OracleSim(SP.n, SP.L, 2002)
    for s in (g, o):
        s.set_shape(SP.kind, SP.params)
        s.set_fugacity(SP.z_p, SP.d_dep, SP.n_trial)
        s.set_moves(SP.d_trans)
    g.set_state(pos)
    o.set_state(pos)
    g.sweep(200, counters=False)
    o.sweep(200)
    sg = _series(g, 120, 10)
    so = _series(o, 120, 10)
    for name, xg, xo in zip(("alpha", "g(contact)", "beta P"), sg, so):
        mg, eg = _blocked(xg)
        mo, eo = _blocked(xo)
        z = (mg - mo) / math.sqrt(eg**2 + eo**2)
        assert abs(z) < 3.0, (name, mg, eg, mo, eo)


@pytest.mark.parametrize("n_trial", [0, 4])
def test_ball_and_shell_regions_sample_the_same_ensemble(n_trial):
    """The insertion region changes the random streams, not the ensemble."""
    import paper_1508_07077_amd as hp

    pos, _ = SP.initial_state()
    series = []
    for region, seed in ((hp.V0_BALL, 3003), (hp.V0_SHELL, 4004)):
        g = hp.Sim(SP.n, SP.L, seed=seed)
        g.set_shape(SP.kind, SP.params)
        g.set_fugacity(SP.z_p, SP.d_dep, n_trial)
        g.set_moves(SP.d_trans)
        g.set_insertion(region)
        g.set_state(pos)
        g.sweep(200, counters=False)
        series.append(_series(g, 200, 10))
    for name, xb, xs in zip(("alpha", "g(contact)", "beta P"), *series):
        mb, eb = _blocked(xb)
        ms, es = _blocked(xs)
        z = (mb - ms) / math.sqrt(eb**2 + es**2)
        assert abs(z) < 3.0, (name, n_trial, mb, eb, ms, es)
