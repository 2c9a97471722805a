"""Pins of the shell insertion region (Sec. III.C): depletants are drawn only in
B(x', R0) minus the ball B(x', r_in + r_dep - sqrt(3) d_trans), which lies
inside the old pose for every translation of at most sqrt(3) d_trans.

S1  the sampler's points are uniform in the shell: radial CDF
    (r^3 - r_i^3) / (R0^3 - r_i^3) (Kolmogorov-Smirnov), isotropic directions,
    block acceptance (pi/4) E[r^2]/R0^2
S2  the mean number of depletants per move is z_p vol(shell)
S3  a single sphere's acceptance is exp(-z_p [vol V_0 - V_lens(delta)]), the same
    closed form as with the full ball (Eq. transition_prob_final); a move longer
    than the shell allows breaks it (the test can see a wrong region)
S4  forward/backward ratio exp(z_p [V_f(M') - V_f(M)]) for every n_trial
S5  V_0 invariance: with neighbours and configurational bias, ball and shell give
    the same acceptance
S6  the two-sphere Asakura-Oosawa pair density with CB on top of the shell
"""
import math

import numpy as np
import pytest
from scipy import integrate, stats

Q, ETA = 0.25, 0.10
D_DEP = Q * 1.0
Z_P = ETA / (math.pi * D_DEP**3 / 6)
R0 = 0.5 + D_DEP / 2
V_B = 4.0 / 3.0 * math.pi * R0**3


def v_lens(d, R=R0):
    if d >= 2 * R:
        return 0.0
    return math.pi * (4 * R + d) * (2 * R - d) ** 2 / 12.0


def _sim(oracle, n, L, seed=1, n_trial=0, d_trans=0.1, shell=True):
    s = oracle.OracleSim(n, L, seed)
    s.set_shape(oracle.SPHERE, [1.0])
    s.set_fugacity(Z_P, D_DEP, n_trial)
    s.set_moves(d_trans)
    s.set_insertion(oracle.V0_SHELL if shell else oracle.V0_BALL)
    return s


def _binom_close(k, n, p, nsig=4.5):
    return abs(k / n - p) <= nsig * math.sqrt(p * (1 - p) / n)


@pytest.mark.parametrize("r_i", [0.45, 0.0])
def test_s1_shell_sampler_distribution(oracle, r_i):
    rng = np.random.default_rng(11)
    words = rng.integers(0, 2**32, size=(60000, 4), dtype=np.uint64)
    span = R0 - r_i
    pts = []
    for w in words:
        ok, e = oracle.shell_candidate(w, r_i, span, R0 * R0)
        if ok:
            pts.append(e)
    pts = np.array(pts)
    acc = len(pts) / len(words)
    er2 = (R0**3 - r_i**3) / (3.0 * (R0 - r_i) * R0**2)
    p_acc = math.pi / 4 * er2
    assert abs(acc - p_acc) < 4.5 * math.sqrt(p_acc * (1 - p_acc) / len(words))
    r = np.linalg.norm(pts, axis=1)
    assert r.min() >= r_i * (1 - 1e-12) and r.max() < R0
    ks = stats.kstest(r, lambda x: (np.clip(x, r_i, R0) ** 3 - r_i**3) / (R0**3 - r_i**3))
    assert ks.pvalue > 1e-3
    u = pts / r[:, None]
    n = len(u)
    assert np.all(np.abs(u.mean(0)) < 4.5 * math.sqrt(1 / 3 / n))
    cov = u.T @ u / n
    assert np.allclose(cov, np.eye(3) / 3, atol=4.5 * math.sqrt(4 / 45 / n))
    # each octant equally often
    oct_ = (u[:, 0] > 0) + 2 * (u[:, 1] > 0) + 4 * (u[:, 2] > 0)
    assert stats.chisquare(np.bincount(oct_, minlength=8)).pvalue > 1e-3


def test_s2_mean_depletants_per_move(oracle):
    d_trans = 0.05
    s = _sim(oracle, 1, 6.9459, d_trans=d_trans)
    ri = 0.5 + D_DEP / 2 - math.sqrt(3) * d_trans
    lam = Z_P * 4 / 3 * math.pi * (R0**3 - ri**3)
    d = s.derived()
    assert abs(d["r_inner"] - ri) < 1e-12 and abs(d["lambda"] - lam) < 1e-9
    s.set_state(np.array([[2.0], [2.0], [2.0]]))
    n = 40000
    _, ndep = s.try_move_many(0, [2.01, 2.0, 2.0], None, 0, n)
    mean = ndep.mean()
    assert abs(ndep.var() - lam) < 0.1 * lam  # Poisson: variance = mean
    assert abs(mean - lam) < 4.5 * math.sqrt(lam / n)
    # the full ball draws z_p vol(B) per move
    assert lam < 0.6 * Z_P * V_B


@pytest.mark.parametrize("delta", [0.01, 0.05, 0.15])
def test_s3_single_sphere_closed_form(oracle, delta):
    exact = math.exp(-Z_P * (V_B - v_lens(delta)))
    s = _sim(oracle, 1, 6.9459, d_trans=0.1)  # shell valid for |move| <= 0.1732
    s.set_state(np.array([[2.0], [2.0], [2.0]]))
    r, _ = s.try_move_many(0, [2.0 + delta, 2.0, 2.0], None, 0, 200000)
    assert _binom_close(int((r == oracle.ACCEPT).sum()), len(r), exact)


def test_s3_too_long_move_breaks_the_shell(oracle):
    """Negative control: a shell sized for d_trans = 0.01 misses blocking
    depletants of a 0.15 move, so acceptance rises far above the closed form."""
    delta = 0.15
    exact = math.exp(-Z_P * (V_B - v_lens(delta)))
    s = _sim(oracle, 1, 6.9459, d_trans=0.01)
    s.set_state(np.array([[2.0], [2.0], [2.0]]))
    r, _ = s.try_move_many(0, [2.0 + delta, 2.0, 2.0], None, 0, 50000)
    assert (r == oracle.ACCEPT).mean() > exact + 0.1


def _two_sphere_acc(oracle, n_trial, r_from, r_to, count, sweep0=0, shell=True):
    s = _sim(oracle, 2, 6.9459, seed=3, n_trial=n_trial, shell=shell)
    c = 3.0
    s.set_state(np.array([[c, c + r_from], [c, c], [c, c]]))
    rs, _ = s.try_move_many(1, [c + r_to, c, c], None, sweep0, count)
    return int((rs == oracle.ACCEPT).sum())


@pytest.mark.parametrize("n_trial", [0, 1, 4])
def test_s4_forward_backward_ratio(oracle, n_trial):
    n = 300000
    kf = _two_sphere_acc(oracle, n_trial, 1.05, 1.15, n)
    kr = _two_sphere_acc(oracle, n_trial, 1.15, 1.05, n, sweep0=10**7)
    pf, pr = kf / n, kr / n
    exact = math.exp(Z_P * (v_lens(1.15) - v_lens(1.05)))
    if n_trial == 0:
        assert _binom_close(kf, n, 0.22385) and _binom_close(kr, n, 0.31373)
    sig = math.sqrt(pf * (1 - pf) / n) / pr + pf / pr**2 * math.sqrt(pr * (1 - pr) / n)
    assert abs(pf / pr - exact) < 4.5 * sig, (pf / pr, exact)


@pytest.mark.parametrize("n_trial", [0, 4])
def test_s5_region_invariance_with_neighbours(oracle, n_trial):
    L = 5.0
    c = 2.0
    centres = np.array([[c, c, c], [c + 1.05, c, c], [c + 0.6, c + 1.0, c], [c - 0.2, c - 0.9, c + 0.5]]).T.copy()
    new = [c - 0.04, c + 0.03, c - 0.02]
    n = 150000
    acc = {}
    for shell in (False, True):
        s = _sim(oracle, 4, L, seed=21, n_trial=n_trial, shell=shell)
        s.set_state(centres)
        r, _ = s.try_move_many(0, new, None, 0, n)
        acc[shell] = (r == oracle.ACCEPT).mean()
    p = 0.5 * (acc[False] + acc[True])
    sig = math.sqrt(2 * p * (1 - p) / n)
    assert abs(acc[False] - acc[True]) < 4.5 * sig, acc


def _pair_window_probs(edges):
    w = [integrate.quad(lambda r: r * r * math.exp(Z_P * v_lens(r)), a, b)[0] for a, b in zip(edges[:-1], edges[1:])]
    w = np.array(w)
    return w / w.sum()


@pytest.mark.slow
def test_s6_asakura_oosawa_pair_density_shell_cb(oracle):
    L = 2.6
    s = _sim(oracle, 2, L, seed=204, n_trial=4, d_trans=0.15)
    s.set_state(np.array([[0.3, 1.6], [0.3, 1.6], [0.3, 1.6]]))
    s.sweep(500)
    rs = np.empty(160000)
    for i in range(len(rs)):
        s.sweep(3)
        pos, _, _ = s.get_state()
        d = pos[:, 1] - pos[:, 0]
        d -= L * np.round(d / L)
        rs[i] = math.sqrt(float(d @ d))
    assert rs.min() >= 1.0
    edges = np.linspace(1.0, 1.3, 7)
    probs = _pair_window_probs(edges)
    nblk = 20
    fr = []
    for b in rs.reshape(nblk, -1):
        w = b[b < 1.3]
        fr.append(np.histogram(w, bins=edges)[0] / max(len(w), 1))
    fr = np.array(fr)
    mean, err = fr.mean(0), fr.std(0, ddof=1) / math.sqrt(nblk)
    z = (mean - probs) / err
    assert np.all(np.abs(z) < 4.5), (mean.round(4), probs.round(4), z.round(2))


def test_s7_invariants_dense_box(oracle):
    from paper_1508_07077_amd import workloads as wl

    sp = wl.StatePoint(wl.SPHERE, (1.0,), 400, 0.30, 0.10, 0.30, n_trial=4, d_trans=0.05, seed=3)
    s = oracle.OracleSim(sp.n, sp.L, 5)
    s.set_shape(oracle.SPHERE, [1.0])
    s.set_fugacity(sp.z_p, sp.d_dep, sp.n_trial)
    s.set_moves(sp.d_trans)
    s.set_insertion(oracle.V0_SHELL)
    pos, _ = sp.initial_state()
    s.set_state(pos)
    c = s.sweep(5)
    assert s.count_overlaps() == 0
    assert c["trials"] == 5 * sp.n
    assert c["accepts"] + c["rej_cell_exit"] + c["rej_overlap"] + c["rej_depletant"] + c["rej_cb_zero"] + \
        c["rej_cb_metropolis"] == c["trials"]
    assert c["accepts"] > 0
