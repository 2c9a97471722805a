"""Pins of the oracle's Monte Carlo chain for oriented colloids (hemispheres,
Sec. V.A; swept disks standing in for the discoids of Sec. V.B).

The sphere pins (P1, P3, P6) fix the chain's logic only where the old and new
poses differ by a translation of a rotation-free body.  These pins repeat them
for bodies with an orientation, where the trial must tell the new pose (with
its new rotation) from the old one (with the old rotation):

O1  single body, fixed translation or rotation, n_trial = 0: acceptance
    exp(-z_p vol(E' minus E)), E and E' the excluded regions (points within
    d_dep/2 of the body) of the old and the new pose       (Eq. transition_prob_final)
O2  single body, configurational bias (n_trial 1 and 4): acceptance equals the
    exact enumeration over W' ~ Bin(n_trial, f_fwd), W ~ Bin(n_trial - 1, f_rev)
    with f_fwd = vol(E minus E') / vol(B), f_rev = vol(E' minus E) / vol(B)
                                                             (Sec. III.D, Eq. pacc_cb)
O3  two bodies, forward/backward acceptance ratio exp(z_p [V_f(M') - V_f(M)])
    for n_trial 0, 1, 4; V_f(M') - V_f(M) = vol(E'_i with E_j) - vol(E_i with E_j)
                                                             (Eq. detailed_bal_product)
O4  the rotation proposal q' = (q + a v)/|q + a v| is symmetric: with no
    depletants a lone body's orientation becomes uniform on the unit
    quaternions, and the flux between orientation bins is the same both ways
                                                             (Sec. III.B: symmetric proposals)

The volumes come from a seeded Monte Carlo quadrature written here in numpy:
rotations through scipy's own quaternion code (scalar-last), and distances to
the body core from closest points (the half ball, the bare disk).  That
distance test is checked first against the oracle's predicate, itself pinned
against dense point clouds in test_oracle_shapes.py.
"""
import math

import numpy as np
import pytest
from scipy import stats
from scipy.spatial.transform import Rotation

HEMI = dict(kind=1, params=[1.0], d_dep=0.15, z_p=0.1 / (math.pi * 0.15**3 / 6))   # eta_r 0.1, q 0.15
DISC = dict(kind=2, params=[0.5, 0.1], d_dep=0.2, z_p=0.2 / (math.pi * 0.2**3 / 6))  # eta_r 0.2, q 0.2


def _rot(q_wxyz):
    w, x, y, z = q_wxyz
    return Rotation.from_quat([x, y, z, w])


def _unit(q):
    q = np.asarray(q, dtype=float)
    return q / np.linalg.norm(q)


def _rcirc(sh):
    return 0.5 * sh["params"][0] if sh["kind"] == 1 else sh["params"][0] + sh["params"][1]


def _core_dist(sh, p):
    """distance of body-frame points p (n, 3) to the body core: the solid half
    ball (hemisphere, face at z = 0, dome toward +z) or the bare disk of the
    swept disk"""
    px, py, pz = p[:, 0], p[:, 1], p[:, 2]
    rho = np.hypot(px, py)
    if sh["kind"] == 1:
        a = 0.5 * sh["params"][0]
        # above the face plane the closest point of the half ball is that of the whole ball
        up = np.maximum(np.linalg.norm(p, axis=1) - a, 0.0)
        # below it the closest point lies in the face disk
        down = np.hypot(np.maximum(rho - a, 0.0), pz)
        return np.where(pz >= 0.0, up, down)
    a = sh["params"][0]
    return np.hypot(np.maximum(rho - a, 0.0), pz)


def _threshold(sh):
    """a depletant overlaps the body when its centre is closer than this to the core"""
    r_dep = 0.5 * sh["d_dep"]
    return r_dep if sh["kind"] == 1 else sh["params"][1] + r_dep


def _in_excluded(sh, y, x, q):
    """points y (n, 3) inside the excluded region of the body at x with orientation q"""
    p = _rot(q).inv().apply(y - np.asarray(x))
    return _core_dist(sh, p) < _threshold(sh)


def _quadrature(sh, centre, regions, n=8_000_000, seed=0, chunk=1_000_000):
    """Monte Carlo volumes (and standard errors) of boolean combinations of
    excluded regions, all inside the ball of radius R0 about `centre`.
    regions: dict name -> function(inside) of a dict of membership arrays."""
    R0 = _rcirc(sh) + 0.5 * sh["d_dep"]
    rng = np.random.default_rng(seed)
    side = 2.0 * R0
    counts = {k: 0 for k in regions}
    done = 0
    while done < n:
        m = min(chunk, n - done)
        y = np.asarray(centre) + rng.uniform(-R0, R0, size=(m, 3))
        for k, f in regions.items():
            counts[k] += int(np.count_nonzero(f(y)))
        done += m
    vol = side**3
    out = {}
    for k, c in counts.items():
        p = c / n
        out[k] = (vol * p, vol * math.sqrt(p * (1 - p) / n))
    return out


def _sim(oracle, sh, pos, quat, n_trial=0, L=8.0, seed=11):
    s = oracle.OracleSim(pos.shape[1], L, seed)
    s.set_shape(sh["kind"], sh["params"])
    s.set_fugacity(sh["z_p"], sh["d_dep"], n_trial)
    s.set_moves(0.05, 0.05, 0.5)
    s.set_state(pos, quat)
    return s


def _close(k, n, p, sig_p, nsig=4.5):
    sig = math.sqrt(p * (1 - p) / n + sig_p**2)
    return abs(k / n - p) <= nsig * sig, (k / n, p, sig)


def test_core_distance_matches_the_oracle_predicate(oracle):
    """the quadrature's numpy test decides like the oracle's (point-cloud pinned) predicate"""
    rng = np.random.default_rng(3)
    for sh in (HEMI, DISC):
        q = _unit(rng.standard_normal(4))
        R0 = _rcirc(sh) + 0.5 * sh["d_dep"]
        v = rng.uniform(-R0, R0, size=(4000, 3))
        mine = _in_excluded(sh, v, np.zeros(3), q)
        d = _core_dist(sh, _rot(q).inv().apply(v))
        checked = 0
        for vi, mi, di in zip(v, mine, d):
            if abs(di - _threshold(sh)) < 1e-9:
                continue
            assert oracle.depletant_overlap(sh["kind"], sh["params"], 0.5 * sh["d_dep"], vi, q) == bool(mi)
            checked += 1
        assert checked > 3900 and 0 < mine.sum() < len(mine)


# fixed moves of one body at x0 with orientation q0: a translation, and a
# rotation about the reference point
X0 = np.array([4.0, 4.0, 4.0])
Q0 = _unit([0.9, 0.2, -0.3, 0.25])
# step sizes give acceptances between about 0.2 and 0.4 without configurational bias
MOVES = {
    ("hemisphere", "translate"): (X0 + np.array([0.025, -0.014, 0.021]), Q0),
    ("hemisphere", "rotate"): (X0, _unit(Q0 + 0.08 * np.array([0.3, -0.5, 0.6, 0.4]))),
    ("discoid", "translate"): (X0 + np.array([0.025, -0.014, 0.021]), Q0),
    ("discoid", "rotate"): (X0, _unit(Q0 + 0.04 * np.array([0.3, -0.5, 0.6, 0.4]))),
}


def _single_volumes(sh, xn, qn, seed):
    return _quadrature(sh, xn, {
        "new_not_old": lambda y: _in_excluded(sh, y, xn, qn) & ~_in_excluded(sh, y, X0, Q0),
    }, seed=seed) | _quadrature(sh, X0, {
        "old_not_new": lambda y: _in_excluded(sh, y, X0, Q0) & ~_in_excluded(sh, y, xn, qn),
    }, seed=seed + 1)


@pytest.mark.parametrize("shape", ["hemisphere", "discoid"])
@pytest.mark.parametrize("move", ["translate", "rotate"])
def test_o1_single_body_acceptance(oracle, shape, move):
    sh = HEMI if shape == "hemisphere" else DISC
    xn, qn = MOVES[shape, move]
    vols = _single_volumes(sh, xn, qn, seed=10)
    V, sV = vols["new_not_old"]
    exact = math.exp(-sh["z_p"] * V)
    s = _sim(oracle, sh, X0.reshape(3, 1).copy(), Q0.reshape(4, 1).copy())
    n = 200000
    r, nd = s.try_move_many(0, xn, qn, 0, n)
    ok, info = _close(int((r == oracle.ACCEPT).sum()), n, exact, exact * sh["z_p"] * sV)
    assert ok, info
    assert 0.15 < exact < 0.5  # an informative test: neither always nor never accepted
    # every proposal drew Poisson(z_p vol B(x', R0)) depletants
    R0 = _rcirc(sh) + 0.5 * sh["d_dep"]
    lam = sh["z_p"] * 4.0 / 3.0 * math.pi * R0**3
    assert abs(nd.mean() - lam) < 5 * math.sqrt(lam / n)


def _cb_enumerate(lam_block, f_fwd, f_rev, n_trial, m_max=80):
    """E[min(1, prod_k W'_k / (1 + W_k))]: m ~ Poisson(lam_block) blocking
    depletants, W'_k ~ Bin(n_trial, f_fwd), W_k ~ Bin(n_trial - 1, f_rev),
    W'_k = 0 rejects.  The product's distribution is kept exactly (fractions)."""
    from fractions import Fraction

    fac = {}
    for wf in range(1, n_trial + 1):
        pf = stats.binom.pmf(wf, n_trial, f_fwd)
        for wr in range(0, n_trial):
            pr = stats.binom.pmf(wr, n_trial - 1, f_rev) if n_trial > 1 else (1.0 if wr == 0 else 0.0)
            if pr == 0.0:
                continue
            key = Fraction(wf, 1 + wr)
            fac[key] = fac.get(key, 0.0) + pf * pr
    total = 0.0
    dist = {Fraction(1): 1.0}
    for m in range(m_max):
        pm = stats.poisson.pmf(m, lam_block)
        total += pm * sum(p * min(1.0, float(v)) for v, p in dist.items())
        nd = {}
        for v, p in dist.items():
            for fv, fp in fac.items():
                k = v * fv
                nd[k] = nd.get(k, 0.0) + p * fp
        dist = {k: p for k, p in nd.items() if p > 1e-300}
        if pm < 1e-16 and m > lam_block:
            break
    return total


# larger moves, so that a re-insertion often lands in E minus E' (f of 0.17 to
# 0.41), at a fugacity that puts about 2.5 blocking depletants in E' minus E
MOVES_CB = {
    ("hemisphere", "translate"): (X0 + np.array([0.35, -0.2, 0.3]), Q0),
    ("hemisphere", "rotate"): (X0, _unit(Q0 + 0.8 * np.array([0.3, -0.5, 0.6, 0.4]))),
    ("discoid", "translate"): (X0 + np.array([0.35, -0.2, 0.3]), Q0),
    ("discoid", "rotate"): (X0, _unit(Q0 + 0.8 * np.array([0.3, -0.5, 0.6, 0.4]))),
}


@pytest.mark.parametrize("shape,move,n_trial", [("hemisphere", "rotate", 1), ("hemisphere", "rotate", 4),
                                                ("hemisphere", "translate", 4), ("discoid", "rotate", 4),
                                                ("discoid", "translate", 1)])
def test_o2_single_body_configurational_bias(oracle, shape, move, n_trial):
    xn, qn = MOVES_CB[shape, move]
    sh = dict(HEMI if shape == "hemisphere" else DISC)
    vols = _single_volumes(sh, xn, qn, seed=20)
    R0 = _rcirc(sh) + 0.5 * sh["d_dep"]
    vb = 4.0 / 3.0 * math.pi * R0**3
    (Vn, sVn), (Vo, sVo) = vols["new_not_old"], vols["old_not_new"]
    # a rigid motion keeps the excluded volume: the two differences agree
    assert abs(Vn - Vo) < 5 * math.hypot(sVn, sVo)
    sh["z_p"] = round(2.5 / Vn, 3)
    exact = _cb_enumerate(sh["z_p"] * Vn, Vo / vb, Vn / vb, n_trial)
    # quadrature uncertainty, propagated by re-evaluating at the volumes moved by one error
    hi = _cb_enumerate(sh["z_p"] * (Vn + sVn), (Vo + sVo) / vb, (Vn + sVn) / vb, n_trial)
    s = _sim(oracle, sh, X0.reshape(3, 1).copy(), Q0.reshape(4, 1).copy(), n_trial=n_trial)
    n = 200000
    r, _ = s.try_move_many(0, xn, qn, 0, n)
    ok, info = _close(int((r == oracle.ACCEPT).sum()), n, exact, abs(hi - exact))
    assert ok, info
    # configurational bias raises the acceptance above the plain scheme's
    assert exact > 1.3 * math.exp(-sh["z_p"] * Vn), (exact, math.exp(-sh["z_p"] * Vn))


# two bodies: body j fixed at the origin's neighbourhood, body i moved
def _two_body(shape):
    if shape == "hemisphere":
        sh = HEMI
        xj, qj = np.array([4.0, 4.0, 4.0]), _unit([1.0, 0.0, 0.0, 0.0])   # dome toward +z
        qi = _unit([0.0, 1.0, 0.0, 0.0])                                   # dome toward -z
        xi = np.array([4.02, 3.99, 3.90])                                  # faces 0.10 apart
        xi2, qi2 = np.array([4.0, 4.01, 3.885]), _unit(qi + 0.06 * np.array([0.2, 0.1, -0.7, 0.5]))
    else:
        sh = DISC
        xj, qj = np.array([4.0, 4.0, 4.0]), _unit([1.0, 0.0, 0.0, 0.0])   # disk in the xy plane
        qi = _unit([0.995, 0.06, 0.05, 0.0])                               # nearly parallel
        xi = np.array([4.05, 3.97, 4.29])                                  # stacked, 0.29 apart
        xi2, qi2 = np.array([4.03, 3.99, 4.305]), _unit(qi + 0.05 * np.array([0.1, -0.6, 0.3, 0.4]))
    return sh, (xj, qj), (xi, qi), (xi2, qi2)


@pytest.mark.parametrize("shape", ["hemisphere", "discoid"])
@pytest.mark.parametrize("n_trial", [0, 1, 4])
def test_o3_two_body_forward_backward_ratio(oracle, shape, n_trial):
    sh, (xj, qj), (xi, qi), (xi2, qi2) = _two_body(shape)
    # the free-volume change: only the overlap of the two excluded regions changes
    vols = _quadrature(sh, xj, {
        "before": lambda y: _in_excluded(sh, y, xj, qj) & _in_excluded(sh, y, xi, qi),
        "after": lambda y: _in_excluded(sh, y, xj, qj) & _in_excluded(sh, y, xi2, qi2),
        "diff": lambda y: _in_excluded(sh, y, xj, qj) & (_in_excluded(sh, y, xi2, qi2) ^ _in_excluded(sh, y, xi, qi)),
    }, seed=30)
    dV = vols["after"][0] - vols["before"][0]
    sdV = vols["diff"][1]  # the error of the difference: the points that change sides
    exact = math.exp(sh["z_p"] * dV)
    assert abs(math.log(exact)) > 0.3  # the move changes the free volume noticeably
    pos = np.stack([xj, xi], axis=1)
    quat = np.stack([qj, qi], axis=1)
    pos2 = np.stack([xj, xi2], axis=1)
    quat2 = np.stack([qj, qi2], axis=1)
    fwd = _sim(oracle, sh, pos, quat, n_trial=n_trial, seed=5)
    rev = _sim(oracle, sh, pos2, quat2, n_trial=n_trial, seed=5)
    assert fwd.count_overlaps() == 0 and rev.count_overlaps() == 0
    n = 300000
    rf, _ = fwd.try_move_many(1, xi2, qi2, 0, n)
    rr, _ = rev.try_move_many(1, xi, qi, 10**7, n)
    pf, pr = (rf == oracle.ACCEPT).mean(), (rr == oracle.ACCEPT).mean()
    ratio = pf / pr
    sig = ratio * math.sqrt((1 - pf) / (pf * n) + (1 - pr) / (pr * n) + (sh["z_p"] * sdV) ** 2)
    assert abs(ratio - exact) < 4.5 * sig, (ratio, exact, sig, pf, pr)


def _s3_marginal_cdf(w):
    """CDF of one component of a uniform unit quaternion: density (2/pi) sqrt(1 - w^2)"""
    w = np.clip(w, -1.0, 1.0)
    return 0.5 + (w * np.sqrt(1 - w * w) + np.arcsin(w)) / math.pi


@pytest.mark.parametrize("shape", ["hemisphere", "discoid"])
def test_o4_rotation_proposal_is_symmetric(oracle, shape):
    """z_p = 0, one body, rotations only: the chain's stationary orientation
    distribution is uniform on the unit quaternions (up to sign), and
    transitions between orientation bins balance."""
    sh = dict(HEMI if shape == "hemisphere" else DISC)
    s = oracle.OracleSim(1, 8.0, 77)
    s.set_shape(sh["kind"], sh["params"])
    s.set_fugacity(0.0, sh["d_dep"], 0)
    s.set_moves(0.05, 0.4, 1.0)
    s.set_state(np.array([[4.0], [4.0], [4.0]]), np.array([[1.0], [0.0], [0.0], [0.0]]))
    # thinned samples for the distribution
    s.sweep(200)
    samples = []
    for _ in range(3000):
        s.sweep(40)
        _, q, _ = s.get_state()
        samples.append(q[:, 0].copy())
    Q = np.array(samples)
    assert np.allclose(np.linalg.norm(Q, axis=1), 1.0, atol=1e-12)
    for comp in range(4):
        assert stats.kstest(Q[:, comp], _s3_marginal_cdf).pvalue > 1e-3, comp
    # the body axis is uniform on the sphere: its z component is uniform in [-1, 1]
    axis_z = Rotation.from_quat(Q[:, [1, 2, 3, 0]]).apply([0.0, 0.0, 1.0])[:, 2]
    assert stats.kstest(axis_z, stats.uniform(-1, 2).cdf).pvalue > 1e-3
    # consecutive states: flux between four bins of the axis z component
    bins = np.linspace(-1, 1, 5)
    prev = None
    flux = np.zeros((4, 4))
    for _ in range(60000):
        s.sweep(1)
        _, q, _ = s.get_state()
        b = min(3, int(np.searchsorted(bins, _rot(q[:, 0]).apply([0, 0, 1.0])[2], side="right") - 1))
        if prev is not None:
            flux[prev, b] += 1
        prev = b
    for a in range(4):
        for b in range(a + 1, 4):
            n_ab, n_ba = flux[a, b], flux[b, a]
            if n_ab + n_ba < 50:
                continue
            # the two counts split binomially around one half
            z = (n_ab - n_ba) / math.sqrt(n_ab + n_ba)
            assert abs(z) < 4.5, (a, b, n_ab, n_ba)
    assert flux.sum() - np.trace(flux) > 1000  # the orientation does move between bins


def _proposals(oracle, q0, n, seed):
    """n rotation proposals from q0, one per stream (sweep index), all accepted"""
    sh = HEMI
    s = oracle.OracleSim(1, 8.0, seed)
    s.set_shape(sh["kind"], sh["params"])
    s.set_fugacity(0.0, sh["d_dep"], 0)
    s.set_moves(0.05, 0.3, 1.0)
    pos = np.array([[4.0], [4.0], [4.0]])
    Q = np.empty((n, 4))
    for k in range(n):
        s.set_state(pos, q0.reshape(4, 1), k)
        s.sweep(1)
        Q[k] = s.get_state()[1][:, 0]
    return Q


def test_o4_rotation_proposal_is_isotropic(oracle):
    """One rotation proposal from a fixed q0 on many streams (one body, z_p = 0,
    so every proposal is accepted): the direction of the step in the tangent
    space of q0 is uniform on the unit sphere (each coordinate uniform in
    [-1, 1]), and the step's angle has the same distribution from any q0.  A
    proposal density that depends only on q.q' is symmetric, which is what the
    acceptance rule assumes (Sec. III.B)."""
    rng = np.random.default_rng(9)
    cos = {}
    for base, q0 in (("identity", np.array([1.0, 0.0, 0.0, 0.0])), ("random", _unit(rng.standard_normal(4)))):
        Q = _proposals(oracle, q0, 12000, 123 if base == "identity" else 321)
        # an orthonormal basis of the tangent space at q0
        B = np.linalg.qr(np.column_stack([q0, rng.standard_normal((4, 3))]))[0][:, 1:]
        t = Q @ B
        u = t / np.linalg.norm(t, axis=1, keepdims=True)
        for c in range(3):
            assert stats.kstest(u[:, c], stats.uniform(-1, 2).cdf).pvalue > 1e-3, (base, c)
        cos[base] = np.clip(Q @ q0, -1, 1)
        assert np.all(cos[base] > 0.5) and cos[base].mean() < 0.999
    assert stats.ks_2samp(cos["identity"], cos["random"]).pvalue > 1e-3
