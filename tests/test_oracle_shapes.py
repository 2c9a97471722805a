"""Pins of the oracle's overlap predicates against brute force on dense point
sets.  The paper gives no overlap algorithm (it only names the shapes: spheres,
hemispheres Sec. V.A, discoids Sec. V.B); the predicates are the contract's
exact distance tests and a GJK distance bracket for colloid pairs.  Rotations
in these tests go through scipy's own quaternion code (scalar-last)."""
import math

import numpy as np
import pytest
from scipy.spatial import cKDTree
from scipy.spatial.transform import Rotation

R_DEP = 0.075


def _rot(q_wxyz):
    w, x, y, z = q_wxyz
    return Rotation.from_quat([x, y, z, w])


def _rand_quat(rng):
    q = rng.standard_normal(4)
    return q / np.linalg.norm(q)


def _fib_hemisphere(a, n):
    i = np.arange(n) + 0.5
    z = i / n  # uniform in z on (0, 1): uniform area on the dome
    phi = i * math.pi * (3.0 - math.sqrt(5.0))
    r = np.sqrt(1 - z * z)
    return a * np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)


def _disk_grid(a, h):
    g = np.arange(-a, a + h, h)
    X, Y = np.meshgrid(g, g)
    m = X**2 + Y**2 <= a * a
    # plus the rim, so the sampled set reaches the edge
    th = np.linspace(0, 2 * math.pi, int(2 * math.pi * a / h) + 1, endpoint=False)
    rim = np.stack([a * np.cos(th), a * np.sin(th)], axis=1)
    pts = np.concatenate([np.stack([X[m], Y[m]], axis=1), rim])
    return np.concatenate([pts, np.zeros((len(pts), 1))], axis=1)


def _hemi_surface(a, h):
    n_dome = int(2 * math.pi * a * a / (h * h) * 2)
    return np.concatenate([_fib_hemisphere(a, n_dome), _disk_grid(a, h)])


@pytest.mark.parametrize("kind", ["hemisphere", "discoid"])
def test_depletant_predicate_vs_point_cloud(oracle, kind):
    rng = np.random.default_rng(21)
    h = 0.004
    if kind == "hemisphere":
        a = 0.5
        params, K = [1.0], oracle.HEMISPHERE
        surf = _hemi_surface(a, h)
        thr = R_DEP
        inside = lambda p: (np.linalg.norm(p, axis=1) <= a) & (p[:, 2] >= 0)
        reach = a + R_DEP
    else:
        a, rs = 0.5, 0.1
        params, K = [a, rs], oracle.DISCOID
        surf = _disk_grid(a, h)
        thr = rs + R_DEP
        inside = lambda p: np.zeros(len(p), dtype=bool)
        reach = a + rs + R_DEP
    tree = cKDTree(surf)
    err = 2.0 * h  # sampled distance exceeds the true one by less than this
    pts = rng.uniform(-1.1 * reach, 1.1 * reach, size=(6000, 3))
    dist, _ = tree.query(pts)
    dist[inside(pts)] = 0.0
    checked = 0
    for p, d in zip(pts, dist):
        if abs(d - thr) < err + 1e-9:
            continue
        q = _rand_quat(rng)
        v = _rot(q).apply(p)  # the same body point seen from the world frame
        got = oracle.depletant_overlap(K, params, R_DEP, v, q)
        assert got == (d < thr), (p, d)
        checked += 1
    assert checked > 5000


def test_sphere_depletant_predicate(oracle):
    rng = np.random.default_rng(4)
    for _ in range(2000):
        v = rng.uniform(-0.7, 0.7, 3)
        r = np.linalg.norm(v)
        if abs(r - 0.575) < 1e-12:
            continue
        assert oracle.depletant_overlap(oracle.SPHERE, [1.0], R_DEP, v) == (r < 0.575)


def _hemi_interior(a, h):
    g = np.arange(-a, a + h, h)
    X, Y, Z = np.meshgrid(g, g, np.arange(h / 2, a, h))
    P = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    return P[np.linalg.norm(P, axis=1) < a]


@pytest.mark.parametrize("kind", ["hemisphere", "discoid"])
def test_pair_overlap_vs_brute_force(oracle, kind):
    rng = np.random.default_rng(5 if kind == "hemisphere" else 6)
    if kind == "hemisphere":
        a, h = 0.5, 0.015
        params, K, reach = [1.0], oracle.HEMISPHERE, 1.0
        surf = _hemi_surface(a, 0.01)
        interior = _hemi_interior(a, h)
        centroid = np.array([0, 0, 3 * a / 8])
    else:
        a, rs, h = 0.5, 0.1, 0.01
        params, K, reach = [a, rs], oracle.DISCOID, 2 * (a + rs)
        disk = _disk_grid(a, h)
    decided = {True: 0, False: 0}
    for trial in range(200):
        qa, qb = _rand_quat(rng), _rand_quat(rng)
        d = rng.standard_normal(3)
        d *= rng.uniform(0.1, 1.0) * reach / np.linalg.norm(d)
        RA, RB = _rot(qa), _rot(qb)
        if kind == "hemisphere":
            A_surf = RA.apply(surf)
            B_surf = RB.apply(surf) + d
            bd, _ = cKDTree(A_surf).query(B_surf, distance_upper_bound=4 * 0.01)
            # an interior point of A strictly inside B certifies overlap
            pa = RA.apply(interior)
            pb = RB.inv().apply(pa - d)
            certain_ov = bool(np.any((np.linalg.norm(pb, axis=1) < a) & (pb[:, 2] > 0)))
            # boundaries apart and no containment certifies separation
            ca_in_b = RB.inv().apply(RA.apply(centroid) - d)
            cb_in_a = RA.inv().apply(RB.apply(centroid) + d)
            contain = (np.linalg.norm(ca_in_b) < a and ca_in_b[2] > 0) or (np.linalg.norm(cb_in_a) < a and cb_in_a[2] > 0)
            certain_sep = bd.min() > 3 * 0.01 and not contain and not certain_ov
        else:
            A = RA.apply(disk)
            B = RB.apply(disk) + d
            ds, _ = cKDTree(A).query(B, distance_upper_bound=2 * rs + 4 * h)
            dmin = ds.min()
            certain_ov = dmin < 2 * rs
            certain_sep = dmin - 2 * h > 2 * rs
        if not (certain_ov or certain_sep):
            continue
        got, near = oracle.pair_overlap(K, params, d, qa, qb)
        assert got == certain_ov, (trial, d, qa, qb)
        decided[certain_ov] += 1
    assert decided[True] > 30 and decided[False] > 30, decided


def test_pair_overlap_symmetric_and_circumsphere(oracle):
    rng = np.random.default_rng(8)
    for K, params, rc in ((oracle.HEMISPHERE, [1.0], 0.5), (oracle.DISCOID, [0.5, 0.1], 0.6)):
        for _ in range(300):
            qa, qb = _rand_quat(rng), _rand_quat(rng)
            d = rng.uniform(-1.3, 1.3, 3)
            ab, _ = oracle.pair_overlap(K, params, d, qa, qb)
            ba, _ = oracle.pair_overlap(K, params, -d, qb, qa)
            assert ab == ba
            if np.linalg.norm(d) >= 2 * rc:
                assert not ab
