"""Seeded synthetic workloads shaped like the paper's systems.

This module holds only input recipes -- box sizes from packing fractions,
fugacities from reservoir packing fractions, overlap-free starting lattices
and random orientations.  It contains none of the Monte Carlo method's
arithmetic, so both the HIP path and the oracle may take their inputs from it.

Relations used (Glaser, Karas & Glotzer, arXiv:1508.07077):
  * reservoir packing fraction phi_p^r = (pi/6) d_dep^3 z_p        (Sec. IV.B, Fig. 5 caption)
  * size ratio q = d_dep / d_colloid                                (Sec. IV.A, Fig. 4 caption)
  * the hemisphere diameter is that of the parent sphere            (Sec. V.A, Fig. 7 caption)
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SPHERE, HEMISPHERE, DISCOID = 0, 1, 2
SHAPE_NAMES = {SPHERE: "sphere", HEMISPHERE: "hemisphere", DISCOID: "discoid"}


def shape_volume(kind: int, params) -> float:
    if kind == SPHERE:
        d = params[0]
        return math.pi * d**3 / 6.0
    if kind == HEMISPHERE:
        d = params[0]
        return math.pi * d**3 / 12.0
    a, r = params
    # disk of radius a swept by a ball of radius r (cylinder + rim by Pappus + caps)
    return 2.0 * math.pi * a * a * r + math.pi**2 * a * r * r + 4.0 / 3.0 * math.pi * r**3


def circumradius(kind: int, params) -> float:
    if kind in (SPHERE, HEMISPHERE):
        return 0.5 * params[0]
    return params[0] + params[1]


def colloid_diameter(kind: int, params) -> float:
    """The length that q multiplies: sphere / parent-sphere diameter, disk diameter."""
    if kind in (SPHERE, HEMISPHERE):
        return params[0]
    return 2.0 * params[0]


def box_length(n: int, kind: int, params, phi_c: float) -> float:
    return (n * shape_volume(kind, params) / phi_c) ** (1.0 / 3.0)


def fugacity(eta_r: float, d_dep: float) -> float:
    """z_p from the reservoir packing fraction eta_r = (pi/6) d_dep^3 z_p."""
    if eta_r <= 0.0:
        return 0.0
    return eta_r / (math.pi * d_dep**3 / 6.0)


def random_quaternions(n: int, rng: np.random.Generator) -> np.ndarray:
    """Uniform unit quaternions, SoA [4][n] (w, x, y, z)."""
    q = rng.standard_normal((4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    return q


def cubic_sites(m: int, L: float, d_min: float) -> np.ndarray:
    """m points of the periodic box [0, L)^3, pairwise (minimum-image) farther
    apart than d_min: the simple-cubic, body-centred or face-centred cubic
    lattice (k^3, 2k^3 or 4k^3 sites) with the largest nearest-neighbour
    distance that holds at least m sites, thinned evenly to m.  ValueError
    when none of the three is loose enough.  Returns [3][m]."""
    best = None
    for per, nn_frac, basis in ((1, 1.0, [(0.0, 0.0, 0.0)]),
                               (2, math.sqrt(3.0) / 2.0, [(0.0, 0.0, 0.0), (0.5, 0.5, 0.5)]),
                               (4, 1.0 / math.sqrt(2.0), [(0.0, 0.0, 0.0), (0.5, 0.5, 0.0),
                                                          (0.5, 0.0, 0.5), (0.0, 0.5, 0.5)])):
        k = max(1, int(math.ceil((m / per) ** (1.0 / 3.0) - 1e-9)))
        while per * k**3 < m:
            k += 1
        nn = nn_frac * L / k
        if best is None or nn > best[0]:
            best = (nn, k, basis)
    nn, k, basis = best
    if nn <= d_min * (1.0 + 1e-6):
        raise ValueError("density too high for an overlap-free cubic lattice")
    a = L / k
    cells = np.arange(k**3)
    ix, iy, iz = cells % k, (cells // k) % k, cells // (k * k)
    pts = np.concatenate([np.stack([(ix + 0.25 + bx) * a, (iy + 0.25 + by) * a, (iz + 0.25 + bz) * a])
                          for bx, by, bz in basis], axis=1)
    keep = (np.arange(m, dtype=np.int64) * pts.shape[1]) // m
    return np.ascontiguousarray(pts[:, keep].astype(np.float64))


def _flip_quaternions(q: np.ndarray) -> np.ndarray:
    """q * (0, 1, 0, 0): the same orientation turned by pi about the body x
    axis, so that the body z axis points the opposite way."""
    w, x, y, z = q
    return np.stack([-x, w, z, -y])


def lattice_state(n: int, L: float, kind: int, params, seed: int):
    """Overlap-free starting state.  Simple-cubic sites (first n of k^3) when
    the spacing exceeds the circumdiameter (any orientation is then safe);
    otherwise spheres on the loosest of sc/bcc/fcc that fits, hemispheres in
    flat-face-to-face pairs (each pair inside a ball of diameter 1.002 d) on
    such a lattice, and discoids as aligned disks in columns.  Returns
    (pos[3][n], quat[4][n] or None)."""
    rng = np.random.default_rng(seed)
    rc = circumradius(kind, params)
    k = int(math.ceil(n ** (1.0 / 3.0) - 1e-9))
    while k**3 < n:
        k += 1
    sp = L / k
    oriented = kind != SPHERE
    if sp > 2.0 * rc * (1.0 + 1e-6):
        idx = np.arange(n)
        ix, iy, iz = idx % k, (idx // k) % k, idx // (k * k)
        pos = np.stack([(ix + 0.5) * sp, (iy + 0.5) * sp, (iz + 0.5) * sp]).astype(np.float64)
        quat = random_quaternions(n, rng) if oriented else None
        return pos, quat
    if kind == SPHERE:
        return cubic_sites(n, L, 2.0 * rc), None
    if kind == HEMISPHERE:
        gap = 1e-3 * 2.0 * rc
        npair = (n + 1) // 2
        centre = cubic_sites(npair, L, 2.0 * rc + gap)
        qa = random_quaternions(npair, rng)
        w, x, y, z = qa
        axis = np.stack([2.0 * (x * z + w * y), 2.0 * (y * z - w * x), 1.0 - 2.0 * (x * x + y * y)])
        pos = np.concatenate([centre + 0.5 * gap * axis, centre - 0.5 * gap * axis], axis=1)[:, :n]
        quat = np.concatenate([qa, _flip_quaternions(qa)], axis=1)[:, :n]
        return np.mod(pos, L), np.ascontiguousarray(quat)
    a, r = params
    # aligned disks (normal along z): in-plane spacing > 2(a + r), vertical spacing > 2 r
    nxy = int(math.floor(L / (2.0 * (a + r) * (1.0 + 1e-6))))
    if nxy < 1:
        raise ValueError("box too small for aligned disks")
    nz = int(math.ceil(n / (nxy * nxy)))
    sz = L / nz
    if sz <= 2.0 * r * (1.0 + 1e-6):
        raise ValueError("density too high for aligned disks")
    sxy = L / nxy
    idx = np.arange(n)
    ix, iy, iz = idx % nxy, (idx // nxy) % nxy, idx // (nxy * nxy)
    pos = np.stack([(ix + 0.5) * sxy, (iy + 0.5) * sxy, (iz + 0.5) * sz]).astype(np.float64)
    quat = np.zeros((4, n), dtype=np.float64)
    quat[0] = 1.0
    return pos, quat


@dataclass
class StatePoint:
    """One simulation: shape, size, density, depletants, moves."""

    kind: int
    params: tuple
    n: int
    phi_c: float
    q: float
    eta_r: float
    n_trial: int = 0
    d_trans: float = 0.1
    a_rot: float = 0.0
    p_rot: float = 0.0
    seed: int = 1
    replica_id: int = 0
    name: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def L(self) -> float:
        return box_length(self.n, self.kind, self.params, self.phi_c)

    @property
    def d_dep(self) -> float:
        return self.q * colloid_diameter(self.kind, self.params)

    @property
    def z_p(self) -> float:
        return fugacity(self.eta_r, self.d_dep)

    def initial_state(self):
        return lattice_state(self.n, self.L, self.kind, self.params, self.seed)


# Step sizes below are frozen from an offline tune toward ~20 % acceptance
# (the paper tunes to 20 %, Sec. V.B).
def c1_spheres_small(n_trial: int = 0) -> StatePoint:
    """Hard spheres d=1, N=64, phi_c=0.10, q=0.25, eta_r=0.10, translation 0.1."""
    return StatePoint(SPHERE, (1.0,), 64, 0.10, 0.25, 0.10, n_trial=n_trial, d_trans=0.1, seed=1,
                      name="spheres N=64 phi_c=0.10 q=0.25 eta_r=0.10")


def c2_hemispheres(eta_r: float = 0.2, n: int = 16384) -> StatePoint:
    """Hemispheres d=1, N=16384, phi_c=0.20, q=0.15, eta_r in 0.1..0.4, translate+rotate."""
    d_trans = {0.1: 0.1, 0.2: 0.07, 0.3: 0.045, 0.4: 0.035}.get(round(eta_r, 2), 0.05)
    return StatePoint(HEMISPHERE, (1.0,), n, 0.20, 0.15, eta_r, n_trial=0, d_trans=d_trans,
                      a_rot=d_trans, p_rot=0.5, seed=1,
                      name=f"hemispheres N={n} phi_c=0.20 q=0.15 eta_r={eta_r}")


def c3_spheres_large(n: int = 1048576, d_trans: float = 0.003) -> StatePoint:
    """Hard spheres d=1, N=1,048,576, phi_c=0.30, q=0.10, eta_r=0.30, n_trial=4."""
    return StatePoint(SPHERE, (1.0,), n, 0.30, 0.10, 0.30, n_trial=4, d_trans=d_trans, seed=1,
                      name=f"spheres N={n} phi_c=0.30 q=0.10 eta_r=0.30 n_trial=4")


def c4_discoid_replicas(count: int = 256, seed: int = 4):
    """Swept disks (a=0.5, r_s=0.1), N log-uniform in [128, 8192], phi_c U[0.05,0.45],
    eta_r U[0, 0.5], q=0.2."""
    rng = np.random.default_rng(seed)
    out = []
    for r in range(count):
        n = int(round(math.exp(rng.uniform(math.log(128), math.log(8192)))))
        phi = float(rng.uniform(0.05, 0.45))
        eta = float(rng.uniform(0.0, 0.5))
        out.append(StatePoint(DISCOID, (0.5, 0.1), n, phi, 0.2, eta, n_trial=0, d_trans=0.02, a_rot=0.02,
                              p_rot=0.5, seed=seed * 1000 + r, replica_id=r,
                              name=f"discoid replica {r}"))
    return out


def c5_request_stream(duration_s: float = 60.0, rate: float = 50.0, seed: int = 5):
    """Poisson arrivals of {sphere, hemisphere, discoid} requests, N log-uniform in
    [256, 65536], phi_c in [0.05, 0.45], eta_r in [0, 0.5], 100 sweeps each."""
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    shapes = [(SPHERE, (1.0,), 0.10), (HEMISPHERE, (1.0,), 0.15), (DISCOID, (0.5, 0.1), 0.2)]
    i = 0
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t > duration_s:
            break
        kind, params, q = shapes[int(rng.integers(0, 3))]
        n = int(round(math.exp(rng.uniform(math.log(256), math.log(65536)))))
        phi = float(rng.uniform(0.05, 0.45))
        eta = float(rng.uniform(0.0, 0.5))
        sp = StatePoint(kind, params, n, phi, q, eta, n_trial=0, d_trans=0.02,
                        a_rot=0.02 if kind != SPHERE else 0.0, p_rot=0.5 if kind != SPHERE else 0.0,
                        seed=seed * 100000 + i, replica_id=i, name=f"request {i}")
        sp.extra["phi_requested"] = phi
        while True:  # cap phi_c at what an overlap-free lattice start holds for this N
            try:
                sp.initial_state()
                break
            except ValueError:
                sp.phi_c *= 0.98
        sp.extra["arrival_s"] = t
        sp.extra["sweeps"] = 100
        reqs.append(sp)
        i += 1
    return reqs
