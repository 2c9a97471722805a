"""Helpers of the GPU parity tests: one handle on each side (the HIP library
through its C-ABI binding, the oracle through ctypes), fed the same seeded
inputs, compared record by record and bit for bit.

Near-contact rule.  The two sides settle colloid pairs of convex shapes with
different exact tests (MPR on the GPU, a GJK distance bracket in the oracle),
so a pair whose separation is within 1e-9 of contact may be decided
differently.  Such a trial may differ, and so may what depends on it, and
nothing else: in the earliest phase with a difference, the first differing
trial of every differing cell must be one that either side decided within
1e-9 of contact (later trials of that cell follow from it); a difference in a
later phase must lie in the light cone of those cells, i.e. within k cells
(periodic Chebyshev distance) of one of them k phases later, because a trial
reads only the cells of its 27-cell stencil and cells of one colour are
independent."""
import numpy as np

TRACE_FIELDS = ("sweep", "cell", "t", "particle", "n_depletants", "resolved", "n_blocking", "w_fwd", "w_rev",
                "phase", "reason", "rotation")


def cells_per_axis(sp) -> int:
    """cells per box side: the largest even n with L / n >= 2 R_circ + d_dep"""
    from paper_1508_07077_amd import workloads as wl

    rcirc = sp.params[0] + sp.params[1] if sp.kind == wl.DISCOID else 0.5 * sp.params[0]
    n = int(np.floor(sp.L / (2.0 * rcirc + sp.d_dep)))
    return n - (n % 2)


def make_pair(sp, pos, quat=None, sweep=0, trace=True, precision=0, region=0):
    import paper_1508_07077_amd as hp
    from oracle import pyoracle

    g = hp.Sim(sp.n, sp.L, sp.seed, sp.replica_id, precision=precision)
    o = pyoracle.OracleSim(sp.n, sp.L, sp.seed, sp.replica_id)
    for s in (g, o):
        s.set_shape(sp.kind, sp.params)
        s.set_fugacity(sp.z_p, sp.d_dep, sp.n_trial)
        s.set_moves(sp.d_trans, sp.a_rot, sp.p_rot)
        s.set_insertion(region)
        s.set_trace(trace)
    g.set_state(pos, quat, sweep)
    o.set_state(pos, quat, sweep)
    g.n_axis = cells_per_axis(sp)
    return g, o


def near_contact_explains(tg, to, n_axis, pg=None, po=None):
    """None if every difference between the two traces of one sweep (and the
    two end states, if given) follows from near-contact trials under the rule
    of this module's docstring; otherwise a message naming the first
    difference it does not explain."""
    bad = np.zeros(len(tg), dtype=bool)
    for f in TRACE_FIELDS:
        bad |= tg[f] != to[f]
    if not bad.any():
        if pg is not None and not np.array_equal(pg, po):
            return "the end states differ while every trial record agrees"
        return None
    near = (tg["near_contact"] | to["near_contact"]).astype(bool)
    # the oracle's record fixes cell and phase (the start states are equal)
    phase = to["phase"].astype(np.int64)
    cell = to["cell"].astype(np.int64)
    t = to["t"].astype(np.int64)
    p0 = int(phase[bad].min())
    seeds = []
    for c in np.unique(cell[bad & (phase == p0)]):
        idx = np.flatnonzero(bad & (cell == c))
        first = idx[np.argmin(t[idx])]
        if not near[first]:
            return (f"phase {p0}, cell {c}: first differing trial {first} was not decided near contact "
                    f"(gpu={tg[first]} oracle={to[first]})")
        seeds.append(int(c))
    seeds = np.array(seeds, dtype=np.int64)
    sx, sy, sz = seeds % n_axis, (seeds // n_axis) % n_axis, seeds // (n_axis * n_axis)

    def cdist(a, b):
        d = np.abs(a - b) % n_axis
        return np.minimum(d, n_axis - d)

    later = np.flatnonzero(bad & (phase > p0))
    for i in later:
        c = cell[i]
        cx, cy, cz = c % n_axis, (c // n_axis) % n_axis, c // (n_axis * n_axis)
        dist = np.maximum(np.maximum(cdist(sx, cx), cdist(sy, cy)), cdist(sz, cz)).min()
        if dist > phase[i] - p0:
            return (f"record {i} (phase {phase[i]}, cell {c}) differs outside the light cone of the "
                    f"near-contact cells {seeds.tolist()} of phase {p0}")
    if pg is not None:
        moved = np.flatnonzero(np.any(pg != po, axis=0))
        allowed = set(tg["particle"][bad].tolist()) | set(to["particle"][bad].tolist())
        stray = [int(j) for j in moved if int(j) not in allowed]
        if stray:
            return f"particles {stray[:5]} end in different places but none of their trials differ"
    return None


def compare_sweeps(g, o, n_sweeps, allow_near=False):
    """Run sweeps on both sides; every trace record and the state must agree.
    With allow_near, differences that the near-contact rule explains are
    tolerated and both sides restart from the oracle's state.  Returns
    (summed GPU counters, number of sweeps with such differences)."""
    tot = None
    diverged = 0
    for _ in range(n_sweeps):
        cg = g.sweep(1)
        co = o.sweep(1)
        tg, to = g.trace(), o.trace()
        pg, qg, swg = g.get_state()
        po, qo, swo = o.get_state()
        assert swg == swo
        assert len(tg) == len(to)
        same = all(np.array_equal(tg[f], to[f]) for f in TRACE_FIELDS)
        same_state = np.array_equal(pg, po) and (qg is None or np.array_equal(qg, qo[:, :]))
        if not (same and same_state):
            if allow_near:
                sg = pg if qg is None else np.vstack([pg, qg])
                so = po if qo is None else np.vstack([po, qo])
                why = near_contact_explains(tg, to, g.n_axis, sg, so)
                if why is None:
                    diverged += 1
                    g.set_state(po, qo if qg is not None else None, swo)
                    continue
                raise AssertionError(why)
            bad = np.zeros(len(tg), dtype=bool)
            for f in TRACE_FIELDS:
                bad |= tg[f] != to[f]
            first = int(np.argmax(bad)) if bad.any() else -1
            msg = []
            if first >= 0:
                msg.append(f"first differing record {first}: gpu={tg[first]} oracle={to[first]}")
            if not same_state:
                d = np.argwhere(pg != po)
                msg.append(f"{len(d)} position entries differ, first {d[:3].tolist()}")
            raise AssertionError("; ".join(msg))
        for k in ("trials", "accepts", "rej_cell_exit", "rej_overlap", "rej_depletant", "rej_cb_zero",
                  "rej_cb_metropolis", "depletants_drawn", "depletants_resolved", "cb_trials"):
            assert cg[k] == co[k], (k, cg[k], co[k])
        tot = cg if tot is None else {k: tot[k] + cg[k] for k in tot}
    return tot, diverged
