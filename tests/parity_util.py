"""Helpers of the GPU parity tests: one handle on each side (the HIP library
through its C-ABI binding, the oracle through ctypes), fed the same seeded
inputs, compared record by record and bit for bit."""
import numpy as np

TRACE_FIELDS = ("sweep", "cell", "t", "particle", "n_depletants", "resolved", "n_blocking", "w_fwd", "w_rev",
                "phase", "reason", "rotation")


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
    return g, o


def compare_sweeps(g, o, n_sweeps, allow_near=False):
    """Run sweeps on both sides; every trace record and the state must agree.
    With allow_near, a disagreement in a trial that either side decided within
    1e-9 of a colloid contact is tolerated: both sides restart from the
    oracle's state.  Returns (summed GPU counters, near-contact divergences)."""
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
            bad = np.zeros(len(tg), dtype=bool)
            for f in TRACE_FIELDS:
                bad |= tg[f] != to[f]
            near = (tg["near_contact"] | to["near_contact"]).astype(bool)
            first = int(np.argmax(bad)) if bad.any() else -1
            if allow_near and bad.any() and near[bad].any():
                diverged += 1
                g.set_state(po, qo if qg is not None else None, swo)
                continue
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
