#!/usr/bin/env python3
"""Benchmark of the implicit-depletant hard-particle Monte Carlo sweep on one MI355X.

Metric: colloid trial moves/s (the JSON ``value``) and depletant overlap checks/s,
with p50/p99 per-sweep latency, on hard spheres N = 1,048,576 at phi_c = 0.30 with
ideal sphere depletants q = 0.10, eta_r = 0.30 and configurational bias
n_trial = 4 (Glaser, Karas & Glotzer, arXiv:1508.07077, Sec. III).  One step = one
sweep (8 checkerboard phases, N trial moves) over the device-resident state.

  python bench.py [--gpus 1] [--steps K] [--warmup W]

The state is built from a simple-cubic lattice and melted (untimed) at zero
fugacity; inputs are synthetic (seeded), shaped like the paper's systems.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 4 SIMD x 16 lanes at 2.4 GHz = VALU lane-instruction issue peak
VALU_PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9

# Algorithmic VALU work per resolved depletant check (lane-instructions), the
# per-unit figure of the roofline: one Philox4x32-10 block yields 2 ball
# candidates, accepted with probability pi/6 each, so a depletant costs
# 1/(2 pi/6) = 0.955 blocks.  A block is 10 rounds of 2 32x32->64 multiplies
# and 4 XORs (60 instructions; the key schedule is wave-uniform and scalar).
# Each candidate: 3 field extractions + 3 int->f64 conversions + 3 offsets
# (9 VALU), 3 squares and 2 adds and 1 compare in f64 (6); each accepted
# candidate: 3 scalings + the old-pose test (3 sub, 3 mul, 2 add, 1 compare)
# (12) + index assignment (2).
#   per depletant = 0.955 * (60 + 2 * 15) + 14 = 100.0 lane-instructions
ALGO_OPS_PER_CHECK = 0.955 * (60 + 2 * 15) + 14


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--melt", type=int, default=20, help="untimed zero-fugacity sweeps from the lattice")
    ap.add_argument("--n", type=int, default=1048576)
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="oracle CPU-baseline budget (0 disables)")
    ap.add_argument("--cpu-n", type=int, default=40000)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device copy (scales the HBM byte counters)")
    return ap.parse_args()


def cpu_baseline(sp_factory, n_sample: int, seconds: float):
    """The oracle (single thread, FP64) on a bounded sample of the workload: a
    smaller box at the same state point, whole sweeps until `seconds` pass."""
    from oracle import pyoracle
    from paper_1508_07077_amd import workloads as wl

    sp = sp_factory(n_sample)
    pos, _ = sp.initial_state()
    o = pyoracle.OracleSim(sp.n, sp.L, sp.seed)
    o.set_shape(pyoracle.SPHERE, sp.params)
    o.set_fugacity(0.0, sp.d_dep, 0)
    o.set_moves(0.1)
    o.set_state(pos)
    o.sweep(20)
    o.set_fugacity(sp.z_p, sp.d_dep, sp.n_trial)
    o.set_moves(sp.d_trans)
    trials = resolved = 0
    sweeps = 0
    t0 = time.perf_counter()
    while True:
        c = o.sweep(1)
        trials += c["trials"]
        resolved += c["depletants_resolved"]
        sweeps += 1
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    return {
        "value": trials / dt,
        "unit": "colloid trial moves/s",
        "depletant_checks_per_s": resolved / dt,
        "cores": 1,
        "kind": "oracle",
        "sample": f"{sweeps} whole sweep(s) of a {sp.n}-sphere box at the same state point "
                  f"(phi_c={sp.phi_c}, q={sp.q}, eta_r={sp.eta_r}, n_trial={sp.n_trial}, delta={sp.d_trans}), "
                  f"single thread, {dt:.1f} s",
        "host_cpus": os.cpu_count(),
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (this build runs on a single MI355X)",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    if args.copy_calibration:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_each_way": src.numel() * 8, "copies": 3}))
        return

    import paper_1508_07077_amd as hp
    from paper_1508_07077_amd import workloads as wl

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    sp = wl.c3_spheres_large(n=args.n)
    pos, _ = sp.initial_state()
    sim = hp.Sim(sp.n, sp.L, sp.seed)
    sim.set_shape(hp.SPHERE, sp.params)
    sim.set_fugacity(0.0, sp.d_dep, 0)
    sim.set_moves(0.1)
    sim.set_state(pos)
    if args.melt:
        sim.sweep(args.melt, counters=False)
    sim.set_fugacity(sp.z_p, sp.d_dep, sp.n_trial)
    sim.set_moves(sp.d_trans)
    sim.ensure_workspace()
    for _ in range(args.warmup):
        sim.sweep(1, counters=True)
    torch.cuda.synchronize()
    tot = None
    lat = []
    phase_ms = 0.0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        c = sim.sweep(1, counters=True)
        lat.append((time.perf_counter() - ts) * 1e3)
        phase_ms += c["phase_kernel_ms"]
        tot = c if tot is None else {k: tot[k] + c[k] for k in tot}
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    moves = tot["trials"] / dt
    checks = tot["depletants_resolved"] / dt
    launches = 8 * args.steps
    avg_phase_s = phase_ms / 1e3 / launches
    achieved = ALGO_OPS_PER_CHECK * (tot["depletants_resolved"] / launches) / avg_phase_s
    line = {
        "metric": "colloid trial moves/s + depletant overlap checks/s (1 GPU); p50/p99 latency",
        "value": moves,
        "unit": "colloid trial moves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"hard spheres N={sp.n} phi_c={sp.phi_c} cubic periodic box L={sp.L:.4f}; "
                        f"sphere depletants q={sp.q} eta_r={sp.eta_r} (z_p={sp.z_p:.3f}); n_trial={sp.n_trial}; "
                        f"translation delta={sp.d_trans}; one step = one sweep of N trial moves",
            "N": sp.n,
            "sweeps_timed": args.steps,
        },
        "depletant_checks_per_s": checks,
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "acceptance": tot["accepts"] / tot["trials"],
        "depletants_per_move": tot["depletants_drawn"] / tot["trials"],
        "resolved_per_move": tot["depletants_resolved"] / tot["trials"],
        "roofline": {
            "bound": "alu",
            "kernel": "phase_kernel<sphere>",
            "achieved": achieved / 1e12,
            "peak": VALU_PEAK_LANE_OPS / 1e12,
            "unit": "T VALU lane-instr/s",
            "frac": achieved / VALU_PEAK_LANE_OPS,
            "traffic": None,
            "avg_launch_ms": avg_phase_s * 1e3,
            "ops_per_check": ALGO_OPS_PER_CHECK,
        },
    }
    if args.cpu_seconds > 0:
        line["cpu_baseline"] = cpu_baseline(lambda n: wl.c3_spheres_large(n=n, d_trans=sp.d_trans), args.cpu_n,
                                            args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
