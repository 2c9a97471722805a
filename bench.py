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

# Minimal VALU work per resolved depletant check (lane-instructions): one
# Philox4x32-10 block yields 2 ball candidates, accepted with probability
# pi/6 each, so a depletant costs 1/(2 pi/6) = 0.955 blocks.  A block is 10
# rounds of 2 32x32->64 multiplies and 2 three-input XORs (40 instructions;
# the key schedule is wave-uniform and scalar).  Each candidate: 3 field
# extractions + 3 int->f64 conversions + 3 offsets (9 VALU), 3 squares, 2 adds
# and 1 compare in f64 (6); each accepted candidate: 3 scalings + the old-pose
# test (3 sub, 3 mul, 2 add, 1 compare) (12) + index assignment (2).
#   per depletant = 0.955 * (40 + 2 * 15) + 14 = 80.9 lane-instructions
ALGO_OPS_PER_CHECK = 0.955 * (40 + 2 * 15) + 14

# Shell insertion region: one candidate per block (40), 4 u32->f64 conversions
# with their offsets and scalings (12), the disk test (3), the radius and its
# r^2 test (5), 2 sqrt(1 - s) + direction + 3 scalings (16): 76 per block,
# accepted with probability (pi/4) E[r^2]/R0^2; + 14 per accepted depletant.
def shell_ops_per_check(R0: float, r_i: float) -> float:
    acc = math.pi / 4 * (R0**3 - r_i**3) / (3.0 * (R0 - r_i) * R0**2)
    return 76.0 / acc + 14.0


# Active VALU lane-instructions of the phase kernels, from rocprofv3 counters
# (SQ_INSTS_VALU x 64 x VALUUtilization per launch) of the kernel sources with
# the digest below, split as the method's work is: a_dep per resolved
# depletant check (timed launches with depletants minus launches of the same
# state at zero fugacity) plus b_move per trial move (the zero-fugacity
# launches).  achieved = (a_dep x resolved checks + b_move x moves) per launch
# / the launch's duration, timed live with HIP events; frac = achieved / peak
# is therefore the share of the VALU's lane-instruction slots the kernel keeps
# busy with active lanes (rocprofv3 VALUBusy x VALUUtilization).  The HBM bytes
# per launch are FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 (the factors a plain
# 256 MiB device copy reads off the same counters).
PROFILED_KERNEL_DIGEST = "115c5d2513932231"
PROFILE = {
    # 1,048,576 spheres, ball region, 212.05 resolved checks per move
    "sphere": {"a_dep": 174.89, "b_move": 15152.8, "valu_instr_per_move": 1212.7, "valu_busy": 78.10,
               "valu_utilization": 67.31, "traffic_bytes_per_launch": 65233511},
    # 16,384 hemispheres at eta_r 0.4, 72.31 resolved checks per move
    "hemisphere": {"a_dep": 393.58, "b_move": 34067.5, "valu_instr_per_move": 2099.3, "valu_busy": 12.54,
                   "valu_utilization": 46.54, "traffic_bytes_per_launch": 4406106},
    # 256 swept-disk replicas, both launch groups of a phase, 56.50 resolved checks per move
    "discoid": {"a_dep": 480.09, "b_move": 29100.9, "valu_instr_per_move": 2306.1,
                "valu_busy": {"replicas of two cells per axis": 0.82, "the others": 43.57},
                "valu_utilization": {"replicas of two cells per axis": 35.06, "the others": 38.14},
                "traffic_bytes_per_phase": 85918366},
}


def kernel_digest() -> str:
    import hashlib

    h = hashlib.sha256()
    for f in ("kernels.hip", "kernels.hpp", "rng.hpp", "geom.hpp"):
        with open(os.path.join(ROOT, "paper_1508_07077_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--melt", type=int, default=200, help="untimed zero-fugacity sweeps from the lattice")
    ap.add_argument("--n", type=int, default=1048576)
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="oracle CPU-baseline budget (0 disables)")
    ap.add_argument("--cpu-n", type=int, default=40000)
    ap.add_argument("--workload", default="c3", choices=["c3", "c1", "c2", "c4", "c5"],
                    help="c3: 1,048,576 spheres (default); c1: 64 spheres, 1000 sweeps; "
                         "c2: 16384 hemispheres, eta_r 0.1..0.4; c4: 256 batched discoid replicas; "
                         "c5: Poisson request stream served with continuous batching")
    ap.add_argument("--v0", default="ball", choices=["ball", "shell"],
                    help="c3: depletant insertion region of the headline run (the other one is timed after it)")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="skip the launch-shape autotuner (default: tune before timing)")
    ap.add_argument("--serve-seconds", type=float, default=10.0, help="c5: length of the arrival trace")
    ap.add_argument("--capacity-requests", type=int, default=60,
                    help="c5: requests of the trace served all at once, batched and one at a time")
    ap.add_argument("--eta", default="0.1,0.2,0.3,0.4",
                    help="c2: comma-separated reservoir packing fractions eta_r to run")
    ap.add_argument("--no-batch", dest="batch", action="store_false",
                    help="c2: skip the leg that sweeps the state points together (value is then one at a time)")
    ap.add_argument("--no-fp32", dest="fp32", action="store_false",
                    help="c2, c3: skip the FP32-guarded companion run")
    ap.add_argument("--no-companion", dest="companion", action="store_false",
                    help="c3: skip the other-insertion-region companion run (profiling)")
    ap.add_argument("--no-alone", dest="alone", action="store_false",
                    help="c4: skip the one-replica-at-a-time comparison")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device copy (scales the HBM byte counters)")
    return ap.parse_args()


def _copy_gbps(torch, n_bytes: int = 1 << 30, reps: int = 5) -> float:
    """HBM bandwidth of a plain device-to-device copy (bytes read + written per
    second, best of `reps`), the practical bound beside the 8 TB/s peak"""
    src = torch.ones(n_bytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * n_bytes / (best * 1e-3) / 1e9


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rate(sp_factory, n_sample: int, seconds: float, threads: int):
    """The oracle (FP64) on a bounded sample of the workload: a smaller box at
    the same state point, whole sweeps until `seconds` pass."""
    from oracle import pyoracle

    sp = sp_factory(n_sample)
    pos, _ = sp.initial_state()
    o = pyoracle.OracleSim(sp.n, sp.L, sp.seed)
    o.set_shape(pyoracle.SPHERE, sp.params)
    o.set_threads(threads)
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
    return sp, trials / dt, resolved / dt, sweeps, dt


def cpu_baseline(sp_factory, n_sample: int, seconds: float):
    """The oracle as it is, timed on this host: with OpenMP threads over the
    active cells of a phase on every core it may use (the same result as one
    thread, bit for bit), and single-threaded beside it."""
    threads = max(1, int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)))
    threads = min(threads, os.cpu_count() or 1)
    sp, m1, c1, s1, d1 = _oracle_rate(sp_factory, n_sample, 0.6 * seconds, 1)
    _, mt, ct, st, dtt = _oracle_rate(sp_factory, n_sample, 0.4 * seconds, threads)
    desc = (f"a {sp.n}-sphere box at the same state point (phi_c={sp.phi_c}, q={sp.q}, eta_r={sp.eta_r}, "
            f"n_trial={sp.n_trial}, delta={sp.d_trans})")
    return {
        "value": mt,
        "unit": "colloid trial moves/s",
        "depletant_checks_per_s": ct,
        "cores": threads,
        "kind": "oracle",
        "sample": f"{st} whole sweep(s) of {desc}, {threads} OpenMP threads over the active cells of a phase, "
                  f"{dtt:.1f} s",
        "single_thread": {"value": m1, "depletant_checks_per_s": c1, "cores": 1,
                          "sample": f"{s1} whole sweep(s) of the same box, one thread, {d1:.1f} s"},
        "nproc": os.cpu_count(),
        "cpu_model": _cpu_model(),
    }


def _oracle_threads() -> int:
    threads = max(1, int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)))
    return min(threads, os.cpu_count() or 1)


def cpu_baseline_states(sps, sweeps: int, seconds: float, what: str, melt: int = 5):
    """The oracle as it is (OpenMP over the active cells of a phase on the
    cores it may use) on a bounded sample of a workload's state points: each
    from its start, `melt` untimed sweeps at zero fugacity, then up to
    `sweeps` timed sweeps, until `seconds` of timed work have passed."""
    from oracle import pyoracle

    threads = _oracle_threads()
    trials = resolved = 0
    timed = 0.0
    done = []
    for sp in sps:
        pos, quat = sp.initial_state()
        o = pyoracle.OracleSim(sp.n, sp.L, sp.seed, sp.replica_id)
        o.set_shape(sp.kind, sp.params)
        o.set_threads(threads)
        o.set_fugacity(0.0, sp.d_dep, 0)
        o.set_moves(0.1, 0.1 if sp.kind != pyoracle.SPHERE else 0.0, sp.p_rot)
        o.set_state(pos, quat)
        if melt:
            o.sweep(melt)
        o.set_fugacity(sp.z_p, sp.d_dep, sp.n_trial)
        o.set_moves(sp.d_trans, sp.a_rot, sp.p_rot)
        n = 0
        t0 = time.perf_counter()
        while n < sweeps and timed + (time.perf_counter() - t0) < seconds:
            c = o.sweep(1)
            trials += c["trials"]
            resolved += c["depletants_resolved"]
            n += 1
        timed += time.perf_counter() - t0
        done.append(n)
        if timed >= seconds:
            break
    return {"value": trials / timed, "unit": "colloid trial moves/s", "depletant_checks_per_s": resolved / timed,
            "cores": threads, "kind": "oracle",
            "sample": f"{what}: {len(done)} state point(s), {sum(done)} timed sweep(s) in all "
                      f"({', '.join(str(x) for x in done)}), after {melt} untimed zero-fugacity sweeps each, "
                      f"{threads} OpenMP threads, {timed:.1f} s",
            "nproc": os.cpu_count()}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the library runs on one MI355X)",
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
    if args.workload != "c3":
        print(json.dumps(OTHER[args.workload](args)), flush=True)
        return
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
    region = hp.V0_SHELL if args.v0 == "shell" else hp.V0_BALL
    sim.set_insertion(region)
    sim.ensure_workspace()
    tuning = sim.autotune(sweeps=2) if args.autotune else None
    tot, lat, phase_ms, dt = _timed_sweeps(torch, sim, args.steps, args.warmup)
    moves = tot["trials"] / dt
    checks = tot["depletants_resolved"] / dt
    launches = 8 * args.steps
    avg_phase_s = phase_ms / 1e3 / launches
    R0 = 0.5 * sp.params[0] + 0.5 * sp.d_dep
    minimal_ops = ALGO_OPS_PER_CHECK if region == hp.V0_BALL else \
        shell_ops_per_check(R0, max(0.0, R0 - math.sqrt(3.0) * sp.d_trans))
    profiled = kernel_digest() == PROFILED_KERNEL_DIGEST
    per_launch_checks = tot["depletants_resolved"] / launches
    per_launch_moves = tot["trials"] / launches
    achieved_minimal = minimal_ops * per_launch_checks / avg_phase_s
    # the same state point with the other insertion region, timed right after
    companion = None
    if args.companion:
        other = hp.V0_BALL if region == hp.V0_SHELL else hp.V0_SHELL
        sim.set_insertion(other)
        sim.ensure_workspace()
        tot2, lat2, _, dt2 = _timed_sweeps(torch, sim, args.steps, args.warmup)
        companion = {
            "insertion_region": "shell" if other == hp.V0_SHELL else "ball",
            "moves_per_s": tot2["trials"] / dt2,
            "depletant_checks_per_s": tot2["depletants_resolved"] / dt2,
            "ms_per_step": dt2 * 1e3 / args.steps,
            "p50_ms": float(np.percentile(lat2, 50)),
            "p99_ms": float(np.percentile(lat2, 99)),
            "acceptance": tot2["accepts"] / tot2["trials"],
            "depletants_per_move": tot2["depletants_drawn"] / tot2["trials"],
        }
    # FP32 geometry with the FP64 guard band, same state point and region as the headline
    fp32 = None
    if args.fp32:
        fp32 = _fp32_companion(hp, torch, sp, sim, region, args, launches)
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
                        f"translation delta={sp.d_trans}; one step = one sweep of N trial moves; "
                        f"depletants inserted in the {args.v0} region",
            "N": sp.n,
            "insertion_region": args.v0,
            "sweeps_timed": args.steps,
        },
        "depletant_checks_per_s": checks,
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "acceptance": tot["accepts"] / tot["trials"],
        "depletants_per_move": tot["depletants_drawn"] / tot["trials"],
        "resolved_per_move": tot["depletants_resolved"] / tot["trials"],
        "pair_tests_per_s": tot["overlap_checks"] / dt,
        "roofline": _roofline("sphere", profiled and region == hp.V0_BALL, per_launch_checks, per_launch_moves,
                              avg_phase_s, "phase_sphere_kernel (one launch per checkerboard colour)",
                              extra={"frac_minimal": achieved_minimal / VALU_PEAK_LANE_OPS,
                                     "ops_per_check_minimal": minimal_ops}),
        "other_insertion_region": companion,
        "fp32_guarded": fp32,
        "launch_tuning": tuning,
    }
    roof = line["roofline"]
    if roof.get("traffic"):
        # the phase kernel's HBM rate beside a plain copy's (not the bound: the kernel is VALU-bound)
        roof["hbm"] = {"achieved_gbps": roof["traffic"] / avg_phase_s / 1e9, "copy_gbps": _copy_gbps(torch),
                       "peak_gbps": 8000.0}
    if args.cpu_seconds > 0:
        line["cpu_baseline"] = cpu_baseline(lambda n: wl.c3_spheres_large(n=n, d_trans=sp.d_trans), args.cpu_n,
                                            args.cpu_seconds)
    print(json.dumps(line), flush=True)


def _roofline(shape, profiled, checks, moves, seconds, kernel, extra=None, per="launch"):
    """The roofline object of the phase kernel: active VALU lane-instructions
    of `checks` resolved depletant checks and `moves` trial moves done in
    `seconds` (one launch, or one batched sweep), against the VALU peak."""
    prof = PROFILE[shape]
    d = {"bound": "alu", "kernel": kernel, "peak": VALU_PEAK_LANE_OPS / 1e12, "unit": "T VALU lane-instr/s",
         "avg_launch_ms" if per == "launch" else "avg_sweep_ms": seconds * 1e3}
    if profiled:
        ops = prof["a_dep"] * checks + prof["b_move"] * moves
        d.update({"achieved": ops / seconds / 1e12, "frac": ops / seconds / VALU_PEAK_LANE_OPS,
                  "basis": "active VALU lane-instructions (rocprofv3 SQ_INSTS_VALU x 64 x VALUUtilization of this "
                           f"kernel): {prof['a_dep']} per resolved depletant check + {prof['b_move']} per trial move",
                  "valu_busy_pct": prof["valu_busy"], "valu_utilization_pct": prof["valu_utilization"],
                  "valu_instr_per_move": prof["valu_instr_per_move"]})
        if "traffic_bytes_per_launch" in prof:
            d["traffic"] = prof["traffic_bytes_per_launch"]
            d["traffic_unit"] = "bytes per launch (rocprofv3 FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0)"
        else:
            d["traffic"] = prof["traffic_bytes_per_phase"]
            d["traffic_unit"] = "bytes per phase, both launch groups (rocprofv3 FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0)"
    else:
        d.update({"achieved": None, "frac": None, "traffic": None,
                  "basis": "kernel sources differ from the profiled ones: no calibration"})
    if extra:
        d.update(extra)
    return d


def _fp32_companion(hp, torch, sp, sim, region, args, launches):
    """the headline state point with FP32 depletant tests and the FP64 guard band"""
    s32 = hp.Sim(sp.n, sp.L, sp.seed, precision=hp.FP32_GUARDED)
    s32.set_shape(hp.SPHERE, sp.params)
    s32.set_fugacity(sp.z_p, sp.d_dep, sp.n_trial)
    s32.set_moves(sp.d_trans)
    s32.set_insertion(region)
    s32.set_state(sim.pos.clone())
    tot3, lat3, phase3, dt3 = _timed_sweeps(torch, s32, args.steps, args.warmup)
    fp32 = {
        "insertion_region": args.v0,
        "moves_per_s": tot3["trials"] / dt3,
        "depletant_checks_per_s": tot3["depletants_resolved"] / dt3,
        "ms_per_step": dt3 * 1e3 / args.steps,
        "avg_launch_ms": phase3 / launches,
        "fp64_fallbacks": tot3["fp64_fallbacks"],
        "fp64_fallbacks_per_depletant": tot3["fp64_fallbacks"] / max(tot3["depletants_drawn"], 1),
        "note": "FP32 depletant tests with a 1e-5 sigma FP64 guard band; decisions equal to FP64",
    }
    s32.close()
    return fp32


def _timed_sweeps(torch, sim, steps, warmup):
    """warmup untimed sweeps, then `steps` timed sweeps of one step each:
    (summed counters, per-step latencies in ms, summed phase-kernel ms, seconds)"""
    for _ in range(warmup):
        sim.sweep(1, counters=True)
    torch.cuda.synchronize()
    tot = None
    lat = []
    phase_ms = 0.0
    t0 = time.perf_counter()
    for _ in range(steps):
        ts = time.perf_counter()
        c = sim.sweep(1, counters=True)
        lat.append((time.perf_counter() - ts) * 1e3)
        phase_ms += c["phase_kernel_ms"]
        tot = c if tot is None else {k: tot[k] + c[k] for k in tot}
    torch.cuda.synchronize()
    return tot, lat, phase_ms, time.perf_counter() - t0


def _prepare(hp, sp):
    """a handle on the lattice start, set up for the untimed zero-fugacity melt"""
    pos, quat = sp.initial_state()
    sim = hp.Sim(sp.n, sp.L, sp.seed, sp.replica_id)
    sim.set_shape(sp.kind, sp.params)
    sim.set_fugacity(0.0, sp.d_dep, 0)
    sim.set_moves(0.1, 0.1 if sp.kind != 0 else 0.0, sp.p_rot)
    sim.set_state(pos, quat)
    return sim


def _finish(sim, sp):
    """after the melt: the state point's depletants and step sizes"""
    sim.set_fugacity(sp.z_p, sp.d_dep, sp.n_trial)
    sim.set_moves(sp.d_trans, sp.a_rot, sp.p_rot)
    sim.ensure_workspace()
    return sim


def _make(hp, sp, melt=20):
    sim = _prepare(hp, sp)
    if melt:
        sim.sweep(melt, counters=False)
    return _finish(sim, sp)


def _group_shapes(shapes):
    """the launch shapes hpmc_autotune_batch chose, one entry per launch group"""
    groups = {}
    for t in shapes:
        key = (t["cells_per_wave"], t["waves_per_block"], t["max_waves"], t["best_ms"], t["default_ms"])
        g = groups.setdefault(key, dict(t, replicas=0))
        g["replicas"] += 1
    return list(groups.values())


def _line(metric_value, tot, dt, steps, warmup, workload, extra):
    d = {
        "metric": "colloid trial moves/s + depletant overlap checks/s (1 GPU); p50/p99 latency",
        "value": metric_value,
        "unit": "colloid trial moves/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": dt * 1e3 / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": workload},
        "depletant_checks_per_s": tot["depletants_resolved"] / dt,
        "acceptance": tot["accepts"] / max(tot["trials"], 1),
    }
    if "overlap_checks" in tot:
        # colloid pair tests executed (spheres: every stencil entry; convex shapes: the narrow phase)
        d["pair_tests_per_s"] = tot["overlap_checks"] / dt
    d.update(extra)
    return d


def bench_c1(args):
    """64 spheres, 1000 sweeps: launch/latency bound.  Throughput from one
    untimed 1000-sweep call (a replayed captured sweep); latency per sweep from
    timed single-sweep calls."""
    import numpy as np
    import torch

    import paper_1508_07077_amd as hp
    from paper_1508_07077_amd import workloads as wl

    sp = wl.c1_spheres_small()
    sim = _make(hp, sp, melt=100)
    sim.sweep(10, counters=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.sweep(1000, counters=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    lat = []
    tot = None
    for _ in range(200):
        ts = time.perf_counter()
        c = sim.sweep(1, counters=True)
        lat.append((time.perf_counter() - ts) * 1e3)
        tot = c if tot is None else {k: tot[k] + c[k] for k in tot}
    extra = {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
             "latency_note": "per-sweep latency of timed single-sweep calls (launch + counter readback)"}
    if args.cpu_seconds > 0:
        extra["cpu_baseline"] = cpu_baseline_states([sp], 1000, args.cpu_seconds, "the same 64-sphere box, 1000 sweeps")
    return _line(1000 * sp.n / dt, {"depletants_resolved": tot["depletants_resolved"] * 1000 / 200,
                                     "accepts": tot["accepts"], "trials": tot["trials"]}, dt, 1000, 10,
                 "hard spheres N=64 phi_c=0.10 q=0.25 eta_r=0.10 delta=0.1, 1000 sweeps (graph replay)", extra)


def bench_c2(args):
    """16384 hemispheres at phi_c = 0.20, q = 0.15, eta_r = 0.1 .. 0.4,
    translate + rotate (p_rot = 0.5), FP64."""
    import numpy as np
    import torch

    import paper_1508_07077_amd as hp
    from paper_1508_07077_amd import workloads as wl

    per = {}
    roofs = {}
    moves = checks = secs = 0.0
    lat = []
    fp32 = {}
    kept = []
    profiled = kernel_digest() == PROFILED_KERNEL_DIGEST
    for eta in [float(x) for x in args.eta.split(",")]:
        sp = wl.c2_hemispheres(eta)
        sim = _make(hp, sp)
        tuning = sim.autotune(sweeps=2) if args.autotune else None
        for _ in range(3):
            sim.sweep(1, counters=True)
        torch.cuda.synchronize()
        tot = None
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ts = time.perf_counter()
            c = sim.sweep(1, counters=True)
            lat.append((time.perf_counter() - ts) * 1e3)
            tot = c if tot is None else {k: tot[k] + c[k] for k in tot}
        dt = time.perf_counter() - t0
        launches = 8 * args.steps
        roof = _roofline("hemisphere", profiled, tot["depletants_resolved"] / launches, tot["trials"] / launches,
                         tot["phase_kernel_ms"] / 1e3 / launches, "phase_oriented_kernel<hemisphere>")
        per[str(eta)] = {"moves_per_s": tot["trials"] / dt, "depletant_checks_per_s": tot["depletants_resolved"] / dt,
                         "acceptance": tot["accepts"] / tot["trials"], "ms_per_sweep": dt * 1e3 / args.steps,
                         "z_p": sp.z_p, "delta": sp.d_trans, "near_contact_trials": tot["near_contact"],
                         "launch_tuning": tuning, "roofline_frac": roof["frac"],
                         "avg_launch_ms": roof["avg_launch_ms"]}
        roofs[str(eta)] = roof
        moves += tot["trials"]
        checks += tot["depletants_resolved"]
        secs += dt
        kept.append(sim)
        if not args.fp32:
            continue
        # the same state point with FP32 depletant predicates and the FP64 guard band
        s32 = hp.Sim(sp.n, sp.L, sp.seed, sp.replica_id, precision=hp.FP32_GUARDED)
        s32.set_shape(sp.kind, sp.params)
        s32.set_fugacity(sp.z_p, sp.d_dep, sp.n_trial)
        s32.set_moves(sp.d_trans, sp.a_rot, sp.p_rot)
        pq, qq, _ = sim.get_state()
        s32.set_state(pq, qq)
        if tuning:
            s32.set_tuning(tuning["cells_per_wave"], tuning["waves_per_block"], tuning["max_waves"])
        t3, _, _, dt3 = _timed_sweeps(torch, s32, args.steps, 3)
        fp32[str(eta)] = {"moves_per_s": t3["trials"] / dt3, "fp64_fallbacks": t3["fp64_fallbacks"],
                          "fp64_fallbacks_per_depletant": t3["fp64_fallbacks"] / max(t3["depletants_drawn"], 1)}
        s32.close()
    if not args.batch:
        for x in kept:
            x.close()
        d = _line(moves / secs, {"depletants_resolved": checks, "accepts": 1, "trials": 1}, secs, len(per) * args.steps,
                  3, f"hemispheres N=16384 phi_c=0.20 q=0.15 eta_r in {{{args.eta}}}, p_rot=0.5, FP64, one at a time",
                  {"per_eta_r": per, "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                   "fp32_guarded_per_eta_r": fp32,
                   "roofline": roofs.get("0.4", roofs[max(roofs)]) if roofs else None})
        d.pop("acceptance")
        return d
    # the state points swept together: one batched launch per phase for all of
    # them (independent replicas, each with its own random streams), which gives
    # the device len(eta) times the independent cells of one state point
    b = hp.Batch(kept)
    btuning = _group_shapes(b.autotune(sweeps=2)) if args.autotune else None
    for _ in range(3):
        b.sweep(1, counters=True)
    torch.cuda.synchronize()
    btot = None
    dev_ms = 0.0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        cs = b.sweep(1, counters=True, as_array=True)
        dev_ms += float(cs["sweep_ms"][0])
        c = {k: int(cs[k].sum()) for k in hp.COUNTERS}
        btot = c if btot is None else {k: btot[k] + c[k] for k in btot}
    bdt = time.perf_counter() - t0
    broof = _roofline("hemisphere", profiled, btot["depletants_resolved"] / args.steps, btot["trials"] / args.steps,
                      dev_ms / 1e3 / args.steps,
                      "phase_oriented_kernel<hemisphere> (one launch per phase for all state points; the time is "
                      "the whole batched sweep on the device, cell lists included)", per="sweep")
    for x in kept:
        x.close()
    one_at_a_time = {"moves_per_s": moves / secs, "depletant_checks_per_s": checks / secs,
                     "note": "each state point swept alone, one after the other"}
    d = _line(btot["trials"] / bdt, btot, bdt, args.steps, 3,
              f"hemispheres N=16384 phi_c=0.20 q=0.15 eta_r in {{{args.eta}}}, p_rot=0.5, FP64, "
              "the state points swept together",
              {"per_eta_r": per, "one_at_a_time": one_at_a_time, "batched_ms_per_sweep": bdt * 1e3 / args.steps,
               "batch_launch_tuning": btuning,
               "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
               "fp32_guarded_per_eta_r": fp32,
               "roofline": broof,
               # one state point alone, per launch (the one with the most depletant work)
               "roofline_one_state_point": roofs.get("0.4", roofs[max(roofs)]) if roofs else None})
    d.pop("acceptance")
    if args.cpu_seconds > 0:
        etas = [float(x) for x in args.eta.split(",")]
        d["cpu_baseline"] = cpu_baseline_states([wl.c2_hemispheres(e) for e in etas], 5, args.cpu_seconds,
                                                "the same 16,384-hemisphere boxes, 5 sweeps per eta_r")
    return d


def bench_c4(args):
    """256 independent discoid replicas (disk 0.5 swept by 0.1), N log-uniform in
    [128, 8192], phi_c U[0.05, 0.45], eta_r U[0, 0.5], q = 0.2, swept together."""
    import numpy as np
    import torch

    import paper_1508_07077_amd as hp
    from paper_1508_07077_amd import workloads as wl

    sps = wl.c4_discoid_replicas()
    sims = [_prepare(hp, sp) for sp in sps]
    hp.Batch(sims).sweep(20, counters=False)  # the untimed melt, all replicas together
    sims = [_finish(x, sp) for x, sp in zip(sims, sps)]
    b = hp.Batch(sims)
    # per launch group: the candidate shapes timed with the group's members swept together
    tuning = _group_shapes(b.autotune(sweeps=2)) if args.autotune else None
    for _ in range(3):
        b.sweep(1, counters=True)
    torch.cuda.synchronize()
    lat = []
    tot = None
    dev_ms = 0.0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        cs = b.sweep(1, counters=True, as_array=True)
        lat.append((time.perf_counter() - ts) * 1e3)
        dev_ms += float(cs["sweep_ms"][0])
        c = {k: int(cs[k].sum()) for k in hp.COUNTERS}
        tot = c if tot is None else {k: tot[k] + c[k] for k in tot}
    dt = time.perf_counter() - t0
    roof = _roofline("discoid", kernel_digest() == PROFILED_KERNEL_DIGEST, tot["depletants_resolved"] / args.steps,
                     tot["trials"] / args.steps, dev_ms / 1e3 / args.steps,
                     "phase_oriented_kernel<discoid> (two launch groups per phase; the time is the whole batched "
                     "sweep on the device, cell lists included)", per="sweep")
    # the same batch, untimed calls of several sweeps: one captured sweep replayed
    torch.cuda.synchronize()
    tg = time.perf_counter()
    b.sweep(args.steps, counters=False)
    torch.cuda.synchronize()
    dtg = time.perf_counter() - tg
    graph = {"moves_per_s": args.steps * sum(x.n for x in sims) / dtg, "ms_per_sweep": dtg * 1e3 / args.steps,
             "note": "one call of `steps` sweeps without counters: a captured batched sweep replayed"}
    alone = None
    # the same replicas swept one at a time (each handle's own launches), for comparison
    for x in (sims if args.alone else []):
        x.sweep(1, counters=False)
    if args.alone:
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(2):
            for x in sims:
                x.sweep(1, counters=False)
        torch.cuda.synchronize()
        dt1 = time.perf_counter() - t1
        alone = {"moves_per_s": 2 * sum(x.n for x in sims) / dt1, "ms_per_sweep": dt1 * 1e3 / 2,
                 "note": "the same replicas, each swept alone in turn (2 sweeps)"}
    return _line(tot["trials"] / dt, tot, dt, args.steps, 3,
                 f"256 swept-disk replicas, N={sum(s.n for s in sps)} in total (128..8192 each), "
                 "phi_c U[0.05,0.45], eta_r U[0,0.5], q=0.2, one launch per kernel for all replicas",
                 {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                  "replicas": len(sps), "launch_tuning": tuning, "graph_replay": graph, "one_at_a_time": alone,
                  "roofline": roof,
                  "cpu_baseline": cpu_baseline_states(sps[::32], 5, args.cpu_seconds,
                                                      "8 of the 256 replicas (every 32nd), 5 sweeps each")
                  if args.cpu_seconds > 0 else None})


def bench_c5(args):
    """Poisson arrivals at 50 req/s of {sphere, hemisphere, discoid} requests,
    N log-uniform in [256, 65536], phi_c in [0.05, 0.45], eta_r in [0, 0.5],
    100 sweeps each, returning g(r), the free-volume fraction and the SDF
    pressure; HBM-budget admission and continuous batching (serve.Server)."""
    import torch

    from paper_1508_07077_amd import serve
    from paper_1508_07077_amd import workloads as wl

    specs = wl.c5_request_stream(duration_s=args.serve_seconds)
    reqs = [serve.Request(sp, sp.extra["sweeps"], sp.extra["arrival_s"], rid=i) for i, sp in enumerate(specs)]
    srv = serve.Server(sweeps_per_tick=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = srv.run(reqs, realtime=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    summ = serve.latency_summary(done)
    errors = sum(1 for r in done if "error" in r.result)
    offered = sum(sp.n * sp.extra["sweeps"] for sp in specs) / args.serve_seconds
    # capacity with every request of a sample available at once: continuous
    # batching against one request at a time, same requests and work
    sample = specs[: args.capacity_requests]
    cap = {}
    for label, max_active in (("batched", 256), ("one_at_a_time", 1)):
        rq = [serve.Request(sp, sp.extra["sweeps"], 0.0, rid=i) for i, sp in enumerate(sample)]
        s2 = serve.Server(sweeps_per_tick=1, max_active=max_active)
        torch.cuda.synchronize()
        tc = time.perf_counter()
        s2.run(rq, realtime=False)
        torch.cuda.synchronize()
        cap[label + "_moves_per_s"] = s2.moves / (time.perf_counter() - tc)
    cap["requests"] = len(sample)
    return {
        "metric": "colloid trial moves/s + depletant overlap checks/s (1 GPU); p50/p99 latency",
        "value": srv.moves / dt,
        "unit": "colloid trial moves/s",
        "n_gpus": 1,
        "steps": len(done),
        "warmup": 0,
        "ms_per_step": dt * 1e3 / max(len(done), 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"request stream: Poisson arrivals 50 req/s for {args.serve_seconds} s, "
                               "{sphere q=0.10, hemisphere q=0.15, discoid q=0.2}, N log-uniform [256, 65536], "
                               "phi_c U[0.05,0.45], eta_r U[0,0.5], 100 sweeps + g(r), alpha, SDF each"},
        "p50_ms": summ["p50_s"] * 1e3,
        "p99_ms": summ["p99_s"] * 1e3,
        "requests": summ["requests"],
        "failed_requests": errors,
        "offered_load_moves_per_s": offered,
        "achieved_moves_per_s": srv.moves / dt,
        "max_active_requests": max((n for _, _, n in srv.ticks), default=0),
        "max_bytes_held": max((u for _, u, _ in srv.ticks), default=0),
        "hbm_budget": srv.budget,
        "latency_note": "per request, arrival to observables returned",
        "capacity": cap,
        "cpu_baseline": cpu_baseline_states(specs[:10], 100, args.cpu_seconds,
                                            "the first 10 requests of the stream, 100 sweeps each (sweeps only)")
        if args.cpu_seconds > 0 else None,
    }


OTHER = {"c1": bench_c1, "c2": bench_c2, "c4": bench_c4, "c5": bench_c5}


if __name__ == "__main__":
    main()
