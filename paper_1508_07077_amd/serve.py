"""Continuous-batching request server for implicit-depletant simulations.

A request is one simulation (shape, N, phi_c, eta_r, number of sweeps) that
returns g(r), the free-volume fraction (phi_p = phi_p^r alpha, the quantity of
Sec. IV.A of Glaser, Karas & Glotzer, arXiv:1508.07077) and the SDF pressure.

Scheduling: requests wait in an arrival queue.  At every tick boundary (one
sweep of every active request) the server admits waiting requests, in arrival
order, while a slot is free and their device memory fits the HBM budget, then
enqueues one batched sweep of every active request (hpmc_sweep_batch: one
launch per kernel for all replicas of a shape kind).  Requests that arrive
while others run join at the next tick, and their work overlaps on the device.
A request whose sweeps are done is measured and retired, which frees its slot
and memory.  Each request keeps its own random streams (seed, replica id), so
its result does not depend on what else is in the batch.

Memory: a request costs exactly what the library asks for (hpmc_workspace_bytes
for its settings) plus its state (24 bytes per colloid, 32 more for
orientations); the server's one batch workspace, sized for max_active slots,
is charged at start.  A request that could never fit is refused with an error;
the sum of what is held never exceeds the budget.

Ticks do not wait for the device: the batch workspace and the descriptor
staging are reused, and hpmc_sweep_batch without counters only enqueues.  The
host waits only when a request is admitted (its state upload and hard-core
check) or retired (its observables).
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import HpmcError, OBS_FREE_VOLUME, OBS_GR, OBS_SDF, Batch, Sim


@dataclass
class Request:
    spec: object                 # workloads.StatePoint
    sweeps: int
    arrival: float               # seconds on the server clock
    rid: int = 0
    admitted: float = -1.0
    finished: float = -1.0
    done_sweeps: int = 0
    sim: object = None
    bytes: int = 0
    result: dict = field(default_factory=dict)


def state_bytes(sp) -> int:
    """device bytes of a request's state: positions (and orientations)"""
    return sp.n * 24 + (sp.n * 32 if sp.kind != 0 else 0)


class Server:
    def __init__(self, hbm_budget: int | None = None, max_active: int = 256, sweeps_per_tick: int = 1,
                 device: str = "cuda:0", obs_probes: int = 50000, keep_state: bool = False):
        import torch

        self.torch = torch
        self.device = device
        free, _total = torch.cuda.mem_get_info(torch.device(device))
        self.budget = int(0.8 * free) if hbm_budget is None else int(hbm_budget)
        self.max_active = max_active
        self.sweeps_per_tick = sweeps_per_tick
        self.obs_probes = obs_probes
        self.keep_state = keep_state
        self.batch = Batch([], capacity=max_active, device=device)
        self.used = self.batch.workspace.numel()
        if self.used > self.budget:
            raise ValueError(f"HBM budget {self.budget} B is smaller than the batch workspace ({self.used} B)")
        self.active: list[Request] = []
        self.waiting: deque[Request] = deque()
        self.finished: list[Request] = []
        self.ticks: list[tuple[float, int, int]] = []  # (time, bytes held, active requests) per tick
        self.t0 = None

    def now(self) -> float:
        return time.perf_counter() - self.t0

    # -- request lifecycle ------------------------------------------------
    def _handle(self, req: Request) -> int:
        """create the request's handle (host only) and return its device bytes"""
        sp = req.spec
        sim = Sim(sp.n, sp.L, sp.seed, sp.replica_id, device=self.device)
        sim.set_shape(sp.kind, sp.params)
        sim.set_fugacity(sp.z_p, sp.d_dep, sp.n_trial)
        sim.set_moves(sp.d_trans, sp.a_rot, sp.p_rot)
        req.sim = sim
        return sim.workspace_bytes() + state_bytes(sp)

    def _refuse(self, req: Request, msg: str):
        req.result = {"error": msg}
        req.finished = self.now()
        if req.sim is not None:
            req.sim.close()
            req.sim = None
        self.finished.append(req)

    def _admit(self):
        while self.waiting and len(self.active) < self.max_active:
            req = self.waiting[0]
            if req.sim is None:
                try:
                    req.bytes = self._handle(req)
                except HpmcError as e:
                    self.waiting.popleft()
                    self._refuse(req, str(e))
                    continue
            if req.bytes > self.budget - self.batch.workspace.numel():
                self.waiting.popleft()
                self._refuse(req, f"needs {req.bytes} B of device memory; the HBM budget leaves "
                                  f"{self.budget - self.batch.workspace.numel()} B for requests")
                continue
            if self.used + req.bytes > self.budget:
                break  # waits for memory (arrival order is kept)
            self.waiting.popleft()
            try:
                pos, quat = req.spec.initial_state()
                req.sim.set_state(pos, quat)
            except HpmcError as e:
                self._refuse(req, str(e))
                continue
            self.used += req.bytes
            req.admitted = self.now()
            self.active.append(req)

    def _measure(self, req: Request):
        sp, sim = req.spec, req.sim
        r_max = min(3.0, 0.5 * sp.L)
        g = sim.observables(OBS_GR, n_bins=60, r_max=r_max)
        fv = sim.observables(OBS_FREE_VOLUME, n_probe=self.obs_probes, obs_seq=1)
        sdf = sim.observables(OBS_SDF, n_bins=20, x_max=0.05, n_fit=6, n_probe=self.obs_probes, obs_seq=2,
                              eps=0.01)
        req.result = {"g_r": g, "r_max": r_max, "alpha": float(fv[0]), "phi_p": float(fv[1]),
                      "beta_P": float(sdf[0]), "beta_P_hard": float(sdf[1]), "beta_P_dep": float(sdf[2])}
        if self.keep_state:
            pos, quat, sweep = sim.get_state()
            req.result.update({"pos": pos, "quat": quat, "sweep": sweep})

    def _retire(self, req: Request):
        try:
            self._measure(req)
        except HpmcError as e:
            req.result = {"error": str(e)}
        req.finished = self.now()
        self.used -= req.bytes
        req.sim.close()
        req.sim = None
        self.finished.append(req)

    # -- main loop --------------------------------------------------------
    def run(self, requests: list[Request], realtime: bool = True) -> list[Request]:
        """Serve `requests` (sorted by arrival).  With realtime, arrivals follow
        the wall clock; otherwise every request is available at once."""
        self.t0 = time.perf_counter()
        pending = deque(sorted(requests, key=lambda r: r.arrival))
        moves = 0
        members = None
        while pending or self.waiting or self.active:
            t = self.now()
            while pending and (not realtime or pending[0].arrival <= t):
                self.waiting.append(pending.popleft())
            self._admit()
            if not self.active:
                if pending:
                    time.sleep(max(0.0, min(0.01, pending[0].arrival - self.now())))
                elif self.waiting:
                    raise RuntimeError("a waiting request cannot be admitted into an empty server")
                continue
            if members != [r.rid for r in self.active]:
                members = [r.rid for r in self.active]
                self.batch.set_members([r.sim for r in self.active])
            k = min([self.sweeps_per_tick] + [r.sweeps - r.done_sweeps for r in self.active])
            self.batch.sweep(k, counters=False)
            self.ticks.append((self.now(), self.used, len(self.active)))
            for r in self.active:
                r.done_sweeps += k
                moves += k * r.spec.n
            done = [r for r in self.active if r.done_sweeps >= r.sweeps]
            if done:
                self.active = [r for r in self.active if r.done_sweeps < r.sweeps]
                for r in done:
                    self._retire(r)
        self.moves = moves
        return self.finished


def latency_summary(finished: list[Request]) -> dict:
    lat = np.array([r.finished - r.arrival for r in finished if r.finished >= 0])
    return {"requests": len(lat), "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean())}
