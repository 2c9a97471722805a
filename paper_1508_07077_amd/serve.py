"""Continuous-batching request server for implicit-depletant simulations.

A request is one simulation (shape, N, phi_c, eta_r, number of sweeps) that
returns g(r), the free-volume fraction (phi_p = phi_p^r alpha, the quantity of
Sec. IV.A of Glaser, Karas & Glotzer, arXiv:1508.07077) and the SDF pressure.

Scheduling: requests wait in an arrival queue; at every tick boundary the
server admits waiting requests while their device memory (state + workspace)
fits the HBM budget and a slot is free, then sweeps every active request
together in one batched call (hpmc_sweep_batch: one launch per kernel for all
replicas of a shape kind), so requests that arrive while others run join the
next tick and their work overlaps on the device.  A request whose sweeps are
done is measured and retired, which frees its slot and memory.  Each request
keeps its own random streams (seed, replica id), so its result does not depend
on what else is in the batch.
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


class Server:
    def __init__(self, hbm_budget: int | None = None, max_active: int = 256, sweeps_per_tick: int = 1,
                 device: str = "cuda:0", obs_probes: int = 50000):
        import torch

        self.torch = torch
        self.device = device
        free, _total = torch.cuda.mem_get_info(torch.device(device))
        self.budget = int(0.8 * free) if hbm_budget is None else int(hbm_budget)
        self.max_active = max_active
        self.sweeps_per_tick = sweeps_per_tick
        self.obs_probes = obs_probes
        self.used = 0
        self.active: list[Request] = []
        self.waiting: deque[Request] = deque()
        self.finished: list[Request] = []
        self.t0 = None

    def now(self) -> float:
        return time.perf_counter() - self.t0

    # -- request lifecycle ------------------------------------------------
    def _open(self, req: Request):
        sp = req.spec
        sim = Sim(sp.n, sp.L, sp.seed, sp.replica_id, device=self.device)
        sim.set_shape(sp.kind, sp.params)
        sim.set_fugacity(sp.z_p, sp.d_dep, sp.n_trial)
        sim.set_moves(sp.d_trans, sp.a_rot, sp.p_rot)
        pos, quat = sp.initial_state()
        sim.set_state(pos, quat)
        req.sim = sim
        req.bytes = sim.workspace.numel() + sim.pos.numel() * 8 + (sim.quat.numel() * 8 if sim.quat is not None else 0)

    def _estimate(self, req: Request) -> int:
        sp = req.spec
        # state + cell-ordered records + cell lists dominate the workspace
        return int(sp.n * (24 + 32 + 12) * (2 if sp.kind != 0 else 1) + 2 ** 20)

    def _admit(self):
        while self.waiting and len(self.active) < self.max_active:
            req = self.waiting[0]
            if self.used + self._estimate(req) > self.budget and self.active:
                break
            self.waiting.popleft()
            try:
                self._open(req)
            except HpmcError as e:
                req.result = {"error": str(e)}
                req.finished = self.now()
                self.finished.append(req)
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

    def _retire(self, req: Request):
        self._measure(req)
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
        while pending or self.waiting or self.active:
            t = self.now()
            while pending and (not realtime or pending[0].arrival <= t):
                self.waiting.append(pending.popleft())
            self._admit()
            if not self.active:
                if pending:
                    time.sleep(max(0.0, min(0.01, pending[0].arrival - self.now())))
                continue
            k = min([self.sweeps_per_tick] + [r.sweeps - r.done_sweeps for r in self.active])
            Batch([r.sim for r in self.active]).sweep(k, counters=False)
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
