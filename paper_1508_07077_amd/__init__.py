"""MI355X implicit-depletant hard-particle Monte Carlo (Glaser, Karas & Glotzer,
arXiv:1508.07077) -- thin ctypes binding of ``libhpmc.so``.

Every step of a sweep runs in the library's HIP kernels; this module only
marshals arguments.  PyTorch provides device memory (state tensors and the
workspace) and the stream.  The C-ABI is declared in ``include/hpmc.h``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhpmc.so")

SPHERE, HEMISPHERE, DISCOID = 0, 1, 2
FP64, FP32_GUARDED = 0, 1
ACCEPT, REJ_CELL_EXIT, REJ_OVERLAP, REJ_DEPLETANT, REJ_CB_ZERO, REJ_CB_METROPOLIS = range(6)
OBS_GR, OBS_FREE_VOLUME, OBS_SDF = 0, 1, 2
V0_BALL, V0_SHELL = 0, 1

ERRORS = {
    -1: "HPMC_EINVAL",
    -2: "HPMC_EBOX",
    -3: "HPMC_EOVERLAP",
    -4: "HPMC_ENOMEM",
    -5: "HPMC_ESTATE",
    -6: "HPMC_EHIP",
    -7: "HPMC_ECAPACITY",
}

EXPORTS = (
    "hpmc_create",
    "hpmc_destroy",
    "hpmc_last_error",
    "hpmc_set_shape",
    "hpmc_set_fugacity",
    "hpmc_set_moves",
    "hpmc_set_insertion",
    "hpmc_workspace_bytes",
    "hpmc_set_workspace",
    "hpmc_set_state",
    "hpmc_get_state",
    "hpmc_set_trace",
    "hpmc_sweep",
    "hpmc_sweep_static",
    "hpmc_observables",
    "hpmc_trace",
    "hpmc_batch_workspace_bytes",
    "hpmc_sweep_batch",
    "hpmc_set_tuning",
    "hpmc_autotune",
    "hpmc_autotune_batch",
    "hpmc_poisson_draw",
)

COUNTERS = (
    "trials",
    "accepts",
    "rej_cell_exit",
    "rej_overlap",
    "rej_depletant",
    "rej_cb_zero",
    "rej_cb_metropolis",
    "depletants_drawn",
    "depletants_resolved",
    "cb_trials",
    "overlap_checks",
    "near_contact",
    "fp64_fallbacks",
)

MOVE_RECORD = np.dtype(
    [
        ("sweep", "<u4"), ("cell", "<u4"), ("t", "<u4"), ("particle", "<u4"),
        ("n_depletants", "<u4"), ("resolved", "<u4"), ("n_blocking", "<u4"),
        ("w_fwd", "<u4"), ("w_rev", "<u4"),
        ("phase", "u1"), ("reason", "u1"), ("rotation", "u1"), ("near_contact", "u1"),
    ]
)


class HpmcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class _Counters(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint64) for f in COUNTERS] + [("phase_kernel_ms", ctypes.c_double),
                                                          ("sweep_ms", ctypes.c_double)]


# the counter record as a numpy structured type (Batch.sweep(as_array=True))
COUNTER_DTYPE = np.dtype([(f, "<u8") for f in COUNTERS] + [("phase_kernel_ms", "<f8"), ("sweep_ms", "<f8")])
assert COUNTER_DTYPE.itemsize == ctypes.sizeof(_Counters)


class _Tuning(ctypes.Structure):
    _fields_ = [
        ("cells_per_wave", ctypes.c_int32),
        ("waves_per_block", ctypes.c_int32),
        ("max_waves", ctypes.c_int32),
        ("candidates", ctypes.c_int32),
        ("best_ms", ctypes.c_double),
        ("default_ms", ctypes.c_double),
    ]


class _ObsParams(ctypes.Structure):
    _fields_ = [
        ("n_bins", ctypes.c_int32), ("n_fit", ctypes.c_int32),
        ("r_max", ctypes.c_double), ("x_max", ctypes.c_double),
        ("n_probe", ctypes.c_int64), ("obs_seq", ctypes.c_uint32), ("pad", ctypes.c_uint32),
        ("eps", ctypes.c_double),
    ]


_lib = None


def lib():
    """Load libhpmc.so; fails loudly when the HIP library has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"HIP library missing: {LIB_PATH} (build it with paper_1508_07077_amd.build.build())")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, u64, u32, dbl, cint = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint32,
                                        ctypes.c_double, ctypes.c_int)
        dp = ctypes.POINTER(ctypes.c_double)
        L.hpmc_create.argtypes = [ctypes.POINTER(vp), i64, dbl, u64, u32, cint, vp]
        L.hpmc_destroy.argtypes = [vp]
        L.hpmc_destroy.restype = None
        L.hpmc_last_error.argtypes = [vp]
        L.hpmc_last_error.restype = ctypes.c_char_p
        L.hpmc_set_shape.argtypes = [vp, cint, dp, cint]
        L.hpmc_set_fugacity.argtypes = [vp, dbl, dbl, cint]
        L.hpmc_set_moves.argtypes = [vp, dbl, dbl, dbl, cint]
        L.hpmc_set_insertion.argtypes = [vp, cint]
        L.hpmc_workspace_bytes.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
        L.hpmc_set_workspace.argtypes = [vp, vp, ctypes.c_size_t]
        L.hpmc_set_state.argtypes = [vp, vp, vp, u64]
        L.hpmc_get_state.argtypes = [vp, ctypes.POINTER(u64)]
        L.hpmc_set_trace.argtypes = [vp, cint]
        L.hpmc_sweep.argtypes = [vp, cint, ctypes.POINTER(_Counters)]
        L.hpmc_sweep_static.argtypes = [vp, cint, ctypes.POINTER(_Counters)]
        L.hpmc_observables.argtypes = [vp, cint, ctypes.POINTER(_ObsParams), dp, i64]
        L.hpmc_trace.argtypes = [vp, vp, i64, ctypes.POINTER(i64)]
        L.hpmc_batch_workspace_bytes.argtypes = [cint, ctypes.POINTER(ctypes.c_size_t)]
        L.hpmc_sweep_batch.argtypes = [ctypes.POINTER(vp), cint, vp, ctypes.c_size_t, cint, ctypes.POINTER(_Counters)]
        L.hpmc_set_tuning.argtypes = [vp, ctypes.POINTER(_Tuning)]
        L.hpmc_autotune.argtypes = [vp, vp, ctypes.c_size_t, cint, ctypes.POINTER(_Tuning)]
        L.hpmc_poisson_draw.argtypes = [vp, dbl, ctypes.POINTER(ctypes.c_int32)]
        L.hpmc_autotune_batch.argtypes = [ctypes.POINTER(vp), cint, vp, ctypes.c_size_t, vp, ctypes.c_size_t, cint,
                                          ctypes.POINTER(_Tuning)]
        for name in EXPORTS:
            if name not in ("hpmc_destroy", "hpmc_last_error"):
                getattr(L, name).restype = cint
        _lib = L
    return _lib


class Sim:
    """One simulation handle.  Device state and workspace are torch tensors on
    ``device``; the library borrows them."""

    def __init__(self, n: int, box_L: float, seed: int, replica_id: int = 0, precision: int = FP64,
                 device: str = "cuda:0", stream=None):
        import torch

        self.torch = torch
        self.device = torch.device(device)
        self.n = int(n)
        self.L = float(box_L)
        # no stream given: the library's own blocking stream (ordered with torch's
        # null-stream work, and capturable into a graph)
        self._stream = stream
        h = ctypes.c_void_p()
        rc = lib().hpmc_create(ctypes.byref(h), self.n, self.L, int(seed) & (2**64 - 1), int(replica_id),
                               int(precision), ctypes.c_void_p(stream.cuda_stream if stream is not None else None))
        if rc != 0:
            raise HpmcError(rc, "hpmc_create")
        self._h = h
        self.workspace = None
        self.pos = None
        self.quat = None
        self.kind = None

    def close(self):
        if getattr(self, "_h", None):
            lib().hpmc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, rc: int, what: str):
        if rc != 0:
            msg = lib().hpmc_last_error(self._h)
            raise HpmcError(rc, f"{what}: {msg.decode() if msg else ''}")

    def set_shape(self, kind: int, params):
        p = np.ascontiguousarray(params, dtype=np.float64)
        self.kind = kind
        self._chk(lib().hpmc_set_shape(self._h, kind, p.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), len(p)),
                  "set_shape")

    def set_fugacity(self, z_p: float, d_dep: float, n_trial: int = 0):
        self._chk(lib().hpmc_set_fugacity(self._h, float(z_p), float(d_dep), int(n_trial)), "set_fugacity")

    def poisson_draw(self, u: float) -> int:
        """The depletant chunk count the sweeps draw for the 52-bit uniform u
        (hpmc_poisson_draw: host evaluation of the device's table)."""
        k = ctypes.c_int32(0)
        self._chk(lib().hpmc_poisson_draw(self._h, float(u), ctypes.byref(k)), "poisson_draw")
        return int(k.value)

    def set_moves(self, d_trans: float, a_rot: float = 0.0, p_rot: float = 0.0, n_select: int = 1):
        self._chk(lib().hpmc_set_moves(self._h, float(d_trans), float(a_rot), float(p_rot), int(n_select)),
                  "set_moves")

    def set_insertion(self, region: int):
        """V0_BALL (circumsphere of the new pose) or V0_SHELL (that ball less the core
        that stays inside the old pose)."""
        self._chk(lib().hpmc_set_insertion(self._h, int(region)), "set_insertion")

    def set_trace(self, enable: bool = True):
        self._chk(lib().hpmc_set_trace(self._h, 1 if enable else 0), "set_trace")
        self.ensure_workspace()

    def workspace_bytes(self) -> int:
        b = ctypes.c_size_t(0)
        self._chk(lib().hpmc_workspace_bytes(self._h, ctypes.byref(b)), "workspace_bytes")
        return int(b.value)

    def ensure_workspace(self):
        need = self.workspace_bytes()
        if self.workspace is None or self.workspace.numel() < need:
            self.workspace = self.torch.empty(need, dtype=self.torch.uint8, device=self.device)
        self._chk(lib().hpmc_set_workspace(self._h, ctypes.c_void_p(self.workspace.data_ptr()),
                                           self.workspace.numel()), "set_workspace")

    def set_state(self, pos, quat=None, sweep: int = 0, workspace: bool = True):
        """pos [3][n], quat [4][n] (oriented shapes): host arrays or device tensors.
        workspace=False allocates no workspace (for sweep_static only)."""
        torch = self.torch
        if workspace:
            self.ensure_workspace()
        self.pos = torch.as_tensor(np.asarray(pos) if not torch.is_tensor(pos) else pos, dtype=torch.float64)
        self.pos = self.pos.reshape(3, self.n).to(self.device).contiguous()
        qptr = None
        if quat is not None:
            q = torch.as_tensor(np.asarray(quat) if not torch.is_tensor(quat) else quat, dtype=torch.float64)
            self.quat = q.reshape(4, self.n).to(self.device).contiguous()
            qptr = ctypes.c_void_p(self.quat.data_ptr())
        torch.cuda.synchronize(self.device)  # the copies above ran on torch's stream
        self._chk(lib().hpmc_set_state(self._h, ctypes.c_void_p(self.pos.data_ptr()), qptr, int(sweep)), "set_state")

    def get_state(self):
        """(pos [3][n] numpy, quat [4][n] numpy or None, sweep index)."""
        sw = ctypes.c_uint64(0)
        self._chk(lib().hpmc_get_state(self._h, ctypes.byref(sw)), "get_state")
        self.torch.cuda.synchronize(self.device)  # sweeps still in flight on the handle's stream
        pos = self.pos.cpu().numpy().copy()
        quat = self.quat.cpu().numpy().copy() if self.quat is not None else None
        return pos, quat, int(sw.value)

    def sweep(self, n_sweeps: int = 1, counters: bool = True):
        c = _Counters()
        self._chk(lib().hpmc_sweep(self._h, int(n_sweeps), ctypes.byref(c) if counters else None), "sweep")
        if counters:
            d = {f: int(getattr(c, f)) for f in COUNTERS}
            d["phase_kernel_ms"] = float(c.phase_kernel_ms)
            d["sweep_ms"] = float(c.sweep_ms)
            return d
        return None

    def sweep_static(self, n_sweeps: int = 1, counters: bool = True):
        """hpmc_sweep_static: the same sweeps with the library's static device
        scratch as workspace (allocates nothing; calls on one device must not
        overlap)."""
        c = _Counters()
        self._chk(lib().hpmc_sweep_static(self._h, int(n_sweeps), ctypes.byref(c) if counters else None),
                  "sweep_static")
        if counters:
            return {f: int(getattr(c, f)) for f in COUNTERS}
        return None

    def set_tuning(self, cells_per_wave: int = 0, waves_per_block: int = 0, max_waves: int = 0):
        """Launch shape of the phase kernels (0 = default); results never depend on it."""
        t = _Tuning(int(cells_per_wave), int(waves_per_block), int(max_waves), 0, 0.0, 0.0)
        self._chk(lib().hpmc_set_tuning(self._h, ctypes.byref(t)), "set_tuning")

    def autotune(self, sweeps: int = 2) -> dict:
        """Time candidate launch shapes on a copy of the state and keep the fastest."""
        n = self.n * (3 + (4 if self.quat is not None else 0))
        scratch = self.torch.empty(n, dtype=self.torch.float64, device=self.device)
        t = _Tuning()
        self._chk(lib().hpmc_autotune(self._h, ctypes.c_void_p(scratch.data_ptr()), scratch.numel() * 8, int(sweeps),
                                      ctypes.byref(t)), "autotune")
        del scratch
        return {f: getattr(t, f) for f, _ in _Tuning._fields_}

    def trace(self) -> np.ndarray:
        cap = self.n * 1024
        buf = np.zeros(cap, dtype=MOVE_RECORD)
        nw = ctypes.c_int64(0)
        self._chk(lib().hpmc_trace(self._h, buf.ctypes.data, cap, ctypes.byref(nw)), "trace")
        return buf[: nw.value].copy()

    def observables(self, kind: int, n_bins: int = 0, r_max: float = 0.0, x_max: float = 0.0, n_fit: int = 0,
                    n_probe: int = 0, obs_seq: int = 0, eps: float = 1e-3) -> np.ndarray:
        p = _ObsParams(n_bins, n_fit, r_max, x_max, n_probe, obs_seq, 0, eps)
        out_len = {OBS_GR: max(n_bins, 1), OBS_FREE_VOLUME: 3, OBS_SDF: 4 + max(n_bins, 0)}[kind]
        out = np.zeros(out_len, dtype=np.float64)
        self._chk(lib().hpmc_observables(self._h, kind, ctypes.byref(p),
                                         out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), out_len),
                  "observables")
        return out


class Batch:
    """Several independent handles swept in shared launches (hpmc_sweep_batch).
    The batch workspace is allocated once for `capacity` handles (default: as
    many as given); set_members changes the membership without reallocating."""

    def __init__(self, sims, capacity: int | None = None, device=None):
        import torch

        self.torch = torch
        self.sims = list(sims)
        cap = max(len(self.sims), int(capacity or 0), 1)
        dev = torch.device(device) if device is not None else self.sims[0].device
        b = ctypes.c_size_t(0)
        rc = lib().hpmc_batch_workspace_bytes(cap, ctypes.byref(b))
        if rc != 0:
            raise HpmcError(rc, "hpmc_batch_workspace_bytes")
        self.capacity = cap
        self.workspace = torch.empty(int(b.value), dtype=torch.uint8, device=dev)
        self.set_members(self.sims)

    def set_members(self, sims):
        if len(sims) > self.capacity:
            raise ValueError(f"{len(sims)} handles exceed the batch capacity {self.capacity}")
        self.sims = list(sims)
        self._handles = (ctypes.c_void_p * max(len(self.sims), 1))(*[s._h.value for s in self.sims])

    def sweep(self, n_sweeps: int = 1, counters: bool = True, as_array: bool = False):
        """Batched sweeps; with counters, one record per member: dicts, or with
        as_array one numpy structured array (COUNTER_DTYPE), which costs no
        per-field Python work for large batches."""
        n = len(self.sims)
        out = (_Counters * n)() if counters else None
        rc = lib().hpmc_sweep_batch(self._handles, n, ctypes.c_void_p(self.workspace.data_ptr()),
                                    self.workspace.numel(), int(n_sweeps), out)
        if rc != 0:
            msg = lib().hpmc_last_error(self.sims[0]._h) if n else b""
            raise HpmcError(rc, f"sweep_batch: {msg.decode() if msg else ''}")
        if not counters:
            return None
        if as_array:
            return np.frombuffer(out, dtype=COUNTER_DTYPE, count=n).copy()
        res = [{f: int(getattr(c, f)) for f in COUNTERS} for c in out]
        for d, c in zip(res, out):
            d["sweep_ms"] = float(c.sweep_ms)
        return res

    def autotune(self, sweeps: int = 2) -> list:
        """Per launch group, time the candidate launch shapes with the group's
        members swept together (on copies of their states) and give them the
        fastest; returns each member's shape (hpmc_autotune_batch)."""
        n = len(self.sims)
        need = sum((s.n * 24 + (s.n * 32 if s.kind != SPHERE else 0) + 255) // 256 * 256 for s in self.sims)
        scratch = self.torch.empty(max(need, 1), dtype=self.torch.uint8, device=self.workspace.device)
        out = (_Tuning * n)()
        rc = lib().hpmc_autotune_batch(self._handles, n, ctypes.c_void_p(self.workspace.data_ptr()),
                                       self.workspace.numel(), ctypes.c_void_p(scratch.data_ptr()), need,
                                       int(sweeps), out)
        del scratch
        if rc != 0:
            msg = lib().hpmc_last_error(self.sims[0]._h) if n else b""
            raise HpmcError(rc, f"autotune_batch: {msg.decode() if msg else ''}")
        return [{f: getattr(t, f) for f, _ in _Tuning._fields_} for t in out]
