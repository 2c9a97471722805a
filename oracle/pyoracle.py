"""ctypes wrapper of the C oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.  It shares no code
with the HIP library; see ``oracle.c`` for what each function follows in the
paper (Glaser, Karas & Glotzer, arXiv:1508.07077, Sec. III).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

SPHERE, HEMISPHERE, DISCOID = 0, 1, 2
ACCEPT, REJ_CELL_EXIT, REJ_OVERLAP, REJ_DEPLETANT, REJ_CB_ZERO, REJ_CB_METROPOLIS = range(6)
OBS_GR, OBS_FREE_VOLUME, OBS_SDF = 0, 1, 2
V0_BALL, V0_SHELL = 0, 1

RECORD_DTYPE = np.dtype(
    [
        ("sweep", "<u4"),
        ("cell", "<u4"),
        ("t", "<u4"),
        ("particle", "<u4"),
        ("n_depletants", "<u4"),
        ("resolved", "<u4"),
        ("n_blocking", "<u4"),
        ("w_fwd", "<u4"),
        ("w_rev", "<u4"),
        ("phase", "u1"),
        ("reason", "u1"),
        ("rotation", "u1"),
        ("near_contact", "u1"),
    ]
)
assert RECORD_DTYPE.itemsize == 40

COUNTER_FIELDS = (
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


class _Counters(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint64) for f in COUNTER_FIELDS]


class _ObsParams(ctypes.Structure):
    _fields_ = [
        ("n_bins", ctypes.c_int32),
        ("n_fit", ctypes.c_int32),
        ("r_max", ctypes.c_double),
        ("x_max", ctypes.c_double),
        ("n_probe", ctypes.c_int64),
        ("obs_seq", ctypes.c_uint32),
        ("pad", ctypes.c_uint32),
        ("eps", ctypes.c_double),
    ]


def build(force: bool = False) -> str:
    """Compile ``liboracle.so`` with gcc (FP64, no contraction, no fast-math)."""
    src = os.path.join(HERE, "oracle.c")
    if not force and os.path.exists(LIB_PATH) and os.path.getmtime(LIB_PATH) >= os.path.getmtime(src):
        return LIB_PATH
    cmd = [
        "gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
        "-Wall", "-shared", "-fPIC", "-o", LIB_PATH + ".tmp", src, "-lm",
    ]
    subprocess.run(cmd, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB_PATH)
        c_d_p = ctypes.POINTER(ctypes.c_double)
        L.orc_create.restype = ctypes.c_void_p
        L.orc_create.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint32]
        L.orc_destroy.argtypes = [ctypes.c_void_p]
        L.orc_last_error.restype = ctypes.c_char_p
        L.orc_last_error.argtypes = [ctypes.c_void_p]
        L.orc_set_shape.argtypes = [ctypes.c_void_p, ctypes.c_int, c_d_p, ctypes.c_int]
        L.orc_set_fugacity.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_double, ctypes.c_int]
        L.orc_set_moves.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int]
        L.orc_set_state.argtypes = [ctypes.c_void_p, c_d_p, c_d_p, ctypes.c_uint64]
        L.orc_get_state.argtypes = [ctypes.c_void_p, c_d_p, c_d_p, ctypes.POINTER(ctypes.c_uint64)]
        L.orc_set_trace.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.orc_set_threads.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.orc_sweep.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(_Counters)]
        L.orc_sweep_cone.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(_Counters)]
        L.orc_trace.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
        L.orc_observables.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(_ObsParams), c_d_p, ctypes.c_int64]
        L.orc_count_overlaps.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]
        L.orc_derived.argtypes = [ctypes.c_void_p, c_d_p, ctypes.c_int]
        L.orc_try_move.argtypes = [
            ctypes.c_void_p, ctypes.c_int64, c_d_p, c_d_p,
            ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p,
        ]
        L.orc_try_move_many.argtypes = [
            ctypes.c_void_p, ctypes.c_int64, c_d_p, c_d_p, ctypes.c_uint32, ctypes.c_int64,
            ctypes.c_void_p, ctypes.c_void_p,
        ]
        L.orc_philox4x32_10.argtypes = [ctypes.POINTER(ctypes.c_uint32)] * 3
        L.orc_poisson_table.argtypes = [ctypes.c_double, c_d_p, ctypes.c_int]
        L.orc_poisson_draw.argtypes = [c_d_p, ctypes.c_int, ctypes.c_double]
        L.orc_ball_candidate.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.POINTER(ctypes.c_int32)]
        L.orc_shell_candidate.argtypes = [ctypes.POINTER(ctypes.c_uint32), ctypes.c_double, ctypes.c_double,
                                          ctypes.c_double, c_d_p]
        L.orc_set_insertion.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.orc_depletant_overlap.argtypes = [ctypes.c_int, c_d_p, ctypes.c_double, c_d_p, c_d_p]
        L.orc_pair_overlap.argtypes = [ctypes.c_int, c_d_p, c_d_p, c_d_p, c_d_p, ctypes.POINTER(ctypes.c_int)]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def philox(ctr, key) -> np.ndarray:
    c = (ctypes.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (ctypes.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return np.array(list(o), dtype=np.uint32)


def poisson_table(lambda_c: float, K: int = 1024) -> np.ndarray:
    F = np.zeros(K, dtype=np.float64)
    lib().orc_poisson_table(float(lambda_c), _dp(F), K)
    return F


def poisson_draw(F: np.ndarray, u: float) -> int:
    F = np.ascontiguousarray(F, dtype=np.float64)
    return int(lib().orc_poisson_draw(_dp(F), len(F), float(u)))


def ball_candidate(wa: int, wb: int):
    m = (ctypes.c_int32 * 3)()
    ok = lib().orc_ball_candidate(wa & 0xFFFFFFFF, wb & 0xFFFFFFFF, m)
    return bool(ok), (m[0], m[1], m[2])


def shell_candidate(words, r_i: float, span: float, R0sq: float):
    w = (ctypes.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in words])
    e = (ctypes.c_double * 3)()
    ok = lib().orc_shell_candidate(w, float(r_i), float(span), float(R0sq), e)
    return bool(ok), (e[0], e[1], e[2])


def depletant_overlap(kind: int, params, r_dep: float, v_world, quat=None) -> bool:
    p = np.ascontiguousarray(params, dtype=np.float64)
    v = np.ascontiguousarray(v_world, dtype=np.float64)
    q = None if quat is None else _dp(np.ascontiguousarray(quat, dtype=np.float64))
    return bool(lib().orc_depletant_overlap(kind, _dp(p), float(r_dep), _dp(v), q))


def pair_overlap(kind: int, params, d_world, qa, qb):
    p = np.ascontiguousarray(params, dtype=np.float64)
    d = np.ascontiguousarray(d_world, dtype=np.float64)
    a = np.ascontiguousarray(qa, dtype=np.float64)
    b = np.ascontiguousarray(qb, dtype=np.float64)
    nc = ctypes.c_int(0)
    r = lib().orc_pair_overlap(kind, _dp(p), _dp(d), _dp(a), _dp(b), ctypes.byref(nc))
    return bool(r), bool(nc.value)


class OracleSim:
    """One simulation handle of the C oracle (host buffers only)."""

    def __init__(self, n: int, box_L: float, seed: int, replica_id: int = 0):
        self.n = int(n)
        self.L = float(box_L)
        self._h = lib().orc_create(self.n, self.L, int(seed) & (2**64 - 1), int(replica_id))
        if not self._h:
            raise ValueError("orc_create failed")
        self.kind = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_destroy(h)
            self._h = None

    def _chk(self, rc: int):
        if rc != 0:
            raise RuntimeError(f"oracle error {rc}: {lib().orc_last_error(self._h).decode()}")

    def set_shape(self, kind: int, params):
        p = np.ascontiguousarray(params, dtype=np.float64)
        self.kind = kind
        self._chk(lib().orc_set_shape(self._h, kind, _dp(p), len(p)))

    def set_fugacity(self, z_p: float, d_dep: float, n_trial: int = 0):
        self._chk(lib().orc_set_fugacity(self._h, float(z_p), float(d_dep), int(n_trial)))

    def set_moves(self, d_trans: float, a_rot: float = 0.0, p_rot: float = 0.0, n_select: int = 1):
        self._chk(lib().orc_set_moves(self._h, float(d_trans), float(a_rot), float(p_rot), int(n_select)))

    def set_insertion(self, region: int):
        self._chk(lib().orc_set_insertion(self._h, int(region)))

    def set_state(self, pos: np.ndarray, quat: np.ndarray | None = None, sweep: int = 0):
        pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(3, self.n)
        qp = None
        if quat is not None:
            quat = np.ascontiguousarray(quat, dtype=np.float64).reshape(4, self.n)
            qp = _dp(quat)
        self._chk(lib().orc_set_state(self._h, _dp(pos), qp, int(sweep)))

    def get_state(self):
        pos = np.zeros((3, self.n), dtype=np.float64)
        quat = np.zeros((4, self.n), dtype=np.float64)
        sw = ctypes.c_uint64(0)
        self._chk(lib().orc_get_state(self._h, _dp(pos), _dp(quat), ctypes.byref(sw)))
        return pos, quat, int(sw.value)

    def set_threads(self, threads: int):
        """OpenMP threads over the active cells of a phase (1 = serial)."""
        self._chk(lib().orc_set_threads(self._h, int(threads)))

    def set_trace(self, enable: bool = True):
        self._chk(lib().orc_set_trace(self._h, 1 if enable else 0))

    def sweep(self, n_sweeps: int = 1) -> dict:
        c = _Counters()
        self._chk(lib().orc_sweep(self._h, int(n_sweeps), ctypes.byref(c)))
        return {f: int(getattr(c, f)) for f in COUNTER_FIELDS}

    def sweep_cone(self, target_cell: int) -> dict:
        """One sweep restricted to the cells that can influence `target_cell`."""
        c = _Counters()
        self._chk(lib().orc_sweep_cone(self._h, int(target_cell), ctypes.byref(c)))
        return {f: int(getattr(c, f)) for f in COUNTER_FIELDS}

    def trace(self) -> np.ndarray:
        cap = self.n * 64
        buf = np.zeros(cap, dtype=RECORD_DTYPE)
        nw = ctypes.c_int64(0)
        self._chk(lib().orc_trace(self._h, buf.ctypes.data, cap, ctypes.byref(nw)))
        return buf[: nw.value].copy()

    def derived(self) -> dict:
        out = np.zeros(14, dtype=np.float64)
        lib().orc_derived(self._h, _dp(out), 14)
        keys = ["n", "w", "inv_w", "R0", "lambda", "n_chunks", "lambda_c", "s_ball", "r_dep", "rcirc", "vol", "halfL",
                "r_inner", "span"]
        return dict(zip(keys, out.tolist()))

    def count_overlaps(self) -> int:
        n = ctypes.c_int64(0)
        self._chk(lib().orc_count_overlaps(self._h, ctypes.byref(n)))
        return int(n.value)

    def try_move(self, j: int, xnew, qnew=None, sweep: int = 0, cell: int = 0, t: int = 0):
        x = np.ascontiguousarray(xnew, dtype=np.float64)
        q = None if qnew is None else _dp(np.ascontiguousarray(qnew, dtype=np.float64))
        rec = np.zeros(1, dtype=RECORD_DTYPE)
        r = lib().orc_try_move(self._h, int(j), _dp(x), q, sweep & 0xFFFFFFFF, cell & 0xFFFFFFFF, t, rec.ctypes.data)
        if r < 0:
            self._chk(r)
        return int(r), rec[0]

    def try_move_many(self, j: int, xnew, qnew=None, sweep0: int = 0, count: int = 1000):
        """Outcome codes and depletant counts of one fixed proposal on `count` streams."""
        x = np.ascontiguousarray(xnew, dtype=np.float64)
        q = None if qnew is None else _dp(np.ascontiguousarray(qnew, dtype=np.float64))
        reasons = np.zeros(count, dtype=np.uint8)
        ndep = np.zeros(count, dtype=np.uint32)
        self._chk(lib().orc_try_move_many(self._h, int(j), _dp(x), q, sweep0 & 0xFFFFFFFF, int(count),
                                          reasons.ctypes.data, ndep.ctypes.data))
        return reasons, ndep

    def observables(self, kind: int, n_bins: int = 0, r_max: float = 0.0, x_max: float = 0.0, n_fit: int = 0,
                    n_probe: int = 0, obs_seq: int = 0, eps: float = 1e-3) -> np.ndarray:
        p = _ObsParams(n_bins, n_fit, r_max, x_max, n_probe, obs_seq, 0, eps)
        out_len = {OBS_GR: max(n_bins, 1), OBS_FREE_VOLUME: 3, OBS_SDF: 4 + max(n_bins, 0)}[kind]
        out = np.zeros(out_len, dtype=np.float64)
        self._chk(lib().orc_observables(self._h, kind, ctypes.byref(p), _dp(out), out_len))
        return out
