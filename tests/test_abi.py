"""The C-ABI library loads on the host and exports every entry point that
include/hpmc.h declares; host-only argument validation works without a GPU
(no device work is launched here)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hpmc.h")


@pytest.fixture(scope="module")
def hp():
    import paper_1508_07077_amd as hp

    if not os.path.exists(hp.LIB_PATH):
        from paper_1508_07077_amd import build

        build.build()
    return hp


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hpmc_[a-z_]+)\s*\(", src)))


def test_header_and_binding_agree(hp):
    assert _declared() == sorted(hp.EXPORTS)


def test_library_exports_every_declared_symbol(hp):
    out = subprocess.run(["nm", "-D", "--defined-only", hp.LIB_PATH], capture_output=True, text=True, check=True).stdout
    syms = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = [s for s in _declared() if s not in syms]
    assert not missing, missing
    L = hp.lib()
    for s in _declared():
        assert getattr(L, s) is not None


ESTATE = -5


def _handle(hp, n=64, L=6.9459):
    h = ctypes.c_void_p()
    assert hp.lib().hpmc_create(ctypes.byref(h), n, L, 1, 0, 0, None) == 0
    return h


def _dp(a):
    return np.ascontiguousarray(a, dtype=np.float64).ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def test_create_validation(hp):
    L = hp.lib()
    h = ctypes.c_void_p()
    assert L.hpmc_create(ctypes.byref(h), 0, 5.0, 1, 0, 0, None) == -1
    assert L.hpmc_create(ctypes.byref(h), 10, -5.0, 1, 0, 0, None) == -1
    assert L.hpmc_create(ctypes.byref(h), 10, 5.0, 1, 0, 7, None) == -1
    assert L.hpmc_create(None, 10, 5.0, 1, 0, 0, None) == -1


def test_parameter_validation_and_errors(hp):
    L = hp.lib()
    h = _handle(hp)
    b = ctypes.c_size_t()
    assert L.hpmc_workspace_bytes(h, ctypes.byref(b)) == -5  # no shape yet
    assert L.hpmc_set_shape(h, 9, _dp([1.0]), 1) == -1
    assert L.hpmc_set_shape(h, 0, _dp([-1.0]), 1) == -1
    assert L.hpmc_set_shape(h, 2, _dp([0.5]), 1) == -1  # discoid needs two radii
    assert L.hpmc_set_shape(h, 0, _dp([1.0]), 1) == 0
    assert L.hpmc_set_fugacity(h, -1.0, 0.25, 0) == -1
    assert b"invalid" in L.hpmc_last_error(h)
    assert L.hpmc_set_fugacity(h, 12.0, 0.25, 300) == -1
    assert L.hpmc_set_fugacity(h, 12.0, 0.25, 4) == 0
    assert L.hpmc_set_moves(h, -0.1, 0.0, 0.0, 1) == -1
    assert L.hpmc_set_moves(h, 0.1, 0.0, 1.5, 1) == -1
    assert L.hpmc_set_moves(h, 0.1, 0.0, 0.0, 0) == -1
    assert L.hpmc_set_moves(h, 0.1, 0.0, 0.0, 1) == 0
    assert L.hpmc_workspace_bytes(h, ctypes.byref(b)) == 0 and b.value > 0
    # no workspace / state: calls that would touch the device refuse first
    c = hp._Counters()
    assert L.hpmc_sweep(h, 1, ctypes.byref(c)) == -5
    assert L.hpmc_set_workspace(h, None, 0) == -1
    assert L.hpmc_set_workspace(h, ctypes.c_void_p(1 << 20), 16) == -4
    sw = ctypes.c_uint64()
    assert L.hpmc_get_state(h, ctypes.byref(sw)) == -5
    n = ctypes.c_int64()
    assert L.hpmc_trace(h, None, 0, ctypes.byref(n)) == -5
    L.hpmc_destroy(h)


def test_box_too_small(hp):
    L = hp.lib()
    h = _handle(hp, n=4, L=1.9)
    assert L.hpmc_set_shape(h, 0, _dp([1.0]), 1) == -2  # 2 cells of width >= d do not fit
    h2 = _handle(hp, n=4, L=2.2)
    assert L.hpmc_set_shape(h2, 0, _dp([1.0]), 1) == 0
    assert L.hpmc_set_fugacity(h2, 10.0, 0.25, 0) == -2  # width 1.25 no longer fits twice
    L.hpmc_destroy(h2)
    L.hpmc_destroy(h)


def test_cell_grid_cap(hp):
    """at most 2^30 - 1 cells: 1022 per axis is the largest grid (every cell
    coordinate below 1024, which the sphere kernel packs in 10 bits); 1024 is refused"""
    L = hp.lib()
    h = _handle(hp, L=1022.5)  # unit spheres, no depletants: cells of width >= 1
    assert L.hpmc_set_shape(h, 0, _dp([1.0]), 1) == 0
    ws = ctypes.c_size_t()
    assert L.hpmc_workspace_bytes(h, ctypes.byref(ws)) == 0
    assert ws.value >= 1022 ** 3 * 4  # the cell counts alone
    L.hpmc_destroy(h)
    h = _handle(hp, L=1024.5)
    assert L.hpmc_set_shape(h, 0, _dp([1.0]), 1) == -2
    L.hpmc_destroy(h)


def test_workspace_grows_with_trace(hp):
    L = hp.lib()
    h = _handle(hp)
    assert L.hpmc_set_shape(h, 0, _dp([1.0]), 1) == 0
    a, b = ctypes.c_size_t(), ctypes.c_size_t()
    L.hpmc_workspace_bytes(h, ctypes.byref(a))
    assert L.hpmc_set_trace(h, 1) == 0
    L.hpmc_workspace_bytes(h, ctypes.byref(b))
    assert b.value >= a.value + 64 * 40
    L.hpmc_destroy(h)


def test_missing_library_fails_loudly(monkeypatch):
    import paper_1508_07077_amd as hp

    monkeypatch.setattr(hp, "LIB_PATH", "/nonexistent/libhpmc.so")
    monkeypatch.setattr(hp, "_lib", None)
    with pytest.raises(ImportError):
        hp.lib()


def test_counter_array_layout(hp):
    """Batch.sweep(as_array=True) reads the C counter records through
    COUNTER_DTYPE: the same fields at the same offsets"""
    import numpy as np

    out = (hp._Counters * 3)()
    for i, c in enumerate(out):
        for j, f in enumerate(hp.COUNTERS):
            setattr(c, f, 1000 * i + j)
        c.phase_kernel_ms = 0.25 * i
        c.sweep_ms = 0.5 + i
    a = np.frombuffer(out, dtype=hp.COUNTER_DTYPE, count=3)
    for i in range(3):
        assert [int(a[f][i]) for f in hp.COUNTERS] == [1000 * i + j for j in range(len(hp.COUNTERS))]
        assert a["phase_kernel_ms"][i] == 0.25 * i and a["sweep_ms"][i] == 0.5 + i


def test_batch_autotune_argument_checks(hp):
    """hpmc_autotune_batch rejects a handle given twice, missing scratch and a
    sweep count out of range before any device work, and handles without a
    workspace or state with ESTATE"""
    L = hp.lib()
    hs = []
    for _ in range(2):
        h = ctypes.c_void_p()
        assert L.hpmc_create(ctypes.byref(h), 100, 20.0, 1, 0, 0, None) == 0
        assert L.hpmc_set_shape(h, 0, _dp([1.0]), 1) == 0
        hs.append(h)
    arr = (ctypes.c_void_p * 2)(hs[0].value, hs[0].value)
    scratch = ctypes.c_void_p(1)
    try:
        assert L.hpmc_autotune_batch(arr, 2, None, 0, scratch, 1 << 20, 1, None) == -1  # handle twice
        arr = (ctypes.c_void_p * 2)(hs[0].value, hs[1].value)
        assert L.hpmc_autotune_batch(arr, 2, None, 0, None, 1 << 20, 1, None) == -1  # no scratch
        assert L.hpmc_autotune_batch(arr, 2, None, 0, scratch, 1 << 20, 0, None) == -1  # sweeps < 1
        assert L.hpmc_autotune_batch(arr, 2, None, 0, scratch, 1 << 20, 65, None) == -1  # sweeps > 64
        assert L.hpmc_autotune_batch(arr, 0, None, 0, scratch, 1 << 20, 1, None) == -1
        rc = L.hpmc_autotune_batch(arr, 2, None, 0, scratch, 1 << 20, 1, None)
        assert rc == ESTATE  # no workspace yet
    finally:
        for h in hs:
            L.hpmc_destroy(h)


def test_poisson_draw_needs_a_table(hp):
    L = hp.lib()
    h = ctypes.c_void_p()
    assert L.hpmc_create(ctypes.byref(h), 100, 20.0, 1, 0, 0, None) == 0
    k = ctypes.c_int32(0)
    try:
        assert L.hpmc_poisson_draw(h, 0.5, ctypes.byref(k)) == ESTATE  # no shape, so no table yet
    finally:
        L.hpmc_destroy(h)
