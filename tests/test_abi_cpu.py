"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every symbol include/nfr.h declares, and rejects bad arguments before any
device work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nfr.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nfr_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    from paper_2504_13379_amd import _lib
    return _lib.lib()


def test_header_declares_entry_points():
    names = _declared()
    for must in ("nfr_apply", "nfr_integrate", "nfr_w_build", "nfr_problem_create", "nfr_context_create"):
        assert must in names


def test_library_exports_every_declared_symbol(L):
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing


def test_status_strings_and_version(L):
    assert L.nfr_status_string(0) == b"NFR_OK"
    assert L.nfr_status_string(-6) == b"NFR_ERR_WORKSPACE"
    a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    assert L.nfr_version(ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)) == 0
    assert (a.value, b.value) == (0, 1)


def test_size_queries(L):
    assert L.nfr_problem_bytes(0) == 0
    assert L.nfr_problem_bytes(1) > 0
    assert L.nfr_problem_bytes(4_000_000) > 0 and L.nfr_problem_bytes(4_000_001) == 0   # largest N
    npad = 32768
    assert L.nfr_w_bytes(32768, 1) == 32768 * npad * 4
    assert L.nfr_w_bytes(1000, 0) == 0
    npad = 1024
    for form in (2, 3):   # 256-byte header + hi and lo halves
        assert L.nfr_w_bytes(1000, form) == 256 + 2 * npad * npad * 2
    for form in (4, 5, 6, -1):   # on-the-fly matrix-core forms and AUTO need no W
        assert L.nfr_w_bytes(1000, form) == 0


def test_problem_layout_and_tune_workspace(L):
    """Packed problem: float4 coordinates | FP64 weights | FP64 coordinates |
    two FP64 maxima | tile order: int32 slot -> node, float4 coordinates, FP64
    weights, float4 bounds of 32- and 16-slot blocks, an FP64 bounding box per
    segment of the deepest bisection level (2^L, L = ceil(log2(ceil(N / 16))))
    and 64-bit sort keys for the next power of two; each 256-byte aligned, N
    padded to 256."""
    a = lambda b: (b + 255) // 256 * 256
    for n in (1, 255, 256, 1000, 65536, 70000):
        npad = (n + 255) // 256 * 256
        np2 = 1 << (npad - 1).bit_length()
        levels = (-(-n // 16) - 1).bit_length()
        assert L.nfr_problem_bytes(n) == (a(npad * 16) + a(npad * 8) + a(3 * npad * 8) + a(16) + a(npad * 4)
                                          + a(npad * 16) + a(npad * 8) + a(npad // 32 * 16) + a(npad // 16 * 16)
                                          + a(48 << levels) + a(np2 * 8))
    assert L.nfr_tune_workspace_size(512, 64) == 0        # n_max below 1024
    assert L.nfr_tune_workspace_size(65536, 1) == 0       # B_max below 2
    assert L.nfr_tune_workspace_size(65536, 64) > L.nfr_tune_workspace_size(65536, 16) > 0


def test_null_arguments_rejected_before_device_work(L):
    from paper_2504_13379_amd import _lib
    k = _lib.NfrKernel(0, 1.0, 0.15, 0.5, 0.4)
    f = _lib.NfrFiring(20.0, 0.2, None)
    st = L.nfr_apply(None, ctypes.byref(k), ctypes.byref(f), 1, None, None, 0, None, None, 0)
    assert st == _lib.NFR_ERR_INVALID_ARG
    assert b"problem" in L.nfr_last_error()
    st = L.nfr_integrate(None, ctypes.byref(k), ctypes.byref(f), 1, None, 0.05, 1, 0, None, None, 0, 0, None, 0)
    assert st == _lib.NFR_ERR_INVALID_ARG
    out = ctypes.c_void_p()
    assert L.nfr_problem_create(None, 10, None, None, None, 0, ctypes.byref(out)) == _lib.NFR_ERR_INVALID_ARG


def test_periodic_problem_rejects_bad_period(L):
    from paper_2504_13379_amd import _lib
    out = ctypes.c_void_p()
    st = L.nfr_problem_create_periodic(None, 10, None, None, -1.0, None, 0, ctypes.byref(out))
    assert st == _lib.NFR_ERR_INVALID_ARG and b"period" in L.nfr_last_error()
    st = L.nfr_problem_create_periodic(None, 10, None, None, float("nan"), None, 0, ctypes.byref(out))
    assert st == _lib.NFR_ERR_NONFINITE
    st = L.nfr_problem_create_periodic(None, 10, None, None, 6.0, None, 0, ctypes.byref(out))
    assert st == _lib.NFR_ERR_INVALID_ARG and b"context" in L.nfr_last_error()
    assert L.nfr_problem_period(None) == -1.0


def test_context_without_gpu_reports_no_device(L):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2504_13379_amd import _lib
    out = ctypes.c_void_p()
    assert L.nfr_context_create(0, None, ctypes.byref(out)) == _lib.NFR_ERR_NO_DEVICE


def test_quadrature_host_validation(L):
    """Sizes, triangle indices and closedness are checked on the host before
    the context is touched (dummy device pointers are never dereferenced)."""
    import numpy as np
    from paper_2504_13379_amd import _lib
    assert L.nfr_quad_workspace_size(100, 196, 5) == 0
    assert L.nfr_quad_workspace_size(100, 196, 58) == 0
    assert L.nfr_quad_workspace_size(20, 36, 32) == 0
    assert L.nfr_quad_workspace_size(100, 196, 32) > 0
    tet = np.array([[0, 2, 1], [0, 1, 3], [1, 2, 3], [0, 3, 2]], dtype=np.int32)
    dummy = ctypes.c_void_p(256)

    def call(tri, star, k=6, n=8):
        tri = np.ascontiguousarray(tri, dtype=np.int32)
        return L.nfr_quad_weights(None, n, dummy, dummy, tri.shape[0], tri.ctypes.data_as(ctypes.c_void_p), star, k,
                                  dummy, None, None, dummy, 1 << 20)
    bad = tet.copy()
    bad[2, 1] = 8
    assert call(bad, 0) == _lib.NFR_ERR_INVALID_ARG and b"outside" in L.nfr_last_error()
    assert call(tet[:3], 0) == _lib.NFR_ERR_INVALID_ARG and b"not closed" in L.nfr_last_error()
    flipped = tet.copy()
    flipped[0] = flipped[0, [0, 2, 1]]
    assert call(flipped, 0) == _lib.NFR_ERR_INVALID_ARG and b"oriented" in L.nfr_last_error()
    assert call(tet, 0, k=9) == _lib.NFR_ERR_INVALID_ARG and b"sizes" in L.nfr_last_error()
    assert call(tet, 0) == _lib.NFR_ERR_INVALID_ARG and b"context" in L.nfr_last_error()
    assert call(tet[:3], 1) == _lib.NFR_ERR_INVALID_ARG and b"context" in L.nfr_last_error()
    # orthogonal projection needs no neighbours: an open mesh passes the host checks
    assert call(tet[:3], _lib.PROJ_ORTHOGONAL) == _lib.NFR_ERR_INVALID_ARG and b"context" in L.nfr_last_error()
    assert call(tet, 3) == _lib.NFR_ERR_INVALID_ARG and b"projection" in L.nfr_last_error()
    assert call(tet, -1) == _lib.NFR_ERR_INVALID_ARG and b"projection" in L.nfr_last_error()


def test_tuning_cache_load_query_clear(L, tmp_path):
    """The planner's workgroup target follows a loaded cache (nearest entry in
    log n and log B) and returns to the built-in 1024 after clearing."""
    from paper_2504_13379_amd import _lib
    assert L.nfr_tune_clear() == 0
    assert L.nfr_tune_target(65536, 16) == 1024
    assert L.nfr_tune_target(65536, 1) == -1 and L.nfr_tune_target(0, 4) == -1
    path = tmp_path / "tune.json"
    path.write_text('{"library": "nfr", "arch": "gfx950", "entries": [\n'
                    ' {"npad": 4096, "B": 4, "target_wgs": 256, "ms": 0.1},\n'
                    ' {"npad": 65536, "B": 64, "target_wgs": 4096, "ms": 2.0}\n]}\n')
    try:
        assert L.nfr_tune_load(str(path).encode()) == 0
        assert L.nfr_tune_target(4000, 4) == 256
        assert L.nfr_tune_target(5000, 2) == 256
        assert L.nfr_tune_target(65536, 64) == 4096
        assert L.nfr_tune_target(60000, 128) == 4096
        bad = tmp_path / "bad.json"
        bad.write_text('{"entries": [{"npad": 1000, "B": 4, "target_wgs": 256}]}')
        assert L.nfr_tune_load(str(bad).encode()) == _lib.NFR_ERR_INVALID_ARG
        assert L.nfr_tune_load(str(tmp_path / "missing.json").encode()) == _lib.NFR_ERR_INVALID_ARG
    finally:
        L.nfr_tune_clear()
    assert L.nfr_tune_target(4000, 4) == 1024
    assert L.nfr_tune_workspace_size(100, 4) == 0 and L.nfr_tune_workspace_size(4096, 4) > 0
