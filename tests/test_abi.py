"""The C-ABI library loads, exports every declared symbol, and validates its
arguments on the host (CPU only: no call here reaches a GPU)."""
import ctypes
import os
import re

import pytest

from paper_2111_14641_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "rbgs.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rbgs_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_expected_calls():
    names = declared_functions()
    for n in ("rbgs_create", "rbgs_destroy", "rbgs_qr", "rbgs_sketch_apply", "rbgs_theta_dense",
              "rbgs_status_string", "rbgs_last_error", "rbgs_profile_enable", "rbgs_profile_get"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(B.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    # the binding exposes the same names
    for name in declared_functions():
        assert name in B._SIGNATURES, name


@pytest.fixture(scope="module")
def lib_and_handle():
    lib = B.load_library()
    h = ctypes.c_void_p()
    assert lib.rbgs_create(ctypes.byref(h), 0) == B.RBGS_OK     # lazy: touches no device
    yield lib, h
    lib.rbgs_destroy(h)


def _qr(lib, h, n=100, m=8, p=4, k=32, kind=0, zeta=8, store=0, math=0, variant=1, iters=2,
        ldw=None, ldq=None, ldr=None, W=0x1000, Q=0x100000, R=0x200000):
    sk = B.rbgs_sketch(kind, zeta, k, 1)
    op = B.rbgs_opts(store, math, variant, iters, None)
    return lib.rbgs_qr(h, W, ldw or n, n, m, p, ctypes.byref(sk), ctypes.byref(op), Q, ldq or n,
                       R, ldr or m, None, None)


@pytest.mark.parametrize("kw,expect", [
    (dict(n=0), B.RBGS_EINVAL),
    (dict(m=0), B.RBGS_EINVAL),
    (dict(m=200, n=100), B.RBGS_EINVAL),          # m > n
    (dict(p=0), B.RBGS_EINVAL),
    (dict(p=33), B.RBGS_EUNSUPPORTED),
    (dict(k=4), B.RBGS_EINVAL),                   # k < m
    (dict(k=104, n=100), B.RBGS_EINVAL),          # k > n
    (dict(k=30), B.RBGS_EINVAL),                  # Gaussian needs k % 4 == 0
    (dict(kind=1, zeta=9), B.RBGS_EINVAL),
    (dict(kind=1, zeta=3, k=32), B.RBGS_EINVAL),  # k % zeta
    (dict(kind=1, k=4096, n=10000), B.RBGS_EINVAL),
    (dict(kind=2, k=32), B.RBGS_EINVAL),          # identity needs k == n
    (dict(kind=7), B.RBGS_EINVAL),
    (dict(store=0, math=1), B.RBGS_EINVAL),       # FP64 storage needs FP64 arithmetic
    (dict(math=5), B.RBGS_EINVAL),
    (dict(store=0, math=2), B.RBGS_EINVAL),       # BF16x3 products need FP32 storage
    (dict(store=2), B.RBGS_EINVAL),
    (dict(variant=4), B.RBGS_EINVAL),
    (dict(iters=0, k=1032, n=2000), B.RBGS_EUNSUPPORTED),           # Householder: k <= 1024
    (dict(iters=0, k=600, n=2000, m=64, p=32), B.RBGS_EUNSUPPORTED),  # and p <= 16 past k = 512
    (dict(iters=-1), B.RBGS_EINVAL),
    (dict(iters=17), B.RBGS_EINVAL),
    (dict(ldw=50), B.RBGS_EINVAL),
    (dict(ldr=4), B.RBGS_EINVAL),
    (dict(Q=0x1000 + 8 * 50), B.RBGS_EINVAL),     # Q partially overlaps W
    (dict(R=0x1000), B.RBGS_EINVAL),              # R overlaps W
])
def test_invalid_arguments_rejected_on_host(lib_and_handle, kw, expect):
    lib, h = lib_and_handle
    assert _qr(lib, h, **kw) == expect
    assert lib.rbgs_last_error(h).decode() != ""


def test_null_arguments(lib_and_handle):
    lib, h = lib_and_handle
    assert _qr(lib, h, W=0) == B.RBGS_EINVAL
    assert lib.rbgs_qr(None, 1, 1, 1, 1, 1, None, None, 1, 1, 1, 1, None, None) == B.RBGS_EINVAL
    assert lib.rbgs_create(None, 0) == B.RBGS_EINVAL
    assert lib.rbgs_destroy(None) == B.RBGS_OK
    assert lib.rbgs_status_string(B.RBGS_EBREAKDOWN).decode().startswith("breakdown")


def test_profile_interface_without_gpu(lib_and_handle):
    lib, h = lib_and_handle
    assert lib.rbgs_profile_enable(h, 1) == B.RBGS_OK
    ms, cnt, by = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
    assert lib.rbgs_profile_get(h, 0, ctypes.byref(ms), ctypes.byref(cnt), ctypes.byref(by)) == B.RBGS_OK
    assert cnt.value == 0
    assert lib.rbgs_profile_get(h, 9, None, None, None) == B.RBGS_EINVAL


def test_batched_validation_on_host(lib_and_handle):
    lib, h = lib_and_handle
    sk = B.rbgs_sketch(1, 8, 0, 1)
    op = B.rbgs_opts(1, 0, 1, 4, None)
    arr = (B.rbgs_problem * 2)()
    arr[0] = B.rbgs_problem(0x1000, 100, 100, 8, 0x100000, 100, 0x200000, 8, 4, 32, 0, 0)
    arr[1] = B.rbgs_problem(0x300000, 50, 50, 80, 0x400000, 50, 0x500000, 80, 4, 96, 0, 0)  # m > n
    assert lib.rbgs_qr_batched(h, 2, arr, ctypes.byref(sk), ctypes.byref(op), 0) == B.RBGS_EINVAL
    assert arr[1].status == B.RBGS_EINVAL
    assert "problem 1" in lib.rbgs_last_error(h).decode()
    assert lib.rbgs_qr_batched(h, 0, arr, ctypes.byref(sk), ctypes.byref(op), 0) == B.RBGS_EINVAL
    for flags in (4, -1):  # graph: RBGS_BATCH_GRAPH | RBGS_BATCH_PERSISTENT at most
        assert lib.rbgs_qr_batched(h, 1, arr, ctypes.byref(sk), ctypes.byref(op), flags) == B.RBGS_EINVAL
    arr[0].p = 33
    assert lib.rbgs_qr_batched(h, 1, arr, ctypes.byref(sk), ctypes.byref(op), 0) == B.RBGS_EUNSUPPORTED
    p, k = ctypes.c_int64(), ctypes.c_int64()
    assert lib.rbgs_autotune(h, 10, 20, ctypes.byref(sk), ctypes.byref(op), ctypes.byref(p),
                             ctypes.byref(k)) == B.RBGS_EINVAL
    assert lib.rbgs_autotune(h, 100, 20, None, ctypes.byref(op), ctypes.byref(p),
                             ctypes.byref(k)) == B.RBGS_EINVAL


def test_cholqr_post_validation_on_host(lib_and_handle):
    lib, h = lib_and_handle
    assert lib.rbgs_cholqr_post(h, 0, None, 10, 10, 4, 0x200000, 4, None, None) == B.RBGS_EINVAL
    assert lib.rbgs_cholqr_post(h, 0, 0x1000, 10, 10, 11, 0x200000, 11, None, None) == B.RBGS_EINVAL
    assert lib.rbgs_cholqr_post(h, 0, 0x1000, 5, 10, 4, 0x200000, 4, None, None) == B.RBGS_EINVAL
    assert lib.rbgs_cholqr_post(h, 3, 0x1000, 10, 10, 4, 0x200000, 4, None, None) == B.RBGS_EINVAL
    assert lib.rbgs_cholqr_post(h, 0, 0x1000, 10, 10, 4, 0x1000 + 8, 4, None, None) == B.RBGS_EINVAL
    assert lib.rbgs_cholqr_post(h, 0, 0x1000, 20000, 20000, 9000, 0x9000000000, 9000, None,
                                None) == B.RBGS_EUNSUPPORTED
