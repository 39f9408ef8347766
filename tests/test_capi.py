"""The C-ABI library loads, exports every function include/ski.h declares, and rejects
invalid arguments before touching the device (no GPU needed)."""

import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ski.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ski_[a-z_A-Z]+)\s*\(", text)))


def _lib():
    from paper_2105_11815_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("libski.so not built")
    return L, L.load()


def test_header_declares_the_boundary():
    names = _declared()
    for must in ["ski_create", "ski_destroy", "ski_params_default", "ski_sketch", "ski_factor",
                 "ski_solve", "ski_gradients", "ski_last_error"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    L, lib = _lib()
    for name in _declared():
        assert hasattr(lib, name), name
    assert sorted(L.EXPORTED) == _declared()


def test_params_default_matches_section6():
    L, lib = _lib()
    p = L.SkiParams()
    lib.ski_params_default(L.SKI_DENSE, C.byref(p))
    assert (p.gamma, p.s, p.hadamard, p.tau_a, p.tau_r, p.it_max, p.rcond) == \
        (1.7, 1, 1, 1e-8, 1e-6, 10000, 1e-12)
    lib.ski_params_default(L.SKI_CSR, C.byref(p))
    assert (p.gamma, p.s, p.hadamard, p.rcond_thres, p.perturb) == (1.4, 2, 0, 1e-10, 1e-10)


def test_struct_layouts_match_header_sizes():
    L, _ = _lib()
    # int64 n,d; int32 kind (+pad); ptr; int64; 3 ptrs; int64
    assert C.sizeof(L.SkiMatrix) == 8 * 2 + 8 + 8 + 8 + 8 * 3 + 8
    assert C.sizeof(L.SkiInfo) == 8 + 4 + 4 + 8 * 5 + 4 * 3 + 4


def test_invalid_arguments_are_rejected_on_the_host():
    L, lib = _lib()
    h = C.c_void_p()
    lib.ski_create(C.byref(h))  # may report EDEVICE without a GPU; the handle still exists
    assert h.value
    p = L.SkiParams()
    lib.ski_params_default(L.SKI_DENSE, C.byref(p))
    fake = C.c_void_p(0x1000)  # never dereferenced: every case fails validation first
    cases = [
        dict(n=10, d=20),                  # n < d
        dict(n=100, d=0),                  # d < 1
        dict(n=100, d=10, lda=5),          # lda < d
    ]
    for cs in cases:
        M = L.SkiMatrix(n=cs["n"], d=cs["d"], kind=L.SKI_DENSE, a=fake.value,
                        lda=cs.get("lda", max(cs["d"], 1)), row_ptr=None, col=None, val=None,
                        nnz=0)
        assert lib.ski_sketch(h, C.byref(M), fake, 1, 1, C.byref(p), None) == L.SKI_EINVAL
        assert lib.ski_last_error(h)
    M = L.SkiMatrix(n=100, d=10, kind=L.SKI_DENSE, a=fake.value, lda=10, row_ptr=None,
                    col=None, val=None, nnz=0)
    for field, val in [("s", 0), ("s", 33), ("m", 5), ("it_max", 0)]:
        q = L.SkiParams()
        lib.ski_params_default(L.SKI_DENSE, C.byref(q))
        setattr(q, field, val)
        assert lib.ski_sketch(h, C.byref(M), fake, 1, 1, C.byref(q), None) == L.SKI_EINVAL, field
    assert lib.ski_sketch(h, C.byref(M), fake, 0, 1, C.byref(p), None) == L.SKI_EINVAL  # k < 1
    # the declared limit m <= 12288 (n' = 32768 would allow more)
    Mbig = L.SkiMatrix(n=20000, d=10, kind=L.SKI_DENSE, a=fake.value, lda=10, row_ptr=None,
                       col=None, val=None, nnz=0)
    q = L.SkiParams()
    lib.ski_params_default(L.SKI_DENSE, C.byref(q))
    q.m = 12289
    assert lib.ski_sketch(h, C.byref(Mbig), fake, 1, 1, C.byref(q), None) == L.SKI_EINVAL
    assert b"12288" in lib.ski_last_error(h)
    Mc = L.SkiMatrix(n=100, d=10, kind=L.SKI_CSR, a=None, lda=0, row_ptr=fake.value,
                     col=fake.value, val=fake.value, nnz=10)
    assert lib.ski_sketch(h, C.byref(Mc), fake, 1, 1, C.byref(p), None) == L.SKI_EINVAL  # H+CSR
    # calls out of order
    assert lib.ski_factor(h, None) == L.SKI_ESTATE
    assert lib.ski_solve(h, 0, fake, 1, 1, fake, 1, None, None) == L.SKI_ESTATE
    lib.ski_destroy(h)


def test_noalloc_sketch_rejects_on_the_host():
    """ski_sketch_noalloc validates sizes against its static scratch before any device
    work, and reports through ski_last_error(NULL)."""
    L, lib = _lib()
    p = L.SkiParams()
    lib.ski_params_default(L.SKI_DENSE, C.byref(p))
    fake = C.c_void_p(0x1000)  # never dereferenced: every case fails validation first
    M = L.SkiMatrix(n=600000, d=4, kind=L.SKI_DENSE, a=fake.value, lda=4, row_ptr=None,
                    col=None, val=None, nnz=0)
    p.m = 64
    # n' = 2^20: a 16-column slab of n' doubles is 128 MiB, above the 64 MiB scratch
    assert lib.ski_sketch_noalloc(C.byref(M), fake, 1, 1, C.byref(p), fake, None) == L.SKI_EINVAL
    assert b"too large" in lib.ski_last_error(None)
    assert lib.ski_sketch_noalloc(None, fake, 1, 1, C.byref(p), fake, None) == L.SKI_EINVAL
    assert b"NULL" in lib.ski_last_error(None)
    Mc = L.SkiMatrix(n=100, d=10, kind=L.SKI_DENSE_COLMAJOR, a=fake.value, lda=100,
                     row_ptr=None, col=None, val=None, nnz=0)
    assert lib.ski_sketch_noalloc(C.byref(Mc), fake, 1, 1, C.byref(p), fake, None) == L.SKI_EINVAL
    q = L.SkiParams()
    lib.ski_params_default(L.SKI_DENSE, C.byref(q))
    q.sketch_prec = L.SKI_FP32
    M2 = L.SkiMatrix(n=100, d=10, kind=L.SKI_DENSE, a=fake.value, lda=10, row_ptr=None,
                     col=None, val=None, nnz=0)
    assert lib.ski_sketch_noalloc(C.byref(M2), fake, 1, 1, C.byref(q), fake, None) == L.SKI_EINVAL
    q.sketch_prec = L.SKI_FP64
    q.hadamard = 2
    assert lib.ski_sketch_noalloc(C.byref(M2), fake, 1, 1, C.byref(q), fake, None) == L.SKI_EINVAL
