"""Python binding of the sketch-and-precondition least-squares solver.

The names follow the C interface (include/ski.h): `Solver.sketch`, `Solver.factor`,
`Solver.solve` run Algorithm 1's Steps 1, 2 and 3-5 in the HIP library on the
current torch stream.  This module only marshals arguments: torch provides the
device memory and the stream; every step of the method runs in libski.so.
"""

import ctypes as C
import warnings

import numpy as np
import torch

from . import _lib as L

_PREC = {"fp64": L.SKI_FP64, "fp32": L.SKI_FP32, "bf16": L.SKI_BF16}
_HASH = {"hash": L.SKI_HASH, "variant": L.SKI_HASH_VARIANT, "sample": L.SKI_SAMPLE_ROWS}
_PANEL = {"auto": L.SKI_QR_AUTO, "householder": L.SKI_QR_HOUSEHOLDER,
          "pivoted": L.SKI_QR_PIVOTED, "pivoted_householder": L.SKI_QR_PIVOTED_HOUSEHOLDER,
          "cod": L.SKI_QR_PIVOTED_COD, "sparse": L.SKI_QR_SPARSE}


class SkiError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{L.STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _check_dev(t, name, dtype):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")


def params(kind="dense", **kw):
    """ski_params with the defaults of Section 6 for `kind`, overridden by kw."""
    lib = L.load()
    p = L.SkiParams()
    lib.ski_params_default(L.SKI_CSR if kind == "csr" else L.SKI_DENSE, C.byref(p))
    for key, val in kw.items():
        if key in ("sketch_prec", "qr_prec") and isinstance(val, str):
            val = _PREC[val]
        if key == "qr_panel" and isinstance(val, str):
            val = _PANEL[val]
        if key == "hash_kind" and isinstance(val, str):
            val = _HASH[val]
        if key == "hadamard":
            val = 2 if val == "dht" else (val if isinstance(val, int) and val == 2 else int(bool(val)))
        if not hasattr(p, key):
            raise KeyError(f"unknown parameter {key}")
        setattr(p, key, val)
    return p


def _matrix(A):
    """ski_matrix for a dense float64 CUDA tensor (row- or column-major) or for
    ('csr', row_ptr, col, val, (n, d)); returns (matrix, kind, tensors to keep alive)."""
    if isinstance(A, tuple) and A[0] == "csr":
        _, rp, ci, va, (n, d) = A
        _check_dev(rp, "row_ptr", torch.int64)
        _check_dev(ci, "col", torch.int32)
        _check_dev(va, "val", torch.float64)
        M = L.SkiMatrix(n=n, d=d, kind=L.SKI_CSR, a=None, lda=0, row_ptr=rp.data_ptr(),
                        col=ci.data_ptr(), val=va.data_ptr(), nnz=va.numel())
        return M, "csr", (rp, ci, va)
    _check_dev(A, "A", torch.float64)
    if A.dim() != 2:
        raise ValueError("A must be 2-D")
    n, d = A.shape
    if A.stride(1) == 1 and (d == 1 or A.stride(0) >= d):
        M = L.SkiMatrix(n=n, d=d, kind=L.SKI_DENSE, a=A.data_ptr(), lda=A.stride(0),
                        row_ptr=None, col=None, val=None, nnz=0)
    elif A.stride(0) == 1 and A.stride(1) >= n:
        # column-major (e.g. a transposed view): the library keeps a row-major copy
        M = L.SkiMatrix(n=n, d=d, kind=L.SKI_DENSE_COLMAJOR, a=A.data_ptr(),
                        lda=A.stride(1), row_ptr=None, col=None, val=None, nnz=0)
    else:
        raise ValueError("A must be row-major or column-major (one unit stride)")
    return M, "dense", (A,)


def sketch_noalloc(A, B, out=None, **kw):
    """S [A B] through ski_sketch_noalloc (no device allocation in the library): A a
    row-major float64 CUDA tensor or ('csr', row_ptr, col, val, (n, d)); B (n,) or (n x k).
    out: an optional contiguous float64 CUDA tensor of m x (d + k).  Returns out."""
    lib = L.load()
    M, kind, keep = _matrix(A)
    _check_dev(B, "B", torch.float64)
    B2 = B.reshape(B.shape[0], -1)
    if B2.stride(1) != 1:
        B2 = B2.contiguous()
    k = B2.shape[1]
    p = params(kind, **kw)
    d = M.d
    m = p.m if p.m > 0 else int(np.ceil(p.gamma * d - 1e-9))
    if out is None:
        out = torch.empty((m, d + k), dtype=torch.float64, device=B2.device)
    _check_dev(out, "out", torch.float64)
    if tuple(out.shape) != (m, d + k) or not out.is_contiguous():
        raise ValueError(f"out must be a contiguous {m} x {d + k} tensor")
    rc = lib.ski_sketch_noalloc(C.byref(M), _ptr(B2), k, B2.stride(0), C.byref(p), _ptr(out),
                                _stream())
    if rc != L.SKI_OK:
        msg = lib.ski_last_error(None)
        raise SkiError(rc, f"ski_sketch_noalloc: {msg.decode() if msg else ''}")
    del keep
    return out


class Solver:
    """One handle of the C library (one problem at a time, one stream at a time)."""

    def __init__(self):
        self._lib = L.load()
        self._h = C.c_void_p()
        rc = self._lib.ski_create(C.byref(self._h))
        if rc != L.SKI_OK:
            raise SkiError(rc, "ski_create failed")
        self._keep = ()
        self.k = 0

    def _raise(self, rc, where):
        msg = self._lib.ski_last_error(self._h)
        raise SkiError(rc, f"{where}: {msg.decode() if msg else ''}")

    def close(self):
        if self._h:
            self._lib.ski_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- Step 1 ------------------------------------------------------------
    def sketch(self, A, B, **kw):
        """A: dense (n x d) float64 CUDA tensor, or ('csr', row_ptr, col, val, (n, d)).
        B: (n,) or (n x k) float64 CUDA tensor.  Parameters as in ski_params."""
        M, kind, keep = _matrix(A)
        _check_dev(B, "B", torch.float64)
        B2 = B.reshape(B.shape[0], -1)
        if B2.stride(1) != 1:
            B2 = B2.contiguous()
        k = B2.shape[1]
        p = params(kind, **kw)
        rc = self._lib.ski_sketch(self._h, C.byref(M), _ptr(B2), k, B2.stride(0), C.byref(p),
                                  _stream())
        if rc != L.SKI_OK:
            self._raise(rc, "ski_sketch")
        self._keep = keep + (B2,)
        self.B = B2
        self.k = k
        self.kind = kind
        return self

    # -- Step 2 ------------------------------------------------------------
    def factor(self):
        rc = self._lib.ski_factor(self._h, _stream())
        if rc != L.SKI_OK:
            self._raise(rc, "ski_factor")
        return self

    # -- Steps 3-5 ---------------------------------------------------------
    def solve(self, out=None):
        """Solve for the right-hand sides given to sketch(); returns (X d x k, infos)."""
        B = self.B
        d = self.dims()["d"]
        X = out if out is not None else torch.empty((d, self.k), dtype=torch.float64,
                                                    device=B.device)
        infos = (L.SkiInfo * self.k)()
        rc = self._lib.ski_solve(self._h, L.SKI_OP_LLS, _ptr(B), self.k, B.stride(0), _ptr(X),
                                 X.stride(0), infos, _stream())
        if rc < 0:
            self._raise(rc, "ski_solve")
        return X, [i.as_dict() for i in infos], rc

    def solve_normal(self, G, tol=None):
        """Z = (A^T A)^-1 G by CG preconditioned with R (the adjoint solve)."""
        _check_dev(G, "G", torch.float64)
        G2 = G.reshape(G.shape[0], -1).contiguous()
        k = G2.shape[1]
        Z = torch.empty_like(G2)
        infos = (L.SkiInfo * k)()
        rc = self._lib.ski_solve(self._h, L.SKI_OP_NORMAL, _ptr(G2), k, G2.stride(0), _ptr(Z),
                                 Z.stride(0), infos, _stream())
        if rc < 0:
            self._raise(rc, "ski_solve(NORMAL)")
        return Z, [i.as_dict() for i in infos], rc

    def gradients(self, X, B, Z, want_A=True, want_B=True):
        n, d = self.dims()["n"], self.dims()["d"]
        k = X.shape[1]
        gA = torch.empty((n, d), dtype=torch.float64, device=X.device) if want_A else None
        gB = torch.empty((n, k), dtype=torch.float64, device=X.device) if want_B else None
        X, B, Z = X.contiguous(), B.reshape(n, -1).contiguous(), Z.contiguous()
        rc = self._lib.ski_gradients(self._h, _ptr(X), k, _ptr(B), k, _ptr(Z), k, k, _ptr(gA),
                                     d, _ptr(gB), k, _stream())
        if rc != L.SKI_OK:
            self._raise(rc, "ski_gradients")
        return gA, gB

    # -- measurement ------------------------------------------------------
    def set_profiling(self, on=True, classes=None):
        """Time every kernel class (on), none (off), or only the named classes."""
        if classes is None:
            rc = self._lib.ski_set_profiling(self._h, 1 if on else 0)
        else:
            mask = 0
            for name in classes:
                mask |= 1 << L.PROF_NAMES.index(name)
            rc = self._lib.ski_set_profiling_mask(self._h, mask if on else 0)
        if rc != L.SKI_OK:
            self._raise(rc, "ski_set_profiling")

    def profile(self):
        """{class name: (total device ms, launches)} since profiling was switched on."""
        ms = np.zeros(L.PROF_CLASSES)
        cnt = np.zeros(L.PROF_CLASSES, dtype=np.int64)
        rc = self._lib.ski_get_profile(self._h, ms.ctypes.data, cnt.ctypes.data)
        if rc != L.SKI_OK:
            self._raise(rc, "ski_get_profile")
        return {name: (float(ms[i]), int(cnt[i])) for i, name in enumerate(L.PROF_NAMES)}

    # -- inspection (host copies) -----------------------------------------
    def dims(self):
        a = np.zeros(6, dtype=np.int64)
        rc = self._lib.ski_get_dims(self._h, a.ctypes.data)
        if rc != L.SKI_OK:
            self._raise(rc, "ski_get_dims")
        return dict(n=int(a[0]), d=int(a[1]), k=int(a[2]), m=int(a[3]), npad=int(a[4]),
                    s=int(a[5]))

    def get_hash(self, sampled=False):
        """The sketch's sparse factor; sampled=True after row sampling (rows has m entries)."""
        dm = self.dims()
        nk = dm["m"] if sampled else dm["npad"] * dm["s"]
        rows = np.zeros(nk, dtype=np.int32)
        neg = np.zeros(nk, dtype=np.int8)
        ptr = np.zeros(dm["m"] + 1, dtype=np.int64)
        src = np.zeros(nk, dtype=np.int32)
        sneg = np.zeros(nk, dtype=np.int8)
        rc = self._lib.ski_get_hash(self._h, rows.ctypes.data, neg.ctypes.data, ptr.ctypes.data,
                                    src.ctypes.data, sneg.ctypes.data)
        if rc != L.SKI_OK:
            self._raise(rc, "ski_get_hash")
        s = 1 if sampled else dm["s"]
        return dict(rows=rows.reshape(-1, s), neg=neg.reshape(-1, s).astype(bool),
                    bucket_ptr=ptr, src=src, src_neg=sneg.astype(bool))

    def get_dsign(self):
        dm = self.dims()
        out = np.zeros(dm["npad"], dtype=np.int8)
        rc = self._lib.ski_get_dsign(self._h, out.ctypes.data)
        if rc != L.SKI_OK:
            self._raise(rc, "ski_get_dsign")
        return out.astype(np.float64)

    def get_SA(self):
        dm = self.dims()
        out = np.zeros((dm["m"], dm["d"] + dm["k"]))
        rc = self._lib.ski_get_SA(self._h, out.ctypes.data)
        if rc != L.SKI_OK:
            self._raise(rc, "ski_get_SA")
        return out

    def get_R(self):
        """(R d x d, c d x k, R^-1); after a pivoted factor R^-1 is R_11^-1 (p x p); after
        the sparse factor R is in position order and R^-1 (not formed) is None."""
        dm = self.dims()
        R = np.zeros((dm["d"], dm["d"]))
        c = np.zeros((dm["d"], dm["k"]))
        try:
            sparse = self.factor_stats()["sparse"]
        except SkiError:
            sparse = False
        if sparse:
            rc = self._lib.ski_get_R(self._h, R.ctypes.data, c.ctypes.data, None)
            if rc != L.SKI_OK:
                self._raise(rc, "ski_get_R")
            return R, c, None
        Ri = np.zeros(dm["d"] * dm["d"])
        rc = self._lib.ski_get_R(self._h, R.ctypes.data, c.ctypes.data, Ri.ctypes.data)
        if rc != L.SKI_OK:
            self._raise(rc, "ski_get_R")
        try:
            p = self.get_pivots()[1]
        except SkiError:
            p = dm["d"]
        return R, c, Ri[: p * p].reshape(p, p)

    def factor_stats(self):
        """{rank, panels, panels_cqr (-1 without pivoting), pivoted, sparse} of the last
        factor; after the sparse factor {rank, leaf_fronts, root, sparse=True}."""
        a = np.zeros(4, dtype=np.int64)
        rc = self._lib.ski_get_factor_stats(self._h, a.ctypes.data)
        if rc != L.SKI_OK:
            self._raise(rc, "ski_get_factor_stats")
        if a[3] == 2:
            return dict(rank=int(a[0]), leaf_fronts=int(a[1]), root=int(a[2]), pivoted=True,
                        sparse=True)
        return dict(rank=int(a[0]), panels=int(a[1]), panels_cqr=int(a[2]), pivoted=bool(a[3]),
                    sparse=False)

    def get_pivots(self):
        """(perm: position j holds column perm[j] of A, rank p) of the last factor."""
        d = self.dims()["d"]
        perm = np.zeros(d, dtype=np.int32)
        rank = np.zeros(1, dtype=np.int64)
        rc = self._lib.ski_get_pivots(self._h, perm.ctypes.data, rank.ctypes.data)
        if rc != L.SKI_OK:
            self._raise(rc, "ski_get_pivots")
        return perm.astype(np.int64), int(rank[0])


def lstsq(A, B, **kw):
    """x = argmin ||A x - B|| through Algorithm 1 on the GPU; returns (X, infos, status)."""
    s = Solver()
    try:
        s.sketch(A, B, **kw).factor()
        return s.solve()
    finally:
        s.close()


def _warn_unconverged(rc, infos, where):
    """A solve that stopped at it_max (SKI_WNOCONV) still returns its last iterate: say so."""
    if rc == L.SKI_WNOCONV:
        cols = [(j, i["iters"], i["tc"]) for j, i in enumerate(infos)
                if i["status"] == L.SKI_WNOCONV]
        warnings.warn(f"{where}: {len(cols)} column(s) reached it_max before the stopping "
                      f"test held (column, iterations, test value): {cols[:8]}",
                      RuntimeWarning, stacklevel=3)


class SkiLstsq(torch.autograd.Function):
    """X = argmin ||A X - B||_F (columnwise) with a hand-written adjoint backward.

    Backward: Z = (A^T A)^-1 G by CG preconditioned with the forward's R, then
    grad_B = A Z and grad_A = (B - A X) Z^T - (A Z) X^T, all in the HIP library.

    float32 (or other floating) inputs are converted to float64 for the library, which
    computes in FP64, and the results are converted back.  A solve (forward or adjoint)
    that stops at it_max raises a RuntimeWarning naming the columns.  The library handle
    (which holds the sketch, R and R^-1) lives as long as the autograd node, so backward
    may run more than once (retain_graph=True); it is released with the graph."""

    @staticmethod
    def forward(ctx, A, B, opts=None):
        opts = dict(opts or {})
        in_dtype = A.dtype
        A64 = A.detach().to(torch.float64).contiguous()
        B64 = B.detach().to(torch.float64).reshape(A.shape[0], -1).contiguous()
        s = Solver()
        s.sketch(A64, B64, **opts).factor()
        X, infos, rc = s.solve()
        _warn_unconverged(rc, infos, "SkiLstsq forward")
        ctx.solver = s
        ctx.save_for_backward(A64, B64, X)
        ctx.b_shape = B.shape
        ctx.in_dtype = in_dtype
        ctx.infos = infos
        out = X if B.dim() == 2 else X[:, 0]
        return out.to(in_dtype)

    @staticmethod
    def backward(ctx, gX):
        A64, B64, X = ctx.saved_tensors
        s = ctx.solver
        G = gX.detach().to(torch.float64).reshape(X.shape).contiguous()
        Z, zinfos, zrc = s.solve_normal(G)
        _warn_unconverged(zrc, zinfos, "SkiLstsq backward (adjoint solve)")
        gA, gB = s.gradients(X, B64, Z, want_A=ctx.needs_input_grad[0],
                             want_B=ctx.needs_input_grad[1])
        if gA is not None:
            gA = gA.to(ctx.in_dtype)
        if gB is not None:
            gB = gB.reshape(ctx.b_shape).to(ctx.in_dtype)
        return gA, gB, None
