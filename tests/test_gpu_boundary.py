"""The C interface on the GPU: non-finite input is rejected with SKI_EINVAL (through the
C ABI itself, by ctypes), and many right-hand sides that stop at different iterations."""

import ctypes as C
import sys

import numpy as np
import pytest

import workloads
from oracle import lls

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ski():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2105_11815_amd as P
    return P


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dense(A, kind=None):
    from paper_2105_11815_amd import _lib as L
    if kind == "col":
        return L.SkiMatrix(n=A.shape[0], d=A.shape[1], kind=L.SKI_DENSE_COLMAJOR,
                           a=A.data_ptr(), lda=A.stride(1), row_ptr=None, col=None, val=None,
                           nnz=0)
    return L.SkiMatrix(n=A.shape[0], d=A.shape[1], kind=L.SKI_DENSE, a=A.data_ptr(),
                       lda=A.stride(0), row_ptr=None, col=None, val=None, nnz=0)


def _params(ski, kind="dense", **kw):
    return ski.params(kind, **kw)


def _sketch_factor(lib, L, M, B, k, p):
    h = C.c_void_p()
    assert lib.ski_create(C.byref(h)) == L.SKI_OK
    rc = lib.ski_sketch(h, C.byref(M), C.c_void_p(B.data_ptr()), k, k, C.byref(p), _stream())
    assert rc == L.SKI_OK, lib.ski_last_error(h)
    return h, lib.ski_factor(h, _stream())


@pytest.mark.parametrize("where,value", [("A", np.nan), ("A", np.inf), ("b", -np.inf),
                                         ("b", np.nan), ("Acol", np.nan)])
def test_nonfinite_dense_input_is_rejected(ski, where, value):
    """A NaN or an infinity in A or b: ski_factor returns SKI_EINVAL (the sketch carries it;
    every row of [A b] enters S [A b]) and the handle refuses to solve."""
    from paper_2105_11815_amd import _lib as L
    lib = L.load()
    _say(f"non-finite {where} = {value}")
    rng = np.random.default_rng(3)
    n, d = 3000, 70
    A = rng.standard_normal((n, d))
    b = rng.standard_normal(n)
    if where in ("A", "Acol"):
        A[1234, 17] = value
    else:
        b[2999] = value
    At = dev(A)
    if where == "Acol":
        At = At.t().contiguous().t()
    bt = dev(b)
    h, rc = _sketch_factor(lib, L, _dense(At, "col" if where == "Acol" else None), bt, 1,
                           _params(ski, s=2, m=150, seed=5))
    assert rc == L.SKI_EINVAL
    assert b"non-finite" in lib.ski_last_error(h)
    X = dev(np.zeros(d))
    assert lib.ski_solve(h, L.SKI_OP_LLS, C.c_void_p(bt.data_ptr()), 1, 1,
                         C.c_void_p(X.data_ptr()), 1, None, _stream()) == L.SKI_ESTATE
    lib.ski_destroy(h)


def test_nonfinite_csr_input_is_rejected(ski):
    from paper_2105_11815_amd import _lib as L
    lib = L.load()
    n, d = 5000, 60
    rp, ci, va, b = workloads.sparse_power_law(n=n, d=d, case=3)
    va = va.copy()
    va[len(va) // 2] = np.nan
    rpt, cit, vat, bt = dev(rp, torch.int64), dev(ci, torch.int32), dev(va), dev(b)
    M = L.SkiMatrix(n=n, d=d, kind=L.SKI_CSR, a=None, lda=0, row_ptr=rpt.data_ptr(),
                    col=cit.data_ptr(), val=vat.data_ptr(), nnz=len(va))
    h, rc = _sketch_factor(lib, L, M, bt, 1, _params(ski, "csr", s=2, m=90, seed=7))
    assert rc == L.SKI_EINVAL
    assert b"non-finite" in lib.ski_last_error(h)
    lib.ski_destroy(h)


@pytest.mark.parametrize("fault", ["col_high", "col_negative", "ptr_decreasing", "ptr_end"])
def test_malformed_csr_is_rejected_before_device_work(ski, fault):
    """A column index outside [0, d) or row offsets that do not rise from 0 to nnz: ski_sketch
    returns SKI_EINVAL from its device check of the structure, before any kernel indexes
    with it; the handle then refuses to factor, and a well-formed call afterwards works."""
    from paper_2105_11815_amd import _lib as L
    lib = L.load()
    _say(f"malformed CSR: {fault}")
    n, d = 4000, 50
    rp, ci, va, b = workloads.sparse_power_law(n=n, d=d, case=3)
    rp, ci = rp.copy(), ci.copy()
    if fault == "col_high":
        ci[len(ci) // 3] = d
    elif fault == "col_negative":
        ci[7] = -1
    elif fault == "ptr_decreasing":
        rp[100] = rp[101] + 1  # row 100 would start after row 101
    else:
        rp[-1] = rp[-1] - 1
    rpt, cit, vat, bt = dev(rp, torch.int64), dev(ci, torch.int32), dev(va), dev(b)
    M = L.SkiMatrix(n=n, d=d, kind=L.SKI_CSR, a=None, lda=0, row_ptr=rpt.data_ptr(),
                    col=cit.data_ptr(), val=vat.data_ptr(), nnz=len(va))
    p = _params(ski, "csr", s=2, m=80, seed=7)
    h = C.c_void_p()
    assert lib.ski_create(C.byref(h)) == L.SKI_OK
    rc = lib.ski_sketch(h, C.byref(M), C.c_void_p(bt.data_ptr()), 1, 1, C.byref(p), _stream())
    assert rc == L.SKI_EINVAL
    assert b"malformed CSR" in lib.ski_last_error(h)
    assert lib.ski_factor(h, _stream()) == L.SKI_ESTATE
    # the same handle with the well-formed matrix
    rp0, ci0, _, _ = workloads.sparse_power_law(n=n, d=d, case=3)
    rpt, cit = dev(rp0, torch.int64), dev(ci0, torch.int32)
    M = L.SkiMatrix(n=n, d=d, kind=L.SKI_CSR, a=None, lda=0, row_ptr=rpt.data_ptr(),
                    col=cit.data_ptr(), val=vat.data_ptr(), nnz=len(va))
    rc = lib.ski_sketch(h, C.byref(M), C.c_void_p(bt.data_ptr()), 1, 1, C.byref(p), _stream())
    assert rc == L.SKI_OK, lib.ski_last_error(h)
    assert lib.ski_factor(h, _stream()) == L.SKI_OK, lib.ski_last_error(h)
    lib.ski_destroy(h)


@pytest.mark.parametrize("form", ["auto", "sparse"])
def test_zero_csr_matrix(ski, form):
    """A = 0 stored with no entries (nnz = 0, every row empty): every x is a least-squares
    solution.  The sparse factor leaves zero rows and columns in R, so x = 0.  The dense
    factor of the same sketch has R = 0, which the perturbed back-solve turns into
    R + 1e-10 I, so x = x_s = 1e10 c, and LSQR stops at once (A^T r_0 = 0), as the oracle's
    solve does."""
    import scipy.sparse as sp
    from oracle import sparse_qr as sq
    from paper_2105_11815_amd import _lib as L
    lib = L.load()
    _say(f"zero CSR matrix, {form} factor")
    n, d, s, m, seed = 600, 25, 2, 40, 17
    b = np.random.default_rng(21).standard_normal(n)
    rpt = dev(np.zeros(n + 1, np.int64), torch.int64)
    cit = dev(np.zeros(1, np.int32), torch.int32)  # nnz = 0: nothing is read from these
    vat = dev(np.zeros(1))
    bt = dev(b)
    M = L.SkiMatrix(n=n, d=d, kind=L.SKI_CSR, a=None, lda=0, row_ptr=rpt.data_ptr(),
                    col=cit.data_ptr(), val=vat.data_ptr(), nnz=0)
    p = _params(ski, "csr", s=s, m=m, seed=seed, qr_panel=form)
    h, rc = _sketch_factor(lib, L, M, bt, 1, p)
    assert rc == L.SKI_OK, lib.ski_last_error(h)
    X = dev(np.zeros(d))
    info = (L.SkiInfo * 1)()
    rc = lib.ski_solve(h, L.SKI_OP_LLS, C.c_void_p(bt.data_ptr()), 1, 1,
                       C.c_void_p(X.data_ptr()), 1, info, _stream())
    lib.ski_destroy(h)
    assert rc == L.SKI_OK and info[0].status == L.SKI_OK and info[0].iters == 0
    assert abs(info[0].rnorm - np.linalg.norm(b)) <= 1e-12 * np.linalg.norm(b)
    x = X.cpu().numpy()
    Az = sp.csr_matrix((n, d))
    if form == "sparse":
        assert np.all(x == 0.0)
        assert np.all(sq.solve(Az, b, seed, m=m, s=s)["x"] == 0.0)
    else:
        X_o, info_o = lls.solve(Az, b, seed, m=m, s=s)
        xo = X_o[:, 0]
        assert np.linalg.norm(xo) > 1e8  # the perturbed back-solve of R = 0
        assert np.linalg.norm(x - xo) <= 1e-12 * np.linalg.norm(xo)


def test_nonfinite_right_hand_sides_at_solve_and_adjoint(ski):
    """ski_solve with a B that holds an infinity (LLS) or a G that holds a NaN (the adjoint):
    SKI_EINVAL from the first norm of the iteration, with no iterations run on it; the
    finite columns of the same call still solve."""
    from paper_2105_11815_amd import _lib as L
    lib = L.load()
    rng = np.random.default_rng(4)
    n, d, k = 3000, 80, 3
    A = rng.standard_normal((n, d))
    B = rng.standard_normal((n, k))
    At, Bt = dev(A), dev(B)
    h, rc = _sketch_factor(lib, L, _dense(At), Bt, k, _params(ski, s=2, m=160, seed=9,
                                                             tau_r=1e-14))
    assert rc == L.SKI_OK
    Bbad = B.copy()
    Bbad[10, 1] = np.inf
    Bb = dev(Bbad)
    X = dev(np.zeros((d, k)))
    infos = (L.SkiInfo * k)()
    rc = lib.ski_solve(h, L.SKI_OP_LLS, C.c_void_p(Bb.data_ptr()), k, k,
                       C.c_void_p(X.data_ptr()), k, infos, _stream())
    assert rc == L.SKI_EINVAL
    assert infos[1].status == L.SKI_EINVAL and infos[1].iters == 0
    assert infos[0].status == L.SKI_OK and infos[2].status == L.SKI_OK
    Xd = lls.lstsq_direct(A, B)
    Xh = X.cpu().numpy()
    for j in (0, 2):
        assert np.linalg.norm(Xh[:, j] - Xd[:, j]) <= 1e-10 * np.linalg.norm(Xd[:, j])
    G = rng.standard_normal((d, k))
    G[5, 2] = np.nan
    Gt = dev(G)
    Z = dev(np.zeros((d, k)))
    rc = lib.ski_solve(h, L.SKI_OP_NORMAL, C.c_void_p(Gt.data_ptr()), k, k,
                       C.c_void_p(Z.data_ptr()), k, infos, _stream())
    assert rc == L.SKI_EINVAL
    assert infos[2].status == L.SKI_EINVAL and infos[2].iters == 0
    assert b"non-finite" in lib.ski_last_error(h)
    # the handle still solves finite input afterwards
    rc = lib.ski_solve(h, L.SKI_OP_LLS, C.c_void_p(Bt.data_ptr()), k, k,
                       C.c_void_p(X.data_ptr()), k, infos, _stream())
    assert rc == L.SKI_OK
    lib.ski_destroy(h)


def test_python_binding_raises_on_nonfinite(ski):
    rng = np.random.default_rng(6)
    A = rng.standard_normal((2000, 30))
    A[7, 3] = np.nan
    with pytest.raises(ski.SkiError) as e:
        ski.lstsq(dev(A), dev(rng.standard_normal(2000)), s=1, m=60, seed=1)
    assert e.value.code == -1


def test_one_hundred_columns_stopping_at_different_iterations(ski):
    """k = 100 right-hand sides (two 64-lane chunks of the step kernels' status vote; the
    products take the general GEMM) that do not all stop together: column 0 is consistent
    (Step 3's early exit, no iteration), the others carry noise from 1e-2 to 10.  Every
    column against the direct solution, the adjoint against the closed form, twice in a
    row on one handle (the arrival counter of the status word is re-armed)."""
    n, d, k = 4000, 150, 100
    _say(f"k={k} right-hand sides n={n} d={d}")
    rng = np.random.default_rng(12)
    A = rng.standard_normal((n, d))
    Xt = rng.standard_normal((d, k))
    noise = np.concatenate([[0.0], np.logspace(-2, 1, k - 1)])
    B = A @ Xt + rng.standard_normal((n, k)) * noise
    G = rng.standard_normal((d, k))
    Xd = lls.lstsq_direct(A, B)
    S = ski.Solver()
    S.sketch(dev(A), dev(B), gamma=1.7, s=3, seed=2005, tau_r=1e-13, it_max=400).factor()
    for rep in range(2):
        X, infos, rc = S.solve()
        its = [i["iters"] for i in infos]
        _say(f"  pass {rep}: status {rc}, iteration counts {sorted(set(its))}")
        assert rc == 0
        assert infos[0]["early_exit"] == 1 and its[0] == 0
        assert min(its[1:]) > 0 and len(set(its)) >= 2
        Xh = X.cpu().numpy()
        for j in range(k):
            err = np.linalg.norm(Xh[:, j] - Xd[:, j]) / np.linalg.norm(Xd[:, j])
            assert err <= 1e-10, (rep, j, err)
        Z, zinfos, zrc = S.solve_normal(dev(G))
        assert zrc == 0
        _, _, Z_ref = lls.grads_closed_form(A, Xh, B, G)
        np.testing.assert_allclose(Z.cpu().numpy(), Z_ref, rtol=0,
                                   atol=1e-10 * np.abs(Z_ref).max())
    S.close()
