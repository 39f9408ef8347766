"""Pins of the oracle's Steps 2-5 of Algorithm 1 and of its adjoint (no GPU)."""

import math
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import workloads
from oracle import lls, sketch as sk


def _small_dense(n=2000, d=60, seed=0, coherent=False):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, d))
    if coherent:
        A[: n // 5] *= 1e3
    b = rng.standard_normal(n)
    return A, b


def test_factor_is_a_qr_of_the_sketch():
    A, b = _small_dense()
    out = sk.sketch_dense(A, b, 102, 3, seed=1)
    SA = out["SA_aug"]
    R, c, rho = lls.factor(SA, A.shape[1])
    assert np.all(np.diag(R) >= 0) and np.allclose(R, np.triu(R))
    # R^T R is the Gram matrix of SA (the defining property of the R factor)
    G = SA[:, :-1].T @ SA[:, :-1]
    np.testing.assert_allclose(R.T @ R, G, rtol=1e-12, atol=1e-12 * np.abs(G).max())
    # R^-1 c solves the sketched problem min ||SA x - Sb|| (LAPACK's SVD-based solver)
    xs = sla.solve_triangular(R, c[:, 0])
    ref = sla.lstsq(SA[:, :-1], SA[:, -1], lapack_driver="gelsd")[0]
    np.testing.assert_allclose(xs, ref, rtol=1e-10)
    # rho is the sketched residual norm
    np.testing.assert_allclose(rho[0], np.linalg.norm(SA[:, :-1] @ ref - SA[:, -1]), rtol=1e-10)


def test_lsqr_matches_library_iterate_for_iterate():
    # LSQR in floating point drifts from any other rounding of the same
    # recurrences as the iterates converge; compare the early iterates of a
    # well-embedded problem, where the drift is at rounding level.
    A, b = _small_dense(n=1500, d=50, seed=2, coherent=True)
    out = sk.sketch_dense(A, b, 150, 2, seed=3)
    R, c, _ = lls.factor(out["SA_aug"], 50)
    xs = sla.solve_triangular(R, c[:, 0])
    r0 = b - A @ xs
    W = spla.LinearOperator(
        (1500, 50),
        matvec=lambda v: A @ sla.solve_triangular(R, v),
        rmatvec=lambda u: sla.solve_triangular(R, A.T @ u, trans="T"))
    for k in [1, 2, 5, 12]:
        delta, rec = lls.lsqr_precond(A, R, r0, 0.0, k)
        ref = spla.lsqr(W, r0, atol=0, btol=0, conlim=0, iter_lim=k)[0]
        np.testing.assert_allclose(delta, ref, rtol=1e-10, atol=1e-13 * np.abs(ref).max())
        assert rec["iters"] == k


def test_lsqr_norm_estimates_are_the_true_norms():
    A, b = _small_dense(n=1200, d=40, seed=4)
    out = sk.sketch_dense(A, b, 68, 2, seed=5)
    R, c, _ = lls.factor(out["SA_aug"], 40)
    xs = sla.solve_triangular(R, c[:, 0])
    r0 = b - A @ xs
    W = A @ np.linalg.inv(R)
    for k in [3, 8]:
        delta, rec = lls.lsqr_precond(A, R, r0, 0.0, k)
        res = r0 - W @ delta
        np.testing.assert_allclose(rec["rnorm"], np.linalg.norm(res), rtol=1e-9)
        np.testing.assert_allclose(rec["arnorm"], np.linalg.norm(W.T @ res), rtol=1e-6)
        assert rec["anorm"] <= np.linalg.norm(W, "fro") * (1 + 1e-12)


def _eps_of_embedding(S_apply, A, b):
    """epsilon with which the sketch embeds range([A b]) (via U = orth([A b]))."""
    U = np.linalg.qr(np.concatenate([A, b[:, None]], axis=1))[0]
    sv = np.linalg.svd(S_apply(U), compute_uv=False)
    return max(1 - sv.min() ** 2, sv.max() ** 2 - 1)


def _explicit_S(out, n, m, s):
    npad = out["npad"]
    H = sla.hadamard(npad) / math.sqrt(npad)
    S_h = np.zeros((m, npad))
    S_h[out["rows"], np.arange(npad)[:, None]] = np.where(out["neg"], -1.0, 1.0) / math.sqrt(s)
    return (S_h @ H @ np.diag(out["dsign"]))[:, :n]


def test_embedding_bounds_and_sketched_residual():
    # m large enough relative to d that the sketch is an epsilon-embedding
    # with epsilon < 1 (Marchenko-Pastur edge (1 + sqrt(d/m))^2 < 2)
    n, d, m, s = 1024, 20, 300, 2
    A, b = _small_dense(n=n, d=d, seed=6, coherent=True)
    out = sk.sketch_dense(A, b, m, s, seed=11)
    S = _explicit_S(out, n, m, s)
    eps = _eps_of_embedding(lambda U: S @ U, A, b)
    assert 0 < eps < 1
    R, c, _ = lls.factor(out["SA_aug"], d)
    sv = np.linalg.svd(A @ np.linalg.inv(R), compute_uv=False)
    assert sv.max() <= 1 / math.sqrt(1 - eps) * (1 + 1e-10)
    assert sv.min() >= 1 / math.sqrt(1 + eps) * (1 - 1e-10)
    # S A R^-1 = Q has orthonormal columns
    Qs = out["SA_aug"][:, :d] @ np.linalg.inv(R)
    np.testing.assert_allclose(Qs.T @ Qs, np.eye(d), atol=1e-12)
    # explicit sketching guarantee, squared form
    xs = sla.solve_triangular(R, c[:, 0])
    xstar = lls.lstsq_direct(A, b)
    lhs = np.linalg.norm(A @ xs - b) ** 2
    rhs = (1 + eps) / (1 - eps) * np.linalg.norm(A @ xstar - b) ** 2
    assert lhs <= rhs * (1 + 1e-12)


def test_lsqr_rate_of_convergence_bound():
    n, d, m, s = 1024, 30, 120, 2
    A, b = _small_dense(n=n, d=d, seed=8, coherent=True)
    out = sk.sketch_dense(A, b, m, s, seed=12)
    R, c, _ = lls.factor(out["SA_aug"], d)
    W = A @ np.linalg.inv(R)
    kap = np.linalg.cond(W.T @ W)
    q = (math.sqrt(kap) - 1) / (math.sqrt(kap) + 1)
    xs = sla.solve_triangular(R, c[:, 0])
    r0 = b - A @ xs
    dstar = np.linalg.lstsq(W, r0, rcond=None)[0]
    e0 = np.linalg.norm(W @ dstar)
    for j in [1, 3, 6, 10]:
        delta, _ = lls.lsqr_precond(A, R, r0, 0.0, j)
        ej = np.linalg.norm(W @ (delta - dstar))
        assert ej <= 2 * q ** j * e0 * (1 + 1e-8) + 1e-13


def test_tiny_workload_solution_equals_direct_solve():
    A, b, xstar_gen = workloads.tiny()
    X, info = lls.solve(A, b, seed=2001, s=1, m=256, tau_r=1e-10)
    assert info["status"] == lls.OK
    x = X[:, 0]
    xd = lls.lstsq_direct(A, b)
    np.testing.assert_allclose(x, xd, rtol=0, atol=1e-10 * np.linalg.norm(xd))
    ref = sla.lstsq(A, b, lapack_driver="gelsd")[0]
    assert np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(ref)
    r = b - A @ x
    assert np.linalg.norm(A.T @ r) / (np.linalg.norm(A) * np.linalg.norm(r)) < 1e-10
    # residual statistics of the workload: ||r*|| ~ 1e-3 sqrt(n - d)
    expect = 1e-3 * math.sqrt(4096 - 64)
    assert abs(np.linalg.norm(r) - expect) < 4 * 1e-3 / math.sqrt(2)
    assert info["records"][0]["iters"] < 60


def tc_error_bound(A, R, rec, tau_r):
    """Bound on ||x - x*|| implied by the (TC-lsqr) test having passed:
    ||W^T r|| <= tau_r ||W||_est ||r||, so ||y - y*|| <= ||W^T r|| / sigma_min(W)^2
    and ||x - x*|| <= ||R^-1|| ||y - y*||."""
    W = A @ np.linalg.inv(R)
    sv = np.linalg.svd(W, compute_uv=False)
    Rinv_norm = 1.0 / np.linalg.svd(R, compute_uv=False).min()
    return Rinv_norm * tau_r * rec["anorm"] * rec["rnorm"] / sv.min() ** 2


@pytest.mark.parametrize("s", [1, 2, 3])
def test_coherent_dense_solution(s):
    A, b = workloads.dense_coherent(n=3000, d=100, case=2)
    xd = lls.lstsq_direct(A, b)
    # at the paper's kind of tolerance, x is as close to x* as the stopping test implies
    X, info = lls.solve(A, b, seed=2002, s=s, gamma=1.7, tau_r=1e-10)
    assert info["status"] == lls.OK
    bound = tc_error_bound(A, info["R"], info["records"][0], 1e-10)
    assert np.linalg.norm(X[:, 0] - xd) <= bound
    # run (nearly) to convergence, x equals the plain definition to 1e-10
    X, info = lls.solve(A, b, seed=2002, s=s, gamma=1.7, tau_r=1e-14)
    assert np.linalg.norm(X[:, 0] - xd) <= 1e-10 * np.linalg.norm(xd)


def test_sparse_solution_and_certificate():
    row_ptr, col, val, b = workloads.sparse_power_law(n=8000, d=200, case=3)
    A = sp.csr_matrix((val, col, row_ptr), shape=(8000, 200))
    X, info = lls.solve(A, b, seed=2003, s=2, gamma=1.5, tau_r=1e-10)
    assert info["status"] == lls.OK
    x = X[:, 0]
    r = b - A @ x
    rec = info["records"][0]
    # ||A^T r|| <= ||R|| ||W^T r|| <= ||R|| tau_r ||W||_est ||r||
    cert = np.linalg.norm(A.T @ r) / (sp.linalg.norm(A) * np.linalg.norm(r))
    Rn = np.linalg.norm(info["R"], 2)
    assert cert <= 1e-10 * Rn * rec["anorm"] / sp.linalg.norm(A) * (1 + 1e-6)
    assert cert < 1e-9
    xd = lls.lstsq_direct(A, b)
    assert np.linalg.norm(x - xd) <= tc_error_bound(A.toarray(), info["R"], rec, 1e-10)
    X, info = lls.solve(A, b, seed=2003, s=2, gamma=1.5, tau_r=1e-14)
    assert np.linalg.norm(X[:, 0] - xd) <= 1e-10 * np.linalg.norm(xd)


def test_workload_power_law_statistics():
    row_ptr, col, val, b = workloads.sparse_power_law(n=40000, d=500, case=3)
    lens = np.diff(row_ptr)
    assert lens.min() >= 1 and lens.max() <= 500
    assert abs(lens[:-500].mean() - 10.0) < 0.6  # mean 10 (power law), minus the identity rows
    for i in range(0, 40000, 997):
        seg = col[row_ptr[i]:row_ptr[i + 1]]
        assert np.all(np.diff(seg) > 0)


def test_early_exit_on_consistent_system():
    rng = np.random.default_rng(9)
    A = rng.standard_normal((1000, 20))
    x = rng.standard_normal(20)
    X, info = lls.solve(A, A @ x, seed=4, m=40, s=1)
    assert info["status"] == lls.WEARLY
    assert np.linalg.norm(X[:, 0] - x) < 1e-10 * np.linalg.norm(x)


def test_rank_guard_and_perturbed_solve():
    rng = np.random.default_rng(10)
    A = rng.standard_normal((800, 16))
    A[:, 5] = A[:, 3]
    X, info = lls.solve(A, rng.standard_normal(800), seed=4, m=32, s=1)
    assert info["status"] == lls.ERANK
    R = np.triu(rng.standard_normal((5, 5))) + 3 * np.eye(5)
    R[2, 2] = 1e-14
    Rp = lls.perturbed(R, 1e-10, 1e-10)
    assert Rp[2, 2] == pytest.approx(1e-14 + 1e-10)
    R[2, 2] = -1e-14
    assert lls.perturbed(R, 1e-10, 1e-10)[2, 2] == pytest.approx(-1e-14 - 1e-10)


def test_iteration_limit_reports_no_convergence():
    A, b = _small_dense(n=1000, d=30, seed=12)
    X, info = lls.solve(A, b, seed=4, m=45, s=1, tau_r=1e-14, it_max=2)
    assert info["status"] == lls.WNOCONV and info["records"][0]["iters"] == 2


def test_gradients_closed_form_and_adjoint_solve():
    A, B, G = workloads.batched(n=600, d=20, k=3, case=5)
    X, info = lls.solve(A, B, seed=5, m=34, s=3, tau_r=1e-12)
    gA, gB, Z = lls.grads_closed_form(A, X, B, G)
    Zp, iters = lls.normal_solve_pcg(A, info["R"], G, tol=1e-13)
    np.testing.assert_allclose(Zp, Z, rtol=1e-9, atol=1e-12)
    # Z satisfies the normal equations
    np.testing.assert_allclose(A.T @ (A @ Z), G, rtol=0, atol=1e-9 * np.abs(G).max())
    # central finite differences of L = sum(X * G) along random directions
    rng = np.random.default_rng(0)
    h = 1e-6
    for _ in range(4):
        dA = rng.standard_normal(A.shape)
        dB = rng.standard_normal(B.shape)
        Xp = lls.lstsq_direct(A + h * dA, B + h * dB)
        Xm = lls.lstsq_direct(A - h * dA, B - h * dB)
        fd = ((Xp - Xm) * G).sum() / (2 * h)
        an = (gA * dA).sum() + (gB * dB).sum()
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))


def test_stored_dense_reference_solves_the_normal_equations():
    # the stored x* of the dense 50000 x 4000 workload (tests/golden/make_dense_xstar.py)
    # must satisfy A^T (b - A x*) = 0 to rounding: the definition of the least-squares
    # solution, checked on a freshly generated A
    path = os.path.join(os.path.dirname(__file__), "golden", "dense_50000x4000_xstar.txt")
    xs = np.loadtxt(path)
    c = workloads.CASES["dense"]
    A, b = workloads.dense_coherent(n=c["n"], d=c["d"], case=c["case"])
    r = b - A @ xs
    cert = np.linalg.norm(A.T @ r) / (np.linalg.norm(A) * np.linalg.norm(r))
    assert xs.shape == (c["d"],)
    assert cert < 1e-13
