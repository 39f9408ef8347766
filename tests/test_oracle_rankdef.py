"""Pins of the oracle's rank-deficient path: the column-pivoted factorisation of the
sketch truncated by rcond (Section 6) and Algorithm 1 with V_1 selecting the columns J
(no GPU).

What pins it, independently of the oracle's own QR-with-pivoting call:
* the numerical rank from the SVD of A (p must equal it);
* the structure of the inputs (zero columns are never selected, one column of
  each copied pair at most);
* the least-squares residual from LAPACK's SVD-based solver (the projection of b
  onto range(A) is unique, whatever the column set);
* closed forms on two-column problems;
* on full-rank input, the unpivoted path's solution.
"""

import numpy as np
import scipy.linalg as sla

import workloads
from oracle import lls, sketch as sk


def _sketch(A, b, seed, gamma=1.7, s=3):
    d = A.shape[1]
    m = lls.sketch_size(gamma, d)
    return sk.sketch_dense(A, b, m, s, seed)["SA_aug"]


def _sketch_aug(A, b, seed, gamma=1.7, s=3):
    d = A.shape[1]
    m = lls.sketch_size(gamma, d)
    return sk.sketch_dense(A, b, m, s, seed)["SA_aug"]


def _svd_residual(A, b, rcond=1e-12):
    """Residual of the truncated-SVD solution (singular values below rcond sigma_1 cut,
    as in the paper's comparison of rank-deficient residuals)."""
    x = sla.lstsq(A, b, cond=rcond, lapack_driver="gelsd")[0]
    return b - A @ x


def test_rank_count_reads_rcond_relative_to_r11():
    R = np.diag([4.0, 2.0, 1e-9, 1e-13, 3.0])
    assert lls.rank_count(R, 1e-12) == 3          # stops at the first entry below 4e-12
    assert lls.rank_count(R * 1e-20, 1e-12) == 3  # a scaled copy has the same rank
    assert lls.rank_count(np.zeros((3, 3)), 1e-12) == 0
    assert lls.rank_count(np.eye(4), 1e-12) == 4


def test_pivoted_factor_reveals_the_rank_of_structured_input():
    A, b, ind = workloads.rank_deficient(n=3000, d=120, rank=90, case=6)
    SA = _sketch(A, b, seed=11)
    R11, c, perm, p, dg = lls.factor_pivoted(SA, 120, 1e-12)
    assert p == 90 == np.linalg.matrix_rank(A)
    J = perm[:p]
    zero_cols = np.flatnonzero(np.abs(A).sum(axis=0) == 0)
    assert zero_cols.size > 0 and not np.isin(J, zero_cols).any()
    # no column of J is an exact copy of another one in J
    AJ = A[:, J]
    _, first = np.unique(AJ.T, axis=0, return_index=True)
    assert first.size == p
    # A_J has full column rank and spans range(A)
    sv = np.linalg.svd(AJ, compute_uv=False)
    assert sv[-1] / sv[0] > 1e-8
    U = np.linalg.svd(A, full_matrices=False)[0][:, :p]
    assert np.linalg.norm(AJ - U @ (U.T @ AJ)) <= 1e-10 * np.linalg.norm(AJ)
    # R11 is the R factor of the selected sketch columns: R11^T R11 = (SA_J)^T SA_J
    SAJ = SA[:, J]
    G = SAJ.T @ SAJ
    assert np.all(np.diag(R11) > 0)
    np.testing.assert_allclose(R11.T @ R11, G, rtol=0, atol=1e-12 * np.abs(G).max())
    # c = Q_1^T S b: R11^-1 c solves min ||SA_J z - Sb|| (LAPACK's SVD solver)
    z = sla.solve_triangular(R11, c[:, 0])
    ref = sla.lstsq(SAJ, SA[:, -1], lapack_driver="gelsd")[0]
    np.testing.assert_allclose(z, ref, rtol=1e-9, atol=1e-12 * np.abs(ref).max())
    # the diagonal past p is at rounding level relative to r_11
    assert np.all(np.abs(dg[p:]) < 1e-12 * abs(dg[0]))


def test_pivoted_solution_is_a_least_squares_solution():
    A, b, _ = workloads.rank_deficient(n=3000, d=120, rank=90, case=7)
    X, info = lls.solve(A, b, seed=12, pivoting=True, tau_r=1e-14, it_max=500)
    assert info["status"] == lls.OK and info["p"] == 90
    x = X[:, 0]
    J = info["J"]
    # zero outside the selected columns, exactly
    out = np.setdiff1d(np.arange(120), J)
    assert np.all(x[out] == 0.0)
    # the residual is the unique least-squares residual
    r = b - A @ x
    r_ref = _svd_residual(A, b)
    np.testing.assert_allclose(r, r_ref, rtol=0, atol=1e-10 * np.linalg.norm(b))
    # x_J is the basic solution on J (plain definition by a QR of A_J)
    xb = lls.basic_solution(A, b, J)
    np.testing.assert_allclose(x, xb, rtol=0, atol=1e-10 * np.abs(xb).max())
    # optimality certificate of Algorithm 1's problem
    assert np.linalg.norm(A.T @ r) <= 1e-10 * np.linalg.norm(A) * np.linalg.norm(r)


def test_pivoted_closed_forms_on_two_columns():
    rng = np.random.default_rng(5)
    a = rng.standard_normal(400)
    b = rng.standard_normal(400)
    # [a, a, 0]: rank 1; x puts a^T b / a^T a on one of the copies
    A = np.stack([a, a, np.zeros(400)], axis=1)
    X, info = lls.solve(A, b, seed=3, pivoting=True, m=40, tau_r=1e-14)
    assert info["p"] == 1 and info["J"][0] in (0, 1)
    x = X[:, 0]
    np.testing.assert_allclose(x.sum(), a @ b / (a @ a), rtol=1e-12)
    assert x[2] == 0.0 and np.count_nonzero(x) == 1
    # the zero matrix: p = 0 and x = 0
    X0, info0 = lls.solve(np.zeros((400, 3)), b, seed=3, pivoting=True, m=40)
    assert info0["p"] == 0 and np.all(X0 == 0.0)
    # [a, 2a + 1e-6 e]: full rank but ill-conditioned; p = 2 and the exact solution
    e = rng.standard_normal(400)
    A2 = np.stack([a, 2 * a + 1e-6 * e], axis=1)
    X2, info2 = lls.solve(A2, b, seed=3, pivoting=True, m=40, tau_r=1e-14)
    assert info2["p"] == 2
    xr = sla.lstsq(A2, b, lapack_driver="gelsd")[0]
    np.testing.assert_allclose(X2[:, 0], xr, rtol=1e-7)


def test_pivoted_path_equals_unpivoted_on_full_rank_input():
    rng = np.random.default_rng(9)
    A = rng.standard_normal((2000, 60))
    A[:400] *= 1e3
    b = rng.standard_normal(2000)
    X1, i1 = lls.solve(A, b, seed=4, tau_r=1e-14, it_max=300)
    X2, i2 = lls.solve(A, b, seed=4, pivoting=True, tau_r=1e-14, it_max=300)
    assert i2["p"] == 60 and sorted(i2["J"]) == list(range(60))
    np.testing.assert_allclose(X2, X1, rtol=1e-10, atol=1e-12 * np.abs(X1).max())
    xr = lls.lstsq_direct(A, b)
    np.testing.assert_allclose(X2[:, 0], xr, rtol=1e-10, atol=1e-12 * np.abs(xr).max())


# ------------------------------------------------------------ minimal-norm form (COD)
def test_cod_factor_structure():
    """S A = Q_1 L^T V_1^T with V_1 orthonormal and spanning the row space of SA (R_12 = 0)."""
    A, b, _ = workloads.rank_deficient(n=3000, d=120, rank=90, case=6)
    SA_aug = _sketch_aug(A, b, seed=11)
    L, V1, c, perm, p = lls.factor_cod(SA_aug, 120, 1e-12)
    assert p == 90
    np.testing.assert_allclose(V1.T @ V1, np.eye(p), rtol=0, atol=1e-13)
    SA = SA_aug[:, :120]
    # every row of SA lies in range(V_1): SA = (SA V_1) V_1^T
    np.testing.assert_allclose(SA @ V1 @ V1.T, SA, rtol=0, atol=1e-12 * np.abs(SA).max())
    # (SA V_1)^T (SA V_1) = L L^T (= R_11^T R_11 with R_11 = L^T)
    G = (SA @ V1).T @ (SA @ V1)
    np.testing.assert_allclose(L @ L.T, G, rtol=0, atol=1e-12 * np.abs(G).max())


def test_cod_gives_the_minimal_norm_solution():
    """The minimal-norm guarantee: with R_12 = 0 the solution is pinv(A) b, which LAPACK's
    SVD-based solver returns (singular values below rcond sigma_1 cut)."""
    A, b, _ = workloads.rank_deficient(n=3000, d=120, rank=90, case=7)
    X, info = lls.solve(A, b, seed=12, cod=True, tau_r=1e-14, it_max=500)
    assert info["status"] == lls.OK and info["p"] == 90
    x = X[:, 0]
    xmin = sla.lstsq(A, b, cond=1e-12, lapack_driver="gelsd")[0]
    np.testing.assert_allclose(x, xmin, rtol=0, atol=1e-10 * np.abs(xmin).max())
    # shorter than the basic solution of the pivoted form, with the same residual
    Xb, ib = lls.solve(A, b, seed=12, pivoting=True, tau_r=1e-14, it_max=500)
    assert np.linalg.norm(x) < np.linalg.norm(Xb[:, 0])
    np.testing.assert_allclose(b - A @ x, b - A @ Xb[:, 0], rtol=0, atol=1e-10 * np.linalg.norm(b))


def test_cod_closed_form_on_copied_columns():
    """[a, a, 0]: the minimal-norm solution splits a^T b / a^T a equally between the copies."""
    rng = np.random.default_rng(5)
    a = rng.standard_normal(400)
    b = rng.standard_normal(400)
    A = np.stack([a, a, np.zeros(400)], axis=1)
    X, info = lls.solve(A, b, seed=3, cod=True, m=40, tau_r=1e-14)
    assert info["p"] == 1
    t = a @ b / (a @ a)
    np.testing.assert_allclose(X[:, 0], [t / 2, t / 2, 0.0], rtol=1e-12, atol=1e-15)


def test_cod_equals_unpivoted_on_full_rank_input():
    rng = np.random.default_rng(9)
    A = rng.standard_normal((2000, 60))
    A[:400] *= 1e3
    b = rng.standard_normal(2000)
    X1, _ = lls.solve(A, b, seed=4, tau_r=1e-14, it_max=300)
    X2, i2 = lls.solve(A, b, seed=4, cod=True, tau_r=1e-14, it_max=300)
    assert i2["p"] == 60
    np.testing.assert_allclose(X2, X1, rtol=1e-10, atol=1e-12 * np.abs(X1).max())
