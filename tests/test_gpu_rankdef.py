"""GPU parity of the rank-deficient path (qr_panel = pivoted): the column-pivoted
factorisation of the sketch truncated by rcond and Algorithm 1 on the kept columns J,
through the C interface, against the FP64 oracle on the same seeded inputs.

The GPU pivots on a random sketch of the trailing columns and the oracle pivots
greedily, so the two may keep different (equally valid) column sets.  Parity compares
what is unique: the rank p (exact), the least-squares residual b - A x (unique for any
minimiser), and x against the oracle's basic solution on the GPU's own J (unique when
A_J has full column rank); the rest is checked for validity (J a set of independent
columns, x exactly zero outside J)."""

import sys

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import workloads
from oracle import lls, sketch as sk

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_X = 1e-10  # max |x - x_ref| / max |x_ref|


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


def _check_valid_J(A, perm, p, d):
    assert sorted(perm.tolist()) == list(range(d))
    J = perm[:p]
    AJ = A[:, J]
    assert not np.any(np.abs(AJ).sum(axis=0) == 0)
    sv = np.linalg.svd(AJ, compute_uv=False)
    assert sv[-1] / sv[0] > 1e-8
    return J


RANKDEF_CASES = [
    # n, d, rank, case: one panel with a ragged tail; several panels and two rounds of
    # the tournament (d > 512); three groups in the first round; full rank, ragged
    (3000, 120, 90, 6),
    (6000, 700, 600, 7),
    (9000, 1300, 1100, 8),
    (4000, 333, 333, 9),
]


@pytest.mark.parametrize("panel", ["pivoted", "pivoted_householder"])
@pytest.mark.parametrize("n,d,r,case", RANKDEF_CASES)
def test_pivoted_solve_parity(ski, n, d, r, case, panel):
    _say(f"pivoted solve n={n} d={d} rank={r} case={case} panel={panel}")
    A, b, _ = workloads.rank_deficient(n, d, r, case=case)
    m = lls.sketch_size(1.7, d)
    seed = 500 + case
    S = ski.Solver()
    S.sketch(dev(A), dev(b), m=m, s=3, seed=seed, hadamard=True, qr_panel=panel,
             tau_r=1e-14, it_max=500)
    S.factor()
    X, infos, rc = S.solve()
    x = X[:, 0].cpu().numpy()
    perm, p = S.get_pivots()
    st = S.factor_stats()
    # CholeskyQR2 factors every panel of a full-rank input; the panel holding the rank
    # boundary fails its checks and is factored by Householder columns
    assert st["pivoted"] and st["panels"] == (d + 63) // 64
    if panel == "pivoted_householder":
        assert st["panels_cqr"] == 0
    elif r == d:
        assert st["panels_cqr"] == st["panels"]
    else:
        assert 0 < st["panels_cqr"] < st["panels"]
    R, c, Rinv = S.get_R()
    SA = S.get_SA()
    S.close()
    assert rc == 0 and infos[0]["status"] == 0
    # the oracle on the same sketch (bit-identical to the GPU's): the same rank
    _, _, _, p_ref, _ = lls.factor_pivoted(SA, d, 1e-12)
    assert p == p_ref == r
    J = _check_valid_J(A, perm, p, d)
    # R_11 is the R factor of the kept sketch columns
    SAJ = SA[:, J]
    G = SAJ.T @ SAJ
    R11 = R[:p, :p]
    np.testing.assert_allclose(R11.T @ R11, G, rtol=0, atol=1e-12 * np.abs(G).max())
    assert Rinv.shape == (p, p)
    np.testing.assert_allclose(Rinv @ R11, np.eye(p), rtol=0, atol=1e-10)
    # x: zero outside J, the basic solution on J
    out = np.setdiff1d(np.arange(d), J)
    assert np.all(x[out] == 0.0)
    xb = lls.basic_solution(A, b, J)
    err = np.abs(x - xb).max() / np.abs(xb).max()
    _say(f"  p={p} iters={infos[0]['iters']} max rel err {err:.2e}")
    assert err <= TOL_X
    # the residual is the oracle's (unique) least-squares residual
    Xo, io = lls.solve(A, b, seed, pivoting=True, m=m, s=3, tau_r=1e-14, it_max=500)
    r_ref = b - A @ Xo[:, 0]
    np.testing.assert_allclose(b - A @ x, r_ref, rtol=0, atol=1e-10 * np.linalg.norm(b))


def test_pivoted_equals_unpivoted_on_full_rank(ski):
    _say("pivoted vs unpivoted, full rank 5000 x 260")
    rng = np.random.default_rng(31)
    A = rng.standard_normal((5000, 260))
    A[:1000] *= 1e3
    b = rng.standard_normal(5000)
    out = []
    for panel in ["auto", "pivoted"]:
        S = ski.Solver()
        S.sketch(dev(A), dev(b), s=3, seed=9, qr_panel=panel, tau_r=1e-14, it_max=400)
        S.factor()
        X, infos, rc = S.solve()
        assert rc == 0
        out.append(X[:, 0].cpu().numpy())
        if panel == "pivoted":
            assert S.get_pivots()[1] == 260
        S.close()
    xr = lls.lstsq_direct(A, b)
    for x in out:
        assert np.abs(x - xr).max() / np.abs(xr).max() <= TOL_X


def test_pivoted_zero_matrix_gives_zero(ski):
    _say("pivoted, A = 0")
    A = np.zeros((2000, 70))
    b = np.random.default_rng(2).standard_normal(2000)
    S = ski.Solver()
    S.sketch(dev(A), dev(b), s=2, seed=3, qr_panel="pivoted")
    S.factor()
    X, infos, rc = S.solve()
    assert S.get_pivots()[1] == 0
    assert rc == 0 and infos[0]["iters"] == 0
    assert torch.all(X == 0).item()
    S.close()


def test_pivoted_multiple_rhs_and_adjoint(ski):
    _say("pivoted, 3 right-hand sides and the adjoint, 4000 x 300 rank 250")
    A, _, _ = workloads.rank_deficient(4000, 300, 250, case=10)
    rng = np.random.default_rng(12)
    B = rng.standard_normal((4000, 3))
    G = rng.standard_normal((300, 3))
    S = ski.Solver()
    S.sketch(dev(A), dev(B), s=3, seed=21, qr_panel="pivoted", tau_r=1e-14, it_max=400)
    S.factor()
    X, infos, rc = S.solve()
    assert rc == 0
    perm, p = S.get_pivots()
    assert p == 250
    J = _check_valid_J(A, perm, p, 300)
    X = X.cpu().numpy()
    out = np.setdiff1d(np.arange(300), J)
    assert np.all(X[out] == 0.0)
    for j in range(3):
        xb = lls.basic_solution(A, B[:, j], J)
        assert np.abs(X[:, j] - xb).max() / np.abs(xb).max() <= TOL_X
    # adjoint with J held fixed: Z_J = (A_J^T A_J)^-1 G_J, zero elsewhere
    Z, zinfo, zrc = S.solve_normal(dev(G))
    Z = Z.cpu().numpy()
    assert np.all(Z[out] == 0.0)
    AJ = A[:, J]
    RJ = np.linalg.qr(AJ, mode="r")
    import scipy.linalg as sla
    Zref = sla.solve_triangular(RJ, sla.solve_triangular(RJ, G[J], trans="T"))
    np.testing.assert_allclose(Z[J], Zref, rtol=0, atol=1e-9 * np.abs(Zref).max())
    S.close()


def test_pivoted_sparse_parity(ski):
    _say("pivoted, CSR 6000 x 200 rank 160")
    A, b, _ = workloads.rank_deficient(6000, 200, 160, case=11)
    # sparsify: copies and zero columns stay dependent (the combinations do not, so the
    # rank is taken from the SVD of the sparsified matrix)
    A[np.abs(A) < 0.8] = 0.0
    Acsr = sp.csr_matrix(A)
    n, d = A.shape
    r = np.linalg.matrix_rank(A)
    S = ski.Solver()
    S.sketch(("csr", dev(Acsr.indptr.astype(np.int64), torch.int64),
              dev(Acsr.indices.astype(np.int32), torch.int32), dev(Acsr.data), (n, d)),
             dev(b), s=2, seed=5, hadamard=False, qr_panel="pivoted", rcond=1e-12,
             tau_r=1e-14, it_max=500)
    S.factor()
    X, infos, rc = S.solve()
    assert rc == 0
    perm, p = S.get_pivots()
    assert p == r
    J = _check_valid_J(A, perm, p, d)
    x = X[:, 0].cpu().numpy()
    xb = lls.basic_solution(A, b, J)
    assert np.all(x[np.setdiff1d(np.arange(d), J)] == 0.0)
    assert np.abs(x - xb).max() / np.abs(xb).max() <= TOL_X
    S.close()


def test_pivoted_rejects_mixed_precision(ski):
    A = np.random.default_rng(1).standard_normal((500, 20))
    b = np.ones(500)
    S = ski.Solver()
    with pytest.raises(ski.SkiError):
        S.sketch(dev(A), dev(b), qr_panel="pivoted", qr_prec="fp32")
    S.close()


def test_full_size_rankdef_optimality(ski):
    """The 50000 x 4000 rank-3500 workload in the launch configuration the benchmark times
    (m = 6800, s = 3): the rank, x exactly zero outside J, the optimality certificate of the
    least-squares problem ||A^T r|| / (||A||_F ||r||) (it vanishes only at a minimiser; J
    spans range(A) when p = rank(A)), and R_11's diagonal ratio as a check that J is a set of
    independent columns."""
    c = workloads.CASES["rankdef"]
    _say(f"full-size rank-deficient {c['n']}x{c['d']} rank {c['rank']}")
    A, b, _ = workloads.rank_deficient(n=c["n"], d=c["d"], rank=c["rank"], case=c["case"])
    At, bt = dev(A), dev(b)
    del A
    S = ski.Solver()
    S.sketch(At, bt, gamma=c["gamma"], m=c["m"], s=c["s"], seed=2006, hadamard=True,
             qr_panel="pivoted", tau_r=1e-14, it_max=400)
    S.factor()
    X, infos, rc = S.solve()
    perm, p = S.get_pivots()
    S.close()
    assert p == c["rank"]
    assert sorted(perm.tolist()) == list(range(c["d"]))
    x = X[:, 0]
    out = torch.as_tensor(perm[p:], device="cuda")
    assert bool((x[out] == 0).all().item())
    r = bt - At @ x
    cert = float((At.T @ r).norm() / (At.norm() * r.norm()))
    _say(f"  iters {infos[0]['iters']} certificate {cert:.2e} cond_est {infos[0]['cond_est']:.2e}")
    assert cert <= 1e-12
    assert infos[0]["cond_est"] < 1e6
    del At, bt
    torch.cuda.empty_cache()


# ------------------------------------------------------------ minimal-norm form (COD)
COD_CASES = [(3000, 120, 90, 6), (6000, 700, 600, 7), (4000, 333, 333, 9)]


@pytest.mark.parametrize("n,d,r,case", COD_CASES)
def test_cod_gives_the_minimal_norm_solution(ski, n, d, r, case):
    """qr_panel = cod: x is the minimal-norm least-squares solution (Section 5's guarantee
    with R_12 = 0), against LAPACK's SVD-based solver (a plain definition, independent of
    the factorisation) and against the oracle's COD form on the same inputs."""
    _say(f"cod n={n} d={d} rank={r} case={case}")
    A, b, _ = workloads.rank_deficient(n, d, r, case=case)
    m = lls.sketch_size(1.7, d)
    seed = 700 + case
    S = ski.Solver()
    S.sketch(dev(A), dev(b), m=m, s=3, seed=seed, hadamard=True, qr_panel="cod",
             tau_r=1e-14, it_max=500)
    S.factor()
    X, infos, rc = S.solve()
    perm, p = S.get_pivots()
    S.close()
    assert rc == 0 and p == r
    x = X[:, 0].cpu().numpy()
    xmin = sla.lstsq(A, b, cond=1e-12, lapack_driver="gelsd")[0]
    err = np.abs(x - xmin).max() / np.abs(xmin).max()
    _say(f"  iters {infos[0]['iters']} max rel err vs minimal-norm {err:.2e}")
    assert err <= TOL_X
    Xo, io = lls.solve(A, b, seed, cod=True, m=m, s=3, tau_r=1e-14, it_max=500)
    assert io["p"] == r
    assert np.abs(x - Xo[:, 0]).max() <= TOL_X * np.abs(xmin).max()


def test_cod_multiple_rhs(ski):
    _say("cod, 3 right-hand sides, 4000 x 300 rank 250")
    A, _, _ = workloads.rank_deficient(4000, 300, 250, case=10)
    rng = np.random.default_rng(12)
    B = rng.standard_normal((4000, 3))
    S = ski.Solver()
    S.sketch(dev(A), dev(B), s=3, seed=21, qr_panel="cod", tau_r=1e-14, it_max=400)
    S.factor()
    X, infos, rc = S.solve()
    S.close()
    assert rc == 0
    X = X.cpu().numpy()
    Xmin = sla.lstsq(A, B, cond=1e-12, lapack_driver="gelsd")[0]
    for j in range(3):
        assert np.abs(X[:, j] - Xmin[:, j]).max() <= TOL_X * np.abs(Xmin[:, j]).max()


def test_full_size_cod_minimal_norm_properties(ski):
    """The 50000 x 4000 rank-3500 workload with qr_panel = cod: the optimality certificate,
    and the conditions that single out the minimal-norm solution among all least-squares
    solutions on this input's structure: x_j = 0 on every zero column (e_j spans a null
    direction) and x_i = x_j for every exact copy a_j = a_i (e_i - e_j is a null direction),
    which the basic solution of the pivoted form violates."""
    c = workloads.CASES["rankdef"]
    _say(f"full-size cod {c['n']}x{c['d']} rank {c['rank']}")
    A, b, ind = workloads.rank_deficient(n=c["n"], d=c["d"], rank=c["rank"], case=c["case"])
    d = c["d"]
    zero = np.flatnonzero(~A.any(axis=0))
    # exact copies of an independent column, matched on their first rows
    key = {tuple(A[:4, i]): i for i in ind}
    dep = np.setdiff1d(np.arange(d), ind)
    copies = [(key[tuple(A[:4, j])], j) for j in dep
              if j not in set(zero) and tuple(A[:4, j]) in key
              and np.array_equal(A[:, key[tuple(A[:4, j])]], A[:, j])]
    assert len(zero) > 0 and len(copies) > 0
    At, bt = dev(A), dev(b)
    del A
    S = ski.Solver()
    S.sketch(At, bt, gamma=c["gamma"], m=c["m"], s=c["s"], seed=2006, hadamard=True,
             qr_panel="cod", tau_r=1e-14, it_max=400)
    S.factor()
    X, infos, rc = S.solve()
    perm, p = S.get_pivots()
    S.close()
    assert rc == 0 and p == c["rank"]
    x = X[:, 0]
    r = bt - At @ x
    cert = float((At.T @ r).norm() / (At.norm() * r.norm()))
    xh = x.cpu().numpy()
    scale = np.abs(xh).max()
    zmax = np.abs(xh[zero]).max() / scale
    cmax = max(abs(xh[i] - xh[j]) for i, j in copies) / scale
    _say(f"  iters {infos[0]['iters']} certificate {cert:.2e} zero cols {zmax:.1e} "
         f"copies {cmax:.1e} ({len(copies)} pairs)")
    assert cert <= 1e-12
    assert zmax <= 1e-12
    assert cmax <= 1e-10
    del At, bt
    torch.cuda.empty_cache()
