"""GPU parity of the sparse QR of the sketch (Section 6, the sparse solver: S A P = Q R with
a fill-reducing ordering P, and sparse substitution for every product with R^-1), through
the C interface, against the oracle (oracle/sparse_qr.py).

* The sparse sketch against the oracle's sketch: identical bits.
* The ordering (integer work) against the oracle's minimum-degree order: identical.
* R and c against the QR of the oracle's column-permuted sketch, within
  1e-12 max|R| sqrt(d); R exactly zero outside the oracle's predicted structure.
* The iteration count at tau_r = 1e-10 within max(2, 1%) of the oracle's sparse solve
  (same sketch, same ordering, same LSQR); x run to stagnation within 1e-10 of LAPACK's
  least-squares solution, as the oracle's is.
Cases: leaves only, leaves and a root, root only (with buckets too wide for the sorted
merge), several right-hand sides, a zero column (perturbed back-solve), a non-finite
entry, and the 40000 x 8000 very sparse workload against the dense factorisation.
"""

import math
import sys

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import workloads
from oracle import lls, sketch as sk, sparse_qr as sq

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


def _csr_arg(rp, ci, va, n, d):
    return ("csr", dev(rp, torch.int64), dev(ci, torch.int32), dev(va), (n, d))


def _inputs(case):
    n, d, per_col = case["n"], case["d"], case["per_col"]
    if per_col is None:
        rp, ci, va, b = workloads.sparse_power_law(n=n, d=d, case=3)
    else:
        rp, ci, va, b = workloads.very_sparse(n, d, per_col)
    k = case["k"]
    B = b[:, None] if k == 1 else np.random.default_rng(n + d).standard_normal((n, k))
    return rp, ci, va, B


# n, d, nonzeros per column (None: the power-law rows), s, m, k, and what the order gives
CASES = {
    "leaves_only": dict(n=2000, d=300, per_col=1, s=3, m=600, k=1),
    "leaves_and_root": dict(n=3000, d=500, per_col=2, s=2, m=700, k=1),
    "leaves_root_k2": dict(n=4000, d=600, per_col=3, s=2, m=840, k=2),
    "root_only_wide_buckets": dict(n=40000, d=100, per_col=None, s=2, m=140, k=1),
}


@pytest.mark.parametrize("name", list(CASES))
def test_sparse_sketch_order_and_factor_match_oracle(ski, name):
    c = CASES[name]
    n, d, s, m, k = c["n"], c["d"], c["s"], c["m"], c["k"]
    _say(f"sparse factor {name}: n={n} d={d} s={s} m={m} k={k}")
    rp, ci, va, B = _inputs(c)
    seed = 11
    ref = sk.sketch_csr(rp, ci, va, n, d, B, m, s, seed)
    S = ski.Solver()
    S.sketch(_csr_arg(rp, ci, va, n, d), dev(B), m=m, s=s, seed=seed, qr_panel="sparse")
    # the sparse sketch sums in the dense sketch's order: the same bits
    np.testing.assert_array_equal(S.get_SA(), ref["SA_aug"])
    S.factor()
    pats = sq.sa_row_patterns(rp, ci, n, d, m, s, seed)
    order, root, L = sq.min_degree(pats, d, 63 - k)
    perm_o, _ = sq.positions(order, root)
    perm, rank = S.get_pivots()
    np.testing.assert_array_equal(perm, perm_o)
    st = S.factor_stats()
    assert st["sparse"] and rank == d
    assert (st["leaf_fronts"], st["root"]) == (len(order), len(root))
    if name == "leaves_only":
        assert len(root) == 0
    elif name.startswith("root_only"):
        assert len(order) == 0
    else:
        assert len(order) > 0 and len(root) > 0
    R, cc, Ri = S.get_R()
    assert Ri is None
    Rref, cref = sq.factor(ref["SA_aug"], d, perm_o)
    # the leaf rows hold nothing outside the predicted structure
    assert np.all(R[~sq.r_structure(order, root, L, d)] == 0.0)
    scale = np.abs(Rref).max()
    np.testing.assert_allclose(R, Rref, rtol=0, atol=1e-12 * scale * math.sqrt(d))
    np.testing.assert_allclose(cc, cref, rtol=0, atol=1e-12 * np.abs(cref).max() * math.sqrt(d))
    S.close()


@pytest.mark.parametrize("name", list(CASES))
def test_sparse_solve_matches_oracle(ski, name):
    """Iterations at tau_r = 1e-10 within max(2, 1%) of the oracle's (same sketch, ordering
    and LSQR); x run to stagnation (tau_r = 1e-14) within 1e-10 of LAPACK's least-squares
    solution, as the oracle's is.  (With a large residual, (TC-lsqr) at 1e-12 pins x only to
    about 1e-10 relative, so two runs stopped there differ by that much.)"""
    c = CASES[name]
    n, d, s, m, k = c["n"], c["d"], c["s"], c["m"], c["k"]
    _say(f"sparse solve {name}: n={n} d={d} s={s} m={m} k={k}")
    rp, ci, va, B = _inputs(c)
    A = sp.csr_matrix((va, ci, rp), shape=(n, d))
    Xd = sla.lstsq(A.toarray(), B)[0]
    seed = 12
    for tau in (1e-10, 1e-14):
        res = sq.solve(A, B, seed, m=m, s=s, dmax=63 - k, tau_r=tau, tau_a=0.0)
        S = ski.Solver()
        S.sketch(_csr_arg(rp, ci, va, n, d), dev(B), m=m, s=s, seed=seed, qr_panel="sparse",
                 tau_r=tau, tau_a=0.0).factor()
        X, infos, rc = S.solve()
        S.close()
        X = X.cpu().numpy()
        for j in range(k):
            xd = Xd[:, j]
            err = np.linalg.norm(X[:, j] - xd) / np.linalg.norm(xd)
            erro = np.linalg.norm(res["x"][:, j] - xd) / np.linalg.norm(xd)
            _say(f"  tau {tau:.0e} column {j}: iters {infos[j]['iters']} (oracle "
                 f"{res['iters'][j]}); x error {err:.2e} (oracle {erro:.2e})")
            if tau == 1e-10:
                # the (TC-lsqr) estimate is not monotone near the threshold, so on a slowly
                # converging problem (about 140 steps here) rounding order moves the step
                # that crosses it by a few: within max(2, 1%) of the oracle's count
                assert infos[j]["status"] == 0
                assert abs(infos[j]["iters"] - res["iters"][j]) <= max(2, 0.01 * res["iters"][j])
            else:
                assert infos[j]["status"] in (0, 1)
                assert err <= 1e-10 and erro <= 1e-10


def test_sparse_zero_column_is_perturbed_and_zero(ski):
    n, d, s, m = 2000, 300, 3, 600
    rp, ci, va, b = workloads.very_sparse(n, d, 2)
    A = sp.csr_matrix((va, ci, rp), shape=(n, d)).tolil()
    A[:, 17] = 0.0
    A = A.tocsr()
    A.eliminate_zeros()
    A.sort_indices()
    rp, ci, va = A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data
    _say(f"sparse zero column n={n} d={d}")
    S = ski.Solver()
    S.sketch(_csr_arg(rp, ci, va, n, d), dev(b), m=m, s=s, seed=13, qr_panel="sparse",
             tau_r=1e-12, tau_a=0.0).factor()
    R, cc, _ = S.get_R()
    perm, _ = S.get_pivots()
    q = int(np.nonzero(perm == 17)[0][0])
    assert np.all(R[q] == 0.0) and np.all(R[:, q] == 0.0)
    X, infos, rc = S.solve()
    S.close()
    x = X[:, 0].cpu().numpy()
    assert x[17] == 0.0
    keep = np.arange(d) != 17
    xd = sla.lstsq(A.toarray()[:, keep], b)[0]
    assert np.linalg.norm(x[keep] - xd) <= 1e-9 * np.linalg.norm(xd)


@pytest.mark.parametrize("where", ["leaf", "root", "rhs"])
def test_sparse_nonfinite_entry_is_reported(ski, where):
    """A NaN in A reaching a leaf front, a NaN in A on a root-only problem, and an infinity in
    b: SKI_EINVAL from ski_factor in each case."""
    if where == "root":
        rp, ci, va, b = workloads.sparse_power_law(n=40000, d=100, case=3)
        n, d, m, s = 40000, 100, 140, 2
    else:
        n, d, m, s = 2000, 300, 600, 3
        rp, ci, va, b = workloads.very_sparse(n, d, 2)
    va, b = va.copy(), b.copy()
    if where == "rhs":
        b[5] = np.inf  # row 5 holds column 5's entry: its sketch rows reach a front
    else:
        va[123] = np.nan
    S = ski.Solver()
    S.sketch(_csr_arg(rp, ci, va, n, d), dev(b), m=m, s=s, seed=14, qr_panel="sparse")
    with pytest.raises(ski.SkiError) as e:
        S.factor()
    assert e.value.code == -1
    S.close()


def test_sparse_repeat_runs_are_bitwise_identical(ski):
    c = CASES["leaves_and_root"]
    rp, ci, va, B = _inputs(c)
    xs = []
    for _ in range(2):
        S = ski.Solver()
        S.sketch(_csr_arg(rp, ci, va, c["n"], c["d"]), dev(B), m=c["m"], s=c["s"], seed=15,
                 qr_panel="sparse", tau_r=1e-10).factor()
        X, infos, rc = S.solve()
        xs.append(X.cpu().numpy().copy())
        S.close()
    np.testing.assert_array_equal(xs[0], xs[1])


def test_full_size_very_sparse_matches_the_dense_factor(ski):
    """The 40000 x 8000 very sparse workload: the ordering against the oracle's, and the
    sparse factorisation against the dense one on the same sketch.  Both preconditioners
    satisfy R^T R = P^T (SA)^T (SA) P, so A P R_sparse^-1 and A R_dense^-1 differ by an
    orthogonal factor and LSQR takes the same steps up to rounding (within max(2, 1%))."""
    c = workloads.CASES["very_sparse"]
    n, d, m, s = c["n"], c["d"], c["m"], c["s"]
    _say(f"full-size very sparse n={n} d={d} m={m} s={s}")
    rp, ci, va, b = workloads.very_sparse(n, d, c["per_col"], case=c["case"])
    A = sp.csr_matrix((va, ci, rp), shape=(n, d))
    seed = 2009
    out = {}
    for form in ("sparse", "auto"):
        S = ski.Solver()
        S.sketch(_csr_arg(rp, ci, va, n, d), dev(b), m=m, s=s, seed=seed, qr_panel=form,
                 tau_r=1e-12, tau_a=0.0).factor()
        if form == "sparse":
            perm, _ = S.get_pivots()
            st = S.factor_stats()
        X, infos, rc = S.solve()
        out[form] = (X[:, 0].cpu().numpy(), infos[0]["iters"], rc)
        S.close()
    pats = sq.sa_row_patterns(rp, ci, n, d, m, s, seed)
    order, root, L = sq.min_degree(pats, d, 62)
    perm_o, _ = sq.positions(order, root)
    np.testing.assert_array_equal(perm, perm_o)
    assert (st["leaf_fronts"], st["root"]) == (len(order), len(root))
    (xs, its, rcs), (xd, itd, rcd) = out["sparse"], out["auto"]
    err = np.linalg.norm(xs - xd) / np.linalg.norm(xd)
    r = b - A @ xs
    cert = np.linalg.norm(A.T @ r) / (sp.linalg.norm(A) * np.linalg.norm(r))
    _say(f"  leaves {len(order)} root {len(root)}; iters sparse {its} dense {itd}; "
         f"x difference {err:.2e}; certificate {cert:.2e}")
    assert rcs == 0 and rcd == 0
    # ~320 steps to 1e-12: the (TC-lsqr) estimate is not monotone near the threshold, and the
    # two forms' rounding (substitution against the explicit inverse) moves the crossing by a
    # few steps; within max(2, 1%)
    assert abs(its - itd) <= max(2, 0.01 * itd)
    assert err <= 1e-9
    assert cert <= 1e-10


def test_sparse_sketch_above_the_dense_row_limit(ski):
    """With the sparse factorisation the sketch may exceed the dense QR's 12288 rows: only the
    root front goes through the dense QR.  40000 x 8000 very sparse at gamma 3 (m 24000):
    the ordering equal to the oracle's, the certificate within 1e-10, and x equal to the
    gamma 1.4 solution (a different sketch, the same least-squares solution)."""
    c = workloads.CASES["very_sparse"]
    n, d, s = c["n"], c["d"], c["s"]
    rp, ci, va, b = workloads.very_sparse(n, d, c["per_col"], case=c["case"])
    A = sp.csr_matrix((va, ci, rp), shape=(n, d))
    xs = {}
    for m in (24000, c["m"]):
        _say(f"very sparse n={n} d={d} m={m}")
        S = ski.Solver()
        S.sketch(_csr_arg(rp, ci, va, n, d), dev(b), m=m, s=s, seed=2010, qr_panel="sparse",
                 tau_r=1e-13, tau_a=0.0).factor()
        if m == 24000:
            perm, _ = S.get_pivots()
            st = S.factor_stats()
        X, infos, rc = S.solve()
        xs[m] = (X[:, 0].cpu().numpy(), infos[0]["iters"])
        S.close()
        assert rc in (0, 1)
    pats = sq.sa_row_patterns(rp, ci, n, d, 24000, s, 2010)
    order, root, L = sq.min_degree(pats, d, 62)
    perm_o, _ = sq.positions(order, root)
    np.testing.assert_array_equal(perm, perm_o)
    assert st["root"] == len(root) and len(root) < d // 2
    x3, it3 = xs[24000]
    x1, it1 = xs[c["m"]]
    r = b - A @ x3
    cert = np.linalg.norm(A.T @ r) / (sp.linalg.norm(A) * np.linalg.norm(r))
    err = np.linalg.norm(x3 - x1) / np.linalg.norm(x1)
    _say(f"  root {len(root)}; iters gamma 3: {it3}, gamma 1.4: {it1}; certificate {cert:.2e}; "
         f"x difference {err:.2e}")
    assert cert <= 1e-10 and err <= 1e-9
    assert it3 < it1


def test_sparse_root_front_above_the_dense_limit_is_refused(ski):
    """100000 x 20000 very sparse at gamma 2: the root front has about 21800 rows, more than
    the dense QR takes; ski_factor refuses it with SKI_EINVAL before any numeric work."""
    n, d = 100000, 20000
    rp, ci, va, b = workloads.very_sparse(n, d, 2)
    S = ski.Solver()
    S.sketch(_csr_arg(rp, ci, va, n, d), dev(b), m=40000, s=2, seed=7, qr_panel="sparse")
    with pytest.raises(ski.SkiError) as e:
        S.factor()
    assert e.value.code == -1 and "root front" in str(e.value)
    S.close()


@pytest.mark.parametrize("kind", ["variant", "sample"])
def test_sparse_factor_with_the_other_sketches(ski, kind):
    """The sparse sketch and ordering under the s-hashing variant (Section 4; a row may land
    twice in one bucket with both signs) and under row sampling (Section 7): the sketch
    bit-exact, the ordering equal to the oracle's; with the variant, x against LAPACK."""
    n, d, per_col = 3000, 500, 2
    s, m = (3, 700) if kind == "variant" else (1, 1500)
    rp, ci, va, b = workloads.very_sparse(n, d, per_col)
    seed = 16
    ref = sk.sketch_csr(rp, ci, va, n, d, b, m, s, seed, kind=kind)
    S = ski.Solver()
    S.sketch(_csr_arg(rp, ci, va, n, d), dev(b), m=m, s=s, seed=seed, qr_panel="sparse",
             hash_kind=kind, tau_r=1e-14, tau_a=0.0, it_max=2000)
    np.testing.assert_array_equal(S.get_SA(), ref["SA_aug"])
    S.factor()
    pats = sq.sa_row_patterns(rp, ci, n, d, m, s, seed, kind=kind)
    order, root, L = sq.min_degree(pats, d, 62)
    perm_o, _ = sq.positions(order, root)
    perm, _ = S.get_pivots()
    np.testing.assert_array_equal(perm, perm_o)
    if kind == "variant":
        X, infos, rc = S.solve()
        A = sp.csr_matrix((va, ci, rp), shape=(n, d))
        xd = sla.lstsq(A.toarray(), b)[0]
        err = np.linalg.norm(X[:, 0].cpu().numpy() - xd) / np.linalg.norm(xd)
        _say(f"  variant: iters {infos[0]['iters']} x error {err:.2e}")
        assert err <= 1e-10
    S.close()


def test_sparse_eight_right_hand_sides(ski):
    """k = 8: fronts of at most 64 columns leave 55 for A (degree cap 55); every column's x
    within 1e-10 of LAPACK's."""
    n, d, per_col, s, m, k = 3000, 500, 2, 2, 700, 8
    rp, ci, va, _ = workloads.very_sparse(n, d, per_col)
    B = np.random.default_rng(8).standard_normal((n, k))
    S = ski.Solver()
    S.sketch(_csr_arg(rp, ci, va, n, d), dev(B), m=m, s=s, seed=17, qr_panel="sparse",
             tau_r=1e-14, tau_a=0.0, it_max=2000).factor()
    pats = sq.sa_row_patterns(rp, ci, n, d, m, s, 17)
    order, root, L = sq.min_degree(pats, d, 63 - k)
    perm, _ = S.get_pivots()
    np.testing.assert_array_equal(perm, sq.positions(order, root)[0])
    X, infos, rc = S.solve()
    S.close()
    A = sp.csr_matrix((va, ci, rp), shape=(n, d))
    Xd = sla.lstsq(A.toarray(), B)[0]
    X = X.cpu().numpy()
    for j in range(k):
        assert np.linalg.norm(X[:, j] - Xd[:, j]) <= 1e-10 * np.linalg.norm(Xd[:, j])


def test_sparse_handle_reused_across_sizes(ski):
    """One handle: a larger problem, a smaller one, the larger again (buffers grown once and
    reused, the structure rebuilt each time); each x within 1e-10 of LAPACK's and the
    second factor's R against the oracle."""
    big = CASES["leaves_root_k2"]
    small = CASES["leaves_only"]
    S = ski.Solver()
    for c in (big, small, big):
        n, d, s, m, k = c["n"], c["d"], c["s"], c["m"], c["k"]
        rp, ci, va, B = _inputs(c)
        S.sketch(_csr_arg(rp, ci, va, n, d), dev(B), m=m, s=s, seed=18, qr_panel="sparse",
                 tau_r=1e-14, tau_a=0.0, it_max=2000).factor()
        if c is small:
            ref = sk.sketch_csr(rp, ci, va, n, d, B, m, s, 18)
            pats = sq.sa_row_patterns(rp, ci, n, d, m, s, 18)
            order, root, L = sq.min_degree(pats, d, 63 - k)
            perm_o, _ = sq.positions(order, root)
            R, cc, _ = S.get_R()
            Rref, cref = sq.factor(ref["SA_aug"], d, perm_o)
            np.testing.assert_allclose(R, Rref, rtol=0, atol=1e-12 * np.abs(Rref).max() * math.sqrt(d))
        X, infos, rc = S.solve()
        A = sp.csr_matrix((va, ci, rp), shape=(n, d))
        Xd = sla.lstsq(A.toarray(), B)[0]
        X = X.cpu().numpy()
        for j in range(k):
            assert np.linalg.norm(X[:, j] - Xd[:, j]) <= 1e-10 * np.linalg.norm(Xd[:, j])
    S.close()


def test_sparse_rank_guard(ski):
    """rcond applies to the whole diagonal of the sparse factor, as without pivoting:
    |r_qq| < rcond |r_11| gives SKI_ERANK."""
    c = CASES["leaves_and_root"]
    rp, ci, va, B = _inputs(c)
    S = ski.Solver()
    S.sketch(_csr_arg(rp, ci, va, c["n"], c["d"]), dev(B), m=c["m"], s=c["s"], seed=19,
             qr_panel="sparse", rcond=0.9)
    with pytest.raises(ski.SkiError) as e:
        S.factor()
    assert e.value.code == -4
    S.close()


def _tall_front_matrix():
    """1000 x 20: rows 0-899 hold column 0 only, rows 900-999 three of the other columns.
    Column 0 then meets all 19 others yet is eliminated second, and its leaf front gathers
    377 rows of the sketch: the front is factored in three chunks of its LDS tile."""
    rng = np.random.default_rng(21)
    n, d = 1000, 20
    rows, cols, vals = [], [], []
    for i in range(900):
        rows.append(i)
        cols.append(0)
        vals.append(rng.standard_normal())
    for i in range(900, n):
        for c in rng.choice(np.arange(1, d), size=3, replace=False):
            rows.append(i)
            cols.append(int(c))
            vals.append(rng.standard_normal())
    A = sp.csr_matrix((vals, (rows, cols)), shape=(n, d))
    A.sort_indices()
    return A, rng.standard_normal(n)


@pytest.mark.parametrize("case", ["tall_front", "d1", "d2"])
def test_sparse_tall_fronts_and_tiny_problems(ski, case):
    if case == "tall_front":
        A, b = _tall_front_matrix()
        m, s = 400, 2
    else:
        d = 1 if case == "d1" else 2
        rng = np.random.default_rng(d)
        A = sp.csr_matrix(rng.standard_normal((50, d)))
        b = rng.standard_normal(50)
        m, s = 3 * d + 1, 2
    n, d = A.shape
    rp, ci, va = A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data
    _say(f"sparse {case}: n={n} d={d} m={m}")
    ref = sk.sketch_csr(rp, ci, va, n, d, b, m, s, 21)
    pats = sq.sa_row_patterns(rp, ci, n, d, m, s, 21)
    order, root, L = sq.min_degree(pats, d, 62)
    perm_o, pos = sq.positions(order, root)
    if case == "tall_front":
        q0 = int(pos[0])
        first = [min(int(pos[c]) for c in p) for p in pats if p]
        assert q0 < len(order) and sum(1 for f in first if f == q0) > 256
    S = ski.Solver()
    S.sketch(_csr_arg(rp, ci, va, n, d), dev(b), m=m, s=s, seed=21, qr_panel="sparse",
             tau_r=1e-14, tau_a=0.0, it_max=500).factor()
    np.testing.assert_array_equal(S.get_SA(), ref["SA_aug"])
    perm, _ = S.get_pivots()
    np.testing.assert_array_equal(perm, perm_o)
    R, cc, _ = S.get_R()
    Rref, cref = sq.factor(ref["SA_aug"], d, perm_o)
    scale = np.abs(Rref).max()
    np.testing.assert_allclose(R, Rref, rtol=0, atol=1e-12 * scale * math.sqrt(d))
    np.testing.assert_allclose(cc, cref, rtol=0, atol=1e-12 * np.abs(cref).max() * math.sqrt(d))
    X, infos, rc = S.solve()
    S.close()
    xd = sla.lstsq(A.toarray(), b)[0]
    x = X[:, 0].cpu().numpy()
    assert np.linalg.norm(x - xd) <= 1e-10 * np.linalg.norm(xd)
