"""Pins of the oracle's random bits and sketch against what the paper and the
mathematics fix (no GPU)."""

import math
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from oracle import philox, sketch as sk

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _kat():
    out = []
    for line in open(os.path.join(GOLD, "philox4x64_10_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        lhs, rhs = line.split("->")
        ins = [int(x, 16) for x in lhs.split()]
        outs = [int(x, 16) for x in rhs.split()]
        out.append((ins, outs))
    return out


def test_mulhilo_against_python_ints():
    rng = np.random.default_rng(0)
    a = rng.integers(0, 2**63, size=200, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    b = rng.integers(0, 2**63, size=200, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    with np.errstate(over="ignore"):
        hi, lo = philox.mulhilo64(a, b)
    for x, y, h, l in zip(a, b, hi, lo):
        p = int(x) * int(y)
        assert int(h) == p >> 64 and int(l) == p & (2**64 - 1)


def test_philox_known_answers():
    for ins, outs in _kat():
        got = philox.philox4x64_10(*[np.uint64(v) for v in ins])
        assert [int(g) for g in got] == outs


def test_philox_matches_numpy_library():
    # numpy advances its counter once before producing a block
    for seed, ctr in [(12345, (5, 7, 0, 0)), (2**64 - 3, (0, 0, 1, 0)), (7, (2**64 - 1, 3, 0, 9))]:
        bg = np.random.Philox(key=np.array([seed, 0], dtype=np.uint64),
                              counter=np.array(ctr, dtype=np.uint64))
        ref = bg.random_raw(4)
        nxt = list(ctr)
        nxt[0] = (nxt[0] + 1) % 2**64
        if nxt[0] == 0:
            nxt[1] += 1
        got = philox.philox4x64_10(*[np.uint64(v) for v in nxt], np.uint64(seed), np.uint64(0))
        assert [int(g) for g in got] == [int(r) for r in ref]


@pytest.mark.parametrize("ncols,m,s", [(4096, 256, 1), (3000, 97, 3), (500, 5, 5), (1000, 7, 2)])
def test_hash_structure(ncols, m, s):
    rows, neg = sk.hash_columns(ncols, m, s, seed=42)
    assert rows.shape == (ncols, s)
    assert rows.min() >= 0 and rows.max() < m
    # s distinct rows per column (sampling without replacement)
    srt = np.sort(rows, axis=1)
    assert np.all(np.diff(srt, axis=1) > 0)
    # explicit S: entries +-1/sqrt(s), exactly s per column, diag(S^T S) = 1
    S = np.zeros((m, ncols))
    S[rows, np.arange(ncols)[:, None]] = np.where(neg, -1.0, 1.0) / math.sqrt(s)
    assert np.all((S != 0).sum(axis=0) == s)
    np.testing.assert_allclose(np.einsum("ij,ij->j", S, S), 1.0, rtol=1e-15)
    ptr, src, sg = sk.hash_csr(rows, neg, m)
    assert ptr[-1] == ncols * s and np.all(np.diff(ptr) >= 0)
    for b in range(min(m, 50)):
        seg = src[ptr[b]:ptr[b + 1]]
        assert np.all(np.diff(seg) > 0)
        assert np.all(np.any(rows[seg] == b, axis=1))


def test_hash_uniform_and_fair_signs():
    ncols, m, s = 200000, 50, 2
    rows, neg = sk.hash_columns(ncols, m, s, seed=7)
    counts = np.bincount(rows.reshape(-1), minlength=m)
    expect = ncols * s / m
    chi2 = ((counts - expect) ** 2 / expect).sum()
    from scipy.stats import chi2 as chi2dist
    assert chi2dist.sf(chi2, m - 1) > 1e-3
    frac = neg.mean()
    assert abs(frac - 0.5) < 4 * math.sqrt(0.25 / neg.size)
    D = sk.d_signs(1 << 16, seed=7)
    assert set(np.unique(D)) == {-1.0, 1.0}
    assert abs(D.mean()) < 4 / math.sqrt(D.size)


def _example1_cases():
    out = []
    for line in open(os.path.join(GOLD, "hashing_example1.txt")):
        if line.startswith("#") or not line.strip():
            continue
        out.append(tuple(int(x) for x in line.split()))
    return out


@pytest.mark.parametrize("r,m,trials", _example1_cases())
def test_example1_rank_probability(r, m, trials):
    p = np.prod([1 - k / m for k in range(1, r)])
    assert p <= math.exp(-r * (r - 1) / (2 * m)) + 1e-15
    hits = 0
    for seed in range(trials):
        rows, _ = sk.hash_columns(r, m, 1, seed=seed + 1)
        A = np.zeros((m, r))
        A[rows[:, 0], np.arange(r)] = 1.0
        hits += np.linalg.matrix_rank(A) == r
    sd = math.sqrt(p * (1 - p) / trials)
    assert abs(hits / trials - p) < 4 * sd


def test_fwht_matches_definition_and_library():
    for n in [1, 2, 4, 8, 64, 256]:
        Hdef = np.array([[sk.hadamard_entry(n, i, j) for j in range(n)] for i in range(n)])
        np.testing.assert_array_equal(Hdef, sla.hadamard(n) / math.sqrt(n))
        X = np.eye(n)
        sk.fwht_inplace(X)
        np.testing.assert_allclose(X / math.sqrt(n), Hdef, rtol=0, atol=1e-15)
    n = 1024
    rng = np.random.default_rng(1)
    x = rng.standard_normal((n, 3))
    y = sk.fwht_inplace(x.copy()) / math.sqrt(n)
    np.testing.assert_allclose(np.linalg.norm(y, axis=0), np.linalg.norm(x, axis=0), rtol=1e-14)
    z = sk.fwht_inplace(y.copy()) / math.sqrt(n)
    np.testing.assert_allclose(z, x, rtol=0, atol=1e-13)


def _tropp_cases():
    out = []
    for line in open(os.path.join(GOLD, "tropp_lemma.txt")):
        if line.startswith("#") or not line.strip():
            continue
        n, r, dl = line.split()
        out.append((int(n), int(r), float(dl)))
    return out


@pytest.mark.parametrize("n,r,delta1", _tropp_cases())
def test_coherence_after_hadamard(n, r, delta1):
    U = np.zeros((n, r))
    U[np.arange(r), np.arange(r)] = 1.0
    bound = math.sqrt(r / n) + math.sqrt(8 * math.log(n / delta1) / n)
    for seed in range(5):
        X = U * sk.d_signs(n, seed)[:, None]
        sk.fwht_inplace(X)
        X /= math.sqrt(n)
        mu = np.linalg.norm(X, axis=1).max()
        assert mu <= bound


@pytest.mark.parametrize("n,d,k,m,s", [(1000, 20, 1, 40, 3), (513, 7, 2, 16, 1), (64, 4, 1, 8, 2)])
def test_sketch_dense_equals_explicit_product(n, d, k, m, s):
    rng = np.random.default_rng(n)
    A = rng.standard_normal((n, d))
    B = rng.standard_normal((n, k))
    out = sk.sketch_dense(A, B, m, s, seed=99)
    npad = out["npad"]
    assert npad == sk.next_pow2(n) and npad >= n
    H = sla.hadamard(npad) / math.sqrt(npad)
    D = np.diag(out["dsign"])
    S_h = np.zeros((m, npad))
    S_h[out["rows"], np.arange(npad)[:, None]] = np.where(out["neg"], -1.0, 1.0) / math.sqrt(s)
    X = np.zeros((npad, d + k))
    X[:n] = np.concatenate([A, B], axis=1)
    ref = S_h @ (H @ (D @ X))
    np.testing.assert_allclose(out["SA_aug"], ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def test_sketch_preserves_norm_in_expectation():
    n, m, s = 256, 32, 2
    rng = np.random.default_rng(3)
    x = rng.standard_normal((n, 1))
    vals = [np.linalg.norm(sk.sketch_dense(x[:, :0], x, m, s, seed=t)["SA_aug"]) ** 2
            for t in range(400)]
    # E||Sx||^2 = ||x||^2; the spread of a hashing sketch is O(||x||^2 / sqrt(m))
    assert abs(np.mean(vals) / np.linalg.norm(x) ** 2 - 1) < 0.05


@pytest.mark.parametrize("n,d,m,s", [(300, 12, 30, 2), (1000, 40, 60, 1)])
def test_sketch_csr_equals_explicit_product(n, d, m, s):
    rng = np.random.default_rng(d)
    A = sp.random(n, d, density=0.1, random_state=rng, format="csr")
    b = rng.standard_normal(n)
    out = sk.sketch_csr(A.indptr, A.indices, A.data, n, d, b, m, s, seed=5)
    S_h = np.zeros((m, n))
    S_h[out["rows"], np.arange(n)[:, None]] = np.where(out["neg"], -1.0, 1.0) / math.sqrt(s)
    ref = S_h @ np.concatenate([A.toarray(), b[:, None]], axis=1)
    np.testing.assert_allclose(out["SA_aug"], ref, rtol=1e-13, atol=1e-13)
