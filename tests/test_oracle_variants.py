"""Pins of the oracle's sketch variants (no GPU): the s-hashing variant (rows drawn with
replacement, Section 4) and row sampling after the transform (the sampled randomised
transform that Section 7 compares hashing against), and the paper's qualitative findings
on them (Section 7, numerical illustrations: hashing beats sampling on coherent input;
s > 1 is needed on semi-coherent sparse input)."""

import math

import numpy as np
import scipy.linalg as sla
from scipy.stats import chisquare

import workloads
from oracle import sketch as sk


def _dense_S(rows, neg, m):
    """S_h as a dense m x ncols matrix, entries added (so a repeated row adds twice)."""
    ncols, s = rows.shape
    S = np.zeros((m, ncols))
    for t in range(s):
        np.add.at(S, (rows[:, t], np.arange(ncols)), np.where(neg[:, t], -1.0, 1.0))
    return S / math.sqrt(s)


def test_variant_with_one_row_is_one_hashing():
    r1, n1 = sk.hash_columns(5000, 37, 1, seed=4)
    r2, n2 = sk.hash_columns(5000, 37, 1, seed=4, replace=True)
    np.testing.assert_array_equal(r1, r2)
    np.testing.assert_array_equal(n1, n2)


def test_variant_is_a_sum_of_one_hashing_matrices():
    # Lemma (decomposition of the variant): T = s^-1/2 (S1 + ... + Ss), Sk independent
    # 1-hashing matrices; here Sk takes word k of each column
    m, s, ncols = 6, 4, 3000
    rows, neg = sk.hash_columns(ncols, m, s, seed=9, replace=True)
    assert (rows[:, :, None] == rows[:, None, :]).sum(axis=(1, 2)).max() > s  # repeats exist
    T = _dense_S(rows, neg, m)
    parts = np.zeros_like(T)
    for t in range(s):
        St = np.zeros((m, ncols))
        St[rows[:, t], np.arange(ncols)] = np.where(neg[:, t], -1.0, 1.0)
        parts += St
    np.testing.assert_array_equal(T, parts / math.sqrt(s))
    # the CSR form holds the same matrix
    ptr, src, sg = sk.hash_csr(rows, neg, m)
    T2 = np.zeros((m, ncols))
    for b in range(m):
        for p in range(ptr[b], ptr[b + 1]):
            T2[b, src[p]] += -1.0 if sg[p] else 1.0
    np.testing.assert_array_equal(T2 / math.sqrt(s), T)
    # E ||T e_j||^2 = 1 and the rows are uniform
    col2 = (T * T).sum(axis=0)
    assert abs(col2.mean() - 1.0) < 0.05
    assert chisquare(np.bincount(rows.ravel(), minlength=m)).pvalue > 1e-3


def test_variant_sketch_equals_the_explicit_product():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((700, 9))
    b = rng.standard_normal(700)
    out = sk.sketch_dense(A, b, 20, 3, seed=5, kind="variant")
    n2 = out["npad"]
    H = np.array([[sk.hadamard_entry(n2, i, j) for j in range(n2)] for i in range(n2)])
    X = np.zeros((n2, 10))
    X[:700, :9] = A
    X[:700, 9] = b
    T = _dense_S(out["rows"], out["neg"], 20)
    ref = T @ (H @ (out["dsign"][:, None] * X))
    np.testing.assert_allclose(out["SA_aug"], ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_row_sampling_selects_rows_of_the_transformed_matrix():
    rng = np.random.default_rng(6)
    A = rng.standard_normal((900, 7))
    b = rng.standard_normal(900)
    m = 50
    out = sk.sketch_dense(A, b, m, 1, seed=8, kind="sample")
    n2 = out["npad"]
    X = np.zeros((n2, 8))
    X[:900, :7] = A
    X[:900, 7] = b
    X *= out["dsign"][:, None]
    sk.fwht_inplace(X)
    r = sk.sample_rows(m, n2, 8)
    np.testing.assert_array_equal(out["SA_aug"], X[r] * (1.0 / math.sqrt(n2)))
    big = sk.sample_rows(200000, 64, 3)
    assert chisquare(np.bincount(big, minlength=64)).pvalue > 1e-3
    # without the transform: rows of [A b] themselves
    out2 = sk.sketch_dense(A, b, m, 1, seed=8, hadamard=False, kind="sample")
    r2 = sk.sample_rows(m, 900, 8)
    np.testing.assert_array_equal(out2["SA_aug"][:, :7], A[r2])


def _kappa_AR(A, SA):
    R = np.linalg.qr(SA, mode="r")
    sv = np.linalg.svd(sla.solve_triangular(R, A.T, trans="T").T, compute_uv=False)
    return sv[0] / sv[-1]


def test_hashing_beats_sampling_on_coherent_input():
    # Section 7, first illustration: at equal m/d, hashing after the randomised transform
    # gives a far better preconditioner than sampling after it
    # (m/d = 2: sampling misses rows that the coherent block needs; m/d = 4: both work,
    # hashing still twice as well conditioned)
    A, b = workloads.coherent_dense(4000, 400)
    for ratio, gap in ((2, 1e6), (4, 1.5)):
        m = ratio * 400
        kh = _kappa_AR(A, sk.sketch_dense(A, b, m, 1, seed=11)["SA_aug"][:, :400])
        ks = _kappa_AR(A, sk.sketch_dense(A, b, m, 1, seed=11, kind="sample")["SA_aug"][:, :400])
        assert kh < 10.0 and ks > gap * kh, (ratio, kh, ks)


def test_s_above_one_is_needed_on_semicoherent_sparse_input():
    # Section 7, second illustration: 1-hashing fails on the semi-coherent sparse type,
    # 2- and 3-hashing give good preconditioners
    A, b = workloads.semico_sparse(4000, 400)
    m = 2 * 400
    k = {s: _kappa_AR(A, sk.sketch_dense(A, b, m, s, seed=13, hadamard=False)["SA_aug"][:, :400])
         for s in (1, 2, 3)}
    assert k[2] < 10 and k[3] < 10 and k[1] > 100 * k[2], k


def test_dht_is_the_hartley_transform():
    # the definition, entry by entry, on small orders; and F F = I for the normalised F
    rng = np.random.default_rng(21)
    for n in (1, 2, 8, 32):
        x = rng.standard_normal((n, 3))
        k = np.arange(n)
        C = np.cos(2 * np.pi * np.outer(k, k) / n) + np.sin(2 * np.pi * np.outer(k, k) / n)
        ref = C @ x
        got = sk.dht_inplace(x.copy())
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * max(1.0, np.abs(ref).max()))
    x = rng.standard_normal((1024, 2))
    np.testing.assert_allclose(sk.dht_inplace(sk.dht_inplace(x.copy())) / 1024, x, atol=1e-13)


def test_dht_sketch_equals_the_explicit_product():
    rng = np.random.default_rng(23)
    A = rng.standard_normal((200, 5))
    b = rng.standard_normal(200)
    out = sk.sketch_dense(A, b, 17, 2, seed=2, transform="dht")
    n2 = out["npad"]
    k = np.arange(n2)
    F = (np.cos(2 * np.pi * np.outer(k, k) / n2) + np.sin(2 * np.pi * np.outer(k, k) / n2)) / math.sqrt(n2)
    X = np.zeros((n2, 6))
    X[:200, :5] = A
    X[:200, 5] = b
    T = _dense_S(out["rows"], out["neg"], 17)
    ref = T @ (F @ (out["dsign"][:, None] * X))
    np.testing.assert_allclose(out["SA_aug"], ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_hashing_beats_sampling_with_the_hartley_transform():
    # the paper's own setting of the comparison (HR-DHT against SR-DHT)
    A, b = workloads.coherent_dense(4000, 400)
    m = 2 * 400
    kh = _kappa_AR(A, sk.sketch_dense(A, b, m, 1, seed=11, transform="dht")["SA_aug"][:, :400])
    ks = _kappa_AR(A, sk.sketch_dense(A, b, m, 1, seed=11, kind="sample",
                                      transform="dht")["SA_aug"][:, :400])
    assert kh < 10.0 and ks > 5 * kh, (kh, ks)
