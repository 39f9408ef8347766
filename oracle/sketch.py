"""Sketching step of Algorithm 1 (Step 1): S [A B] for dense and sparse A.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Definitions followed
--------------------
* s-hashing matrix (Section 2.2, Definition of s-hashing): independently for
  every column j, s rows are drawn uniformly WITHOUT replacement from [m] and
  the entries there are +-1/sqrt(s) with independent fair signs.
* HRHT (Section 4.3, Definition of the Hashed-Randomised-Hadamard-Transform):
  S = S_h H D with D a random +-1 diagonal, H the normalised Walsh-Hadamard
  matrix H_ij = n^-1/2 (-1)^<(i-1)_2, (j-1)_2>, and S_h independent of D.
* HR-DHT (Section 6, the paper's dense software): S = S_h F D with F the
  normalised discrete Hartley transform, F_kj = n^-1/2 cas(2 pi k j / n),
  cas = cos + sin, applied here to the zero-padded n' rows like H; it is
  computed through the discrete Fourier transform (DHT = Re - Im of the DFT).
* Sparse input (Section 6, sparse variant): S is an s-hashing matrix alone.
* Step 1 of Algorithm 1 sketches b with the same S (the augmented column).
* s-hashing variant (Section 4, Definition of the s-hashing variant): the s
  rows of a column are drawn WITH replacement; a row drawn twice receives both
  +-1/sqrt(s) contributions.
* Row sampling (Section 7, the sampled transform of Blendenpik that the paper
  compares against): every sketch row is one row of H D [A b] (or of [A b]
  without H), drawn uniformly with replacement, with value 1.

Readings of the paper taken here (each also listed in the design notes):
* H needs a power-of-two order, so the rows are zero-padded to
  n' = 2^ceil(log2 n); the padded rows are hashed too, since H makes them
  nonzero.  HD is orthogonal, so the least-squares solution is unchanged.
* The random bits come from Philox4x64-10 with key (seed, 0):
  - hash of column j: blocks at counter (j, blk, 0, 0), blk = 0, 1, ...,
    words taken in order; a word w proposes row floor((w >> 32) * m / 2^32)
    (multiply-shift on the high half) with sign -1 iff bit 0 of w is set; a
    proposal equal to a row already taken for this column is rejected; the
    column stops at s accepted rows.
  - sign d_i of D: bit (i mod 64) of word ((i >> 6) mod 4) of the block at
    counter (i >> 8, 0, 1, 0); d_i = -1 iff that bit is set.
  - hash of column j in the variant: the same words, none rejected: the column
    takes the rows of its first s words.
  - sampled row of sketch row i: word 0 of the block at counter (i, 0, 2, 0),
    row floor((w >> 32) * n / 2^32) over the n rows sampled from (n' with H).
* The scalars of H and S_h are applied once, at the end, as the single FP64
  factor 1 / sqrt(n' * s) (dense) or 1 / sqrt(s) (sparse); for row sampling
  1 / sqrt(n') (H's normalisation) or 1.
* The Walsh-Hadamard transform is applied by butterflies (x, y) -> (x+y, x-y)
  over row-index bit 0, then bit 1, and so on; the bucket sums run over the
  bucket's columns in ascending order, starting from +0.0.  Fixing both orders
  makes the sketch reproducible to the last bit.  A row that a column of the
  variant drew twice is added twice, the positive entry before the negative.
"""

import math

import numpy as np

from .philox import philox4x64_10

_MASK32 = np.uint64(0xFFFFFFFF)


def next_pow2(n):
    """Smallest power of two >= n (n >= 1)."""
    p = 1
    while p < n:
        p *= 2
    return p


def hash_columns(ncols, m, s, seed, replace=False):
    """Rows and sign bits of an s-hashing matrix with m rows and ncols columns
    (with replace=True, of the s-hashing variant).

    Returns (rows, neg): int64 [ncols, s] rows in the order they were accepted
    and bool [ncols, s], True where the entry is negative."""
    if not (1 <= s <= m):
        raise ValueError("need 1 <= s <= m")
    if replace:
        rows = np.empty((ncols, s), dtype=np.int64)
        neg = np.empty((ncols, s), dtype=bool)
        j = np.arange(ncols, dtype=np.uint64)
        mm = np.uint64(m)
        for t in range(s):
            w = philox4x64_10(j, np.uint64(t // 4), 0, 0, np.uint64(seed), 0)[t % 4]
            rows[:, t] = (((w >> np.uint64(32)) * mm) >> np.uint64(32)).astype(np.int64)
            neg[:, t] = (w & np.uint64(1)) == 1
        return rows, neg
    rows = np.full((ncols, s), -1, dtype=np.int64)
    neg = np.zeros((ncols, s), dtype=bool)
    count = np.zeros(ncols, dtype=np.int64)
    active = np.arange(ncols, dtype=np.int64)
    blk = 0
    mm = np.uint64(m)
    while active.size:
        words = philox4x64_10(active.astype(np.uint64), np.uint64(blk), 0, 0,
                              np.uint64(seed), 0)
        for w in words:
            need = count[active] < s
            cand = (((w >> np.uint64(32)) * mm) >> np.uint64(32)).astype(np.int64)
            dup = (rows[active] == cand[:, None]).any(axis=1)
            take = need & ~dup
            cols = active[take]
            slot = count[cols]
            rows[cols, slot] = cand[take]
            neg[cols, slot] = (w[take] & np.uint64(1)) == 1
            count[cols] += 1
        active = active[count[active] < s]
        blk += 1
    return rows, neg


def sample_rows(m, nrows, seed):
    """The row of [A b] (or of H D [A b]) that each of the m sketch rows samples."""
    i = np.arange(m, dtype=np.uint64)
    w = philox4x64_10(i, 0, np.uint64(2), 0, np.uint64(seed), 0)[0]
    return (((w >> np.uint64(32)) * np.uint64(nrows)) >> np.uint64(32)).astype(np.int64)


def d_signs(nrows, seed):
    """The +-1 diagonal of D, as float64 of length nrows."""
    i = np.arange(nrows, dtype=np.int64)
    q = (i >> 8).astype(np.uint64)
    words = np.stack(philox4x64_10(q, 0, np.uint64(1), 0, np.uint64(seed), 0))
    w = words[(i >> 6) & 3, np.arange(nrows)]
    bit = (w >> (i & 63).astype(np.uint64)) & np.uint64(1)
    return np.where(bit == 1, -1.0, 1.0)


def hash_csr(rows, neg, m):
    """Bucket-sorted form of the hashing matrix: for each sketch row (bucket) b,
    the columns j with S_h[b, j] != 0, ascending, and their sign bits.

    Returns (bucket_ptr int64[m+1], src int64[ncols*s], neg bool[ncols*s]).
    Inside a bucket the entries ascend by column, then sign bit (a row that a
    column of the variant drew twice)."""
    ncols, s = rows.shape
    b = rows.reshape(-1)
    j = np.repeat(np.arange(ncols, dtype=np.int64), s)
    sg = neg.reshape(-1)
    order = np.lexsort((sg, j, b))
    counts = np.bincount(b, minlength=m)
    ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=ptr[1:])
    return ptr, j[order], sg[order]


def fwht_inplace(X):
    """Unnormalised Walsh-Hadamard transform along axis 0 (length a power of
    two), by butterflies over row-index bit 0, then bit 1, ..."""
    n = X.shape[0]
    h = 1
    while h < n:
        V = X.reshape(n // (2 * h), 2, h, -1)
        x = V[:, 0].copy()
        y = V[:, 1]
        V[:, 0] = x + y
        V[:, 1] = x - y
        h *= 2
    return X


def dht_inplace(X):
    """Unnormalised discrete Hartley transform along axis 0: X_k = sum_j x_j cas(2 pi k j / n),
    computed as Re - Im of the discrete Fourier transform (numpy's FFT)."""
    F = np.fft.fft(X, axis=0)
    X[...] = F.real - F.imag
    return X


def bucket_sum(ptr, src, neg, rows_of):
    """out[b] = sum over the bucket's entries, ascending, of +-rows_of(src).

    rows_of(idx) returns the dense rows for the index array idx.  The sum is
    taken entry by entry in bucket order, starting from +0.0."""
    m = ptr.size - 1
    lens = np.diff(ptr)
    width = rows_of(np.zeros(0, dtype=np.int64)).shape[1]
    acc = np.zeros((m, width))
    for t in range(int(lens.max()) if m else 0):
        b = np.nonzero(lens > t)[0]
        p = ptr[b] + t
        r = rows_of(src[p])
        acc[b] = np.where(neg[p][:, None], acc[b] - r, acc[b] + r)
    return acc


def _sketch_structure(nrows, m, s, seed, kind):
    """(rows, neg, bucket_ptr, src, src_neg) of S_h for kind "hash", "variant" or
    "sample" (rows/neg are per column of S_h; for sampling, the sampled rows)."""
    if kind == "sample":
        r = sample_rows(m, nrows, seed)
        ptr = np.arange(m + 1, dtype=np.int64)
        return r, np.zeros(m, dtype=bool), ptr, r.copy(), np.zeros(m, dtype=bool)
    rows, neg = hash_columns(nrows, m, s, seed, replace=(kind == "variant"))
    ptr, src, sg = hash_csr(rows, neg, m)
    return rows, neg, ptr, src, sg


def sketch_dense(A, B, m, s, seed, hadamard=True, kind="hash", transform="wht"):
    """S [A B] for dense A (n x d) and B (n x k), S = S_h H D (or S_h alone).

    kind: "hash" (s-hashing), "variant" (the s-hashing variant) or "sample"
    (row sampling, s ignored).  transform (with hadamard=True): "wht" (the
    Walsh-Hadamard H) or "dht" (the Hartley F).  Returns dict with SA_aug
    (m x (d+k)), and the hashing/sign arrays."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64).reshape(A.shape[0], -1)
    n, d = A.shape
    if hadamard:
        npad = next_pow2(n)
        X = np.zeros((npad, d + B.shape[1]))
        X[:n, :d] = A
        X[:n, d:] = B
        D = d_signs(npad, seed)
        X *= D[:, None]
        if transform == "dht":
            dht_inplace(X)
        else:
            fwht_inplace(X)
        scale = 1.0 / math.sqrt(float(npad * (1 if kind == "sample" else s)))
    else:
        npad = n
        X = np.concatenate([A, B], axis=1)
        D = None
        scale = 1.0 if kind == "sample" else 1.0 / math.sqrt(float(s))
    rows, neg, ptr, src, sg = _sketch_structure(npad, m, s, seed, kind)
    SA = bucket_sum(ptr, src, sg, lambda idx: X[idx]) * scale
    return dict(SA_aug=SA, rows=rows, neg=neg, bucket_ptr=ptr, src=src,
                src_neg=sg, dsign=D, npad=npad, scale=scale)


def sketch_csr(row_ptr, col, val, n, d, B, m, s, seed, kind="hash"):
    """S [A B] for sparse A in CSR form (no Hadamard; Section 6, sparse input).

    Only the stored entries are added, in bucket order; adding an absent
    (zero) entry would leave the sum unchanged."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    val = np.asarray(val, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64).reshape(n, -1)
    k = B.shape[1]
    rows, neg, ptr, src, sg = _sketch_structure(n, m, s, seed, kind)
    lens = np.diff(ptr)
    acc = np.zeros((m, d + k))
    for t in range(int(lens.max()) if m else 0):
        b = np.nonzero(lens > t)[0]
        p = ptr[b] + t
        i = src[p]
        sgn = np.where(sg[p], -1.0, 1.0)
        nnz_i = row_ptr[i + 1] - row_ptr[i]
        bb = np.repeat(b, nnz_i)
        ss = np.repeat(sgn, nnz_i)
        starts = np.repeat(row_ptr[i], nnz_i)
        offs = np.arange(nnz_i.sum()) - np.repeat(np.cumsum(nnz_i) - nnz_i, nnz_i)
        e = starts + offs
        cc = col[e]
        vv = val[e]
        cur = acc[bb, cc]
        acc[bb, cc] = np.where(ss < 0, cur - vv, cur + vv)
        cur = acc[b, d:]
        acc[b, d:] = np.where(sg[p][:, None], cur - B[i], cur + B[i])
    scale = 1.0 if kind == "sample" else 1.0 / math.sqrt(float(s))
    return dict(SA_aug=acc * scale, rows=rows, neg=neg, bucket_ptr=ptr,
                src=src, src_neg=sg, dsign=None, npad=n, scale=scale)


def hadamard_entry(n, i, j):
    """H_ij of the definition (0-based i, j): n^-1/2 (-1)^popcount(i & j)."""
    return (-1.0) ** bin(i & j).count("1") / math.sqrt(n)
