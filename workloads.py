"""Seeded synthetic inputs shaped like the paper's test problems.

This module holds only input generation: none of the method's arithmetic.  The
tests, the smoke check and the benchmark draw their inputs from here, and the
same arrays are handed to the GPU library and to the CPU oracle.

Recipes (host numpy Generator(PCG64(1000 + case)) unless stated):

* tiny      4096 x 64 dense, A ~ N(0,1), x* ~ N(0,1), b = A x* + 1e-3 N(0,1);
            Hadamard, s = 1, m = 256.
* dense     50000 x 4000 dense, A ~ N(0,1) with rows 0 .. 0.2n-1 scaled by 1e3
            (a coherent block, standing in for the paper's dense test sets);
            b ~ N(0,1); Hadamard, s = 3, gamma = 1.7 (m = 6800).
* sparse    200000 x 5000 CSR: row lengths k in [1, 500] with P(k) ~ k^-1.6725
            (mean 10), distinct uniform columns per row (sorted), values
            N(0,1), plus 1e-6 added at (n-d+j, j) for full rank; b = 1 (the
            paper's rule for b); no Hadamard, s = 2, gamma = 1.5 (m = 7500).
            Stands in for the paper's sparse random test set, which used
            MATLAB's sprandn.
* illcond   50000 x 7000 dense A = U diag(sigma) V^T with sigma_i =
            10^(-8 i/(d-1)) and U, V from QR of Gaussian matrices; b = 1.
* batched   20000 x 1000 dense N(0,1) with 32 right-hand sides B ~ N(0,1) and
            a loss weight G ~ N(0,1) (d x 32).
* rankdef   50000 x 4000 dense of rank 3500: 3500 independent N(0,1) columns
            and 500 dependent ones, a third each of zero columns, exact copies
            of an independent column and combinations of three independent
            columns with N(0,1) weights, all shuffled; rows 0 .. 0.2n-1 scaled
            by 1e3 as in `dense`; b ~ N(0,1); Hadamard, s = 3, gamma = 1.7.
            Stands in for the paper's rank-deficient test matrices (Table 2),
            which come from the Florida collection.

* coherent  the paper's coherent dense type [I_d; 0] + 1e-8 J (J all ones),
            4000 x 400 in its sketch comparisons; b = 1.
* inco_sparse  a stand-in for MATLAB's sprandn(n, d, 0.01, 1e-6) (which is not
            available): 1% of the entries N(0,1) at uniform positions, plus one
            entry per column so that no column is empty, then columns scaled by
            10^(-6 j/(d-1)) for a condition number near 1e6.
* very_sparse  n x d CSR with a few stored entries per column (default 40000 x
            8000, 2 per column): column j holds row j and per_col - 1 further
            distinct uniform rows, values N(0,1); b ~ N(0,1); no Hadamard,
            s = 2, gamma = 1.4 (m = 11200).  Stands in for the very sparse
            matrices of the Florida collection on which the paper's sparse
            solver relies on a sparse QR of the sketch (such a sketch keeps a
            few entries per column, and its R stays sparse).
* semico_sparse  the paper's semi-coherent type [B 0; 0 I_{d/2}] + 1e-8 J with B
            an inco_sparse matrix of (n - d/2) x d/2 (the matrix of the paper's
            s = 1, 2, 3 comparison), as dense float64.

Every generator takes (n, d) so that the same recipe runs at test sizes.
"""

import numpy as np

CASES = {
    "tiny": dict(n=4096, d=64, s=1, m=256, hadamard=True, case=1),
    "dense": dict(n=50000, d=4000, s=3, gamma=1.7, m=6800, hadamard=True, case=2),
    "sparse": dict(n=200000, d=5000, s=2, gamma=1.5, m=7500, hadamard=False, case=3),
    "illcond": dict(n=50000, d=7000, s=3, gamma=1.7, m=11900, hadamard=True, case=4),
    "batched": dict(n=20000, d=1000, s=3, gamma=1.7, m=1700, hadamard=True, case=5, k=32),
    "rankdef": dict(n=50000, d=4000, rank=3500, s=3, gamma=1.7, m=6800, hadamard=True, case=6),
    "very_sparse": dict(n=40000, d=8000, s=2, gamma=1.4, m=11200, hadamard=False, case=9,
                        per_col=2),
}

POWER_LAW_ALPHA = 1.6725
MAX_ROW_NNZ = 500


def rng_for(case, salt=0):
    return np.random.Generator(np.random.PCG64(1000 + case + 7919 * salt))


def tiny(n=4096, d=64, case=1):
    rng = rng_for(case)
    A = rng.standard_normal((n, d))
    xstar = rng.standard_normal(d)
    b = A @ xstar + 1e-3 * rng.standard_normal(n)
    return A, b, xstar


def dense_coherent(n=50000, d=4000, case=2, frac=0.2, scale=1e3):
    rng = rng_for(case)
    A = rng.standard_normal((n, d))
    A[: int(frac * n)] *= scale
    b = rng.standard_normal(n)
    return A, b


def power_law_lengths(rng, n, alpha=POWER_LAW_ALPHA, kmax=MAX_ROW_NNZ, d=None):
    k = np.arange(1, kmax + 1)
    p = k ** (-alpha)
    p /= p.sum()
    lens = rng.choice(k, size=n, p=p)
    if d is not None:
        lens = np.minimum(lens, d)
    return lens


def sparse_power_law(n=200000, d=5000, case=3, identity_eps=1e-6):
    """CSR arrays (row_ptr int64, col int32, val float64) and b = 1."""
    rng = rng_for(case)
    lens = power_law_lengths(rng, n, d=d)
    row_of = np.repeat(np.arange(n, dtype=np.int64), lens)
    cols = rng.integers(0, d, size=row_of.size, dtype=np.int64)
    # redraw duplicate columns within a row until every row's columns are distinct
    while True:
        order = np.lexsort((cols, row_of))
        r_s, c_s = row_of[order], cols[order]
        dup = np.zeros(r_s.size, dtype=bool)
        dup[1:] = (r_s[1:] == r_s[:-1]) & (c_s[1:] == c_s[:-1])
        if not dup.any():
            row_of, cols = r_s, c_s
            break
        idx = order[dup]
        cols[idx] = rng.integers(0, d, size=idx.size, dtype=np.int64)
    vals = rng.standard_normal(row_of.size)
    # identity rows: + eps at (n - d + j, j), merged with any stored entry
    ir = np.arange(n - d, n, dtype=np.int64)
    ic = np.arange(d, dtype=np.int64)
    key = row_of * d + cols
    ikey = ir * d + ic
    hit = np.isin(key, ikey)
    vals[hit] += identity_eps
    have = np.isin(ikey, key)
    row_of = np.concatenate([row_of, ir[~have]])
    cols = np.concatenate([cols, ic[~have]])
    vals = np.concatenate([vals, np.full((~have).sum(), identity_eps)])
    order = np.lexsort((cols, row_of))
    row_of, cols, vals = row_of[order], cols[order], vals[order]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(row_of, minlength=n), out=row_ptr[1:])
    b = np.ones(n)
    return row_ptr, cols.astype(np.int32), vals, b


def illcond(n=50000, d=7000, case=4, decades=8.0, device="cpu"):
    """A = U diag(sigma) V^T, sigma geometric from 1 to 10^-decades; b = 1.

    Uses torch for the two orthonormal factors so that the full-size matrix
    can be generated on the accelerator; returns a torch tensor on `device`."""
    import torch
    g = torch.Generator(device="cpu")
    g.manual_seed(1000 + case)
    G1 = torch.randn(n, d, generator=g, dtype=torch.float64)
    G2 = torch.randn(d, d, generator=g, dtype=torch.float64)
    G1, G2 = G1.to(device), G2.to(device)
    U = torch.linalg.qr(G1, mode="reduced").Q
    V = torch.linalg.qr(G2, mode="reduced").Q
    sigma = 10.0 ** (-decades * torch.arange(d, dtype=torch.float64, device=device) / max(d - 1, 1))
    A = (U * sigma) @ V.T.contiguous()
    b = torch.ones(n, dtype=torch.float64, device=device)
    return A.contiguous(), b


def batched(n=20000, d=1000, k=32, case=5):
    rng = rng_for(case)
    A = rng.standard_normal((n, d))
    B = rng.standard_normal((n, k))
    G = rng.standard_normal((d, k))
    return A, B, G


def rank_deficient(n=50000, d=4000, rank=3500, case=6, frac=0.2, scale=1e3):
    """Dense A of rank `rank` (the recipe `rankdef` above) and b.

    Returns (A, b, independent) where `independent` lists the columns of A that
    are the independent Gaussian ones."""
    rng = rng_for(case)
    base = rng.standard_normal((n, rank))
    base[: int(frac * n)] *= scale
    ndep = d - rank
    nz = ndep // 3
    ncp = ndep // 3
    ncb = ndep - nz - ncp
    A = np.empty((n, d))
    A[:, :rank] = base
    A[:, rank:rank + nz] = 0.0
    A[:, rank + nz:rank + nz + ncp] = base[:, rng.integers(0, rank, ncp)]
    idx = rng.integers(0, rank, (ncb, 3))
    w = rng.standard_normal((ncb, 3))
    for j in range(ncb):
        A[:, rank + nz + ncp + j] = base[:, idx[j]] @ w[j]
    del base
    order = rng.permutation(d)
    A = np.ascontiguousarray(A[:, order])  # column j of A is column order[j] above
    b = rng.standard_normal(n)
    return A, b, np.flatnonzero(order < rank)


def coherent_dense(n=4000, d=400):
    """[I_d; 0] + 1e-8 J and b = 1."""
    A = np.full((n, d), 1e-8)
    A[np.arange(d), np.arange(d)] += 1.0
    return A, np.ones(n)


def inco_sparse(n=4000, d=400, case=7, density=0.01, decades=6.0):
    """Dense float64 form of the incoherent sparse stand-in (see the recipe)."""
    rng = rng_for(case)
    A = np.zeros((n, d))
    nnz = int(round(density * n * d))
    r = rng.integers(0, n, nnz)
    c = rng.integers(0, d, nnz)
    A[r, c] = rng.standard_normal(nnz)
    A[rng.integers(0, n, d), np.arange(d)] = rng.standard_normal(d)
    A *= 10.0 ** (-decades * np.arange(d) / max(d - 1, 1))
    return A


def semico_sparse(n=4000, d=400, case=8):
    """[B 0; 0 I_{d/2}] + 1e-8 J with B = inco_sparse((n - d/2), d/2); b = 1."""
    h = d // 2
    A = np.full((n, d), 1e-8)
    A[: n - h, :h] += inco_sparse(n - h, h, case=case)
    A[n - h + np.arange(h), h + np.arange(h)] += 1.0
    return A, np.ones(n)


def very_sparse(n=40000, d=8000, per_col=2, case=9):
    """CSR arrays (row_ptr int64, col int32, val float64) and b ~ N(0,1): column j
    holds row j and per_col - 1 further distinct rows drawn uniformly."""
    rng = rng_for(case)
    rows = np.empty((d, per_col), dtype=np.int64)
    rows[:, 0] = np.arange(d)
    if per_col > 1:
        rows[:, 1:] = rng.integers(0, n, size=(d, per_col - 1))
        # redraw any row that repeats within its column
        while True:
            srt = np.sort(rows, axis=1)
            bad = (srt[:, 1:] == srt[:, :-1]).any(axis=1)
            if not bad.any():
                break
            idx = np.nonzero(bad)[0]
            rows[idx, 1:] = rng.integers(0, n, size=(idx.size, per_col - 1))
    cols = np.repeat(np.arange(d, dtype=np.int64), per_col)
    row_of = rows.ravel()
    vals = rng.standard_normal(row_of.size)
    order = np.lexsort((cols, row_of))
    row_of, cols, vals = row_of[order], cols[order], vals[order]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(row_of, minlength=n), out=row_ptr[1:])
    b = rng.standard_normal(n)
    return row_ptr, cols.astype(np.int32), vals, b
