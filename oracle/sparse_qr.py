"""Step 2 of Algorithm 1 in the sparse form of Section 6 (the sparse solver): a
sparse QR of the sketch, S A P = Q R with P a fill-reducing column ordering, and
the solve that uses it.

TEST INFRASTRUCTURE ONLY (see the package docstring).

What is computed, and from which definition
-------------------------------------------
* Pattern of SA.  For S = S_h (s-hashing, Section 2.2; no transform for sparse
  input, Section 6), entry (b, j) of SA is structurally present iff some stored
  A_ij has row i hashed to bucket b.  Each row of SA is one clique ("element") of
  the column graph of (SA)^T (SA).
* Column ordering.  The paper's sparse solver leaves the ordering to its sparse
  QR, set to a minimum-degree heuristic on that column graph (parameter
  `ordering`, Section 6).  The oracle takes the exact minimum-degree rule that
  such heuristics approximate: repeatedly eliminate an uneliminated column of
  smallest degree in the elimination graph (ties: smallest column index), and
  join its neighbours into a clique.  Elimination stops as soon as the smallest
  degree exceeds `dmax`; the columns left (the root) follow in increasing index.
  Positions: position q of the factorisation holds column perm[q].
* Structure of R.  Row q < L (an eliminated column) of R is structurally non-zero
  only at q and at the positions of the neighbours the column had when it was
  eliminated (R^T R = P^T (SA)^T (SA) P, so R is the Cholesky factor of that
  matrix up to row signs, whose structure the elimination graph gives).  The
  trailing root block is treated as dense.
* R itself: by definition the triangular factor of the Householder QR of the
  column-permuted sketch S [A P, B], with non-negative diagonal (lls.factor).
* The solve: Steps 3-5 on the permuted matrix A P with that R (lls), x = P x_P.
  Every division by r_ii follows the perturbed back-solve of lls.perturbed.
"""

import numpy as np

from . import lls
from . import sketch as sk


def sa_row_patterns(row_ptr, col, n, d, m, s, seed, kind="hash"):
    """Column lists (ascending) of the rows of S_h A for A in CSR form: row b of
    SA holds column j iff a stored A_ij has row i in bucket b.  kind "hash" or
    "variant" (the s-hashing variant, Section 4), or "sample" (row sampling, Section 7:
    row b of SA is the sampled row of A)."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    if kind == "sample":
        picked = sk.sample_rows(m, n, seed)
        return [sorted(int(c) for c in col[row_ptr[i]:row_ptr[i + 1]]) for i in picked]
    rows, neg = sk.hash_columns(n, m, s, seed, replace=(kind == "variant"))
    pats = [set() for _ in range(m)]
    for i in range(n):
        cols_i = col[row_ptr[i]:row_ptr[i + 1]]
        if len(cols_i) == 0:
            continue
        for b in rows[i]:
            pats[int(b)].update(int(c) for c in cols_i)
    return [sorted(p) for p in pats]


def min_degree(row_patterns, d, dmax):
    """Exact minimum-degree elimination on the column graph whose cliques are the
    given rows.  Returns (order, root, L): the eliminated columns in elimination
    order, the remaining columns in increasing index, and for each eliminated
    column j the sorted list L[j] of its neighbours at elimination."""
    adj = [set() for _ in range(d)]
    for r in row_patterns:
        for a in r:
            adj[a].update(r)
    for a in range(d):
        adj[a].discard(a)
    alive = set(range(d))
    order, L = [], {}
    while alive:
        j = min(alive, key=lambda v: (len(adj[v]), v))
        if len(adj[j]) > dmax:
            break
        nb = set(adj[j])
        order.append(j)
        L[j] = sorted(nb)
        alive.remove(j)
        for a in nb:
            adj[a].update(nb)
            adj[a].discard(a)
            adj[a].discard(j)
        adj[j] = set()
    return order, sorted(alive), L


def positions(order, root):
    """perm (position -> column) and its inverse pos (column -> position)."""
    perm = np.array(list(order) + list(root), dtype=np.int64)
    pos = np.empty_like(perm)
    pos[perm] = np.arange(len(perm))
    return perm, pos


def r_structure(order, root, L, d):
    """Boolean d x d structure of R in position space: the eliminated rows at
    their diagonal and their neighbours' positions, the root block dense upper."""
    perm, pos = positions(order, root)
    S = np.zeros((d, d), dtype=bool)
    for q, j in enumerate(order):
        S[q, q] = True
        for a in L[j]:
            S[q, pos[a]] = True
    nl = len(order)
    S[nl:, nl:] = np.triu(np.ones((d - nl, d - nl), dtype=bool))
    return S


def elimination_tree(order, root, L):
    """parent[q] for the eliminated positions q < L: the smallest position among
    the neighbours at elimination (-1 if none); positions >= L are the root."""
    perm, pos = positions(order, root)
    parent = np.full(len(order), -1, dtype=np.int64)
    for q, j in enumerate(order):
        if L[j]:
            parent[q] = min(int(pos[a]) for a in L[j])
    return parent


def factor(SA_aug, d, perm):
    """R (d x d, position space) and c of the QR of the column-permuted sketch
    S [A P, B], non-negative diagonal (lls.factor).

    A column of the sketch with no entry at all (a zero column of A) has degree 0,
    so the ordering puts it first among its ties and its front holds no row: its
    row and column of R are zero.  R of the other columns is then the QR of the
    sketch without it, in the same order (the factorisation of a matrix with a zero
    column is otherwise not unique)."""
    SA_aug = np.asarray(SA_aug, dtype=np.float64)
    perm = np.asarray(perm, dtype=np.int64)
    live = np.array([bool(np.any(SA_aug[:, j] != 0)) for j in perm], dtype=bool)
    q = np.nonzero(live)[0]
    cols = np.concatenate([perm[q], np.arange(d, SA_aug.shape[1])])
    Rq, cq, _ = lls.factor(SA_aug[:, cols], len(q))
    R = np.zeros((d, d))
    c = np.zeros((d, SA_aug.shape[1] - d))
    R[np.ix_(q, q)] = Rq
    c[q] = cq
    return R, c


def solve(A_csr, B, seed, m=None, gamma=1.4, s=2, dmax=62, tau_a=1e-8,
          tau_r=1e-6, it_max=10000, rcond_thres=1e-10, perturb=1e-10):
    """The sparse solver end to end for one or more right-hand sides: sketch,
    ordering, factor, Steps 3-5 on A P, x = P x_P.  Returns a dict with x
    (d x k), iters, status per column and the factor's pieces."""
    A = A_csr.tocsr()
    n, d = A.shape
    B = np.asarray(B, dtype=np.float64).reshape(n, -1)
    m = lls.sketch_size(gamma, d, m)
    skd = sk.sketch_csr(A.indptr, A.indices, A.data, n, d, B, m, s, seed)
    pats = sa_row_patterns(A.indptr, A.indices, n, d, m, s, seed)
    order, root, L = min_degree(pats, d, dmax)
    perm, pos = positions(order, root)
    R, c = factor(skd["SA_aug"], d, perm)
    Rp = lls.perturbed(R, rcond_thres, perturb)
    AP = A[:, perm]
    X = np.zeros((d, B.shape[1]))
    iters, status = [], []
    for t in range(B.shape[1]):
        x, rec = lls.solve_with_factor(AP, B[:, t], Rp, c[:, t], tau_a=tau_a, tau_r=tau_r,
                                       it_max=it_max)
        X[perm, t] = x
        iters.append(rec["iters"])
        status.append(rec["status"])
    return dict(x=X, iters=iters, status=status, R=R, c=c, perm=perm, order=order,
                root=root, L=L, SA_aug=skd["SA_aug"], patterns=pats, m=m)
