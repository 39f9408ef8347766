"""Pins of the oracle's sparse form of Step 2 (Section 6: the sparse QR of the sketch
with a fill-reducing ordering, and the solve on the permuted matrix), no GPU.

What pins it, independently of the oracle's own code:
* hand-derived minimum-degree orders on a path, a star and a clique;
* at every step of the ordering, each remaining column's degree recomputed from
  scratch by the fill-path lemma (u and v are adjacent in the elimination graph
  iff the column graph has a path between them whose inner vertices are all
  eliminated) and the choice checked against it, the neighbour sets too;
* on trees, the ordering never fills (a leaf always has the least degree);
* the predicted structure of R against the non-zero pattern of numpy's Cholesky
  factor of P^T (SA)^T (SA) P, and R against that factor up to row signs;
* the solution against LAPACK's least-squares solver, with and without a root,
  and with a zero column of A (the perturbed back-solve of Section 6).
"""

import itertools

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

import workloads
from oracle import lls, sketch as sk, sparse_qr as sq


def _csr(n, d, per_col, case=9):
    rp, col, val, b = workloads.very_sparse(n, d, per_col, case=case)
    return sp.csr_matrix((val, col, rp), shape=(n, d)), b


def test_min_degree_hand_derived_orders():
    # path 0-1-2-3-4: an end has degree 1; each elimination exposes the next end
    order, root, L = sq.min_degree([[0, 1], [1, 2], [2, 3], [3, 4]], 5, 10)
    assert order == [0, 1, 2, 3, 4] and root == []
    assert [L[j] for j in order] == [[1], [2], [3], [4], []]
    # star with centre 0: leaves 1, 2, 3 first (degree 1); then the centre and leaf 4
    # both have degree 1 and the smaller index, the centre, goes first
    order, root, L = sq.min_degree([[0, 1], [0, 2], [0, 3], [0, 4]], 5, 10)
    assert order == [1, 2, 3, 0, 4]
    assert [L[j] for j in order] == [[0], [0], [0], [4], []]
    # one row holding three columns: a triangle, eliminated by index
    order, root, L = sq.min_degree([[0, 1, 2]], 3, 10)
    assert order == [0, 1, 2] and [L[j] for j in order] == [[1, 2], [2], []]
    # the cap: on the star every degree is >= 1, so dmax = 0 eliminates nothing
    order, root, L = sq.min_degree([[0, 1], [0, 2], [0, 3], [0, 4]], 5, 0)
    assert order == [] and root == [0, 1, 2, 3, 4]
    # an isolated column (no row) has degree 0 and goes first
    order, root, L = sq.min_degree([[1, 2]], 3, 10)
    assert order == [0, 1, 2] and L[0] == []


def _fill_path_neighbours(adj0, eliminated, v, alive):
    """Columns u != v adjacent to v after eliminating `eliminated`: a path from v to u
    whose inner vertices are all eliminated (breadth-first through them)."""
    seen, out, stack = {v}, set(), [v]
    while stack:
        x = stack.pop()
        for y in adj0[x]:
            if y in seen:
                continue
            seen.add(y)
            if y in eliminated:
                stack.append(y)
            elif y in alive:
                out.add(y)
    return out


def test_min_degree_against_fill_path_lemma():
    rng = np.random.default_rng(5)
    for trial in range(40):
        d = int(rng.integers(2, 10))
        nrows = int(rng.integers(1, 9))
        rows = [sorted(set(rng.integers(0, d, size=int(rng.integers(1, 4))).tolist()))
                for _ in range(nrows)]
        dmax = int(rng.integers(0, d + 1))
        order, root, L = sq.min_degree(rows, d, dmax)
        adj0 = [set() for _ in range(d)]
        for r in rows:
            for a, b in itertools.permutations(r, 2):
                adj0[a].add(b)
        elim, alive = set(), set(range(d))
        for j in order:
            deg = {v: len(_fill_path_neighbours(adj0, elim, v, alive)) for v in alive}
            best = min(alive, key=lambda v: (deg[v], v))
            assert j == best and deg[j] <= dmax
            assert L[j] == sorted(_fill_path_neighbours(adj0, elim, j, alive))
            elim.add(j)
            alive.remove(j)
        assert sorted(alive) == root
        if alive:
            deg = [len(_fill_path_neighbours(adj0, elim, v, alive)) for v in alive]
            assert min(deg) > dmax


def test_min_degree_never_fills_a_tree():
    rng = np.random.default_rng(11)
    for d in (2, 7, 30, 120):
        parent = [int(rng.integers(0, v)) for v in range(1, d)]
        edges = [[p, v] for v, p in zip(range(1, d), parent)]
        order, root, L = sq.min_degree(edges, d, d)
        assert root == [] and len(order) == d
        nb = {v: set() for v in range(d)}
        for a, b in edges:
            nb[a].add(b)
            nb[b].add(a)
        for j in order:
            assert len(L[j]) <= 1 and set(L[j]) <= nb[j]


def _sketch_csr(A, b, m, s, seed):
    A = A.tocsr()
    n, d = A.shape
    return sk.sketch_csr(A.indptr, A.indices, A.data, n, d, b, m, s, seed)["SA_aug"]


def test_structure_and_r_against_cholesky():
    for (n, d, per_col, s, dmax) in ((600, 120, 2, 2, 62), (600, 120, 3, 2, 8),
                                     (300, 60, 2, 2, 3)):
        A, b = _csr(n, d, per_col)
        m = lls.sketch_size(1.4, d)
        pats = sq.sa_row_patterns(A.indptr, A.indices, n, d, m, s, 7)
        SA = _sketch_csr(A, b, m, s, 7)
        # the pattern: exactly the structurally present entries of the sketch
        P = np.zeros((m, d), dtype=bool)
        for i, r in enumerate(pats):
            P[i, r] = True
        assert np.array_equal(P, SA[:, :d] != 0)
        order, root, L = sq.min_degree(pats, d, dmax)
        perm, pos = sq.positions(order, root)
        G = SA[:, perm].T @ SA[:, perm]
        C = np.linalg.cholesky(G).T  # upper, positive diagonal
        S = sq.r_structure(order, root, L, d)
        nl = len(order)
        tiny = 1e-13 * np.abs(C).max()
        assert np.all(np.abs(C[~S]) <= tiny)
        assert np.array_equal(np.abs(C[:nl]) > tiny, S[:nl])
        R, c = sq.factor(SA, d, perm)
        assert np.allclose(R, C, rtol=0, atol=1e-11 * np.abs(C).max())
        # the elimination tree: a parent is later than its child, and L[j] (minus the
        # parent) lies inside the parent's L (the clique passed up)
        parent = sq.elimination_tree(order, root, L)
        for q, j in enumerate(order):
            if parent[q] >= 0:
                assert parent[q] > q
                if parent[q] < nl:
                    jp = order[parent[q]]
                    assert set(L[j]) - {jp} <= set(L[jp])


def test_sparse_solve_matches_lapack():
    for (n, d, per_col, dmax) in ((2000, 300, 2, 62), (2000, 300, 3, 62), (1500, 200, 2, 4)):
        A, b = _csr(n, d, per_col)
        res = sq.solve(A, b, seed=3, dmax=dmax, tau_r=1e-12, tau_a=0.0)
        x = sla.lstsq(A.toarray(), b)[0]
        assert np.linalg.norm(res["x"][:, 0] - x) <= 1e-9 * np.linalg.norm(x)
        assert res["status"] == [lls.OK]
        if dmax == 4:
            assert len(res["root"]) > 0


def test_zero_column_gets_zero_row_and_x_zero():
    A, b = _csr(1500, 200, 2)
    A = A.tolil()
    A[:, 17] = 0.0
    A = A.tocsr()
    A.eliminate_zeros()
    res = sq.solve(A, b, seed=4, tau_r=1e-12, tau_a=0.0)
    pos17 = int(np.nonzero(res["perm"] == 17)[0][0])
    assert np.all(res["R"][pos17] == 0) and np.all(res["R"][:, pos17] == 0)
    assert res["x"][17, 0] == 0.0
    keep = np.arange(200) != 17
    x = sla.lstsq(A.toarray()[:, keep], b)[0]
    assert np.linalg.norm(res["x"][keep, 0] - x) <= 1e-9 * np.linalg.norm(x)


def test_patterns_of_the_other_sketches():
    # row sampling: each row of SA is one row of A, so the pattern is exactly the nonzeros;
    # the s-hashing variant: a row drawn twice into one bucket with both signs cancels, so
    # the pattern holds the nonzeros and, at most, such exact zeros
    n, d = 3000, 500
    A, b = _csr(n, d, 2)
    for kind, s, m in (("sample", 1, 1500), ("variant", 3, 700)):
        SA = sk.sketch_csr(A.indptr, A.indices, A.data, n, d, b, m, s, 16, kind=kind)["SA_aug"]
        pats = sq.sa_row_patterns(A.indptr, A.indices, n, d, m, s, 16, kind=kind)
        P = np.zeros((m, d), dtype=bool)
        for i, r in enumerate(pats):
            P[i, r] = True
        nz = SA[:, :d] != 0
        assert np.all(P >= nz)
        if kind == "sample":
            assert np.array_equal(P, nz)
        else:
            assert (P & ~nz).sum() <= 2
