"""The host symbolic phase of the sparse QR of the sketch (Section 6, the sparse solver),
built with the host compiler and run on the CPU: no GPU needed.

Against the oracle (oracle/sparse_qr.py): the minimum-degree order and the root, the
structure of R and the elimination tree.  Against their definitions, written out here:
each sketch row's front and local columns, the fronts' row sources and sizes, the
contribution blocks and where their columns land in the parent, the factorisation levels,
the transposed lists of R^-T and the two solve schedules.  Also the error returns.
"""

import ctypes as C
import os
import shutil
import subprocess

import numpy as np
import pytest

import workloads
from oracle import lls
from oracle import sparse_qr as sq

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2105_11815_amd", "csrc")


@pytest.fixture(scope="module")
def sym(tmp_path_factory):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    out = str(tmp_path_factory.mktemp("sym") / "libsym.so")
    subprocess.run([cxx, "-O2", "-std=c++17", "-shared", "-fPIC", "-I", CSRC,
                    os.path.join(HERE, "symbolic_shim.cpp"),
                    os.path.join(CSRC, "sparse_symbolic.cpp"), "-o", out], check=True)
    lib = C.CDLL(out)
    P = C.c_void_p
    lib.sym_run.argtypes = [C.c_int64] * 3 + [P, P, P, C.c_int64, C.c_int, C.c_int]
    lib.sym_error.restype = C.c_char_p
    lib.sym_sizes.argtypes = [P]
    lib.sym_get.argtypes = [P] * 17
    lib.sym_sched.argtypes = [C.c_int, P, P, P, P]
    return lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def run(lib, pats, d, k=1, dmax=None, groups=16):
    """The symbolic phase on row patterns (sorted column lists); returns a dict of its
    arrays, or the error message."""
    dmax = 63 - k if dmax is None else dmax
    m = len(pats)
    rl = np.array([len(p) for p in pats], np.int32)
    rs = np.zeros(m, np.int64)
    if m > 1:
        rs[1:] = np.cumsum(rl)[:-1]
    col = np.concatenate([np.array(p, np.int32) for p in pats]) if rl.sum() else np.zeros(1, np.int32)
    nv = max(1, int(rl.sum()))
    if lib.sym_run(m, d, k, _ptr(rs), _ptr(rl), _ptr(col), nv, dmax, groups) != 0:
        return lib.sym_error().decode()
    sz = np.zeros(13, np.int64)
    lib.sym_sizes(_ptr(sz))
    nl, nnzl, nsrc, _, _, nlev, nt, nup, nlo, ngu, ngl, nlbu, nlbl = (int(x) for x in sz)
    a = dict(perm=np.zeros(d, np.int32), lptr=np.zeros(nl + 1, np.int64),
             lcol=np.zeros(max(nnzl, 1), np.int32), relmap=np.zeros(max(nnzl, 1), np.int32),
             parent=np.zeros(max(nl, 1), np.int32), nrows=np.zeros(nl + 1, np.int32),
             cbrows=np.zeros(max(nl, 1), np.int32), cboff=np.zeros(max(nl, 1), np.int64),
             src_ptr=np.zeros(nl + 2, np.int64), src_a=np.zeros(max(nsrc, 1), np.int32),
             src_b=np.zeros(max(nsrc, 1), np.int32), ent_lc=np.zeros(nv, np.int32),
             lev_ptr=np.zeros(max(nlev, 1), np.int64), lev_front=np.zeros(max(nl, 1), np.int32),
             tptr=np.zeros(d + 1, np.int64), trow=np.zeros(max(nt, 1), np.int32),
             tent=np.zeros(max(nt, 1), np.int64))
    keys = ["perm", "lptr", "lcol", "relmap", "parent", "nrows", "cbrows", "cboff", "src_ptr",
            "src_a", "src_b", "ent_lc", "lev_ptr", "lev_front", "tptr", "trow", "tent"]
    lib.sym_get(*[_ptr(a[x]) for x in keys])
    for name, n_rows, n_g, n_lb, up in (("up", nup, ngu, nlbu, 1), ("lo", nlo, ngl, nlbl, 0)):
        rows, gptr = np.zeros(max(n_rows, 1), np.int32), np.zeros(max(n_g, 1), np.int64)
        lbptr, lb = np.zeros(max(n_g, 1), np.int64), np.zeros(max(n_lb, 1), np.int64)
        lib.sym_sched(up, _ptr(rows), _ptr(gptr), _ptr(lbptr), _ptr(lb))
        a[name] = (rows[:n_rows], gptr[:n_g], lbptr[:n_g], lb[:n_lb])
    a.update(nl=nl, nnzl=nnzl, lcol=a["lcol"][:nnzl], relmap=a["relmap"][:nnzl],
             parent=a["parent"][:nl], cbrows=a["cbrows"][:nl], cboff=a["cboff"][:nl],
             src_a=a["src_a"][:nsrc], src_b=a["src_b"][:nsrc], lev_ptr=a["lev_ptr"][:nlev],
             lev_front=a["lev_front"][:nl], trow=a["trow"][:nt], tent=a["tent"][:nt],
             rs=rs, k=k)
    return a


def check_against_oracle(a, pats, d, dmax):
    """Order, root, R's structure and the elimination tree equal the oracle's."""
    order, root, L = sq.min_degree(pats, d, dmax)
    perm, pos = sq.positions(order, root)
    nl = a["nl"]
    assert nl == len(order)
    assert np.array_equal(a["perm"], np.asarray(perm))
    for q, j in enumerate(order):
        got = a["lcol"][a["lptr"][q]:a["lptr"][q + 1]]
        assert np.array_equal(got, np.sort([pos[u] for u in L[j]]).astype(np.int32))
    assert np.array_equal(a["parent"], np.asarray(sq.elimination_tree(order, root, L)))
    return pos


def check_structure(a, pats, d, pos):
    """The fronts' assembly data against their definitions."""
    nl, k = a["nl"], a["k"]
    ROOT = nl
    lptr, lcol = a["lptr"], a["lcol"]
    cols = [[q] + list(lcol[lptr[q]:lptr[q + 1]]) for q in range(nl)]  # local columns
    front_of = lambda p: -1 if p < 0 else (p if p < nl else ROOT)
    # each non-empty sketch row: its front is its first position's; local columns
    own = [[] for _ in range(nl + 1)]
    for r, p in enumerate(pats):
        if not p:
            continue
        ps = [pos[c] for c in p]
        f = min(ps) if min(ps) < nl else ROOT
        own[f].append(r)
        for u, c in enumerate(p):
            lc = pos[c] - nl if f == ROOT else cols[f].index(pos[c])
            assert a["ent_lc"][a["rs"][r] + u] == lc
    kids = [[] for _ in range(nl + 1)]
    for q in range(nl):
        pf = front_of(a["parent"][q])
        if pf >= 0:
            kids[pf].append(q)
    # sizes and contribution blocks, children before parents (children have lower positions)
    off = 0
    for q in range(nl + 1):
        rows = len(own[q]) + sum(int(a["cbrows"][c]) for c in kids[q])
        assert a["nrows"][q] == rows
        if q < nl:
            assert a["cbrows"][q] == max(0, min(rows, len(cols[q])) - 1)
            assert a["cboff"][q] == off
            off += int(a["cbrows"][q]) * (len(cols[q]) - 1 + k)
    # row sources: own rows ascending, then each child's contribution rows
    for q in range(nl + 1):
        want = [(r, -1) for r in own[q]] + [(c, t) for c in kids[q] for t in range(a["cbrows"][c])]
        s0, s1 = a["src_ptr"][q], a["src_ptr"][q + 1]
        assert list(zip(a["src_a"][s0:s1].tolist(), a["src_b"][s0:s1].tolist())) == want
    # where a child's columns land in its parent front
    for q in range(nl):
        pf = front_of(a["parent"][q])
        for e in range(lptr[q], lptr[q + 1]):
            want = lcol[e] - nl if pf == ROOT else (cols[pf].index(lcol[e]) if pf >= 0 else -1)
            assert a["relmap"][e] == want
    # levels: every leaf front once, each after its leaf children
    level = np.full(nl, -1)
    lp = a["lev_ptr"]
    for l in range(len(lp) - 1):
        for f in a["lev_front"][lp[l]:lp[l + 1]]:
            level[f] = l
    assert np.all(level >= 0) and sorted(a["lev_front"].tolist()) == list(range(nl))
    for q in range(nl):
        for c in kids[q]:
            assert level[c] < level[q]
    # transposed lists: for each position, the leaf rows holding it, ascending
    for p in range(d):
        t0, t1 = a["tptr"][p], a["tptr"][p + 1]
        want = [(f, e) for f in range(nl) for e in range(lptr[f], lptr[f + 1]) if lcol[e] == p]
        assert list(zip(a["trow"][t0:t1].tolist(), a["tent"][t0:t1].tolist())) == want
    # solve schedules: every leaf row once; within a group, by level, whole trees; a row's
    # leaf parent (R^-1, top-down) or leaf children (R^-T, bottom-up) come in earlier levels
    for name, before in (("up", lambda q: [a["parent"][q]] if 0 <= a["parent"][q] < nl else []),
                         ("lo", lambda q: kids[q] if q < nl else [])):
        rows, gptr, lbptr, lb = a[name]
        assert sorted(rows.tolist()) == list(range(nl))
        where = {}
        for g in range(len(gptr) - 1):
            bounds = lb[lbptr[g]:lbptr[g + 1]]
            assert bounds[0] == gptr[g] and bounds[-1] == gptr[g + 1]
            for li in range(len(bounds) - 1):
                for i in range(bounds[li], bounds[li + 1]):
                    where[int(rows[i])] = (g, li)
        for q in range(nl):
            for b in before(q):
                assert where[b][0] == where[q][0] and where[b][1] < where[q][1]


def test_random_patterns_against_oracle_and_definitions(sym):
    rng = np.random.default_rng(5)
    for trial in range(160):
        d = int(rng.integers(1, 40))
        m = int(rng.integers(1, 60))
        k = int(rng.integers(1, 4))
        pats = [sorted(set(rng.integers(0, d, size=int(rng.integers(0, 6))).tolist()))
                for _ in range(m)]
        dmax = 63 - k if trial % 3 else int(rng.integers(-1, 6))
        a = run(sym, pats, d, k, dmax, groups=int(rng.integers(1, 9)))
        assert isinstance(a, dict), a
        pos = check_against_oracle(a, pats, d, dmax)
        check_structure(a, pats, d, pos)


@pytest.mark.parametrize("n,d,per_col,s,m", [(2000, 300, 2, 3, 600), (3000, 400, 2, 2, 560),
                                             (2500, 200, 3, 1, 400)])
def test_sketch_patterns_of_very_sparse_matrices(sym, n, d, per_col, s, m):
    """The row patterns the sparse sketch gives for the very sparse workload's kind of
    matrix (the hashing of the oracle's sketch)."""
    rp, ci, _, _ = workloads.very_sparse(n, d, per_col)
    pats = sq.sa_row_patterns(rp, ci, n, d, m, s, 11)
    a = run(sym, pats, d, 1, 62, groups=64)
    pos = check_against_oracle(a, pats, d, 62)
    check_structure(a, pats, d, pos)


def test_errors(sym):
    assert "outside [0, d)" in run(sym, [[0, 1], [1, 5]], 4)
    assert "outside [0, d)" in run(sym, [[-1, 2]], 4)
    assert "1 <= k <= 32" in run(sym, [[0]], 2, k=33, dmax=0)
    assert "degree cap" in run(sym, [[0]], 2, k=1, dmax=63)
    assert "degree cap" in run(sym, [[0]], 2, k=1, dmax=-2)
