"""Steps 2-5 of Algorithm 1 (generic sketching algorithm) and the adjoint.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Steps
-----
2. Factor the sketch: S[A b] = Q [R c; 0 rho] by Householder QR without
   pivoting (the usual QR that the algorithm's factorisation remark allows for
   full-rank SA; V-hat = I, p = d).  The sign of diag(R) is normalised to be
   non-negative (a row sign flip of [R c] does not change x).
3. x_s = R^-1 c; terminate early if ||A x_s - b|| <= tau_a.
4. LSQR (Paige and Saunders, 1982) on W = A R^-1, started from y_0 = c, i.e.
   on the residual r_0 = b - A x_s, stopped by (TC-lsqr):
       ||W^T (W y_k - b)|| / (||W|| ||W y_k - b||) <= tau_r
   with the LSQR estimates of both norms and the running Frobenius estimate
   ||B_k||_F of ||W||.
5. x = R^-1 (c + delta).

Guards (Section 6): a rank check on diag(R), read as relative
(|r_qq| >= rcond |r_11|), and the perturbed back-solve: when the diagonal
ratio max|r_ii| / min|r_ii| reaches 1/rcond_thres, every division by r_ii
becomes a division by r_ii + copysign(perturb, r_ii).

The adjoint solves (A^T A) Z = G by conjugate gradients on the preconditioned
normal equations R^-T A^T A R^-1 (R Z) = R^-T G with the same R.  With the
residual r = B - A X and the loss sum(X * G), the gradients are
grad_B = A Z and grad_A = r Z^T - (A Z) X^T.

Rank-deficient input (Step 2 in the form S A V-hat = Q R, Section 6, parameter
rcond): a column-pivoted QR of SA, truncated to its leading p x p block R11.
The oracle pivots greedily (LAPACK's xGEQP3, largest remaining column norm
first) in place of the randomised pivoting of R-CPQR; both choose a valid
column set, and the quantities that parity compares (p, the residual, and the
solution on a given column set) do not depend on which.  V_1 holds the first
p pivots J, so x_s = V_1 R11^-1 Q_1^T S b, W = A V_1 R11^-1 = A_J R11^-1 and
x = V_1 R11^-1 y vanishes outside J.

Minimal-norm form (cod=True): the complete orthogonal decomposition with R_12 = 0
that the factorisation remark lists and the minimal-norm guarantee of Section 5 (the
theorem on the minimal Euclidean norm solution) needs.
The truncated rows Rtop = [R11 R12] of the pivoted QR are factored as Rtop^T = Y L;
then S A = Q_1 L^T V_1^T with V_1 = Pi Y orthonormal, and Algorithm 1 runs with
P = V_1 L^-T.  range(P) = range((SA)^T) = range(A^T) under an embedding, so the LSQR
solution is the minimal-norm least-squares solution.
"""

import math

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

# status codes shared in meaning (not in code) with the C interface
OK, WNOCONV, WEARLY, EINVAL, ERANK = 0, 1, 2, -1, -4


def factor(SA_aug, d):
    """Householder QR of the m x (d+k) sketch; returns (R d x d, c d x k, rho)."""
    R_aug = np.linalg.qr(SA_aug, mode="r")
    sgn = np.sign(np.diag(R_aug[:d, :d])).copy()
    sgn[sgn == 0] = 1.0
    R = sgn[:, None] * R_aug[:d, :d]
    c = sgn[:, None] * R_aug[:d, d:]
    rho = None
    if R_aug.shape[0] > d:
        rho = np.linalg.norm(R_aug[d:, d:], axis=0)
    return np.triu(R), c, rho


def rank_ok(R, rcond):
    dg = np.abs(np.diag(R))
    return bool(dg.size == 0 or (dg[0] > 0 and np.all(dg >= rcond * dg[0])))


def rank_count(R, rcond):
    """p = the number of leading diagonal entries with |r_qq| >= rcond |r_11|.

    Reading of Section 6 (parameter rcond): the threshold is taken relative to
    |r_11|, and R11 ends at the first diagonal entry below it, so that R11 is
    never ill-conditioned by a small pivot in its middle.  Greedy pivoting
    gives a non-increasing |diag(R)|, where this is the largest such q."""
    dg = np.abs(np.diag(R))
    if dg.size == 0 or not dg[0] > 0:
        return 0
    bad = np.flatnonzero(~(dg >= rcond * dg[0]))
    return int(bad[0]) if bad.size else int(dg.size)


def factor_pivoted(SA_aug, d, rcond):
    """Step 2 with column pivoting: S A P = Q R, truncated to R11 (p x p).

    Returns (R11, c = (Q_1^T S b) p x k, perm d, p, diag(R) of the full
    factorisation).  perm[:p] are the columns that V_1 selects.  Signs are
    normalised so that diag(R11) >= 0."""
    SA = np.asarray(SA_aug[:, :d], dtype=np.float64)
    SB = np.asarray(SA_aug[:, d:], dtype=np.float64)
    Q, R, perm = sla.qr(SA, mode="economic", pivoting=True)
    p = rank_count(R, rcond)
    sgn = np.sign(np.diag(R)[:p]).copy()
    sgn[sgn == 0] = 1.0
    R11 = np.triu(sgn[:, None] * R[:p, :p])
    c = sgn[:, None] * (Q[:, :p].T @ SB)
    return R11, c, np.asarray(perm, dtype=np.int64), p, np.diag(R).copy()


def solve_pivoted_with_factor(A, b, R11, c, J, tau_a=1e-8, tau_r=1e-6, it_max=10000):
    """Steps 3-5 with V_1 = the columns J: LSQR on W = A_J R11^-1.

    Returns x (d, zero outside J) and the record of the one right-hand side."""
    d = A.shape[1]
    x = np.zeros(d)
    if len(J) == 0:
        r = np.asarray(b, dtype=np.float64)
        return x, dict(iters=0, status=OK, rnorm=float(np.linalg.norm(r)), arnorm=0.0,
                       anorm=0.0, tc=0.0, xs=x.copy())
    AJ = A[:, J]
    xJ, rec = solve_with_factor(AJ, b, R11, c, tau_a, tau_r, it_max)
    x[J] = xJ
    xs = np.zeros(d)
    xs[J] = rec["xs"]
    rec["xs"] = xs
    return x, rec


def factor_cod(SA_aug, d, rcond):
    """Step 2 as a complete orthogonal decomposition (the factorisation remark allows it;
    R_12 = 0 is what the minimal-norm guarantee needs).

    The column-pivoted QR S A Pi = Q R is truncated at p (as in factor_pivoted); its top
    rows Rtop = [R11 R12] (p x d, full row rank) are factored as Rtop^T = Y L (a QR of the
    d x p matrix, L upper triangular).  Then S A = Q_1 L^T (Pi Y)^T: V_1 = Pi Y has
    orthonormal columns, the p x p factor is L^T and R_12 = 0.

    Returns (L, V1 d x p, c = (Q_1^T S b) p x k, perm, p)."""
    SA = np.asarray(SA_aug[:, :d], dtype=np.float64)
    SB = np.asarray(SA_aug[:, d:], dtype=np.float64)
    Q, R, perm = sla.qr(SA, mode="economic", pivoting=True)
    p = rank_count(R, rcond)
    c = Q[:, :p].T @ SB
    if p == 0:
        return np.zeros((0, 0)), np.zeros((d, 0)), c, np.asarray(perm, dtype=np.int64), 0
    Y, L = np.linalg.qr(R[:p, :].T, mode="reduced")
    V1 = np.zeros((d, p))
    V1[np.asarray(perm)] = Y
    return L, V1, c, np.asarray(perm, dtype=np.int64), p


def solve_cod_with_factor(A, b, L, V1, c, tau_a=1e-8, tau_r=1e-6, it_max=10000):
    """Steps 3-5 of Algorithm 1 with V_1 and R_11 = L^T from factor_cod:
    P = V_1 L^-T, x_s = P c, LSQR on W = A P from y_0 = c, x = P (c + delta)."""
    d = A.shape[1]
    p = L.shape[0]
    if p == 0:
        r = np.asarray(b, dtype=np.float64)
        return np.zeros(d), dict(iters=0, status=OK, rnorm=float(np.linalg.norm(r)),
                                 arnorm=0.0, anorm=0.0, tc=0.0, xs=np.zeros(d))
    Pm = lambda y: V1 @ sla.solve_triangular(L, y, lower=False, trans="T")   # V_1 L^-T y
    PTm = lambda g: sla.solve_triangular(L, V1.T @ g, lower=False)          # L^-1 V_1^T g
    xs = Pm(c)
    r0 = b - A @ xs
    if np.linalg.norm(r0) <= tau_a:
        return xs, dict(iters=0, status=WEARLY, rnorm=float(np.linalg.norm(r0)), arnorm=0.0,
                        anorm=0.0, tc=0.0, xs=xs)
    delta, rec = lsqr_op(A, Pm, PTm, p, r0, tau_r, it_max)
    x = Pm(c + delta)
    rec["status"] = OK if rec["converged"] else WNOCONV
    rec["xs"] = xs
    return x, rec


def perturbed(R, rcond_thres, perturb):
    """R with its diagonal moved away from zero when it looks singular."""
    dg = np.abs(np.diag(R))
    if perturb > 0 and dg.size and (dg.min() == 0 or dg.max() / dg.min() >= 1.0 / rcond_thres):
        R = R.copy()
        i = np.arange(R.shape[0])
        R[i, i] = R[i, i] + np.copysign(perturb, R[i, i])
    return R


def _matvecs(A):
    if sp.issparse(A):
        A = A.tocsr()
        AT = A.T.tocsr()
        return (lambda z: A @ z), (lambda u: AT @ u)
    return (lambda z: A @ z), (lambda u: A.T @ u)


def lsqr_precond(A, R, r0, tau_r, it_max):
    """LSQR on min ||W delta - r0||, W = A R^-1.  Returns delta and a record."""
    Rs = lambda v: sla.solve_triangular(R, v, lower=False)           # R^-1 v
    RTs = lambda g: sla.solve_triangular(R, g, lower=False, trans="T")  # R^-T g
    return lsqr_op(A, Rs, RTs, R.shape[0], r0, tau_r, it_max)


def lsqr_op(A, Rs, RTs, d, r0, tau_r, it_max):
    """LSQR (Paige and Saunders) on min ||W delta - r0|| with W = A P, P given by its
    products Rs(v) = P v and RTs(g) = P^T g (P is d_A x d).  Returns delta (length d)."""
    Amul, ATmul = _matvecs(A)
    delta = np.zeros(d)
    beta = float(np.linalg.norm(r0))
    rec = dict(iters=0, rnorm=beta, arnorm=0.0, anorm=0.0, tc=0.0, converged=True)
    if beta == 0.0:
        return delta, rec
    u = r0 / beta
    v = RTs(ATmul(u))
    alpha = float(np.linalg.norm(v))
    if alpha == 0.0:
        return delta, rec
    v = v / alpha
    h = v.copy()
    phibar, rhobar, anorm2 = beta, alpha, 0.0
    rec["converged"] = False
    for it in range(1, it_max + 1):
        # bidiagonalisation: beta u = W v - alpha u ; alpha v = W^T u - beta v
        u = Amul(Rs(v)) - alpha * u
        beta = float(np.linalg.norm(u))
        if beta > 0.0:
            u = u / beta
        anorm2 += alpha * alpha + beta * beta
        v = RTs(ATmul(u)) - beta * v
        alpha = float(np.linalg.norm(v))
        if alpha > 0.0:
            v = v / alpha
        # plane rotation eliminating the subdiagonal beta
        rho = math.sqrt(rhobar * rhobar + beta * beta)
        cs, sn = rhobar / rho, beta / rho
        theta = sn * alpha
        rhobar = -cs * alpha
        phi = cs * phibar
        phibar = sn * phibar
        delta = delta + (phi / rho) * h
        h = v - (theta / rho) * h
        rnorm = phibar
        arnorm = phibar * alpha * abs(cs)
        anorm = math.sqrt(anorm2)
        tc = arnorm / (anorm * rnorm) if rnorm > 0 and anorm > 0 else 0.0
        rec.update(iters=it, rnorm=rnorm, arnorm=arnorm, anorm=anorm, tc=tc)
        if rnorm == 0.0 or arnorm == 0.0 or tc <= tau_r:
            rec["converged"] = True
            break
    return delta, rec


def solve_with_factor(A, b, R, c, tau_a=1e-8, tau_r=1e-6, it_max=10000):
    """Steps 3-5 for one right-hand side, given R and c = (Q^T S b)[:d]."""
    xs = sla.solve_triangular(R, c, lower=False)
    r0 = b - A @ xs
    if np.linalg.norm(r0) <= tau_a:
        return xs, dict(iters=0, status=WEARLY, rnorm=float(np.linalg.norm(r0)),
                        arnorm=0.0, anorm=0.0, tc=0.0, xs=xs)
    delta, rec = lsqr_precond(A, R, r0, tau_r, it_max)
    x = sla.solve_triangular(R, c + delta, lower=False)
    rec["status"] = OK if rec["converged"] else WNOCONV
    rec["xs"] = xs
    return x, rec


def default_params(sparse):
    """Defaults of Section 6 (dense: gamma 1.7, s 1; sparse: gamma 1.4, s 2)."""
    if sparse:
        return dict(gamma=1.4, s=2, hadamard=False, tau_a=1e-8, tau_r=1e-6,
                    it_max=10000, rcond=0.0, rcond_thres=1e-10, perturb=1e-10)
    return dict(gamma=1.7, s=1, hadamard=True, tau_a=1e-8, tau_r=1e-6,
                it_max=10000, rcond=1e-12, rcond_thres=1e-10, perturb=0.0)


def sketch_size(gamma, d, m=None):
    return int(m) if m else int(math.ceil(gamma * d - 1e-9))


def solve(A, B, seed, sparse=None, **kw):
    """Algorithm 1 end to end (dense or scipy CSR A, B n x k).

    Returns (X d x k, info dict)."""
    from . import sketch as sk
    if sparse is None:
        sparse = sp.issparse(A)
    p = default_params(sparse)
    p.update(kw)
    n, d = A.shape
    B2 = np.asarray(B, dtype=np.float64).reshape(n, -1)
    m = sketch_size(p["gamma"], d, p.get("m"))
    if n < d or m < d or p["s"] > m:
        return None, dict(status=EINVAL)
    if sparse:
        Ac = A.tocsr()
        out = sk.sketch_csr(Ac.indptr, Ac.indices, Ac.data, n, d, B2, m, p["s"], seed,
                            kind=p.get("hash_kind", "hash"))
    else:
        out = sk.sketch_dense(A, B2, m, p["s"], seed, hadamard=p["hadamard"],
                              kind=p.get("hash_kind", "hash"),
                              transform=p.get("transform", "wht"))
    X = np.zeros((d, B2.shape[1]))
    recs = []
    extra = {}
    if p.get("cod"):
        L, V1, c, perm, rank = factor_cod(out["SA_aug"], d, p["rcond"])
        R = L
        extra = dict(perm=perm, p=rank, V1=V1)
        for j in range(B2.shape[1]):
            X[:, j], rec = solve_cod_with_factor(A, B2[:, j], L, V1, c[:, j], p["tau_a"],
                                                 p["tau_r"], p["it_max"])
            recs.append(rec)
    elif p.get("pivoting"):
        R, c, perm, rank, dg = factor_pivoted(out["SA_aug"], d, p["rcond"])
        R = perturbed(R, p["rcond_thres"], p["perturb"])
        J = perm[:rank]
        extra = dict(perm=perm, p=rank, J=J, diag_full=dg)
        for j in range(B2.shape[1]):
            X[:, j], rec = solve_pivoted_with_factor(A, B2[:, j], R, c[:, j], J, p["tau_a"],
                                                     p["tau_r"], p["it_max"])
            recs.append(rec)
    else:
        R, c, _ = factor(out["SA_aug"], d)
        if p["rcond"] > 0 and not rank_ok(R, p["rcond"]):
            return None, dict(status=ERANK, R=R, sketch=out)
        R = perturbed(R, p["rcond_thres"], p["perturb"])
        for j in range(B2.shape[1]):
            X[:, j], rec = solve_with_factor(A, B2[:, j], R, c[:, j], p["tau_a"],
                                             p["tau_r"], p["it_max"])
            recs.append(rec)
    if any(r["status"] == WNOCONV for r in recs):
        status = WNOCONV
    elif all(r["status"] == WEARLY for r in recs):
        status = WEARLY
    else:
        status = OK
    return X, dict(status=status, R=R, c=c, m=m, records=recs, sketch=out, **extra)


def lstsq_direct(A, B):
    """The plain definition: x* = argmin ||A x - b|| by Householder QR of A."""
    A = A.toarray() if sp.issparse(A) else np.asarray(A, dtype=np.float64)
    Q, R = np.linalg.qr(A, mode="reduced")
    return sla.solve_triangular(R, Q.T @ B, lower=False)


def basic_solution(A, b, J):
    """The plain definition on a column set J: x_J = argmin ||A_J z - b|| (A_J of full
    column rank), x = 0 outside J, by Householder QR of A_J."""
    A = A.toarray() if sp.issparse(A) else np.asarray(A, dtype=np.float64)
    x = np.zeros(A.shape[1])
    J = np.asarray(J, dtype=np.int64)
    if J.size:
        x[J] = lstsq_direct(A[:, J], b)
    return x


def normal_solve_pcg(A, R, G, tol=1e-12, it_max=1000):
    """Z = (A^T A)^-1 G by CG on R^-T A^T A R^-1 y = R^-T g, z = R^-1 y."""
    Amul, ATmul = _matvecs(A)
    G = np.asarray(G, dtype=np.float64).reshape(R.shape[0], -1)
    Z = np.zeros_like(G)
    iters = []
    for j in range(G.shape[1]):
        Mop = lambda y: sla.solve_triangular(
            R, ATmul(Amul(sla.solve_triangular(R, y, lower=False))), lower=False, trans="T")
        rhs = sla.solve_triangular(R, G[:, j], lower=False, trans="T")
        y = np.zeros_like(rhs)
        r = rhs.copy()
        pdir = r.copy()
        rr = float(r @ r)
        stop = (tol * float(np.linalg.norm(rhs))) ** 2
        it = 0
        while it < it_max and rr > stop:
            q = Mop(pdir)
            a = rr / float(pdir @ q)
            y = y + a * pdir
            r = r - a * q
            rr_new = float(r @ r)
            pdir = r + (rr_new / rr) * pdir
            rr = rr_new
            it += 1
        Z[:, j] = sla.solve_triangular(R, y, lower=False)
        iters.append(it)
    return Z, iters


def grads_from_Z(A, X, B, Z):
    """grad_A = (B - A X) Z^T - (A Z) X^T and grad_B = A Z for loss sum(X * G)."""
    A = np.asarray(A, dtype=np.float64)
    AZ = A @ Z
    return (B - A @ X) @ Z.T - AZ @ X.T, AZ


def grads_closed_form(A, X, B, G):
    """Reference gradient from a dense QR of A: Z = R_A^-1 R_A^-T G."""
    A = np.asarray(A, dtype=np.float64)
    RA = np.linalg.qr(A, mode="r")
    Z = sla.solve_triangular(RA, sla.solve_triangular(RA, G, lower=False, trans="T"), lower=False)
    gA, gB = grads_from_Z(A, X, B, Z)
    return gA, gB, Z
