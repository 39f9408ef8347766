/*
 * ski.h -- C interface of the MI355X (gfx950) sketch-and-precondition solver for
 * overdetermined linear least squares  min_x ||A x - b||_2  (A n x d, n >= d).
 *
 * Method: Cartis, Fiala and Shao, "Hashing embeddings of optimal dimension, with
 * applications to linear least squares", Algorithm 1 (generic sketching
 * algorithm) with the dense and sparse variants of Section 6:
 *   ski_sketch  -- Step 1: S [A B], with S = S_h H D for dense A (Definition of
 *                  HRHT, Section 4.3; Walsh-Hadamard H, rows zero-padded to a
 *                  power of two n') and S = S_h for sparse A; S_h is an s-hashing
 *                  matrix (Definition of s-hashing, Section 2.2).
 *   ski_factor  -- Step 2: Householder QR of the m x (d+k) sketch (no pivoting,
 *                  V-hat = I, p = d), giving R and c = (Q^T S B)[0:d].
 *   ski_solve   -- Steps 3-5: x_s = R^-1 c and the early exit on tau_a, LSQR on
 *                  W = A R^-1 stopped by (TC-lsqr) with tau_r, x = R^-1 y.
 *                  With op = SKI_OP_NORMAL it solves (A^T A) Z = G instead, by
 *                  conjugate gradients preconditioned with the same R (the adjoint
 *                  used for differentiation; not in the paper).
 *   ski_gradients -- grad_B = A Z and grad_A = (B - A X) Z^T - (A Z) X^T for the
 *                  loss sum(X .* G) once Z = (A^T A)^-1 G is known.
 *
 * Conventions
 *   - All matrix/vector arguments of ski_sketch/ski_solve/ski_gradients are DEVICE
 *     pointers; dense matrices are row-major with an explicit leading dimension
 *     (element (i, j) of an n x d matrix at p[i * ld + j]).
 *   - `stream` is a hipStream_t (passed as void*); every call is ordered on it.
 *     ski_sketch is asynchronous for dense A; for CSR A it waits once for a device check
 *     of the CSR structure, and with qr_panel = SKI_QR_SPARSE once more, to size the
 *     sparse sketch from its entry count.  ski_factor synchronises the stream before it returns
 *     (it reads diag(R) for the rank guard and the perturbation, and the device's checks
 *     of the sketch; with qr_panel = SKI_QR_PIVOTED it also waits once per 64-column panel
 *     for that panel's CholeskyQR2 check).  ski_solve returns after LSQR (or CG) has
 *     stopped: it polls a status word in mapped host memory once per iteration, one
 *     iteration behind the device.  The getters synchronise the device.
 *   - Return value: 0 (SKI_OK) on success, > 0 a warning, < 0 an error; the
 *     message of the last error is available from ski_last_error.  No C++
 *     exception crosses this interface.
 *   - A handle may be used from one host thread and one stream at a time.
 */
#ifndef SKI_H
#define SKI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ski_handle_s* ski_handle;

enum ski_status {
    SKI_OK = 0,
    SKI_WNOCONV = 1,   /* it_max reached before (TC-lsqr) held; X holds the last iterate */
    SKI_WEARLY = 2,    /* Step 3 terminated early: ||A x_s - b|| <= tau_a, X = x_s       */
    SKI_EINVAL = -1,   /* invalid argument (sizes, leading dimensions, NULL pointers), or
                          a non-finite entry in A, B or G (see ski_factor, ski_solve)       */
    SKI_ENOMEM = -2,   /* device allocation failed                                         */
    SKI_EDEVICE = -3,  /* a HIP call failed                                                */
    SKI_ERANK = -4,    /* rank guard: some |r_qq| < rcond |r_11| (A looks rank deficient)  */
    SKI_ESTATE = -5    /* calls out of order (e.g. ski_factor before ski_sketch)           */
};

enum ski_kind { SKI_DENSE = 0, SKI_DENSE_COLMAJOR = 1, SKI_CSR = 2 };
enum ski_prec { SKI_FP64 = 0, SKI_FP32 = 1, SKI_BF16 = 2 };
enum ski_op { SKI_OP_LLS = 0, SKI_OP_NORMAL = 1 };
enum ski_hash_kind { SKI_HASH = 0, SKI_HASH_VARIANT = 1, SKI_SAMPLE_ROWS = 2 };
enum ski_qr_panel {
    SKI_QR_AUTO = 0,
    SKI_QR_HOUSEHOLDER = 1,
    SKI_QR_PIVOTED = 2,
    SKI_QR_PIVOTED_HOUSEHOLDER = 3,
    SKI_QR_PIVOTED_COD = 4,
    SKI_QR_SPARSE = 5
};

/* The data matrix.  Dense: `a` (n x d, row-major, leading dimension lda >= d).
 * Dense column-major (SKI_DENSE_COLMAJOR): entry (i, j) at a[j lda + i], lda >= n;
 * ski_sketch transposes it once, in stream order, into a row-major copy that the handle
 * owns (n d doubles, kept until the next ski_sketch or ski_destroy), and every later call
 * reads the copy, so this A may change or be freed once ski_sketch's work on the stream is
 * done; gradients with respect to A are returned row-major as for SKI_DENSE.
 * CSR: row_ptr[n+1] (int64, row_ptr[0] = 0), col[nnz] (int32 in [0, d), distinct
 * within a row), val[nnz].  For SKI_DENSE and SKI_CSR the caller owns the arrays and must
 * keep them alive and unmodified from ski_sketch until the last ski_solve/ski_gradients
 * call on the handle: LSQR streams A directly, the handle keeps pointers, not copies. */
typedef struct {
    int64_t n, d;
    int32_t kind;
    const double* a;
    int64_t lda;
    const int64_t* row_ptr;
    const int32_t* col;
    const double* val;
    int64_t nnz;
} ski_matrix;

/* Parameters (defaults of Section 6 from ski_params_default).
 *   gamma, m     sketch rows m = ceil(gamma d) unless m > 0 is given; d <= m <= 12288
 *                (the column-by-column Householder panel, which every QR falls back to,
 *                keeps a column's m entries in the registers of one 512-thread workgroup,
 *                24 per thread).  With qr_panel = SKI_QR_SPARSE any m >= d is taken, and
 *                the limit of 12288 applies to the rows of the dense root front instead
 *                (ski_factor returns SKI_EINVAL above it).
 *   s            nonzeros per column of S_h, 1 <= s <= min(m, 32).
 *   hadamard     1: S = S_h H D (dense only); 0: S = S_h; 2: S = S_h F D with F the
 *                discrete Hartley transform of the paper's dense software (Section 6,
 *                HR-DHT), on the zero-padded n' rows; needs n' <= 2^24 and FP64 sketch
 *                and QR; computed through the DFT, so it matches a reference to rounding.
 *   seed         Philox4x64-10 key (seed, 0) for S_h and D.
 *   sketch_prec  arithmetic of H D A and of the hashing sums, and the type of the
 *                transform's intermediate (FP64; FP32; BF16 storage with FP32 arithmetic).
 *                The sketch is stored in the type the QR reads: FP64 when qr_prec = FP64
 *                (which makes the sketch FP64 whatever sketch_prec says), FP32 otherwise
 *                (an FP64 sketch is then rounded once, when it is written).
 *   qr_prec      arithmetic of the QR of the sketch (FP64/FP32/BF16 MFMA inputs,
 *                FP32 accumulation for BF16); R is always used in FP64.
 *   tau_a        early exit when ||A x_s - b|| <= tau_a (absolute).
 *   tau_r        (TC-lsqr) tolerance.
 *   it_max       LSQR iteration limit.
 *   rcond        rank guard |r_qq| >= rcond |r_11| (0 disables); failure -> SKI_ERANK.
 *   rcond_thres, perturb  if max|r_ii|/min|r_ii| >= 1/rcond_thres and perturb > 0,
 *                every division by r_ii becomes a division by r_ii + copysign(perturb, r_ii).
 *   qr_panel     how each 64-column panel of the Householder QR is factored:
 *                SKI_QR_AUTO (default): CholeskyQR2 of the panel, with the Householder
 *                vectors reconstructed from its orthonormal factor; if any panel is too
 *                ill-conditioned for that (checked on the device), the whole factorisation
 *                is repeated with the column-by-column panel.  SKI_QR_HOUSEHOLDER: the
 *                column-by-column panel only.  Both give the same R up to rounding.
 *                SKI_QR_PIVOTED: the rank-revealing form of Step 2, S A V-hat = Q R with
 *                V-hat a column permutation (Section 6: randomised column-pivoted QR,
 *                parameter rcond).  Each panel's 64 pivots are chosen by greedy column
 *                pivoting on a 72-row random sketch of the trailing columns (a
 *                tournament over groups of 512 columns), the panel is factored by
 *                CholeskyQR2 in FP64 (its columns saved first; a panel whose CholeskyQR2
 *                checks fail, such as the one holding the rank boundary, is restored and
 *                factored by Householder columns; one host synchronisation per panel),
 *                and the sketch is updated from R_12.  SKI_QR_PIVOTED_HOUSEHOLDER: the
 *                same with Householder-column panels only (no per-panel synchronisation).
 *                SKI_QR_SPARSE (CSR A only, FP64, k <= 32): the sparse form of Step 2 in
 *                Section 6, S A P = Q R with P a fill-reducing column ordering, and every
 *                product with R^-1 or R^-T a sparse substitution instead of an explicit
 *                inverse.  ski_sketch keeps S A sparse (rows of ascending columns, entries
 *                summed in the dense sketch's order, so equal to it bit for bit).
 *                ski_factor orders the columns by exact minimum degree on the column graph
 *                of (SA)^T (SA) (smallest degree first, ties by smallest column index),
 *                stopping once the smallest degree exceeds 63 - k; the columns left form
 *                one dense root, placed last in increasing index.  Each eliminated column
 *                is one front of a multifrontal QR (its rows, and the contribution blocks
 *                of its children in the elimination tree, factored by Householder
 *                reflections); the root front is factored by the dense QR above and its
 *                R^-1 formed explicitly.  R (d x d in position order: upper, row q sparse
 *                for q below the root) and V-hat = P are returned by ski_get_R and
 *                ski_get_pivots; ski_get_factor_stats gives the leaf fronts and the root
 *                size.  No rank detection: rank = d, and the guards rcond and
 *                rcond_thres/perturb act on the whole diagonal as without pivoting.  The
 *                ordering and the symbolic structure are computed on the host.  Non-finite
 *                entries are found as the fronts are assembled; a sketch row with no entry
 *                of A carries only B's values and reaches no front, so a non-finite B there
 *                is reported by ski_solve.
 *                SKI_QR_PIVOTED_COD: the minimal-norm form (the complete orthogonal
 *                decomposition that the factorisation remark allows, with R_12 = 0): the
 *                SKI_QR_PIVOTED factorisation truncated at p, then a QR of the transposed
 *                top rows Rtop^T = Y L (d x p, Rtop = [R_11 R_12]); S A = Q_1 L^T V_1^T
 *                with V_1 = Pi Y, and Steps 3-5 use P = V_1 L^-T = Pi Rtop^T (L^T L)^-1,
 *                held as an explicit d x p matrix.  range(P) = range(A^T) under an
 *                embedding, so x is the minimal-norm least-squares solution (Section 5's
 *                minimal-norm guarantee).  The diagonal perturbation does not apply.
 *                The rank p is the number of leading diagonal entries with
 *                |r_qq| >= rcond |r_11| (with rcond = 0: the leading non-zero ones);
 *                R_11 is the leading p x p block, V_1 the first p pivots J, and Steps
 *                3-5 use W = A V_1 R_11^-1, so x is zero outside J.  Needs qr_prec =
 *                SKI_FP64; the rank guard (SKI_ERANK) does not apply.
 *   hash_kind    the sparse factor of S: SKI_HASH (default), the s-hashing matrix of
 *                Section 2.2 (s distinct rows per column); SKI_HASH_VARIANT, the s-hashing
 *                variant of Section 4 (s rows drawn with replacement, a repeated row gets
 *                both +-1/sqrt(s) entries); SKI_SAMPLE_ROWS, row sampling (each sketch row
 *                is one row of H D [A b], or of [A b] without H, drawn uniformly with
 *                replacement, value 1: the sampled transform that Section 7 compares
 *                hashing against; needs s = 1).  The sketch is scaled by 1/sqrt(n') with
 *                H and left unscaled without it. */
typedef struct {
    double gamma;
    int64_t m;
    int32_t s;
    int32_t hadamard;
    uint64_t seed;
    int32_t sketch_prec;
    int32_t qr_prec;
    double tau_a;
    double tau_r;
    int64_t it_max;
    double rcond;
    double rcond_thres;
    double perturb;
    int32_t qr_panel;
    int32_t hash_kind;
} ski_params;

/* Per right-hand side result of ski_solve. */
typedef struct {
    int64_t iters;      /* LSQR (or CG) iterations taken                              */
    int32_t status;     /* SKI_OK, SKI_WNOCONV or SKI_WEARLY for this column           */
    int32_t early_exit; /* 1 if Step 3 terminated                                       */
    double rnorm;       /* LSQR estimate of ||A x - b|| (CG: ||rhs - M y||)           */
    double arnorm;      /* LSQR estimate of ||W^T (W y - b)||                          */
    double wnorm_est;   /* running Frobenius estimate of ||W||                         */
    double tc;          /* arnorm / (wnorm_est * rnorm), the (TC-lsqr) value           */
    double cond_est;    /* max|r_ii| / min|r_ii| of the R used                          */
    float ms_sketch, ms_factor, ms_solve; /* device time of the three calls (ms)       */
} ski_info;

int ski_create(ski_handle* h);
int ski_destroy(ski_handle h);

/* Fill *p with the defaults of Section 6 for `kind` (SKI_DENSE: gamma 1.7, s 1,
 * Hadamard on, rcond 1e-12, no perturbation; SKI_CSR: gamma 1.4, s 2, no Hadamard,
 * rcond_thres 1e-10, perturb 1e-10; both tau_a 1e-8, tau_r 1e-6, it_max 1e4). */
void ski_params_default(int32_t kind, ski_params* p);

/* Step 1.  Draws S from (m, s, seed), forms S [A B] (B: n x k, device, leading
 * dimension ldb >= k; k >= 1) and keeps it in the handle.  Errors (all found on the host,
 * before any device work): SKI_EINVAL for n < d, d < 1, m < d, m > n' (dense with
 * Hadamard) or m > n, m > 12288 (except with SKI_QR_SPARSE), s out of range, k < 1, bad
 * leading dimensions, Hadamard requested for CSR; SKI_ENOMEM.  For CSR A, SKI_EINVAL also
 * when the structure is malformed (row_ptr not rising from 0 to nnz, or a column index
 * outside [0, d)): a device pass over row_ptr and col checks it before any other work on
 * A.  Non-finite entries of A and B are not looked for here (that would cost a pass over
 * the values); they are reported by ski_factor. */
int ski_sketch(ski_handle h, const ski_matrix* A, const double* B, int32_t k, int64_t ldb,
               const ski_params* p, void* stream);

/* Step 2.  Householder QR of the sketch; forms R (FP64, diag(R) >= 0), c, and the
 * explicit inverse of R used by every later product with R^-1 (any nonsingular P
 * applied consistently keeps the implicit sketching guarantee).  SKI_ERANK if the
 * rank guard fails (the handle then holds R but cannot solve).  SKI_EINVAL if the sketch
 * holds a NaN or an infinity: with a transform, or with hashing, every row of [A B]
 * enters S [A B] with a +-1 weight, so a non-finite entry anywhere in A or B shows up
 * there (the check rides on the QR's first pass over the sketch); under row sampling
 * without a transform only the sampled rows are seen, and ski_solve reports the rest.
 * The handle cannot solve after an error.  With qr_panel =
 * SKI_QR_PIVOTED: the column-pivoted factorisation and its truncation to R_11
 * (p x p, p from rcond); p = 0 (a numerically zero A) gives x = 0.  Synchronises the
 * stream. */
int ski_factor(ski_handle h, void* stream);

/* Steps 3-5 (op = SKI_OP_LLS): B is n x k (ldb), X is d x k (ldx).  The k columns are
 * solved together but stop independently.  info: host array of k entries, or NULL.
 * Returns the worst status over the columns (SKI_WNOCONV > SKI_WEARLY > SKI_OK).
 * op = SKI_OP_NORMAL: B is G (d x k, ldb) and X receives Z = (A^T A)^-1 G; the CG
 * stops when ||rhs - M y|| <= tau_r ||rhs|| for M = R^-T A^T A R^-1.
 * SKI_EINVAL (the column's info status too) when a column's iteration meets a non-finite
 * value: a NaN or infinity in B (LLS) or G (NORMAL), found at the first norm, so that no
 * iterations run on it. */
int ski_solve(ski_handle h, int32_t op, const double* B, int32_t k, int64_t ldb,
              double* X, int64_t ldx, ski_info* info, void* stream);

/* grad_B = A Z (n x k, ldgb) and grad_A = (B - A X) Z^T - (A Z) X^T (n x d, ldga) for
 * dense A.  Either output may be NULL.  X, Z: d x k; B: n x k.  After a pivoted factor
 * SKI_OP_NORMAL gives Z = V_1 (A_J^T A_J)^-1 G_J (zero outside the kept columns J), the
 * adjoint of the solution on J with J held fixed. */
int ski_gradients(ski_handle h, const double* X, int64_t ldx, const double* B, int64_t ldb,
                  const double* Z, int64_t ldz, int32_t k, double* grad_A, int64_t ldga,
                  double* grad_B, int64_t ldgb, void* stream);

/* Message of the handle's last error.  With h = NULL: the message of the last failed
 * ski_sketch_noalloc call on this host thread ("null handle" if there is none). */
const char* ski_last_error(ski_handle h);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): Step 1 as ski_sketch computes it, with
 * no handle and no allocation.  Writes SA = S [A B] (m x (d+k), FP64, row-major,
 * leading dimension d+k; caller-owned device buffer) for the S that (m, s, seed,
 * hadamard, hash_kind) define; the result equals the sketch ski_sketch forms from the
 * same arguments, bit for bit.  A: SKI_DENSE (row-major) or SKI_CSR; B: n x k device
 * (ldb >= k).  hadamard must be 0 or 1; sketch_prec and qr_prec must be SKI_FP64.  A CSR
 * structure is taken as given (this call never waits, so it cannot check it as ski_sketch
 * does): with a malformed one the call may read outside the arrays.
 * Scratch: the hash keys, their bucket sort, the D sign bits and the transform's column
 * slab live in one static device array of 64 MiB that the library holds on every GPU it
 * runs on until the process ends (its address is looked up on the first call on each
 * device, which must be the current device).  Limit: the hash buffers (10 bytes per key,
 * n' s keys, plus 4 m bytes per 4096 keys and 4 (m + 1) bytes) and, with the Hadamard
 * transform, a slab of 16 columns of n' doubles (n' <= 2^19) must fit in it; larger
 * problems are refused with SKI_EINVAL before any device work.  Every call on one GPU
 * shares that array: calls that overlap on one GPU (two streams, two threads) race and
 * must be serialised by the caller.  Asynchronous on `stream`; nothing is synchronised.
 * Returns SKI_OK, SKI_EINVAL (arguments, sizes; message from ski_last_error(NULL)) or
 * SKI_EDEVICE (a launch failed). */
int ski_sketch_noalloc(const ski_matrix* A, const double* B, int32_t k, int64_t ldb,
                       const ski_params* p, double* SA, void* stream);

/* Test and inspection getters: HOST copies, synchronous.
 *   dims: n, d, k, m, n' (padded rows, = n without Hadamard), s.
 *   hash: rows[n'*s] and neg[n'*s] per column in acceptance order; the bucket-sorted
 *         form bucket_ptr[m+1], src[n'*s] (column index), src_neg[n'*s].  Any pointer
 *         may be NULL.  With SKI_SAMPLE_ROWS: rows[m] = the row each sketch row samples,
 *         neg[m] = 0, src[m] = rows, src_neg[m] = 0.
 *   dsign: the diagonal of D as int8 (+1 / -1), n' entries (dense with Hadamard only).
 *   SA: the sketch m x (d+k) row-major, converted to double.
 *   R: d x d row-major (upper triangle, zeros below); c: d x k; Rinv: d x d (after a
 *      pivoted factor: R of the permuted sketch S A P, and Rinv = R_11^-1, p x p; after
 *      SKI_QR_PIVOTED_COD: Rinv = L^-1, p x p, for Rtop^T = Y L; after SKI_QR_SPARSE: R
 *      of S A P in position order, c likewise, and Rinv is not formed: SKI_ESTATE if
 *      Rinv is not NULL).  With SKI_QR_SPARSE, SA is returned dense. */
/* Kernel timing for measurement (not needed to solve).  ski_set_profiling(h, 1) makes the
 * library record a HIP event pair on the launch stream around every launch of the kernel
 * classes below (clearing earlier totals); ski_get_profile returns, per class, the summed
 * device time in ms and the number of launches since profiling was switched on.
 * Classes: 0 fused dense LSQR pass, 1 its partial-sum reduction, 2 triangular GEMV with
 * R^-1 / R^-T, 3 CSR product A z, 4 CSR product A^T u, 5 LSQR scalar step, 6 hashing
 * (Philox + bucket sort), 7 dense sketch with the Hadamard mix (transform passes and
 * hashing gather, by column slabs), 8 hashing gather without the Hadamard mix (dense or
 * CSR), 9 whole QR of the sketch with CholeskyQR2 panels, 10 explicit R^-1, 11 whole QR
 * with column-by-column Householder panels, 12 whole column-pivoted QR (pivot sketch,
 * selection, moves, panels, updates), 13 sparse sketch (SKI_QR_SPARSE), 14 its symbolic
 * phase and leaf fronts, 15 its root front (assembly and dense QR); the sparse
 * factor's triangular solves are timed as class 2.  ms[] and count[] hold SKI_PROF_CLASSES
 * entries.  ski_set_profiling(h, 1) times every class; ski_set_profiling_mask times only
 * the classes whose bit is set (bit c for class c; 0 switches profiling off), which keeps
 * the event records out of the other launches. */
#define SKI_PROF_CLASSES 16
int ski_set_profiling(ski_handle h, int32_t on);
int ski_set_profiling_mask(ski_handle h, uint32_t mask);
int ski_get_profile(ski_handle h, double* ms, int64_t* count);

int ski_get_dims(ski_handle h, int64_t dims[6]);
int ski_get_hash(ski_handle h, int32_t* rows, int8_t* neg, int64_t* bucket_ptr, int32_t* src,
                 int8_t* src_neg);
int ski_get_dsign(ski_handle h, int8_t* dsign);
int ski_get_SA(ski_handle h, double* SA);
int ski_get_R(ski_handle h, double* R, double* c, double* Rinv);
/* After ski_factor: perm[d] (position j of the factorisation holds column perm[j] of A;
 * the identity without pivoting) and the rank p (d without pivoting).  Either pointer
 * may be NULL.  SKI_ESTATE before a successful ski_factor. */
int ski_get_pivots(ski_handle h, int32_t* perm, int64_t* rank);
/* After ski_factor: stats[0] = rank p, stats[1] = number of 64-column panels,
 * stats[2] = panels that CholeskyQR2 factored in a pivoted factorisation (-1 without
 * pivoting), stats[3] = 1 if the factorisation pivoted.  After SKI_QR_SPARSE: stats[1] =
 * leaf fronts (eliminated columns), stats[2] = root columns, stats[3] = 2.  SKI_ESTATE
 * before ski_factor. */
int ski_get_factor_stats(ski_handle h, int64_t stats[4]);

#ifdef __cplusplus
}
#endif

#endif /* SKI_H */
