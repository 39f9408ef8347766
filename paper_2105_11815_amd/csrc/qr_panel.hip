// Panel factorisation for the blocked Householder QR of the sketch (Step 2 of
// Algorithm 1), built from wide kernels instead of a column-by-column chain.
//
// A panel P (mr x nb, nb <= 64, column-major inside the working copy) is factored by
// CholeskyQR2 (Yamamoto, Nakatsukasa, Yanagisawa and Fukaya, 2015):
//   G1 = P^T P,  R1 = chol(G1),  Q1 = P R1^-1,  G2 = Q1^T Q1,  R2 = chol(G2),
//   R  = R2 R1,  Q = Q1 R2^-1  (orthonormal to working precision).
// The Householder form of the same factorisation is then recovered from Q by a LU
// factorisation with sign-chosen pivots (Ballard, Demmel, Grigori, Jacquelin, Knight and
// Nguyen, "Reconstructing Householder vectors from tall-skinny QR", 2015):
//   [I; 0] - Q S = V U',  S = diag(s_k) chosen during the elimination so that every pivot
//   is 1 + |q_kk| >= 1,
// which gives the unit lower trapezoidal reflectors V, tau_k = U'_kk, and R_h = S R with
// P = (I - V T V^T) [R_h; 0].  The result is exactly what the column-by-column panel
// writes (R_h on and above the diagonal, V below it, the taus), so the trailing updates
// are unchanged.
//
// CholeskyQR2 is accurate only while cond(P) stays well below u^-1/2.  Both Cholesky
// factorisations check their pivots and the second Gram matrix must be close to the
// identity; any failure sets a flag that the host reads after the factorisation, which
// then repeats with the column-by-column Householder panel.
//
// Kernels per panel: Gram partials on MFMA over 64-row chunks, their fixed-order
// reduction, the first Cholesky and R1^-1, Q1 = P R1^-1 with the Gram partials of Q1 (MFMA),
// the reduction, the second Cholesky with the reconstruction and the panel's T, and
// V2 = Q1(nb:, :) M (MFMA).  The 64 x 64 factorisations are blocked (8 x 8 diagonal
// blocks, register-resident on one wavefront; the block row and the trailing update on
// all 256 threads), and the triangular inverses use recursive doubling, so that each
// runs in a few dozen barrier steps.  All sums have a fixed order: the result is
// deterministic.  T = U' V1^-T is written out, so the trailing updates apply it as a
// GEMM.
#include "ski_internal.h"
#include "tile64.h"

namespace ski {

namespace {

using namespace tile;
constexpr int GR = 64;       // rows per workgroup of the Gram / apply / V2 kernels
constexpr int RSL = 16;      // slices of the partial-sum reduction
constexpr double EPS_SERIES = 1e-8;  // |G2 - I| below which R2 comes from the series
constexpr double EPS_FIRST = 1e-11;  // ... from its first-order term alone
// One CholeskyQR pass leaves Q1 = P R1^-1 orthonormal to about u kappa(R1)^2.  When
// ||R1||_F ||R1^-1||_F (>= kappa_2(R1)) is at most ONE_PASS_KF in FP64, that is 1e-12 or
// less, and the second pass (Q1, its Gram matrix, R2) is skipped: the reconstruction then
// works on Q1's top block P_top R1^-1 and V2 = P(nb:, :) R1^-1 M.
constexpr double ONE_PASS_KF = 96.0;

// x if keep, else +0.0, without a branch (a select can be turned into a branch around the
// load, which then waits at once; integer masking keeps the loads together)
template <typename T>
__device__ __forceinline__ T keep_or_zero(T x, bool keep) {
    if constexpr (sizeof(T) == 8) {
        const uint64_t b = __builtin_bit_cast(uint64_t, x) & (keep ? ~0ull : 0ull);
        return __builtin_bit_cast(T, b);
    } else {
        const uint32_t b = __builtin_bit_cast(uint32_t, x) & (keep ? ~0u : 0u);
        return __builtin_bit_cast(T, b);
    }
}

// rows [r0, r1) of an nb-column column-major block -> sh[GR][PP], zero padded (r1 > r0).
// Thread t takes row r0 + t%64 of the columns t/64 + 4q: all 16 loads are issued before the
// first is used (addresses clamped into the block, masked values zeroed).
template <typename T>
__device__ __forceinline__ void stage_chunk(const T* __restrict__ P, int64_t ldp, int64_t r0,
                                            int64_t r1, int nb, T (*sh)[PP], int t) {
    const int rr = t & (GR - 1), c0 = t / GR;
    const int64_t r = r0 + rr;
    const bool rok = r < r1;
    const int64_t rc = rok ? r : r1 - 1;
    T v[PB / 4];
#pragma unroll
    for (int q = 0; q < PB / 4; ++q) {
        const int c = c0 + 4 * q;
        v[q] = P[(int64_t)(c < nb ? c : nb - 1) * ldp + rc];
    }
#pragma unroll
    for (int q = 0; q < PB / 4; ++q) sh[rr][c0 + 4 * q] = keep_or_zero(v[q], rok && c0 + 4 * q < nb);
}

// a full row-major PB x PB tile -> LDS, the loads issued together
template <typename T>
__device__ __forceinline__ void load_tile(const T* __restrict__ src, T (*dst)[PP], int t) {
    T v[PB * PB / 256];
#pragma unroll
    for (int q = 0; q < PB * PB / 256; ++q) v[q] = src[t + 256 * q];
#pragma unroll
    for (int q = 0; q < PB * PB / 256; ++q) {
        const int o = t + 256 * q;
        dst[o / PB][o % PB] = v[q];
    }
}

// sh[GR][PP] -> rows [r0, r1), columns < nb of a column-major block
template <typename T>
__device__ __forceinline__ void store_chunk(T (*sh)[PP], int64_t r0, int64_t r1, int nb,
                                            T* __restrict__ P, int64_t ldp, int t) {
    for (int o = t; o < GR * PB; o += 256) {
        const int rr = o % GR, c = o / GR;
        if (r0 + rr < r1 && c < nb) P[c * ldp + r0 + rr] = sh[rr][c];
    }
}

// X^T Y (PB x PB) of two staged chunks on MFMA -> Gp: wave w owns the tile row w
template <typename T>
__device__ __forceinline__ void chunk_atb(T (*X)[PP], T (*Y)[PP], T* __restrict__ Gp, int t) {
    using A4 = typename MF<T>::A4;
    const int l = t & 63, w = t >> 6, li = l & 15, lk = l >> 4;
    A4 acc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = (A4){0, 0, 0, 0};
#pragma unroll 4
    for (int s = 0; s < GR / 4; ++s) {
        const T a = X[4 * s + lk][16 * w + li];
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] = MF<T>::mma(a, Y[4 * s + lk][16 * q + li], acc[q]);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) Gp[(16 * w + MF<T>::row(r, l)) * PB + 16 * q + li] = acc[q][r];
}

template <typename T>
__device__ __forceinline__ void chunk_gram(T (*sh)[PP], T* __restrict__ Gp, int t) {
    chunk_atb(sh, sh, Gp, t);
}

// sh <- sh X for the staged chunk and an upper triangular X (PB x PB in Xs) on MFMA;
// wave w owns the tile row w.  Synchronises before overwriting sh.
template <typename T>
__device__ __forceinline__ void chunk_times_upper(T (*sh)[PP], T (*Xs)[PP], int t) {
    using A4 = typename MF<T>::A4;
    const int l = t & 63, w = t >> 6, li = l & 15, lk = l >> 4;
    A4 acc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = (A4){0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < 4; ++q)
        for (int s = 0; s < 4 * (q + 1); ++s)  // X(k, 16q + j) = 0 for k >= 16 (q + 1)
            acc[q] = MF<T>::mma(sh[16 * w + li][4 * s + lk], Xs[4 * s + lk][16 * q + li], acc[q]);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) sh[16 * w + MF<T>::row(r, l)][16 * q + li] = acc[q][r];
    __syncthreads();
}

// The panel chain is the QR's critical path, and its kernels share CUs with the trailing
// products of the second stream: their waves ask for the highest issue priority.
__device__ __forceinline__ void chain_priority() { __builtin_amdgcn_s_setprio(3); }

// Gram partials: workgroup b sums P^T P over the rows [b GR, (b+1) GR) -> Gp[b] (PB x PB)
template <typename T>
__global__ __launch_bounds__(256) void k_cqr_gram(const T* __restrict__ P, int64_t ldp, int64_t mr,
                                                  int nb, T* __restrict__ Gp) {
    chain_priority();
    __shared__ T sh[GR][PP];
    const int t = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * GR, r1 = std::min<int64_t>(mr, r0 + GR);
    stage_chunk(P, ldp, r0, r1, nb, sh, t);
    __syncthreads();
    chunk_gram(sh, Gp + (int64_t)blockIdx.x * PB * PB, t);
}

// G = sum of the nch partials: slice q of an entry sums the partials q, q + RSL, ... in
// ascending order, then the slices are added in ascending order.  A slice's loads (at most
// RMAX: nch <= RSL RMAX covers m <= 16384) are issued together, indices clamped, and only
// the valid ones summed, so the sum costs one memory round trip instead of one per term.
constexpr int RMAX = 16;
template <typename T>
__global__ __launch_bounds__(256) void k_cqr_reduce(const T* __restrict__ Gp, int nch,
                                                    T* __restrict__ G,
                                                    const int* __restrict__ skip) {
    chain_priority();
    if (skip && *skip) return;
    __shared__ T part[RSL][256 / RSL];
    constexpr int EPB = 256 / RSL;  // entries per workgroup
    const int t = threadIdx.x, el = t % EPB, sl = t / EPB;
    const int e = blockIdx.x * EPB + el;
    T v[RMAX];
#pragma unroll
    for (int u = 0; u < RMAX; ++u) {
        const int c = sl + RSL * u;
        v[u] = Gp[(int64_t)(c < nch ? c : nch - 1) * PB * PB + e];
    }
    T s = 0;
#pragma unroll
    for (int u = 0; u < RMAX; ++u)
        if (sl + RSL * u < nch) s += v[u];
    part[sl][el] = s;
    __syncthreads();
    if (t < EPB) {
        T a = 0;
#pragma unroll
        for (int q = 0; q < RSL; ++q) a += part[q][t];
        G[e] = a;
    }
}

// ---------------------------------------------------------------- kernels

// first Cholesky: G (PB x PB, identity beyond nb) -> R1 and R1^-1 (row-major PB x PB), and
// the one-pass decision for this panel
template <typename T>
__global__ __launch_bounds__(256) void k_cqr_chol1(const T* __restrict__ G, int nb,
                                                   T* __restrict__ R1, T* __restrict__ R1i,
                                                   int* __restrict__ flag,
                                                   int* __restrict__ one_pass) {
    chain_priority();
    __shared__ T A[PB][PP];
    __shared__ int bad;
    const int t = threadIdx.x;
    if (t == 0) bad = 0;
    {
        T v[PB * PB / 256];
#pragma unroll
        for (int q = 0; q < PB * PB / 256; ++q) v[q] = G[t + 256 * q];
#pragma unroll
        for (int q = 0; q < PB * PB / 256; ++q) {
            const int o = t + 256 * q, i = o / PB, j = o % PB;
            A[i][j] = (i < nb && j < nb) ? v[q] : (i == j ? (T)1 : (T)0);
        }
    }
    __syncthreads();
    tile_chol(A, t, &bad);
    T nr = 0, ni = 0;  // squared Frobenius norms of R1 and R1^-1 (this thread's entries)
    for (int o = t; o < PB * PB; o += 256) {
        const T x = A[o / PB][o % PB];
        R1[o] = x;
        nr += x * x;
    }
    tile_trinv(A, t, false);
    for (int o = t; o < PB * PB; o += 256) {
        const T x = A[o / PB][o % PB];
        R1i[o] = x;
        ni += x * x;
    }
    __shared__ T red[2][4];
    nr = wave_sum(nr);
    ni = wave_sum(ni);
    if ((t & 63) == 0) {
        red[0][t >> 6] = nr;
        red[1][t >> 6] = ni;
    }
    __syncthreads();
    if (t == 0) {
        const T kf2 = ((red[0][0] + red[0][1]) + (red[0][2] + red[0][3])) *
                      ((red[1][0] + red[1][1]) + (red[1][2] + red[1][3]));
        const bool one = sizeof(T) == 8 && !bad && kf2 <= (T)(ONE_PASS_KF * ONE_PASS_KF);
        one_pass[0] = one ? 1 : 0;
        if (bad) flag[0] = 1;
    }
}

// Q1 = P R1^-1 over the rows [b GR, (b+1) GR) (column-major, ld ldq) and the Gram partial
// of those rows of Q1
template <typename T>
__global__ __launch_bounds__(256) void k_cqr_apply_gram(const T* __restrict__ P, int64_t ldp,
                                                        int64_t mr, int nb,
                                                        const T* __restrict__ Ri,
                                                        T* __restrict__ Q, int64_t ldq,
                                                        T* __restrict__ Gp,
                                                        const int* __restrict__ one_pass) {
    chain_priority();
    if (*one_pass) return;
    __shared__ T Xs[PB][PP];
    __shared__ T sh[GR][PP];
    const int t = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * GR, r1 = std::min<int64_t>(mr, r0 + GR);
    load_tile(Ri, Xs, t);
    stage_chunk(P, ldp, r0, r1, nb, sh, t);
    __syncthreads();
    chunk_times_upper(sh, Xs, t);
    store_chunk(sh, r0, r1, nb, Q, ldq, t);
    chunk_gram(sh, Gp + (int64_t)blockIdx.x * PB * PB, t);
}

// Second Cholesky and the Householder reconstruction:
//   check G2 ~ I, R2 = chol(G2), R = R2 R1, Qt = Q1(0:nb, :) R2^-1,
//   LU with sign-chosen pivots of [I - Qt S] -> L1 (unit lower), U' (upper), S,
//   M = -R2^-1 S U'^-1 (for V2 = Q1(nb:, :) M),  T = U' L1^-T.
// Writes the panel's top block (S R on and above the diagonal, L1 below), tau = diag(U'),
// M and T (row-major PB x PB).
template <typename T>
__global__ __launch_bounds__(256) void k_cqr_chol2(const T* __restrict__ G, int nb,
                                                   const T* __restrict__ R1,
                                                   const T* __restrict__ Q, int64_t ldq,
                                                   T* __restrict__ Pt, int64_t ldp,
                                                   T* __restrict__ tau, T* __restrict__ Mx,
                                                   T* __restrict__ Tx, int* __restrict__ flag,
                                                   const T* __restrict__ R1i,
                                                   const int* __restrict__ one_pass) {
    chain_priority();
    __shared__ T A[PB][PP];  // G2 -> R2 -> R2^-1 -> M
    __shared__ T B[PB][PP];  // R1 -> R = R2 R1
    __shared__ T C[PB][PP];  // Q1 top -> Qt -> L1 and the eliminated Qt
    __shared__ T D[PB][PP];  // R2 copy -> U'^-1 -> L1^-T -> T
    __shared__ T sg[PB];
    __shared__ int bad;
    const int t = threadIdx.x;
    int off = 0, big = 0, second = 0;
    if (*one_pass) {
        // one CholeskyQR pass: R = R1, "R2^-1" := R1^-1 (so that M below comes out as
        // -R1^-1 S U'^-1, for V2 = P(nb:, :) M), Qt = P_top R1^-1 from the panel's own top
        // block (read before it is overwritten at the end)
        T rv[PB * PB / 256], iv[PB * PB / 256], pv[PB * PB / 256];
#pragma unroll
        for (int q = 0; q < PB * PB / 256; ++q) {
            const int o = t + 256 * q, r = o % PB, c = o / PB;
            rv[q] = R1[o];
            iv[q] = R1i[o];
            pv[q] = Pt[(int64_t)(c < nb ? c : nb - 1) * ldp + (r < nb ? r : nb - 1)];
        }
#pragma unroll
        for (int q = 0; q < PB * PB / 256; ++q) {
            const int o = t + 256 * q, i = o / PB, j = o % PB;
            B[i][j] = rv[q];
            A[i][j] = iv[q];
            const int r = o % PB, c = o / PB;
            C[r][c] = keep_or_zero(pv[q], r < nb && c < nb);
        }
        if (t == 0) bad = 0;
        __syncthreads();
        tile_mma(C, t, [&](int i, int k) { return C[i][k]; }, [&](int k, int j) { return A[k][j]; },
                 KFullUpper{}, [](int, int, T v) { return v; });
    } else {
        // all loads first (Q1's top block walked column-major for coalescing; rows and
        // columns beyond nb are clamped and zeroed)
        T gv[PB * PB / 256], rv[PB * PB / 256], qv[PB * PB / 256];
#pragma unroll
        for (int q = 0; q < PB * PB / 256; ++q) {
            const int o = t + 256 * q, r = o % PB, c = o / PB;
            gv[q] = G[o];
            rv[q] = R1[o];
            qv[q] = Q[(int64_t)(c < nb ? c : nb - 1) * ldq + (r < nb ? r : nb - 1)];
        }
#pragma unroll
        for (int q = 0; q < PB * PB / 256; ++q) {
            const int o = t + 256 * q, i = o / PB, j = o % PB;
            const T g = (i < nb && j < nb) ? gv[q] : (i == j ? (T)1 : (T)0);
            A[i][j] = g;
            // G2 must be close to the identity for the second step to be accurate
            const T e = fabs(g - (i == j ? (T)1 : (T)0));
            off |= !(e <= (T)0.01);
            big |= !(e <= (T)EPS_SERIES);
            second |= !(e <= (T)EPS_FIRST);
            B[i][j] = rv[q];
            const int r = o % PB, c = o / PB;
            C[r][c] = keep_or_zero(qv[q], r < nb && c < nb);
        }
        if (t == 0) bad = 0;
        off = __syncthreads_or(off);
        big = __syncthreads_or(big);
        second = __syncthreads_or(second);
        if (!second) {
            // |G2 - I| <= EPS_FIRST: to first order R2 = I + F, R2^-1 = I - F with
            // F = up(G2 - I); the neglected terms are O(|G2 - I|^2), below 1e-18
            tile_eval(D, t, [&](int i, int j) {
                const T e = A[i][j] - (i == j ? (T)1 : (T)0);
                return i < j ? e : (i == j ? e * (T)0.5 : (T)0);
            });
            // R = R1 + F R1
            tile_mma(B, t, [&](int i, int k) { return D[i][k]; }, [&](int k, int j) { return B[k][j]; },
                     KFullUpper{}, [&](int i, int j, T v) { return B[i][j] + v; });
            tile_eval(A, t, [&](int i, int j) { return (i == j ? (T)1 : (T)0) - D[i][j]; });
        } else if (big) {
            tile_chol(A, t, &bad);
            // R = R2 R1 (both upper)
            tile_mma(B, t, [&](int i, int k) { return A[i][k]; }, [&](int k, int j) { return B[k][j]; },
                     KFullUpper{}, [](int, int, T v) { return v; });
            tile_trinv(A, t, false);
        } else {
            // G2 = I + E with |E| <= EPS_SERIES: R2 = I + F where F + F^T + F^T F = E is solved
            // by two steps of F <- up(E - F^T F) (up: strict upper part plus half the diagonal),
            // and R2^-1 = I - F + F^2; both are exact to O(|E|^3), far below rounding
            auto up = [](int i, int j, T x) { return i < j ? x : (i == j ? x * (T)0.5 : (T)0); };
            tile_eval(D, t, [&](int i, int j) { return up(i, j, A[i][j] - (i == j ? (T)1 : (T)0)); });
            tile_mma(A, t, [&](int i, int k) { return D[k][i]; }, [&](int k, int j) { return D[k][j]; },
                     KFull{}, [&](int i, int j, T v) {
                         return (i == j ? (T)1 : (T)0) +
                                up(i, j, A[i][j] - (i == j ? (T)1 : (T)0) - v);
                     });
            // R = R2 R1 (both upper)
            tile_mma(B, t, [&](int i, int k) { return A[i][k]; }, [&](int k, int j) { return B[k][j]; },
                     KFullUpper{}, [](int, int, T v) { return v; });
            // R2^-1 = I - F + F F with F = R2 - I
            tile_mma(A, t, [&](int i, int k) { return A[i][k] - (i == k ? (T)1 : (T)0); },
                     [&](int k, int j) { return A[k][j] - (k == j ? (T)1 : (T)0); }, KFullUpper{},
                     [&](int i, int j, T v) {
                         return (i == j ? (T)1 : (T)0) - (A[i][j] - (i == j ? (T)1 : (T)0)) + v;
                     });
        }
        // Qt = Q1top R2^-1
        tile_mma(C, t, [&](int i, int k) { return C[i][k]; }, [&](int k, int j) { return A[k][j]; },
                 KFullUpper{}, [](int, int, T v) { return v; });
    }  // two passes
    tile_lu_signed(C, sg, t);
    // U'(k, c) = delta_kc - s_c C(k, c) on and above the diagonal; then U'^-1 in place
    tile_eval(D, t, [&](int i, int j) {
        return i <= j ? (i == j ? (T)1 : (T)0) - sg[j] * C[i][j] : (T)0;
    });
    tile_trinv(D, t, false);
    // M = -R2^-1 S U'^-1
    tile_mma(A, t, [&](int i, int k) { return A[i][k] * sg[k]; },
             [&](int k, int j) { return D[k][j]; }, KFullUpper{},
             [](int, int, T v) { return -v; });
    for (int o = t; o < PB * PB; o += 256) Mx[o] = A[o / PB][o % PB];
    // L1^T (unit upper), inverted in place; U' again (into A)
    tile_eval(D, t, [&](int i, int j) { return i < j ? C[j][i] : (i == j ? (T)1 : (T)0); });
    tile_eval(A, t, [&](int i, int j) {
        return i <= j ? (i == j ? (T)1 : (T)0) - sg[j] * C[i][j] : (T)0;
    });
    tile_trinv(D, t, true);
    // T = U' L1^-T
    tile_mma(D, t, [&](int i, int k) { return A[i][k]; }, [&](int k, int j) { return D[k][j]; },
             KFullUpper{}, [](int, int, T v) { return v; });
    for (int o = t; o < PB * PB; o += 256) {
        const int i = o % PB, c = o / PB;  // column-major walk of the panel's top block
        if (i < nb && c < nb) Pt[c * ldp + i] = i <= c ? sg[i] * B[i][c] : C[i][c];
        Tx[o] = D[o / PB][o % PB];
    }
    if (t < nb) tau[t] = (T)1 - sg[t] * C[t][t];
    if (t == 0 && (bad || off)) flag[0] = 1;
}

// Gram partials of panel p after the previous panel's block reflector (V, T; rows [jq, m))
// is applied to it: with W = V^T C (reduced beforehand) and Y = T^T W,
//   C <- C - V Y  over the rows [jq, m),
// written back (rows [jq, j0) are rows of R), and the Gram partials of the updated rows
// [j0, m) (the panel to factor).  Chunk b covers the rows [jq + b GR, jq + (b+1) GR); its
// Gram partial goes to Gp[b - 1] (chunk 0 is the block of R rows).
template <typename T>
__global__ __launch_bounds__(256) void k_cqr_update_gram(T* __restrict__ Ac, int64_t m, int64_t jq,
                                                         int64_t j0, int nb,
                                                         const T* __restrict__ V,
                                                         const T* __restrict__ Tq,
                                                         const T* __restrict__ W,
                                                         T* __restrict__ Gp) {
    using A4 = typename MF<T>::A4;
    chain_priority();
    // two tiles (66.5 KB in FP64), so that a workgroup fits on a CU beside two workgroups
    // of the trailing update; V's MFMA operands go straight to registers
    __shared__ T Ys[PB][PP];  // T, then Y = T^T W
    __shared__ T Cs[PB][PP];  // W, then the chunk of C
    const int t = threadIdx.x, l = t & 63, w = t >> 6, li = l & 15, lk = l >> 4;
    const int64_t mq = m - jq;
    const int64_t r0 = (int64_t)blockIdx.x * GR, r1 = std::min<int64_t>(mq, r0 + GR);
    // this wave's operands of the chunk of V: row r0 + 16 w + li, columns 4 u + lk
    const int64_t rv = r0 + 16 * w + li;
    const bool vok = rv < r1;
    const int64_t rvc = vok ? rv : r1 - 1;
    T vf[PB / 4];
#pragma unroll
    for (int u = 0; u < PB / 4; ++u) vf[u] = V[(int64_t)(4 * u + lk) * mq + rvc];
    load_tile(Tq, Ys, t);
    load_tile(W, Cs, t);
    __syncthreads();
    // Y = T^T W (T upper), in place
    tile_mma(Ys, t, [&](int i, int k) { return Ys[k][i]; }, [&](int k, int j) { return Cs[k][j]; },
             KLowerFull{}, [](int, int, T v) { return v; });
    stage_chunk(Ac + j0 * m + jq, m, r0, r1, nb, Cs, t);
    __syncthreads();
    // C <- C - V Y: wave w owns the tile row w (the MFMA sequence of tile_mma)
    A4 acc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        acc[q] = (A4){0, 0, 0, 0};
#pragma unroll
        for (int u = 0; u < PB / 4; ++u)
            acc[q] = MF<T>::mma(keep_or_zero(vf[u], vok), Ys[4 * u + lk][16 * q + li], acc[q]);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            T& c = Cs[16 * w + MF<T>::row(r, l)][16 * q + li];
            c = c - acc[q][r];  // each entry is read and written by its own lane only
        }
    __syncthreads();
    store_chunk(Cs, r0, r1, nb, Ac + j0 * m + jq, m, t);
    if (blockIdx.x > 0) chunk_gram(Cs, Gp + (int64_t)(blockIdx.x - 1) * PB * PB, t);
}

// The panel's reflectors: V2 = Q1 M below the top block (P R1^-1 M after one pass), L1
// (unit lower) in it.  Chunk b
// covers the panel rows [b GR, (b+1) GR): V2 rows go into the panel, the explicit V (unit
// diagonal, zeros above) into Vout (column-major, ld mr), and with a next panel of nbn
// columns the partial products V^T C_next of those rows into Gp[b].
template <typename T>
__global__ __launch_bounds__(256) void k_cqr_v2x(const T* __restrict__ Q, int64_t ldq, int64_t mr,
                                                 int nb, const T* __restrict__ Mx,
                                                 T* __restrict__ P, int64_t ldp,
                                                 T* __restrict__ Vout, int nbn,
                                                 T* __restrict__ Gp,
                                                 const int* __restrict__ one_pass) {
    using A4 = typename MF<T>::A4;
    chain_priority();
    // two tiles (66.5 KB in FP64), so that a workgroup fits on a CU beside two workgroups
    // of the trailing update; the chunk's MFMA operands go straight to registers, and V2
    // replaces M in its tile once the product is formed
    __shared__ T Xs[PB][PP];  // M, then V2's chunk
    __shared__ T Cs[PB][PP];  // the next panel's chunk
    const int t = threadIdx.x, l = t & 63, w = t >> 6, li = l & 15, lk = l >> 4;
    const int64_t r0 = (int64_t)blockIdx.x * GR, r1 = std::min<int64_t>(mr, r0 + GR);
    // one pass: V2 = P(nb:, :) M with M = -R1^-1 S U'^-1 (rows < nb of the product unused:
    // the panel's top block, already overwritten, gives L1 below); else V2 = Q1(nb:, :) M.
    // This wave's operands: row r0 + 16 w + li of the chunk, columns 4 u + lk.
    const bool one = *one_pass != 0;
    const T* src = one ? (const T*)P : Q;
    const int64_t lds = one ? ldp : ldq;
    const int64_t ra = r0 + 16 * w + li;
    const bool aok = ra < r1;
    const int64_t rac = aok ? ra : r1 - 1;
    T af[PB / 4];
#pragma unroll
    for (int u = 0; u < PB / 4; ++u) {
        const int c = 4 * u + lk;
        af[u] = keep_or_zero(src[(int64_t)(c < nb ? c : nb - 1) * lds + rac], aok && c < nb);
    }
    load_tile(Mx, Xs, t);
    if (nbn > 0) stage_chunk(P + (int64_t)nb * ldp, ldp, r0, r1, nbn, Cs, t);
    __syncthreads();
    // chunk x M (M upper: tile column q needs k < 16 q + 16), wave w owns the tile row w
    A4 acc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        acc[q] = (A4){0, 0, 0, 0};
#pragma unroll
        for (int u = 0; u < 4 * q + 4; ++u)
            acc[q] = MF<T>::mma(af[u], Xs[4 * u + lk][16 * q + li], acc[q]);
    }
    T vals[16];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = 16 * w + MF<T>::row(r, l), j = 16 * q + li;
            const int64_t rr = r0 + i;
            T v = acc[q][r];
            if (rr >= r1 || j >= nb) v = (T)0;
            else if (rr < nb) v = rr == j ? (T)1 : (rr > j ? P[j * ldp + rr] : (T)0);
            vals[4 * q + r] = v;
        }
    __syncthreads();  // every wave has read M
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) Xs[16 * w + MF<T>::row(r, l)][16 * q + li] = vals[4 * q + r];
    __syncthreads();
    for (int o = t; o < GR * PB; o += 256) {
        const int rr = o % GR, c = o / GR;
        const int64_t r = r0 + rr;
        if (r < r1 && c < nb) {
            if (r >= nb) P[c * ldp + r] = Xs[rr][c];
            Vout[c * mr + r] = Xs[rr][c];
        }
    }
    if (nbn > 0) chunk_atb(Xs, Cs, Gp + (int64_t)blockIdx.x * PB * PB, t);
}

__global__ void k_set_flag(int* flag, int v) {
    if (threadIdx.x == 0) flag[0] = v;
}

}  // namespace

int64_t cqr_num_chunks(int64_t m) { return (m + GR - 1) / GR; }

template <typename T>
hipError_t cqr_gram_update(T* Ac, int64_t m, int64_t jq, int64_t j0, int nb, const T* V,
                           const T* Tq, const CqrWs& w, hipStream_t st) {
    if (nb < 1 || nb > PB || m - j0 < nb) return hipErrorInvalidValue;
    if (cqr_num_chunks(m) > RSL * RMAX) return hipErrorInvalidValue;
    const int64_t mr = m - j0;
    const int nch = (int)((mr + GR - 1) / GR);
    const unsigned nred = PB * PB / (256 / RSL);
    if (jq < 0) {
        hipLaunchKernelGGL((k_cqr_gram<T>), dim3(nch), dim3(256), 0, st, Ac + j0 * m + j0, m, mr,
                           nb, (T*)w.Gp);
    } else {
        if (j0 - jq != PB) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_cqr_update_gram<T>), dim3(nch + 1), dim3(256), 0, st, Ac, m, jq, j0,
                           nb, V, Tq, (const T*)w.W, (T*)w.Gp);
    }
    hipLaunchKernelGGL((k_cqr_reduce<T>), dim3(nred), dim3(256), 0, st, (const T*)w.Gp, nch,
                       (T*)w.G, (const int*)nullptr);
    return hipGetLastError();
}

template <typename T>
hipError_t cqr_factor_panel(T* Ac, int64_t m, int64_t j0, int nb, const CqrWs& w, T* Tout,
                            hipStream_t st) {
    if (nb < 1 || nb > PB) return hipErrorInvalidValue;
    const int64_t mr = m - j0;
    if (mr < nb) return hipErrorInvalidValue;
    T* P = Ac + j0 * m + j0;
    T* Q = (T*)w.Q1;
    T* Gp = (T*)w.Gp;
    T* G = (T*)w.G;
    T* R1 = (T*)w.R1;
    T* R1i = (T*)w.R1i;
    const int nch = (int)((mr + GR - 1) / GR);
    const unsigned nred = PB * PB / (256 / RSL);
    hipLaunchKernelGGL((k_cqr_chol1<T>), dim3(1), dim3(256), 0, st, G, nb, R1, R1i, w.flag,
                       w.one_pass);
    // the second pass's kernels return at once when the first Cholesky chose one pass
    hipLaunchKernelGGL((k_cqr_apply_gram<T>), dim3(nch), dim3(256), 0, st, P, m, mr, nb, R1i, Q,
                       m, Gp, (const int*)w.one_pass);
    hipLaunchKernelGGL((k_cqr_reduce<T>), dim3(nred), dim3(256), 0, st, Gp, nch, G,
                       (const int*)w.one_pass);
    hipLaunchKernelGGL((k_cqr_chol2<T>), dim3(1), dim3(256), 0, st, G, nb, R1, Q, m, P, m,
                       (T*)w.tau + j0, (T*)w.Mx, Tout, w.flag, (const T*)R1i,
                       (const int*)w.one_pass);
    return hipGetLastError();
}

template <typename T>
hipError_t cqr_finish_panel(T* Ac, int64_t m, int64_t j0, int nb, int nbn, const CqrWs& w,
                            T* Vout, hipStream_t st) {
    if (nb < 1 || nb > PB || nbn < 0 || nbn > PB) return hipErrorInvalidValue;
    const int64_t mr = m - j0;
    const int nch = (int)((mr + GR - 1) / GR);
    hipLaunchKernelGGL((k_cqr_v2x<T>), dim3(nch), dim3(256), 0, st, (const T*)w.Q1, m, mr, nb,
                       (const T*)w.Mx, Ac + j0 * m + j0, m, Vout, nbn, (T*)w.Gp,
                       (const int*)w.one_pass);
    if (nbn > 0)
        hipLaunchKernelGGL((k_cqr_reduce<T>), dim3(PB * PB / (256 / RSL)), dim3(256), 0, st,
                           (const T*)w.Gp, nch, (T*)w.W, (const int*)nullptr);
    return hipGetLastError();
}

hipError_t cqr_clear_flag(int* flag, hipStream_t st) {
    hipLaunchKernelGGL(k_set_flag, dim3(1), dim3(64), 0, st, flag, 0);
    return hipGetLastError();
}

#define SKI_CQR_INST(T)                                                                     \
    template hipError_t cqr_gram_update<T>(T*, int64_t, int64_t, int64_t, int, const T*,     \
                                           const T*, const CqrWs&, hipStream_t);             \
    template hipError_t cqr_factor_panel<T>(T*, int64_t, int64_t, int, const CqrWs&, T*,      \
                                            hipStream_t);                                    \
    template hipError_t cqr_finish_panel<T>(T*, int64_t, int64_t, int, int, const CqrWs&, T*, \
                                            hipStream_t);
SKI_CQR_INST(double)
SKI_CQR_INST(float)
#undef SKI_CQR_INST

}  // namespace ski
