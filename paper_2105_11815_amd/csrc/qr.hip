// Step 2 of Algorithm 1: Householder QR (no pivoting) of the m x (d+k) sketch [SA Sb],
// blocked as in LAPACK's DGEQRF (the factorisation the paper's dense solver uses when A
// has full rank), giving R in the upper triangle and Q^T S b in the last k columns.
//
// Reflectors follow the LAPACK convention: for x = [alpha; x2],
//   beta = -sign(alpha) ||x||, tau = (beta - alpha)/beta, v = [1; x2/(alpha - beta)],
// H = I - tau v v^T; a block H_1 ... H_b = I - V T V^T with T upper triangular (forward,
// columnwise compact-WY); Q^T C = C - V T^T V^T C.
//
// Layout: the factorisation works on a column-major copy of the sketch (column j holds m
// contiguous entries), so that a panel's columns stream contiguously.  Reflectors are
// stored in place below the diagonal with an implicit unit diagonal.
//
// Blocking: outer panels of NBP = 64 columns.  Inside a panel, leaves of 4 columns are
// factored by one workgroup with the leaf's rows in registers (one block reduction per
// column gives the squared norm below the diagonal and the inner products with the other
// leaf columns); the leaf's T is formed in the same kernel.  The leaf's block reflector
// is then applied to each remaining panel column by one workgroup per column (4 inner
// products, T^T, the rank-4 update).  After a panel, its reflectors are copied out
// explicitly (V^T, nb x (m - j0)), T is formed from V^T V and the taus, and the trailing
// columns get Q^T through three MFMA GEMMs on the transposed operands:
//   W^T = C^T V,  W2^T = W^T T,  C^T -= W2^T V^T.
// Every sum has a fixed order: the factorisation is deterministic.
#include "ski_internal.h"

#include <type_traits>

namespace ski {

namespace {

constexpr int NBL = 4;     // leaf width
constexpr int LFT = 512;   // leaf threads
constexpr int LT = 512;    // threads of the narrow update
constexpr int NBP = 64;    // outer panel width

// block reduction of N values over a workgroup of NT threads, in a fixed order
template <typename T, int N, int NT>
__device__ __forceinline__ void block_reduce(T (&v)[N], T (*sh)[N], int tid) {
    const int lane = tid & 63, wv = tid >> 6;
#pragma unroll
    for (int c = 0; c < N; ++c) v[c] = wave_sum(v[c]);
    if (lane == 0)
#pragma unroll
        for (int c = 0; c < N; ++c) sh[wv][c] = v[c];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < N; ++c) {
        T a = 0;
        for (int q = 0; q < NT / 64; ++q) a += sh[q][c];
        v[c] = a;
    }
}

// leaf: factor columns [jc, jc+w) over rows [jc, m) of the column-major matrix (ld = m);
// taus -> tau[jc..], the leaf's T (w x w, zero-padded to NBL x NBL, row-major) -> Tl
template <typename T, int RPT>
__global__ __launch_bounds__(LFT) void k_qr_leaf(T* __restrict__ Ac, int64_t m, int64_t jc, int w,
                                                T* __restrict__ tau, T* __restrict__ Tl) {
    __shared__ T red[2][LFT / 64][NBL];
    __shared__ T rowb[2][NBL];
    __shared__ T gsh[LFT / 64][NBL * NBL];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t mrem = m - jc;
    T* base = Ac + jc * m + jc;  // element (r, c) of the leaf at base[c * m + r]
    T P[RPT][NBL];
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
        const int64_t r = tid + (int64_t)LFT * u;
#pragma unroll
        for (int c = 0; c < NBL; ++c) P[u][c] = (r < mrem && c < w) ? base[c * m + r] : (T)0;
    }
    T taus[NBL];
#pragma unroll
    for (int c = 0; c < NBL; ++c) taus[c] = 0;
#pragma unroll
    for (int jj = 0; jj < NBL; ++jj) {
        if (jj >= w) break;
        const int buf = jj & 1;
        T s[NBL];
#pragma unroll
        for (int c = 0; c < NBL; ++c) s[c] = 0;
#pragma unroll
        for (int u = 0; u < RPT; ++u) {
            const int64_t r = tid + (int64_t)LFT * u;
            if (r > jj && r < mrem) {
#pragma unroll
                for (int c = 0; c < NBL; ++c)
                    if (c >= jj) s[c] += P[u][jj] * P[u][c];
            }
        }
#pragma unroll
        for (int c = 0; c < NBL; ++c) {
            if (c >= jj) {
                T v = wave_sum(s[c]);
                if (lane == 0) red[buf][wv][c] = v;
            }
        }
        if (tid == jj) {
#pragma unroll
            for (int c = 0; c < NBL; ++c) rowb[buf][c] = P[0][c];
        }
        __syncthreads();
        T tot[NBL];
#pragma unroll
        for (int c = 0; c < NBL; ++c) {
            T a = 0;
            if (c >= jj)
                for (int q = 0; q < LFT / 64; ++q) a += red[buf][q][c];
            tot[c] = a;
        }
        const T alpha = rowb[buf][jj];
        const T xn2 = tot[jj];
        T beta, tj, scal;
        if (xn2 == (T)0) {
            tj = 0;
            beta = alpha;
            scal = 0;
        } else {
            beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
            tj = (beta - alpha) / beta;
            scal = (T)1 / (alpha - beta);
        }
        taus[jj] = tj;
        T wc[NBL];
#pragma unroll
        for (int c = 0; c < NBL; ++c) wc[c] = (c > jj) ? rowb[buf][c] + tot[c] * scal : (T)0;
#pragma unroll
        for (int u = 0; u < RPT; ++u) {
            const int64_t r = tid + (int64_t)LFT * u;
            if (r > jj && r < mrem) {
                const T v = P[u][jj] * scal;
#pragma unroll
                for (int c = 0; c < NBL; ++c)
                    if (c > jj) P[u][c] -= tj * v * wc[c];
                P[u][jj] = v;
            } else if (r == jj) {
#pragma unroll
                for (int c = 0; c < NBL; ++c)
                    if (c > jj) P[u][c] -= tj * wc[c];
                P[u][jj] = beta;
            }
        }
    }
    // write back R (upper) and the reflectors (below the diagonal)
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
        const int64_t r = tid + (int64_t)LFT * u;
        if (r < mrem)
#pragma unroll
            for (int c = 0; c < NBL; ++c)
                if (c < w) base[c * m + r] = P[u][c];
    }
    // leaf T: G = V^T V over the explicit reflectors, then the forward recurrence
    T g[NBL * NBL];
#pragma unroll
    for (int q = 0; q < NBL * NBL; ++q) g[q] = 0;
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
        const int64_t r = tid + (int64_t)LFT * u;
        if (r < mrem) {
            T v[NBL];
#pragma unroll
            for (int c = 0; c < NBL; ++c)
                v[c] = (c >= w) ? (T)0 : (r < c ? (T)0 : (r == c ? (T)1 : P[u][c]));
#pragma unroll
            for (int a = 0; a < NBL; ++a)
#pragma unroll
                for (int b = a + 1; b < NBL; ++b) g[a * NBL + b] += v[a] * v[b];
        }
    }
#pragma unroll
    for (int a = 0; a < NBL; ++a)
#pragma unroll
        for (int b = a + 1; b < NBL; ++b) {
            T t = wave_sum(g[a * NBL + b]);
            if (lane == 0) gsh[wv][a * NBL + b] = t;
        }
    __syncthreads();
    if (tid == 0) {
        T G[NBL * NBL], Tm[NBL * NBL];
#pragma unroll
        for (int q = 0; q < NBL * NBL; ++q) {
            T a = 0;
            const int qa = q / NBL, qb = q % NBL;
            if (qa < qb)
                for (int wq = 0; wq < LFT / 64; ++wq) a += gsh[wq][q];
            G[q] = a;
            Tm[q] = 0;
        }
#pragma unroll
        for (int i = 0; i < NBL; ++i) {
            if (i < w) {
#pragma unroll
                for (int a = 0; a < NBL; ++a) {
                    if (a < i) {
                        T y = 0;
#pragma unroll
                        for (int b = 0; b < NBL; ++b)
                            if (b >= a && b < i) y += Tm[a * NBL + b] * G[b * NBL + i];
                        Tm[a * NBL + i] = -taus[i] * y;
                    }
                }
                Tm[i * NBL + i] = taus[i];
                tau[jc + i] = taus[i];
            }
        }
#pragma unroll
        for (int a = 0; a < NBL; ++a)
#pragma unroll
            for (int b = 0; b < NBL; ++b)
                Tl[a * NBL + b] = Tm[a * NBL + b];
    }
}

// Q_leaf^T applied to one trailing column per workgroup: c = c0 + blockIdx.x,
// W = V^T C_c (w values), W2 = T^T W, C_c -= V W2, over rows [jc, m).  The column and
// the leaf's reflectors stay in registers between the reduction and the update.
template <typename T, int RPT>
__global__ __launch_bounds__(LT) void k_narrow_apply(T* __restrict__ Ac, int64_t m, int64_t jc,
                                                     int w, const T* __restrict__ Tl,
                                                     int64_t c0) {
    __shared__ T sh[LT / 64][NBL];
    const int tid = threadIdx.x;
    const int64_t mrem = m - jc;
    const T* V = Ac + jc * m + jc;
    T* C = Ac + (c0 + blockIdx.x) * m + jc;
    T cv[RPT], vv[RPT][NBL];
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
        const int64_t r = tid + (int64_t)LT * u;
        const bool ok = r < mrem;
        cv[u] = ok ? C[r] : (T)0;
#pragma unroll
        for (int a = 0; a < NBL; ++a)
            vv[u][a] = (ok && a < w) ? (r < a ? (T)0 : (r == a ? (T)1 : V[a * m + r])) : (T)0;
    }
    T acc[NBL];
#pragma unroll
    for (int a = 0; a < NBL; ++a) {
        T s = 0;
#pragma unroll
        for (int u = 0; u < RPT; ++u) s += vv[u][a] * cv[u];
        acc[a] = s;
    }
    block_reduce<T, NBL, LT>(acc, sh, tid);
    T w2[NBL];
#pragma unroll
    for (int a = 0; a < NBL; ++a) {
        T s = 0;
#pragma unroll
        for (int b = 0; b < NBL; ++b)
            if (b <= a && a < w) s += Tl[b * NBL + a] * acc[b];
        w2[a] = s;
    }
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
        const int64_t r = tid + (int64_t)LT * u;
        if (r < mrem) {
            T s = 0;
#pragma unroll
            for (int a = 0; a < NBL; ++a) s += vv[u][a] * w2[a];
            C[r] = cv[u] - s;
        }
    }
}

// [V^T; C_next^T] of a panel: rows c < nb hold the explicit reflectors v_c (unit diagonal,
// zeros above), rows nb + c hold the next panel's column nx0 + c, all over the rows
// [j0, m) of the matrix (leading dimension mr = m - j0)
template <typename T>
__global__ __launch_bounds__(256) void k_make_VC(const T* __restrict__ Ac, int64_t m, int64_t j0,
                                                 int nb, int64_t nx0, T* __restrict__ VC) {
    const int64_t mr = m - j0;
    const int c = blockIdx.y;
    const bool isv = c < nb;
    const T* col = isv ? Ac + (j0 + c) * m + j0 : Ac + (nx0 + (c - nb)) * m + j0;
    for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < mr; r += (int64_t)gridDim.x * 256)
        VC[c * mr + r] = isv ? (r < c ? (T)0 : (r == c ? (T)1 : col[r])) : col[r];
}

// W2^T = W^T T for the panel's T without forming T: T^-1 = diag(1/tau) + striu(V^T V), so
// each row x of W2^T solves x T^-1 = w, i.e. x_j = tau_j (w_j - sum_{i<j} x_i G_ij); a
// reflector with tau = 0 (the identity) contributes x_j = 0.  One thread per row.
template <typename T>
__global__ __launch_bounds__(256) void k_apply_Tinv(const T* __restrict__ Wt, int64_t n, int nb,
                                                    const T* __restrict__ G, int ldg,
                                                    const T* __restrict__ tau,
                                                    T* __restrict__ W2t) {
    __shared__ T Gs[NBP * NBP];
    __shared__ T ts[NBP];
    for (int o = threadIdx.x; o < nb * nb; o += 256) Gs[o] = G[(o / nb) * ldg + (o % nb)];
    for (int o = threadIdx.x; o < nb; o += 256) ts[o] = tau[o];
    __syncthreads();
    const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (row >= n) return;
    const T* w = Wt + row * nb;
    T* x = W2t + row * nb;
    T xs[NBP];
#pragma unroll
    for (int j = 0; j < NBP; ++j) {
        if (j < nb) {
            T sacc = w[j];
#pragma unroll
            for (int i = 0; i < j; ++i) sacc -= xs[i] * Gs[i * nb + j];
            xs[j] = ts[j] * sacc;
            x[j] = xs[j];
        }
    }
}

// row-major m x n -> column-major (ld m), 64 x 64 tiles through LDS.  *nonfinite is set
// to 1 when an entry is not finite (a NaN or an infinity anywhere in [A B] reaches the
// sketch: each row of the transformed matrix enters s sketch rows with a +-1 weight, so
// this check costs no pass of its own)
template <typename T>
__global__ __launch_bounds__(256) void k_to_colmajor(const T* __restrict__ A, int64_t m,
                                                     int64_t n, T* __restrict__ Ac,
                                                     int* __restrict__ nonfinite) {
    __shared__ T tile[64][65];
    const int64_t r0 = (int64_t)blockIdx.y * 64, c0 = (int64_t)blockIdx.x * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    int bad = 0;
    for (int i = ty; i < 64; i += 4) {
        const int64_t r = r0 + i, c = c0 + tx;
        if (r < m && c < n) {
            const T v = A[r * n + c];
            bad |= !isfinite(v);
            tile[i][tx] = v;
        }
    }
    if (__syncthreads_or(bad) && threadIdx.x == 0) *nonfinite = 1;
    for (int i = ty; i < 64; i += 4) {
        const int64_t c = c0 + i, r = r0 + tx;
        if (r < m && c < n) Ac[c * m + r] = tile[tx][i];
    }
}

template <typename T, int RPT>
void leaf_launch(T* Ac, int64_t m, int64_t jc, int w, T* tau, T* Tl, hipStream_t st) {
    hipLaunchKernelGGL((k_qr_leaf<T, RPT>), dim3(1), dim3(LFT), 0, st, Ac, m, jc, w, tau, Tl);
}

template <typename T>
hipError_t launch_leaf(T* Ac, int64_t m, int64_t jc, int w, T* tau, T* Tl, hipStream_t st) {
    const int64_t rpt = (m - jc + LFT - 1) / LFT;
    if (rpt <= 1)
        leaf_launch<T, 1>(Ac, m, jc, w, tau, Tl, st);
    else if (rpt <= 2)
        leaf_launch<T, 2>(Ac, m, jc, w, tau, Tl, st);
    else if (rpt <= 4)
        leaf_launch<T, 4>(Ac, m, jc, w, tau, Tl, st);
    else if (rpt <= 8)
        leaf_launch<T, 8>(Ac, m, jc, w, tau, Tl, st);
    else if (rpt <= 12)
        leaf_launch<T, 12>(Ac, m, jc, w, tau, Tl, st);
    else if (rpt <= 16)
        leaf_launch<T, 16>(Ac, m, jc, w, tau, Tl, st);
    else if (rpt <= 24)
        leaf_launch<T, 24>(Ac, m, jc, w, tau, Tl, st);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

template <typename T, int RPT>
void narrow_launch(T* Ac, int64_t m, int64_t jc, int w, const T* Tl, int nc, hipStream_t st) {
    hipLaunchKernelGGL((k_narrow_apply<T, RPT>), dim3((unsigned)nc), dim3(LT), 0, st, Ac, m, jc, w,
                       Tl, jc + w);
}

template <typename T>
hipError_t launch_narrow(T* Ac, int64_t m, int64_t jc, int w, const T* Tl, int nc,
                         hipStream_t st) {
    const int64_t rpt = (m - jc + LT - 1) / LT;
    if (rpt <= 1)
        narrow_launch<T, 1>(Ac, m, jc, w, Tl, nc, st);
    else if (rpt <= 2)
        narrow_launch<T, 2>(Ac, m, jc, w, Tl, nc, st);
    else if (rpt <= 4)
        narrow_launch<T, 4>(Ac, m, jc, w, Tl, nc, st);
    else if (rpt <= 8)
        narrow_launch<T, 8>(Ac, m, jc, w, Tl, nc, st);
    else if (rpt <= 12)
        narrow_launch<T, 12>(Ac, m, jc, w, Tl, nc, st);
    else if (rpt <= 16)
        narrow_launch<T, 16>(Ac, m, jc, w, Tl, nc, st);
    else if (rpt <= 24)
        narrow_launch<T, 24>(Ac, m, jc, w, Tl, nc, st);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

template <typename T>
hipError_t gemm_t(bool ta, bool tb, int64_t M, int64_t N, int64_t K, T alpha, const T* A,
                  int64_t lda, const T* B, int64_t ldb, T beta, T* C, int64_t ldc, bool bf16,
                  GemmWs& ws, hipStream_t st) {
    if constexpr (sizeof(T) == 8)
        return gemm_f64(ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, ws, st, 0);
    else
        return gemm_f32(ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, bf16, ws, st, 0);
}

// C -= A B for one panel's K <= 64 reflectors: the tile kernel that reads C once
// (rank_update.hip); the BF16 form keeps the general GEMM, which rounds its operands
template <typename T>
hipError_t rank_update_t(int64_t M, int64_t N, int K, const T* A, int64_t lda, const T* B,
                         int64_t ldb, T* C, int64_t ldc, bool bf16, GemmWs& ws, hipStream_t st) {
    if (!bf16 && K <= 64) return launch_rank_update<T>(M, N, K, A, lda, B, ldb, C, ldc, st);
    return gemm_t<T>(false, false, M, N, K, (T)-1, A, lda, B, ldb, (T)1, C, ldc, bf16, ws, st);
}

// W = C V^T for one panel's K <= 64 reflectors (C: M x N, V: K x N, row-major views):
// the tile kernel with fixed-order partial sums over ranges of N (rank_update.hip); the
// BF16 form keeps the general GEMM
template <typename T>
hipError_t rank_project_t(int64_t M, int64_t N, int K, const T* C, int64_t ldc, const T* V,
                          int64_t ldv, T* W, int64_t ldw, bool bf16, GemmWs& ws, hipStream_t st) {
    if (!bf16 && K <= 64 && rank_project_ws_bytes(M, N, sizeof(T)) <= ws.bytes)
        return launch_rank_project<T>(M, N, K, C, ldc, V, ldv, W, ldw, ws.part, ws.bytes, st);
    return gemm_t<T>(false, true, M, K, N, (T)1, C, ldc, V, ldv, (T)0, W, ldw, bf16, ws, st);
}

template <typename T>
hipError_t launch_Tinv(const T* Wt, int64_t n, int nb, const T* G, int ldg, const T* tau, T* W2t,
                       hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_apply_Tinv<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, Wt, n,
                       nb, G, ldg, tau, W2t);
    return hipGetLastError();
}

// queue block column [j0, j0 + nb) of R_h^-1 on the third stream once the panel's
// columns of R_h are final (FP64 only)
template <typename T>
hipError_t queue_rinv(T* Ac, int64_t m, int64_t d, int64_t j0, int nb, QrWs& ws, hipStream_t st) {
    if constexpr (std::is_same<T, double>::value) {
        if (!ws.Xinv) return hipSuccess;
        SKI_HIP(hipEventRecord(ws.evP, st));
        SKI_HIP(hipStreamWaitEvent(ws.st3, ws.evP, 0));
        return rinv_block(Ac, m, j0, nb, ws.Xinv, d, ws.Zinv, ws.g3, ws.st3);
    }
    return hipSuccess;
}

// the caller's stream waits for every block of R_h^-1
inline hipError_t join_rinv(const QrWs& ws, hipStream_t st) {
    if (!ws.Xinv) return hipSuccess;
    SKI_HIP(hipEventRecord(ws.evI, ws.st3));
    return hipStreamWaitEvent(st, ws.evI, 0);
}

// Column-by-column panels with a look-ahead of one panel.  After panel p is factored, one
// GEMM gives both V^T V (for T) and V^T C of the next panel's columns; those columns are
// updated on the caller's stream, so panel p+1 can be factored at once, while the
// remaining columns are updated on a second stream.  Events keep the order of the updates
// that every column receives (Q_1^T, Q_2^T, ... in sequence).  T is never formed:
// W2^T = W^T T is applied through T^-1 = diag(1/tau) + striu(V^T V).
template <typename T>
hipError_t qr_impl_hh(T* Ac, int64_t m, int64_t ncols, int64_t d, QrWs& ws, bool bf16,
                      hipStream_t st) {
    T* tau = (T*)ws.tau;
    T* Tl = (T*)ws.Tl;
    T* VCb[2] = {(T*)ws.Vt, (T*)ws.Vt2};  // [V^T; C_next^T], 2 NBP x m each
    T* GWb[2] = {(T*)ws.Tp, (T*)ws.Tp2};  // [V^T V; W_next^T], 2 NBP x NBP each
    hipStream_t s2 = ws.st2;
    int64_t p = 0;
    bool pending_rest = false;  // a remaining-columns update is queued on s2
    for (int64_t j0 = 0; j0 < d; j0 += NBP, ++p) {
        const int nb = (int)std::min<int64_t>(NBP, d - j0);
        T* VC = VCb[p & 1];
        T* GW = GWb[p & 1];
        for (int jl = 0; jl < nb; jl += NBL) {
            const int64_t jc = j0 + jl;
            const int w = std::min(NBL, nb - jl);
            SKI_HIP(launch_leaf<T>(Ac, m, jc, w, tau, Tl, st));
            const int nc = nb - jl - w;
            if (nc > 0) SKI_HIP(launch_narrow<T>(Ac, m, jc, w, Tl, nc, st));
        }
        SKI_HIP(queue_rinv<T>(Ac, m, d, j0, nb, ws, st));
        if (ncols - j0 - nb <= 0) break;
        const int64_t mr = m - j0;
        const int64_t nx0 = j0 + nb;
        const int64_t nx1 = std::min<int64_t>(j0 + 2 * NBP, d);  // next panel's columns
        const int ncn = (int)std::max<int64_t>(0, nx1 - nx0);
        // the previous panel's remaining-columns update covered the next panel: wait for it
        if (pending_rest) SKI_HIP(hipStreamWaitEvent(st, ws.evE[(p - 1) & 1], 0));
        pending_rest = false;
        hipLaunchKernelGGL((k_make_VC<T>),
                           dim3((unsigned)std::min<int64_t>((mr + 255) / 256, 64),
                                (unsigned)(nb + ncn)),
                           dim3(256), 0, st, Ac, m, j0, nb, nx0, VC);
        SKI_HIP(hipGetLastError());
        // [V^T V; W_next^T] = [V^T; C_next^T] V
        SKI_HIP(gemm_t<T>(false, true, nb + ncn, nb, mr, (T)1, VC, mr, VC, mr, (T)0, GW, nb,
                          false, ws.g, st));
        SKI_HIP(hipEventRecord(ws.evF[p & 1], st));
        if (ncn > 0) {
            T* W2n = (T*)ws.W2t;
            SKI_HIP(launch_Tinv<T>(GW + (int64_t)nb * nb, ncn, nb, GW, nb, tau + j0, W2n, st));
            SKI_HIP(rank_update_t<T>(ncn, mr, nb, W2n, nb, VC, mr, Ac + nx0 * m + j0, m, bf16,
                                     ws.g, st));
        }
        if (nx1 < ncols) {
            const int64_t nrest = ncols - nx1;
            T* Ct = Ac + nx1 * m + j0;
            SKI_HIP(hipStreamWaitEvent(s2, ws.evF[p & 1], 0));
            SKI_HIP(rank_project_t<T>(nrest, mr, nb, Ct, m, VC, mr, (T*)ws.Wt2, nb, bf16, ws.g2,
                                      s2));
            SKI_HIP(launch_Tinv<T>((T*)ws.Wt2, nrest, nb, GW, nb, tau + j0, (T*)ws.W2t2, s2));
            SKI_HIP(rank_update_t<T>(nrest, mr, nb, (T*)ws.W2t2, nb, VC, mr, Ct, m, bf16, ws.g2,
                                     s2));
            SKI_HIP(hipEventRecord(ws.evE[p & 1], s2));
            pending_rest = true;
        }
    }
    if (pending_rest) SKI_HIP(hipStreamWaitEvent(st, ws.evE[(p - 1) & 1], 0));
    return join_rinv(ws, st);
}

// CholeskyQR2 panels.  The look-ahead is fused into the panel kernels: the finished panel
// p leaves its explicit reflectors V, its T and W = V^T C_{p+1}; the Gram kernel of panel
// p+1 applies C_{p+1} -= V (T^T W) chunk by chunk before summing its Gram matrix.  The
// columns beyond panel p+1 get Q_p^T on the second stream (W = C^T V, W T and the rank-nb
// update as MFMA GEMMs); events keep every column's updates in panel order.
template <typename T>
hipError_t qr_impl_cqr(T* Ac, int64_t m, int64_t ncols, int64_t d, QrWs& ws, bool bf16,
                       hipStream_t st) {
    T* Vb[2] = {(T*)ws.Vt, (T*)ws.Vt2};  // explicit V of a panel, column-major (ld m - j0)
    T* Tb[2] = {(T*)ws.cqr.Tx, (T*)ws.cqr.Tx + NBP * NBP};
    hipStream_t s2 = ws.st2;
    SKI_HIP(cqr_clear_flag(ws.cqr.flag, st));
    int64_t p = 0;
    bool pending_rest = false;  // the previous panel's remaining-columns update is on s2
    for (int64_t j0 = 0; j0 < d; j0 += NBP, ++p) {
        const int nb = (int)std::min<int64_t>(NBP, d - j0);
        const int64_t mr = m - j0;
        if (p == 0)
            SKI_HIP(cqr_gram_update<T>(Ac, m, -1, j0, nb, nullptr, nullptr, ws.cqr, st));
        else
            SKI_HIP(cqr_gram_update<T>(Ac, m, j0 - NBP, j0, nb, Vb[(p - 1) & 1], Tb[(p - 1) & 1],
                                       ws.cqr, st));
        SKI_HIP(cqr_factor_panel<T>(Ac, m, j0, nb, ws.cqr, Tb[p & 1], st));
        SKI_HIP(queue_rinv<T>(Ac, m, d, j0, nb, ws, st));
        const int64_t nx0 = j0 + nb;
        const int64_t nx1 = std::min<int64_t>(nx0 + NBP, d);  // next panel's columns
        const int nbn = (int)std::max<int64_t>(0, nx1 - nx0);
        // V^T C_next needs the previous panel's update of the next panel's columns
        if (pending_rest) SKI_HIP(hipStreamWaitEvent(st, ws.evE[(p - 1) & 1], 0));
        pending_rest = false;
        SKI_HIP(cqr_finish_panel<T>(Ac, m, j0, nb, nbn, ws.cqr, Vb[p & 1], st));
        if (nx1 < ncols) {
            const int64_t nrest = ncols - nx1;
            T* Ct = Ac + nx1 * m + j0;
            T* V = Vb[p & 1];
            SKI_HIP(hipEventRecord(ws.evF[p & 1], st));
            SKI_HIP(hipStreamWaitEvent(s2, ws.evF[p & 1], 0));
            SKI_HIP(rank_project_t<T>(nrest, mr, nb, Ct, m, V, mr, (T*)ws.Wt2, nb, bf16, ws.g2,
                                      s2));
            SKI_HIP(gemm_t<T>(false, false, nrest, nb, nb, (T)1, (T*)ws.Wt2, nb, Tb[p & 1], NBP,
                              (T)0, (T*)ws.W2t2, nb, false, ws.g2, s2));
            SKI_HIP(rank_update_t<T>(nrest, mr, nb, (T*)ws.W2t2, nb, V, mr, Ct, m, bf16, ws.g2,
                                     s2));
            SKI_HIP(hipEventRecord(ws.evE[p & 1], s2));
            pending_rest = true;
        }
    }
    if (pending_rest) SKI_HIP(hipStreamWaitEvent(st, ws.evE[(p - 1) & 1], 0));
    return join_rinv(ws, st);
}

// Column-pivoted panels (FP64): before each panel its pivots are chosen on the sketch of
// the trailing columns and moved to the front.  The panel is factored by CholeskyQR2 with
// Householder reconstruction when `cqr` is set: its columns are saved first, the host reads
// the panel's failure flag (published into a polled host word, once per panel), and a
// failed panel (the one that holds the rank boundary, typically) is restored and factored
// column by column.
// The trailing matrix (with the ride-along columns) then gets Q^T: W = C^T V and W2 = W T
// on the caller's stream, then the panel's rows of C (R_12, which the sketch update needs)
// there too, while the rows below go to the second stream; the sketch update and the next
// selection overlap that bulk update, and the next column moves wait for it.
hipError_t qr_impl_pivoted(double* Ac, int64_t m, int64_t ncols, int64_t d, QrWs& ws, PivWs& pw,
                           uint64_t seed, bool cqr, HostFlag& pf, int* panels_cqr,
                           hipStream_t st) {
    using T = double;
    T* tau = (T*)ws.tau;
    T* Tl = (T*)ws.Tl;
    T* VC = (T*)ws.Vt;
    T* GW = (T*)ws.Tp;
    T* Tq = (T*)ws.cqr.Tx;
    hipStream_t s2 = ws.st2;
    if (panels_cqr) *panels_cqr = 0;
    SKI_HIP(piv_init(Ac, m, d, seed, pw, ws.g, st));
    int64_t p = 0;
    bool pending = false;  // a bulk update is queued on s2
    for (int64_t j0 = 0; j0 < d; j0 += NBP, ++p) {
        const int nb = (int)std::min<int64_t>(NBP, d - j0);
        const int64_t mr = m - j0;
        SKI_HIP(piv_select(j0, d, nb, pw, st));
        // the moved columns, and the panel, need the previous panel's bulk update
        if (pending) SKI_HIP(hipStreamWaitEvent(st, ws.evE[(p - 1) & 1], 0));
        pending = false;
        SKI_HIP(piv_apply(Ac, m, j0, nb, pw, st));
        bool done = false;
        if (cqr) {
            // the staging buffer of the moves is free again: keep the panel's columns there
            SKI_HIP(hipMemcpyAsync(pw.tA, Ac + j0 * m, (size_t)nb * m * sizeof(T),
                                   hipMemcpyDeviceToDevice, st));
            SKI_HIP(cqr_clear_flag(ws.cqr.flag, st));
            SKI_HIP(cqr_gram_update<T>(Ac, m, -1, j0, nb, nullptr, nullptr, ws.cqr, st));
            SKI_HIP(cqr_factor_panel<T>(Ac, m, j0, nb, ws.cqr, Tq, st));
            SKI_HIP(cqr_finish_panel<T>(Ac, m, j0, nb, 0, ws.cqr, VC, st));
            int failed = 0;
            SKI_HIP(launch_publish_flag(ws.cqr.flag, pf, st));
            SKI_HIP(wait_flag(pf, st, &failed));
            if (failed == 0) {
                done = true;
                if (panels_cqr) ++*panels_cqr;
            } else {
                SKI_HIP(hipMemcpyAsync(Ac + j0 * m, pw.tA, (size_t)nb * m * sizeof(T),
                                       hipMemcpyDeviceToDevice, st));
            }
        }
        const int64_t nrest = ncols - j0 - nb;
        T* Ct = Ac + (j0 + nb) * m + j0;
        if (!done) {
            for (int jl = 0; jl < nb; jl += NBL) {
                const int64_t jc = j0 + jl;
                const int w = std::min(NBL, nb - jl);
                SKI_HIP(launch_leaf<T>(Ac, m, jc, w, tau, Tl, st));
                const int nc = nb - jl - w;
                if (nc > 0) SKI_HIP(launch_narrow<T>(Ac, m, jc, w, Tl, nc, st));
            }
        }
        if (nrest <= 0) break;
        // W = C^T V and W2 = W T (explicit V, ld mr, and T from CholeskyQR2; or the explicit
        // reflectors and T^-1 = diag(1/tau) + striu(V^T V) of the column-by-column panel)
        if (!done) {
            hipLaunchKernelGGL((k_make_VC<T>),
                               dim3((unsigned)std::min<int64_t>((mr + 255) / 256, 64),
                                    (unsigned)nb),
                               dim3(256), 0, st, Ac, m, j0, nb, j0 + nb, VC);
            SKI_HIP(hipGetLastError());
            SKI_HIP(gemm_t<T>(false, true, nb, nb, mr, (T)1, VC, mr, VC, mr, (T)0, GW, nb, false,
                              ws.g, st));
        }
        SKI_HIP(rank_project_t<T>(nrest, mr, nb, Ct, m, VC, mr, (T*)ws.Wt2, nb, false, ws.g, st));
        if (done)
            SKI_HIP(gemm_t<T>(false, false, nrest, nb, nb, (T)1, (T*)ws.Wt2, nb, Tq, NBP, (T)0,
                              (T*)ws.W2t2, nb, false, ws.g, st));
        else
            SKI_HIP(launch_Tinv<T>((T*)ws.Wt2, nrest, nb, GW, nb, tau + j0, (T*)ws.W2t2, st));
        // C -= V W2^T: the panel's rows here, the rows below on the second stream
        SKI_HIP(gemm_t<T>(false, false, nrest, nb, nb, (T)-1, (T*)ws.W2t2, nb, VC, mr, (T)1, Ct,
                          m, false, ws.g, st));
        if (mr > nb) {
            SKI_HIP(hipEventRecord(ws.evF[p & 1], st));
            SKI_HIP(hipStreamWaitEvent(s2, ws.evF[p & 1], 0));
            SKI_HIP(rank_update_t<T>(nrest, mr - nb, nb, (T*)ws.W2t2, nb, VC + nb, mr, Ct + nb, m,
                                     false, ws.g2, s2));
            SKI_HIP(hipEventRecord(ws.evE[p & 1], s2));
            pending = true;
        }
        SKI_HIP(piv_update_sketch(Ac, m, j0, nb, d, pw, ws.g, st));
    }
    if (pending) SKI_HIP(hipStreamWaitEvent(st, ws.evE[(p - 1) & 1], 0));
    return hipSuccess;
}

template <typename T>
hipError_t qr_impl(const T* SA, int64_t m, int64_t ncols, int64_t d, QrWs& ws, bool bf16,
                   hipStream_t st) {
    T* Ac = (T*)ws.Ac;  // column-major working copy, ld = m
    SKI_HIP(cqr_clear_flag(ws.nonfinite, st));
    hipLaunchKernelGGL((k_to_colmajor<T>),
                       dim3((unsigned)((ncols + 63) / 64), (unsigned)((m + 63) / 64)), dim3(256), 0,
                       st, SA, m, ncols, Ac, ws.nonfinite);
    SKI_HIP(hipGetLastError());
    if (ws.cqr_panels) return qr_impl_cqr<T>(Ac, m, ncols, d, ws, bf16, st);
    return qr_impl_hh<T>(Ac, m, ncols, d, ws, bf16, st);
}

template <typename T>
__global__ __launch_bounds__(256) void k_extract_Rc(const T* __restrict__ Ac, int64_t m, int64_t d,
                                                    int64_t k, double* __restrict__ R,
                                                    double* __restrict__ c) {
    const int64_t i = blockIdx.x;
    const double dg = (double)Ac[i * m + i];
    const double sg = dg < 0 ? -1.0 : 1.0;
    for (int64_t j = threadIdx.x; j < d; j += 256)
        R[i * d + j] = j < i ? 0.0 : sg * (double)Ac[j * m + i];
    for (int64_t j = threadIdx.x; j < k; j += 256) c[i * k + j] = sg * (double)Ac[(d + j) * m + i];
}

}  // namespace

namespace {

// the workspace's layout from a base address (each piece 256-byte aligned); returns the end
uintptr_t qr_ws_layout(Prec prec, uintptr_t base, int64_t m, int64_t ncols, QrWs& ws) {
    const size_t e = prec == Prec::F64 ? 8 : 4;
    uintptr_t p = base;
    auto take = [&](size_t count) {
        void* q = (void*)p;
        p += ((count * e + 255) / 256) * 256;
        return q;
    };
    ws.Ac = take((size_t)m * ncols);
    ws.Vt = take(2 * (size_t)NBP * m);   // [V^T; C_next^T], two alternating
    ws.Vt2 = take(2 * (size_t)NBP * m);
    ws.W2t = take((size_t)NBP * NBP);    // look-ahead product
    ws.Wt2 = take((size_t)ncols * NBP);  // remaining-columns products
    ws.W2t2 = take((size_t)ncols * NBP);
    ws.Tp = take(2 * NBP * NBP);         // [V^T V; W_next^T], two alternating
    ws.Tp2 = take(2 * NBP * NBP);
    ws.Tl = take(NBL * NBL);
    ws.tau = take((size_t)ncols);
    ws.cqr.Q1 = take((size_t)NBP * m);
    ws.cqr.Gp = take((size_t)cqr_num_chunks(m) * NBP * NBP);
    ws.cqr.G = take(NBP * NBP);
    ws.cqr.R1 = take(NBP * NBP);
    ws.cqr.R1i = take(NBP * NBP);
    ws.cqr.Mx = take(NBP * NBP);
    ws.cqr.Tx = take(2 * NBP * NBP);
    ws.cqr.W = take(NBP * NBP);
    ws.cqr.tau = ws.tau;
    ws.cqr.flag = (int*)take(1);
    ws.cqr.one_pass = (int*)take(1);
    ws.nonfinite = (int*)take(1);
    return p;
}

}  // namespace

// the size is the layout's own end, so the two cannot disagree
size_t qr_ws_bytes(Prec prec, int64_t m, int64_t ncols, size_t* gemm_bytes) {
    const size_t e = prec == Prec::F64 ? 8 : 4;
    *gemm_bytes = gemm_ws_bytes(2 * NBP, NBP, m, e);
    QrWs w;
    return (size_t)qr_ws_layout(prec, 0, m, ncols, w);
}

void qr_ws_carve(Prec prec, void* base, int64_t m, int64_t ncols, QrWs& ws) {
    qr_ws_layout(prec, (uintptr_t)base, m, ncols, ws);
}

hipError_t qr_factor(Prec prec, const void* SA, int64_t m, int64_t ncols, int64_t d, QrWs& ws,
                     hipStream_t st) {
    if (prec == Prec::F64) return qr_impl<double>((const double*)SA, m, ncols, d, ws, false, st);
    return qr_impl<float>((const float*)SA, m, ncols, d, ws, prec == Prec::BF16, st);
}

hipError_t qr_factor_pivoted(const double* SA, int64_t m, int64_t ncols, int64_t d, QrWs& ws,
                             PivWs& pw, uint64_t seed, bool cqr, HostFlag& pf, int* panels_cqr,
                             hipStream_t st) {
    double* Ac = (double*)ws.Ac;
    SKI_HIP(cqr_clear_flag(ws.nonfinite, st));
    hipLaunchKernelGGL((k_to_colmajor<double>),
                       dim3((unsigned)((ncols + 63) / 64), (unsigned)((m + 63) / 64)), dim3(256), 0,
                       st, SA, m, ncols, Ac, ws.nonfinite);
    SKI_HIP(hipGetLastError());
    return qr_impl_pivoted(Ac, m, ncols, d, ws, pw, seed, cqr, pf, panels_cqr, st);
}

namespace {

__global__ void k_publish_flag(const int* __restrict__ src, int32_t* dst, int32_t seq) {
    if (threadIdx.x == 0) *(volatile int32_t*)dst = (int32_t)(seq << 1) | (*src != 0 ? 1 : 0);
}

}  // namespace

hipError_t launch_publish_flag(const int* src, HostFlag& f, hipStream_t st) {
    if (!f.dev) return hipErrorInvalidValue;
    f.seq = (f.seq + 1) & 0x3fffffff;
    hipLaunchKernelGGL(k_publish_flag, dim3(1), dim3(64), 0, st, src, f.dev, f.seq);
    return hipGetLastError();
}

hipError_t wait_flag(HostFlag& f, hipStream_t st, int* flag) {
    auto fresh = [&](int* out) {
        const int32_t w = *f.host;
        if ((w >> 1) != f.seq) return false;
        *out = w & 1;
        return true;
    };
    for (uint32_t spin = 1;; ++spin) {
        if (fresh(flag)) return hipSuccess;
        if ((spin & 255) == 0) {
            const hipError_t q = hipStreamQuery(st);
            if (q == hipErrorNotReady) continue;
            if (q != hipSuccess) return q;
            // the stream has drained: the word must be there once its writes are visible
            SKI_HIP(hipStreamSynchronize(st));
            return fresh(flag) ? hipSuccess : hipErrorUnknown;
        }
    }
}

hipError_t launch_extract_Rc(Prec prec, const QrWs& ws, int64_t m, int64_t d, int64_t k, double* R,
                             double* c, hipStream_t st) {
    if (prec == Prec::F64)
        hipLaunchKernelGGL((k_extract_Rc<double>), dim3((unsigned)d), dim3(256), 0, st,
                           (const double*)ws.Ac, m, d, k, R, c);
    else
        hipLaunchKernelGGL((k_extract_Rc<float>), dim3((unsigned)d), dim3(256), 0, st,
                           (const float*)ws.Ac, m, d, k, R, c);
    return hipGetLastError();
}

}  // namespace ski
