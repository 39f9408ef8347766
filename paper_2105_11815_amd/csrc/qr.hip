// Step 2 of Algorithm 1: Householder QR (no pivoting) of the m x (d+k) sketch
// [SA Sb], in place, blocked as in LAPACK's DGEQRF (the factorisation the paper's dense
// solver uses when A is full rank), so that R sits in the upper triangle and Q^T S b in
// the last k columns.
//
// Reflectors follow the LAPACK convention: for x = [alpha; x2],
//   beta = -sign(alpha) ||x||, tau = (beta - alpha)/beta, v = [1; x2/(alpha - beta)],
// H = I - tau v v^T, and are stored in place below the diagonal (implicit unit diagonal).
// A block of reflectors H_1 ... H_b = I - V T V^T with T upper triangular (the forward
// columnwise compact-WY form); applying Q^T to C is C - V T^T V^T C.
//
// Blocking: outer panels of NB columns.  Inside a panel, leaves of 4 columns are factored
// by one workgroup with the leaf's rows held in registers (one reduction per column: the
// squared norm below the diagonal and the column's inner products with the other leaf
// columns); each leaf's block reflector is applied to the rest of the panel by two small
// streaming kernels (partial V^T C over row blocks, then a fixed-order sum, T^T and the
// rank-4 update).  After the panel, T is formed from V^T V and the taus, and the
// trailing columns (including the right-hand sides) get Q^T through three MFMA GEMMs.
// Every sum is in a fixed order: the factorisation is deterministic.
#include "ski_internal.h"

namespace ski {

namespace {

constexpr int NBL = 4;       // leaf width
constexpr int LT = 512;      // leaf threads
constexpr int NBP = 64;      // outer panel width
constexpr int RB = 64;       // rows per workgroup in the narrow kernels

template <typename T>
__device__ __forceinline__ T vval(const T* SA, int64_t ld, int64_t r, int64_t c) {
    // element (r, c) of the explicit reflector block whose origin is at SA
    if (r < c) return (T)0;
    if (r == c) return (T)1;
    return SA[r * ld + c];
}

// leaf: factor columns [jc, jc+w) (w <= NBL) over rows [jc, m); taus -> tau[jc..]
template <typename T, int RPT>
__global__ __launch_bounds__(LT) void k_qr_leaf(T* __restrict__ SA, int64_t ld, int64_t m,
                                                int64_t jc, int w, T* __restrict__ tau) {
    __shared__ T red[2][LT / 64][NBL];
    __shared__ T rowb[2][NBL];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t mrem = m - jc;
    T* base = SA + jc * ld + jc;
    T P[RPT][NBL];
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
        const int64_t r = tid + (int64_t)LT * u;
#pragma unroll
        for (int c = 0; c < NBL; ++c) P[u][c] = (r < mrem && c < w) ? base[r * ld + c] : (T)0;
    }
    // fully unrolled over the leaf's columns so that every register-array index is static
#pragma unroll
    for (int jj = 0; jj < NBL; ++jj) {
        if (jj >= w) break;
        const int buf = jj & 1;
        T s[NBL];
#pragma unroll
        for (int c = 0; c < NBL; ++c) s[c] = 0;
#pragma unroll
        for (int u = 0; u < RPT; ++u) {
            const int64_t r = tid + (int64_t)LT * u;
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
                for (int q = 0; q < LT / 64; ++q) a += red[buf][q][c];
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
        T wc[NBL];
#pragma unroll
        for (int c = 0; c < NBL; ++c) wc[c] = (c > jj) ? rowb[buf][c] + tot[c] * scal : (T)0;
#pragma unroll
        for (int u = 0; u < RPT; ++u) {
            const int64_t r = tid + (int64_t)LT * u;
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
        if (tid == 0) tau[jc + jj] = tj;
    }
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
        const int64_t r = tid + (int64_t)LT * u;
        if (r < mrem)
#pragma unroll
            for (int c = 0; c < NBL; ++c)
                if (c < w) base[r * ld + c] = P[u][c];
    }
}

// partial W_g = V^T C over row block g: V = reflector block at (r0, vc) of width w,
// C = columns [c0, c0+nc) over rows [r0, m).  part: [G][w][nc]
template <typename T>
__global__ __launch_bounds__(256) void k_narrow_partial(const T* __restrict__ SA, int64_t ld,
                                                        int64_t r0, int64_t m, int64_t vc, int w,
                                                        int64_t c0, int nc, T* __restrict__ part) {
    const int64_t g = blockIdx.x;
    const int64_t rb0 = g * RB, rb1 = std::min<int64_t>(m - r0, rb0 + RB);
    const T* V = SA + r0 * ld + vc;
    const T* C = SA + r0 * ld + c0;
    for (int o = threadIdx.x; o < w * nc; o += 256) {
        const int a = o / nc, c = o - a * nc;
        T acc = 0;
        for (int64_t r = rb0; r < rb1; ++r) acc += vval(V, ld, r, (int64_t)a) * C[r * ld + c];
        part[(g * w + a) * nc + c] = acc;
    }
}

// W = sum_g part_g (fixed order), W2 = T^T W with T the leaf block (tau-based recurrence
// rebuilt from the leaf's V: T is passed precomputed in Tl[w][w])
template <typename T>
__global__ __launch_bounds__(256) void k_narrow_reduce(const T* __restrict__ part, int64_t G,
                                                       int w, int nc, const T* __restrict__ Tl,
                                                       int ldt, T* __restrict__ W2) {
    __shared__ T Ws[NBL * NBP];
    for (int o = threadIdx.x; o < w * nc; o += 256) {
        T s = 0;
        for (int64_t g = 0; g < G; ++g) s += part[g * w * nc + o];
        Ws[o] = s;
    }
    __syncthreads();
    for (int o = threadIdx.x; o < w * nc; o += 256) {
        const int a = o / nc, c = o - a * nc;
        T s = 0;
        for (int b = 0; b <= a; ++b) s += Tl[b * ldt + a] * Ws[b * nc + c];
        W2[o] = s;
    }
}

// C -= V W2 over rows [r0, m)
template <typename T>
__global__ __launch_bounds__(256) void k_narrow_update(T* __restrict__ SA, int64_t ld, int64_t r0,
                                                       int64_t m, int64_t vc, int w, int64_t c0,
                                                       int nc, const T* __restrict__ W2) {
    const int64_t rows = m - r0;
    const T* V = SA + r0 * ld + vc;
    T* C = SA + r0 * ld + c0;
    const int64_t total = rows * nc;
    for (int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x; o < total;
         o += (int64_t)gridDim.x * 256) {
        const int64_t r = o / nc;
        const int c = (int)(o - r * nc);
        T s = 0;
        for (int a = 0; a < w; ++a) s += vval(V, ld, r, (int64_t)a) * W2[a * nc + c];
        C[r * ld + c] -= s;
    }
}

// partial Gram matrix of the panel's reflectors: G_g = V^T V over row block g (upper)
template <typename T>
__global__ __launch_bounds__(256) void k_gram_partial(const T* __restrict__ SA, int64_t ld,
                                                      int64_t j0, int64_t m, int nb,
                                                      T* __restrict__ part) {
    const int64_t g = blockIdx.x;
    const int64_t rb0 = g * RB, rb1 = std::min<int64_t>(m - j0, rb0 + RB);
    const T* V = SA + j0 * ld + j0;
    for (int o = threadIdx.x; o < nb * nb; o += 256) {
        const int a = o / nb, b = o - a * nb;
        T acc = 0;
        if (a < b)
            for (int64_t r = std::max<int64_t>(rb0, b); r < rb1; ++r)
                acc += vval(V, ld, r, (int64_t)a) * vval(V, ld, r, (int64_t)b);
        part[g * nb * nb + o] = acc;
    }
}

// T of the panel from G = V^T V and tau: T_ii = tau_i, T[0:i, i] = -tau_i T[0:i,0:i] G[0:i, i]
template <typename T>
__global__ __launch_bounds__(256) void k_form_T(const T* __restrict__ part, int64_t G, int nb,
                                                const T* __restrict__ tau, T* __restrict__ Tp) {
    __shared__ T Gs[NBP * NBP];
    __shared__ T Ts[NBP * NBP];
    for (int o = threadIdx.x; o < nb * nb; o += 256) {
        T s = 0;
        for (int64_t g = 0; g < G; ++g) s += part[g * nb * nb + o];
        Gs[o] = s;
        Ts[o] = 0;
    }
    __syncthreads();
    for (int i = 0; i < nb; ++i) {
        const T ti = tau[i];
        // y = T[0:i,0:i] G[0:i, i]; T[0:i, i] = -ti y
        if (threadIdx.x < i) {
            const int a = threadIdx.x;
            T y = 0;
            for (int b = a; b < i; ++b) y += Ts[a * nb + b] * Gs[b * nb + i];
            Ts[a * nb + i] = -ti * y;
        }
        if (threadIdx.x == 0) Ts[i * nb + i] = ti;
        __syncthreads();
    }
    for (int o = threadIdx.x; o < nb * nb; o += 256) Tp[o] = Ts[o];
}

// leaf T (w x w) from the leaf's reflectors, computed the same way on one row-block pass
template <typename T>
hipError_t leaf_T(const T* SA, int64_t ld, int64_t jc, int64_t m, int w, const T* tau, T* part,
                  T* Tl, hipStream_t st) {
    const int64_t G = (m - jc + RB - 1) / RB;
    hipLaunchKernelGGL((k_gram_partial<T>), dim3((unsigned)G), dim3(256), 0, st, SA, ld, jc, m, w,
                       part);
    hipLaunchKernelGGL((k_form_T<T>), dim3(1), dim3(256), 0, st, part, G, w, tau + jc, Tl);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_leaf(T* SA, int64_t ld, int64_t m, int64_t jc, int w, T* tau, hipStream_t st) {
    const int64_t mrem = m - jc;
    const int64_t rpt = (mrem + LT - 1) / LT;
#define SKI_LEAF(R)                                                                            \
    hipLaunchKernelGGL((k_qr_leaf<T, R>), dim3(1), dim3(LT), 0, st, SA, ld, m, jc, w, tau); \
    return hipGetLastError()
    if (rpt <= 1) { SKI_LEAF(1); }
    if (rpt <= 2) { SKI_LEAF(2); }
    if (rpt <= 4) { SKI_LEAF(4); }
    if (rpt <= 8) { SKI_LEAF(8); }
    if (rpt <= 12) { SKI_LEAF(12); }
    if (rpt <= 16) { SKI_LEAF(16); }
    if (rpt <= 24) { SKI_LEAF(24); }
#undef SKI_LEAF
    return hipErrorInvalidValue;
}

template <typename T>
hipError_t gemm_t(bool ta, bool tb, int64_t M, int64_t N, int64_t K, T alpha, const T* A,
                  int64_t lda, const T* B, int64_t ldb, T beta, T* C, int64_t ldc, bool bf16,
                  GemmWs& ws, hipStream_t st, int unitA) {
    if constexpr (sizeof(T) == 8)
        return gemm_f64(ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, ws, st, unitA);
    else
        return gemm_f32(ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, bf16, ws, st, unitA);
}

template <typename T>
hipError_t qr_impl(T* SA, int64_t m, int64_t ncols, int64_t d, QrWs& ws, bool bf16,
                   hipStream_t st) {
    const int64_t ld = ncols;
    T* tau = (T*)ws.ddiag;
    T* Tp = (T*)ws.T;      // NBP x NBP panel T
    T* Tl = (T*)ws.Y;      // NBL x NBL leaf T
    T* W = (T*)ws.W;       // NBP x ncols
    T* W2 = W + (int64_t)NBP * ncols;
    T* part = (T*)ws.V;    // partial sums of the narrow kernels
    for (int64_t j0 = 0; j0 < d; j0 += NBP) {
        const int nb = (int)std::min<int64_t>(NBP, d - j0);
        for (int jl = 0; jl < nb; jl += NBL) {
            const int64_t jc = j0 + jl;
            const int w = std::min(NBL, nb - jl);
            SKI_HIP(launch_leaf<T>(SA, ld, m, jc, w, tau, st));
            const int nc = nb - jl - w;
            if (nc > 0) {
                SKI_HIP(leaf_T<T>(SA, ld, jc, m, w, tau, part, Tl, st));
                const int64_t G = (m - jc + RB - 1) / RB;
                hipLaunchKernelGGL((k_narrow_partial<T>), dim3((unsigned)G), dim3(256), 0, st, SA,
                                   ld, jc, m, jc, w, jc + w, nc, part);
                hipLaunchKernelGGL((k_narrow_reduce<T>), dim3(1), dim3(256), 0, st, part, G, w, nc,
                                   Tl, w, W2);
                const int64_t tot = (m - jc) * nc;
                const unsigned gu = (unsigned)std::min<int64_t>((tot + 255) / 256, 4096);
                hipLaunchKernelGGL((k_narrow_update<T>), dim3(gu), dim3(256), 0, st, SA, ld, jc, m,
                                   jc, w, jc + w, nc, W2);
                SKI_HIP(hipGetLastError());
            }
        }
        const int64_t n_rem = ncols - j0 - nb;
        if (n_rem > 0) {
            // T of the panel from V^T V
            const int64_t G = (m - j0 + RB - 1) / RB;
            hipLaunchKernelGGL((k_gram_partial<T>), dim3((unsigned)G), dim3(256), 0, st, SA, ld, j0,
                               m, nb, part);
            hipLaunchKernelGGL((k_form_T<T>), dim3(1), dim3(256), 0, st, part, G, nb, tau + j0, Tp);
            SKI_HIP(hipGetLastError());
            const T* V = SA + j0 * ld + j0;
            T* C = SA + j0 * ld + j0 + nb;
            const int64_t mr = m - j0;
            // W = V^T C ; W2 = T^T W ; C -= V W2
            SKI_HIP(gemm_t<T>(true, false, nb, n_rem, mr, (T)1, V, ld, C, ld, (T)0, W, n_rem, bf16,
                              ws.g, st, 1));
            SKI_HIP(gemm_t<T>(true, false, nb, n_rem, nb, (T)1, Tp, nb, W, n_rem, (T)0, W2, n_rem,
                              false, ws.g, st, 0));
            SKI_HIP(gemm_t<T>(false, false, mr, n_rem, nb, (T)-1, V, ld, W2, n_rem, (T)1, C, ld,
                              bf16, ws.g, st, 1));
        }
    }
    return hipSuccess;
}

template <typename T>
__global__ __launch_bounds__(256) void k_extract_Rc(const T* __restrict__ SA, int64_t ld,
                                                    int64_t d, int64_t k, double* __restrict__ R,
                                                    double* __restrict__ c) {
    const int64_t i = blockIdx.x;
    const double dg = (double)SA[i * ld + i];
    const double sg = dg < 0 ? -1.0 : 1.0;
    for (int64_t j = threadIdx.x; j < d; j += 256)
        R[i * d + j] = j < i ? 0.0 : sg * (double)SA[i * ld + j];
    for (int64_t j = threadIdx.x; j < k; j += 256) c[i * k + j] = sg * (double)SA[i * ld + d + j];
}

}  // namespace

size_t qr_ws_bytes(Prec prec, int64_t m, int64_t ncols, int64_t d, size_t* gemm_bytes) {
    const size_t e = prec == Prec::F64 ? 8 : 4;
    const int64_t G = (m + RB - 1) / RB;
    size_t part = (size_t)G * std::max<int64_t>((int64_t)NBL * NBP, (int64_t)NBP * NBP) * e;
    // split-K partials of the V^T C product
    *gemm_bytes = gemm_ws_bytes(NBP, ncols, m, e);
    return part;
}

hipError_t qr_factor(Prec prec, void* SA, int64_t m, int64_t ncols, int64_t d, QrWs& ws,
                     hipStream_t st) {
    if (prec == Prec::F64) return qr_impl<double>((double*)SA, m, ncols, d, ws, false, st);
    return qr_impl<float>((float*)SA, m, ncols, d, ws, prec == Prec::BF16, st);
}

hipError_t launch_extract_Rc(Prec prec, const void* SA, int64_t ldsa, int64_t d, int64_t k,
                             double* R, double* c, hipStream_t st) {
    if (prec == Prec::F64)
        hipLaunchKernelGGL((k_extract_Rc<double>), dim3((unsigned)d), dim3(256), 0, st,
                           (const double*)SA, ldsa, d, k, R, c);
    else
        hipLaunchKernelGGL((k_extract_Rc<float>), dim3((unsigned)d), dim3(256), 0, st,
                           (const float*)SA, ldsa, d, k, R, c);
    return hipGetLastError();
}

}  // namespace ski
