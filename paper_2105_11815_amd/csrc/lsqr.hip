// Steps 3-5 of Algorithm 1 on the GPU, all in FP64: x_s = R^-1 c with the early exit on
// ||A x_s - b|| <= tau_a, LSQR (Paige and Saunders) on W = A R^-1 started from y_0 = c,
// stopped by (TC-lsqr), and x = R^-1 (c + delta); plus CG on the preconditioned normal
// equations for the adjoint.
//
// R^-1 is formed once (blocked triangular inversion on the MFMA GEMM) and kept both
// row-major and transposed, so z = R^-1 v and R^-T g are triangle-only streaming GEMVs.
// Any nonsingular P applied consistently as W = A P and x = P y keeps the implicit
// sketching guarantee, so the explicit inverse is an exact preconditioner.
//
// One LSQR iteration for a dense A and one right-hand side reads A once: the fused pass
// computes u_hat = A z - (alpha/beta) u_hat_old row by row and, with the row still in
// registers, accumulates g = A^T u_hat into per-workgroup partials that a second kernel
// sums in a fixed order.  The scalar recurrences run on the device; the host only reads a
// status word every few iterations.  Every reduction has a fixed order: results are
// bitwise reproducible run to run.
#include "ski_internal.h"
#include "lsqr.h"
#include "tile64.h"

namespace ski {

namespace {

constexpr int DB = 64;  // diagonal block of the triangular inversion

// invert the 64 x 64 diagonal blocks of upper-triangular R (diag + diag_add) into X (row-major
// d x d): one workgroup per block, recursive doubling on the block in LDS; a partial last
// block is padded with the identity
__global__ __launch_bounds__(256) void k_trtri_diag(const double* __restrict__ R, int64_t d,
                                                    const double* __restrict__ diag_add,
                                                    double* __restrict__ X) {
    using namespace tile;
    __shared__ double Rs[PB][PP];
    const int t = threadIdx.x;
    const int64_t b0 = (int64_t)blockIdx.x * DB;
    const int nb = (int)std::min<int64_t>(DB, d - b0);
    for (int o = t; o < PB * PB; o += 256) {
        const int i = o / PB, j = o % PB;
        double v = i == j ? 1.0 : 0.0;
        if (i < nb && j < nb && i <= j) {
            v = R[(b0 + i) * d + b0 + j];
            if (i == j && diag_add) v += diag_add[b0 + i];
        }
        Rs[i][j] = v;
    }
    __syncthreads();
    tile_trinv(Rs, t, false);
    for (int o = t; o < PB * PB; o += 256) {
        const int i = o / PB, j = o % PB;
        if (i < nb && j < nb) X[(b0 + i) * d + b0 + j] = i <= j ? Rs[i][j] : 0.0;
    }
}

// X: zero the strictly lower triangle; XT = X^T; 64 x 64 tiles through LDS so that both
// the reads and the transposed writes are row-contiguous
__global__ __launch_bounds__(256) void k_zero_lower_and_transpose(double* __restrict__ X,
                                                                  int64_t d,
                                                                  double* __restrict__ XT) {
    __shared__ double tl[64][65];
    const int64_t r0 = (int64_t)blockIdx.y * 64, c0 = (int64_t)blockIdx.x * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int i = ty; i < 64; i += 4) {
        const int64_t r = r0 + i, c = c0 + tx;
        if (r < d && c < d) {
            const double v = c < r ? 0.0 : X[r * d + c];
            X[r * d + c] = v;
            tl[i][tx] = v;
        }
    }
    __syncthreads();
    for (int i = ty; i < 64; i += 4) {
        const int64_t c = c0 + i, r = r0 + tx;
        if (r < d && c < d) XT[c * d + r] = tl[tx][i];
    }
}

__global__ __launch_bounds__(256) void k_fill_f64(double* p, int64_t n, double v) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        p[i] = v;
}

hipError_t trtri_rec(const double* R, int64_t d, int64_t lo, int64_t hi, double* X, double* tmp,
                     GemmWs& ws, hipStream_t st) {
    const int64_t n = hi - lo;
    if (n <= DB) return hipSuccess;  // diagonal blocks done by k_trtri_diag
    int64_t mid = lo + ((n / 2 + DB - 1) / DB) * DB;
    if (mid >= hi) mid = hi - DB;
    SKI_HIP(trtri_rec(R, d, lo, mid, X, tmp, ws, st));
    SKI_HIP(trtri_rec(R, d, mid, hi, X, tmp, ws, st));
    const int64_t n1 = mid - lo, n2 = hi - mid;
    // X12 = -X11 (R12 X22): tmp = R12 X22 (n1 x n2), then X12 = -X11 tmp
    // (X22 and X11 are upper triangular: the GEMMs skip their zero blocks)
    SKI_HIP(gemm_f64(false, false, n1, n2, n2, 1.0, R + lo * d + mid, d, X + mid * d + mid, d, 0.0,
                     tmp, n2, ws, st, 0, GEMM_B_UPPER));
    SKI_HIP(gemm_f64(false, false, n1, n2, n1, -1.0, X + lo * d + lo, d, tmp, n2, 0.0,
                     X + lo * d + mid, d, ws, st, 0, GEMM_A_UPPER));
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// triangular GEMV y = s * M x over the triangle only: a workgroup of four waves takes the
// row pair (i, d-1-i), so every workgroup reads d+1 entries; every lane issues its loads
// for both rows before it adds.  With PERM (a column-pivoted factor), the upper product
// scatters its output to y[perm[i]] and the lower one gathers its input from x[perm[j]].
constexpr int TG = 256;
template <bool PERM>
__global__ __launch_bounds__(TG) void k_tri_gemv(const double* __restrict__ M, int64_t d, int upper,
                                                 const double* __restrict__ x, int64_t ldx,
                                                 double* __restrict__ y, int64_t ldy, double s,
                                                 const int32_t* __restrict__ done,
                                                 const int32_t* __restrict__ perm) {
    if (done && *done) return;
    auto xi = [&](int64_t j) -> int64_t { return (PERM && !upper) ? (int64_t)perm[j] : j; };
    auto yi = [&](int64_t i) -> int64_t { return (PERM && upper) ? (int64_t)perm[i] : i; };
    __shared__ double sh[TG / 64][2];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t npairs = (d + 1) / 2;
    for (int64_t p = blockIdx.x; p < npairs; p += gridDim.x) {
        const int64_t i0 = p, i1 = d - 1 - p;
        const bool two = i1 != i0;
        double acc[2] = {0.0, 0.0};
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            if (t == 1 && !two) break;
            const int64_t i = t ? i1 : i0;
            const int64_t j0 = upper ? i : 0, j1 = upper ? d : i + 1;
            const double* row = M + i * d;
            double a = 0;
            int64_t j = j0 + tid;
            for (; j + 3 * TG < j1; j += 4 * TG) {
                const double m0 = row[j], m1 = row[j + TG], m2 = row[j + 2 * TG], m3 = row[j + 3 * TG];
                const double x0 = x[xi(j) * ldx], x1 = x[xi(j + TG) * ldx];
                const double x2 = x[xi(j + 2 * TG) * ldx], x3 = x[xi(j + 3 * TG) * ldx];
                a += m0 * x0 + m1 * x1 + m2 * x2 + m3 * x3;
            }
            for (; j < j1; j += TG) a += row[j] * x[xi(j) * ldx];
            acc[t] = a;
        }
        acc[0] = wave_sum(acc[0]);
        acc[1] = wave_sum(acc[1]);
        if (lane == 0) {
            sh[wv][0] = acc[0];
            sh[wv][1] = acc[1];
        }
        __syncthreads();
        if (tid == 0) {
            y[yi(i0) * ldy] = s * (((sh[0][0] + sh[1][0]) + sh[2][0]) + sh[3][0]);
            if (two) y[yi(i1) * ldy] = s * (((sh[0][1] + sh[1][1]) + sh[2][1]) + sh[3][1]);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// fused dense pass: u = A z - coef * u_old (in place), g partials and ||u||^2 partials.
// A is streamed once with non-temporal loads (it is not reused before it leaves the
// caches); with VEC = 2 each lane loads 16-byte column pairs (needs an even lda and a
// 16-byte aligned A).  One row per step: its dot product is reduced across the
// workgroup while the next row's loads are in flight; the row stays in registers for
// g += A[i,:]^T u_i.
typedef double dvec2 __attribute__((ext_vector_type(2)));

template <int VEC>
struct RowT;
template <>
struct RowT<1> {
    using type = double;
};
template <>
struct RowT<2> {
    using type = dvec2;
};

template <int CPT, int VEC>
__global__ __launch_bounds__(256) void k_lsqr_pass(const double* __restrict__ A, int64_t lda,
                                                   int64_t n, int64_t d,
                                                   const double* __restrict__ z,
                                                   double* __restrict__ u,
                                                   const LsqrState* __restrict__ stt,
                                                   int64_t rows_per_wg, double* __restrict__ gpart,
                                                   double* __restrict__ upart, int use_coef_m1) {
    if (stt->done) return;
    using V = typename RowT<VEC>::type;
    constexpr int H = CPT / VEC;  // vector loads per row per thread
    __shared__ double red[2][4];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const double coef = use_coef_m1 ? -1.0 : stt->coef;
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_wg;
    const int64_t r1 = std::min(n, r0 + rows_per_wg);
    // thread's columns: VEC consecutive columns starting at VEC * (tid + 256 q), q < H
    V zr[H], g[H], cur[H], nxt[H];
    double uo = 0.0, un = 0.0;
#pragma unroll
    for (int q = 0; q < H; ++q) {
        const int64_t c = VEC * (tid + 256 * (int64_t)q);
        V zv, zero;
        if constexpr (VEC == 1) {
            zv = c < d ? z[c] : 0.0;
            zero = 0.0;
        } else {
            zv = dvec2{c < d ? z[c] : 0.0, c + 1 < d ? z[c + 1] : 0.0};
            zero = dvec2{0.0, 0.0};
        }
        zr[q] = zv;
        g[q] = zero;
    }
    auto load = [&](V (&dst)[H], double& uu, int64_t r) {
#pragma unroll
        for (int q = 0; q < H; ++q) {
            const int64_t c = VEC * (tid + 256 * (int64_t)q);
            if constexpr (VEC == 1) {
                dst[q] = (c < d && r < r1) ? __builtin_nontemporal_load(A + r * lda + c) : 0.0;
            } else {
                // d is even on this path, so a pair is either fully inside or fully outside
                dst[q] = (c < d && r < r1)
                             ? __builtin_nontemporal_load((const dvec2*)(A + r * lda + c))
                             : dvec2{0.0, 0.0};
            }
        }
        uu = r < r1 ? u[r] : 0.0;
    };
    double usq = 0.0;
    int buf = 0;
    if (r0 < r1) load(cur, uo, r0);
    for (int64_t r = r0; r < r1; ++r) {
        if (r + 1 < r1) load(nxt, un, r + 1);
        double p = 0.0;
#pragma unroll
        for (int q = 0; q < H; ++q) {
            if constexpr (VEC == 1)
                p += cur[q] * zr[q];
            else
                p += cur[q].x * zr[q].x + cur[q].y * zr[q].y;
        }
        p = wave_sum(p);
        if (lane == 0) red[buf][wv] = p;
        __syncthreads();
        const double dt = (red[buf][0] + red[buf][1]) + (red[buf][2] + red[buf][3]);
        const double u0 = dt - coef * uo;
#pragma unroll
        for (int q = 0; q < H; ++q) g[q] += cur[q] * u0;
        if (tid == 0) {
            u[r] = u0;
            usq += u0 * u0;
        }
#pragma unroll
        for (int q = 0; q < H; ++q) cur[q] = nxt[q];
        uo = un;
        buf ^= 1;
    }
#pragma unroll
    for (int q = 0; q < H; ++q) {
        const int64_t c = VEC * (tid + 256 * (int64_t)q);
        if constexpr (VEC == 1) {
            if (c < d) gpart[(int64_t)blockIdx.x * d + c] = g[q];
        } else {
            if (c < d) gpart[(int64_t)blockIdx.x * d + c] = g[q].x;
            if (c + 1 < d) gpart[(int64_t)blockIdx.x * d + c + 1] = g[q].y;
        }
    }
    if (tid == 0) upart[blockIdx.x] = usq;
}

// g[c] = sum_g gpart[g][c] and beta2 = sum_g upart[g], each in a fixed order: a
// workgroup sums RC columns; lane t takes column t % RC and the partial rows
// g = t / RC, t / RC + RR, ... (RR = 256 / RC row slots, 128-byte segments per row), then
// the RR slot sums of a column are added in slot order.  Workgroup 0 also sums the
// norm partials.
constexpr int RC = 16;
constexpr int RR = 256 / RC;
__global__ __launch_bounds__(256) void k_reduce_pass(const double* __restrict__ gpart,
                                                     const double* __restrict__ upart,
                                                     int64_t G, int64_t d,
                                                     double* __restrict__ g,
                                                     LsqrState* __restrict__ stt) {
    if (stt->done) return;
    __shared__ double part[RR][RC];
    const int t = threadIdx.x;
    const int cl = t % RC, slot = t / RC;
    const int64_t c = (int64_t)blockIdx.x * RC + cl;
    double s = 0;
    if (c < d) {
        int64_t gq = slot;
        for (; gq + 7 * RR < G; gq += 8 * RR) {
            double a[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) a[u] = gpart[(gq + u * RR) * d + c];
#pragma unroll
            for (int u = 0; u < 8; ++u) s += a[u];
        }
        for (; gq < G; gq += RR) s += gpart[gq * d + c];
    }
    part[slot][cl] = s;
    __syncthreads();
    if (t < RC && c < d) {
        double tot = 0;
        for (int j = 0; j < RR; ++j) tot += part[j][t];
        g[c] = tot;
    }
    if (blockIdx.x == 0) {
        __shared__ double us[256];
        const int64_t u0 = t * G / 256, u1 = (t + 1) * G / 256;
        double su = 0;
        for (int64_t i = u0; i < u1; ++i) su += upart[i];
        us[t] = su;
        __syncthreads();
        for (int off = 128; off > 0; off >>= 1) {
            if (t < off) us[t] = us[t] + us[t + off];
            __syncthreads();
        }
        if (t == 0) stt->beta2 = us[0];
    }
}

// ---------------------------------------------------------------------------
// CSR products (k right-hand sides, vectors row-major with leading dimension k)
// u[i] = (A z)[i] - coef_j u[i] for the SP_R rows of a workgroup; squared-norm partial per
// workgroup.  The rows' nonzeros are contiguous, so all 256 threads stream them in chunks of
// SP_CH (eight loads per thread issued together, then the gathers of z) and leave the
// products in LDS; then lane l of a row's SP_L adds the row's products l, l + SP_L, ... in
// order.  A long row (the power-law workloads reach 500 entries) thus costs a few LDS reads
// per lane instead of a chain of dependent global loads that holds up its workgroup.
constexpr int SP_CH = 2048;
constexpr int SP_R = 64;           // rows per workgroup
constexpr int SP_L = 256 / SP_R;   // lanes per row
__global__ __launch_bounds__(256) void k_spmv_csr(const int64_t* __restrict__ rp,
                                                  const int32_t* __restrict__ ci,
                                                  const double* __restrict__ va, int64_t n, int k,
                                                  const double* __restrict__ z,
                                                  double* __restrict__ u,
                                                  const LsqrState* __restrict__ stt,
                                                  int use_coef_m1, double* __restrict__ upart) {
    __shared__ double prod[SP_CH];
    __shared__ double red[SP_R];
    constexpr int PT = SP_CH / 256;
    const int t = threadIdx.x, grp = t / SP_L, gl = t % SP_L;
    const int64_t r0 = (int64_t)blockIdx.x * SP_R;
    const int64_t i = r0 + grp;
    const int64_t rl = r0 + SP_R < n ? r0 + SP_R : n;
    const int64_t e0 = rp[r0], e1 = rp[rl];                // the workgroup's nonzeros
    const int64_t rb = i < n ? rp[i] : e1, re = i < n ? rp[i + 1] : e1;  // this row's
    const int64_t iu = i < n ? i : n - 1;
    for (int j = 0; j < k; ++j) {
        const bool act = !stt[j].done;
        double sq = 0.0;
        if (act) {
            // the old u, loaded now (clamped row) so that it arrives with the nonzeros
            const double uo = u[iu * k + j];
            double acc = 0.0;
            for (int64_t c0 = e0; c0 < e1; c0 += SP_CH) {
                const int64_t c1 = c0 + SP_CH < e1 ? c0 + SP_CH : e1;
                int cv[PT];
                double vv[PT], zv[PT];
#pragma unroll
                for (int q = 0; q < PT; ++q) {
                    const int64_t e = c0 + t + 256 * q;
                    const int64_t ec = e < c1 ? e : c1 - 1;
                    cv[q] = ci[ec];
                    vv[q] = va[ec];
                }
                // keep the index arithmetic below from being interleaved with the loads
                // (each use would wait for its own load)
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int q = 0; q < PT; ++q) zv[q] = z[(int64_t)cv[q] * k + j];
#pragma unroll
                for (int q = 0; q < PT; ++q) prod[t + 256 * q] = vv[q] * zv[q];
                __syncthreads();
                // this lane's entries rb + gl + SP_L s that lie in [c0, c1), in increasing order
                const int64_t lo = rb > c0 ? rb : c0, hi = re < c1 ? re : c1;
                int64_t e = rb + gl;
                if (e < lo) e += (lo - e + SP_L - 1) / SP_L * SP_L;
                for (; e + 3 * SP_L < hi; e += 4 * SP_L) {
                    const double a0 = prod[e - c0], a1 = prod[e + SP_L - c0];
                    const double a2 = prod[e + 2 * SP_L - c0], a3 = prod[e + 3 * SP_L - c0];
                    acc += a0;
                    acc += a1;
                    acc += a2;
                    acc += a3;
                }
                for (; e < hi; e += SP_L) acc += prod[e - c0];
                __syncthreads();
            }
#pragma unroll
            for (int o = 1; o < SP_L; o <<= 1) acc += __shfl_xor(acc, o, 64);
            if (i < n && gl == 0) {
                const double coef = use_coef_m1 ? -1.0 : stt[j].coef;
                const double v = acc - coef * uo;
                u[i * k + j] = v;
                sq = v * v;
            }
        }
        if (gl == 0) red[grp] = sq;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0;
            for (int q = 0; q < SP_R; ++q) s += red[q];
            upart[(int64_t)blockIdx.x * k + j] = s;
        }
        __syncthreads();
    }
}

// g = A^T u through CSR(A^T): one wave per column of A
__global__ __launch_bounds__(256) void k_spmv_csrT(const int32_t* __restrict__ tp,
                                                   const int32_t* __restrict__ ti,
                                                   const double* __restrict__ tv, int64_t d, int k,
                                                   const double* __restrict__ u,
                                                   double* __restrict__ g,
                                                   const LsqrState* __restrict__ stt) {
    const int lane = threadIdx.x & 63;
    const int64_t c = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6;
    if (c >= d) return;
    for (int j = 0; j < k; ++j) {
        if (stt[j].done) continue;
        double acc = 0;
        for (int64_t e = tp[c] + lane; e < tp[c + 1]; e += 64) acc += tv[e] * u[(int64_t)ti[e] * k + j];
        acc = wave_sum(acc);
        if (lane == 0) g[c * k + j] = acc;
    }
}

// beta2_j = sum of the G partials of column j: one workgroup per column; thread t sums
// the partials t, t + 1024, ... in order, then the wave sums and the 16 wave totals are
// added in a fixed order
__global__ __launch_bounds__(1024) void k_reduce_upart(const double* __restrict__ upart, int64_t G,
                                                       int k, LsqrState* __restrict__ stt) {
    __shared__ double sh[16];
    const int j = blockIdx.x;
    if (stt[j].done) return;
    double s = 0;
    for (int64_t q = threadIdx.x; q < G; q += 1024) s += upart[q * k + j];
    s = wave_sum(s);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) sh[wv] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0;
        for (int q = 0; q < 16; ++q) t += sh[q];
        stt[j].beta2 = t;
    }
}

// row index of every stored entry (for CSR(A^T))
__global__ __launch_bounds__(256) void k_csr_keys(const int64_t* __restrict__ rp,
                                                  const int32_t* __restrict__ ci, int64_t n,
                                                  uint64_t* __restrict__ keys) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e)
        keys[e] = ((uint64_t)(uint32_t)ci[e] << 32) | (uint64_t)e;
}

__global__ __launch_bounds__(256) void k_csrT_fill(const int32_t* __restrict__ payload, int64_t nnz,
                                                   const int64_t* __restrict__ rp, int64_t n,
                                                   const double* __restrict__ va,
                                                   int32_t* __restrict__ ti,
                                                   double* __restrict__ tv) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= nnz) return;
    const int64_t e = (uint32_t)payload[p];
    // row of entry e: last i with rp[i] <= e
    int64_t lo = 0, hi = n;
    while (hi - lo > 1) {
        int64_t mid = (lo + hi) >> 1;
        if (rp[mid] <= e)
            lo = mid;
        else
            hi = mid;
    }
    ti[p] = (int32_t)lo;
    tv[p] = va[e];
}

// ---------------------------------------------------------------------------
// dense multi-RHS helpers
// u = t - coef_j u (n x k) and squared-norm partials per column
__global__ __launch_bounds__(256) void k_combine_u(const double* __restrict__ t,
                                                   double* __restrict__ u, int64_t n, int k,
                                                   const LsqrState* __restrict__ stt,
                                                   int use_coef_m1, double* __restrict__ upart,
                                                   int64_t rows_per_wg) {
    __shared__ double red[256];
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_wg, r1 = std::min(n, r0 + rows_per_wg);
    // thread layout: column j = tid % k' over k' = min(k, 256) lanes, row stride 256 / k'
    for (int j0 = 0; j0 < k; j0 += 256) {
        const int kk = std::min(256, k - j0);
        const int rstride = 256 / kk;
        const int j = j0 + threadIdx.x % kk;
        const int rr = threadIdx.x / kk;
        double sq = 0;
        if (threadIdx.x < kk * rstride && !stt[j].done) {
            const double coef = use_coef_m1 ? -1.0 : stt[j].coef;
            for (int64_t i = r0 + rr; i < r1; i += rstride) {
                const double v = t[i * k + j] - coef * u[i * k + j];
                u[i * k + j] = v;
                sq += v * v;
            }
        }
        red[threadIdx.x] = sq;
        __syncthreads();
        if (threadIdx.x < kk) {
            double s = 0;
            for (int q = 0; q < rstride; ++q) s += red[q * kk + threadIdx.x];
            upart[(int64_t)blockIdx.x * k + j0 + threadIdx.x] = s;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// on-device LSQR scalars, one workgroup per right-hand side j; vectors have stride k
__device__ double block_sum(double v, double* sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wv] = v;
    __syncthreads();
    double s = 0;
    const int nw = blockDim.x >> 6;
    for (int q = 0; q < nw; ++q) s += sh[q];
    return s;
}

// entries per thread kept in registers by the step kernels (1024 threads: d <= 4096)
constexpr int STEP_REG = 4;

// init: beta_1 u_1 = r_0 (u holds r_0, beta2 = ||r_0||^2), wp = R^-T A^T r_0
__global__ __launch_bounds__(1024) void k_lsqr_init(LsqrState* __restrict__ stt, int64_t d, int k,
                                                    const double* __restrict__ wp,
                                                    double* __restrict__ v, double* __restrict__ h,
                                                    double* __restrict__ delta, double tau_a) {
    __shared__ double sh[16];
    const int j = blockIdx.x;
    LsqrState& S = stt[j];
    if (S.done) return;
    const double beta = sqrt(S.beta2);
    if (!isfinite(beta)) {  // r_0 is not finite: the right-hand side holds a NaN or infinity
        if (threadIdx.x == 0) {
            S.rnorm = beta;
            S.done = 1;
            S.status = SKI_EINVAL;
        }
        return;
    }
    if (beta <= tau_a) {  // Step 3: early exit with x_s
        if (threadIdx.x == 0) {
            S.rnorm = beta;
            S.done = 1;
            S.status = SKI_WEARLY;
            S.early = 1;
        }
        return;
    }
    double ss = 0;
    for (int64_t i = threadIdx.x; i < d; i += blockDim.x) {
        const double w = wp[i * k + j] / beta;
        ss += w * w;
    }
    const double alpha = sqrt(block_sum(ss, sh));
    for (int64_t i = threadIdx.x; i < d; i += blockDim.x) {
        const double w = alpha > 0 ? (wp[i * k + j] / beta) / alpha : 0.0;
        v[i * k + j] = w;
        h[i * k + j] = w;
        delta[i * k + j] = 0.0;
    }
    if (threadIdx.x == 0) {
        S.alpha = alpha;
        S.beta = beta;
        S.phibar = beta;
        S.rhobar = alpha;
        S.anorm2 = 0.0;
        S.coef = alpha / beta;
        S.iters = 0;
        S.arnorm = 0.0;
        S.tc = 0.0;
        S.rnorm = beta;
        if (alpha == 0.0) {  // A^T r_0 = 0: x_s is optimal
            S.done = 1;
            S.status = SKI_OK;
        } else if (!isfinite(alpha)) {
            S.done = 1;
            S.status = SKI_EINVAL;
        }
    }
}

// Status word of a step over k > 1 columns (one workgroup each), without a kernel of its
// own: every workgroup counts itself in once its column's state is written (release); in
// the last one (acquire) the first wave reads the columns' done flags, one per lane, and
// a vote ANDs them; it writes the word and re-arms the counter for the next step.  No
// workgroup waits for another.
__device__ __forceinline__ void post_all_done(LsqrState* stt, int k, int32_t* word,
                                              uint32_t* cnt) {
    __shared__ int last;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        last = atomicAdd(cnt, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (!last || threadIdx.x >= 64) return;
    __threadfence();
    int all = 1;
    for (int j0 = 0; j0 < k; j0 += 64) {
        const int j = j0 + (int)threadIdx.x;
        const int jc = j < k ? j : k - 1;
        const int dn =
            __hip_atomic_load(&stt[jc].done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ? 1 : 0;
        all &= __all(dn) ? 1 : 0;
    }
    if (threadIdx.x == 0) {
        *word = all;
        __hip_atomic_store(cnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// one step: u_hat holds W v - alpha u (beta2 = its squared norm), wp = R^-T A^T u_hat
template <int SR>
__global__ __launch_bounds__(1024) void k_lsqr_step(LsqrState* __restrict__ stt, int64_t d, int k,
                                                    const double* __restrict__ wp,
                                                    double* __restrict__ v, double* __restrict__ h,
                                                    double* __restrict__ delta, double tau_r,
                                                    int64_t it_max, int32_t* hflag,
                                                    uint32_t* cnt) {
    __shared__ double sh[16];
    const int j = blockIdx.x;
    LsqrState& S = stt[j];
    if (S.done) {
        if (cnt)
            post_all_done(stt, k, hflag, cnt);
        else if (hflag && threadIdx.x == 0)
            *hflag = 1;
        return;
    }
    const double beta = sqrt(S.beta2);
    const double alpha_old = S.alpha;
    const double rhobar = S.rhobar, phibar = S.phibar, anorm2_old = S.anorm2;
    const int64_t iters_old = S.iters;
    const double ib = beta > 0 ? 1.0 / beta : 0.0;
    // d <= SR * blockDim: each thread's entries are loaded once, all loads issued together
    // (indices clamped), and stay in registers between the norm and the update; the
    // per-thread sums run over the same entries in the same order as the general loops
    const bool reg = d <= (int64_t)SR * blockDim.x;
    double wv[SR], vv[SR], hv[SR], dv[SR];
    double ss = 0;
    if (reg) {
#pragma unroll
        for (int u = 0; u < SR; ++u) {
            const int64_t i = threadIdx.x + (int64_t)u * blockDim.x;
            const int64_t o = (i < d ? i : d - 1) * k + j;
            wv[u] = wp[o];
            vv[u] = v[o];
            hv[u] = h[o];
            dv[u] = delta[o];
        }
#pragma unroll
        for (int u = 0; u < SR; ++u) {
            const double w = wv[u] * ib - beta * vv[u];
            if (threadIdx.x + (int64_t)u * blockDim.x < d) ss += w * w;
        }
    } else {
        for (int64_t i = threadIdx.x; i < d; i += blockDim.x) {
            const double w = wp[i * k + j] * ib - beta * v[i * k + j];
            ss += w * w;
        }
    }
    const double alpha = sqrt(block_sum(ss, sh));
    const double ia = alpha > 0 ? 1.0 / alpha : 0.0;
    // plane rotation eliminating beta
    const double rho = sqrt(rhobar * rhobar + beta * beta);
    const double cs = rhobar / rho, sn = beta / rho;
    const double theta = sn * alpha;
    const double phi = cs * phibar;
    const double t1 = phi / rho, t2 = theta / rho;
    if (reg) {
#pragma unroll
        for (int u = 0; u < SR; ++u) {
            const int64_t i = threadIdx.x + (int64_t)u * blockDim.x;
            if (i < d) {
                const double vn = (wv[u] * ib - beta * vv[u]) * ia;
                delta[i * k + j] = dv[u] + t1 * hv[u];
                h[i * k + j] = vn - t2 * hv[u];
                v[i * k + j] = vn;
            }
        }
    } else {
        for (int64_t i = threadIdx.x; i < d; i += blockDim.x) {
            const double w = wp[i * k + j] * ib - beta * v[i * k + j];
            const double vn = w * ia;
            const double hi = h[i * k + j];
            delta[i * k + j] += t1 * hi;
            h[i * k + j] = vn - t2 * hi;
            v[i * k + j] = vn;
        }
    }
    if (threadIdx.x == 0) {
        const double anorm2 = anorm2_old + alpha_old * alpha_old + beta * beta;
        const double phibar_n = sn * phibar;
        const double arnorm = phibar_n * alpha * fabs(cs);
        const double anorm = sqrt(anorm2);
        const double tc = (phibar_n > 0 && anorm > 0) ? arnorm / (anorm * phibar_n) : 0.0;
        S.anorm2 = anorm2;
        S.rhobar = -cs * alpha;
        S.phibar = phibar_n;
        S.alpha = alpha;
        S.beta = beta;
        S.coef = beta > 0 ? alpha / beta : 0.0;
        S.rnorm = phibar_n;
        S.arnorm = arnorm;
        S.tc = tc;
        S.iters = iters_old + 1;
        if (!isfinite(alpha) || !isfinite(beta) || !isfinite(tc)) {
            // a non-finite iterate never meets (TC-lsqr): stop at once
            S.done = 1;
            S.status = SKI_EINVAL;
        } else if (phibar_n == 0.0 || arnorm == 0.0 || tc <= tau_r) {
            S.done = 1;
            S.status = SKI_OK;
        } else if (iters_old + 1 >= it_max) {
            S.done = 1;
            S.status = SKI_WNOCONV;
        }
        // one right-hand side: this workgroup's state is the whole status word
        if (hflag && !cnt) *hflag = S.done;
    }
    if (cnt) post_all_done(stt, k, hflag, cnt);
}

// y = c + delta (per column) for the final x = R^-1 y, x_s when the early exit was taken
__global__ __launch_bounds__(256) void k_final_y(const LsqrState* __restrict__ stt, int64_t d, int k,
                                                 const double* __restrict__ c,
                                                 const double* __restrict__ delta,
                                                 double* __restrict__ y) {
    const int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (o >= d * k) return;
    const int j = (int)(o % k);
    y[o] = stt[j].early ? c[o] : c[o] + delta[o];
}

// rows through a permutation: scatter dst[perm[i]] = src[i] or gather dst[i] = src[perm[i]]
// (rows x cols, row-major with the given leading dimensions)
__global__ __launch_bounds__(256) void k_permute_rows(const double* __restrict__ src, int64_t lds,
                                                      double* __restrict__ dst, int64_t ldd,
                                                      const int32_t* __restrict__ perm,
                                                      int64_t rows, int64_t cols, int scatter) {
    const int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (o >= rows * cols) return;
    const int64_t i = o / cols, j = o - i * cols;
    if (scatter)
        dst[(int64_t)perm[i] * ldd + j] = src[i * lds + j];
    else
        dst[i * ldd + j] = src[(int64_t)perm[i] * lds + j];
}

__global__ __launch_bounds__(256) void k_fill_rows(double* __restrict__ y, int64_t rows,
                                                   int64_t cols, int64_t ldy, double v) {
    const int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (o >= rows * cols) return;
    const int64_t i = o / cols, j = o - i * cols;
    y[i * ldy + j] = v;
}

__global__ __launch_bounds__(256) void k_scale_copy(const double* __restrict__ x, int64_t rows,
                                                    int64_t cols, int64_t ldx, double s,
                                                    double* __restrict__ y, int64_t ldy) {
    const int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (o >= rows * cols) return;
    const int64_t i = o / cols, j = o - i * cols;
    y[i * ldy + j] = s * x[i * ldx + j];
}

// CG scalars on M y = rhs (M = R^-T A^T A R^-1), one workgroup per column
__global__ __launch_bounds__(1024) void k_cg_init(LsqrState* __restrict__ stt, int64_t d, int k,
                                                  const double* __restrict__ rhs,
                                                  double* __restrict__ r, double* __restrict__ p,
                                                  double* __restrict__ y, double tol) {
    __shared__ double sh[16];
    const int j = blockIdx.x;
    LsqrState& S = stt[j];
    double ss = 0;
    for (int64_t i = threadIdx.x; i < d; i += blockDim.x) {
        const double v = rhs[i * k + j];
        r[i * k + j] = v;
        p[i * k + j] = v;
        y[i * k + j] = 0.0;
        ss += v * v;
    }
    const double rr = block_sum(ss, sh);
    if (threadIdx.x == 0) {
        S.rr = rr;
        S.stop2 = tol * tol * rr;
        S.iters = 0;
        S.rnorm = sqrt(rr);
        S.done = (rr <= S.stop2 || rr == 0.0 || !isfinite(rr)) ? 1 : 0;
        S.status = isfinite(rr) ? SKI_OK : SKI_EINVAL;
        S.early = 0;
    }
}

__global__ __launch_bounds__(1024) void k_cg_step(LsqrState* __restrict__ stt, int64_t d, int k,
                                                  const double* __restrict__ q,
                                                  double* __restrict__ r, double* __restrict__ p,
                                                  double* __restrict__ y, int64_t it_max,
                                                  int32_t* word, uint32_t* cnt) {
    __shared__ double sh[16];
    const int j = blockIdx.x;
    LsqrState& S = stt[j];
    if (S.done) {
        if (cnt) post_all_done(stt, k, word, cnt);
        return;
    }
    const double rr_old = S.rr, stop2 = S.stop2;
    const int64_t iters_old = S.iters;
    // as in the LSQR step: registers for d <= STEP_REG * blockDim, the same sums otherwise
    const bool reg = d <= (int64_t)STEP_REG * blockDim.x;
    double pv[STEP_REG], qv[STEP_REG], rv[STEP_REG], yv[STEP_REG];
    double pq = 0;
    if (reg) {
#pragma unroll
        for (int u = 0; u < STEP_REG; ++u) {
            const int64_t i = threadIdx.x + (int64_t)u * blockDim.x;
            const int64_t o = (i < d ? i : d - 1) * k + j;
            pv[u] = p[o];
            qv[u] = q[o];
            rv[u] = r[o];
            yv[u] = y[o];
        }
#pragma unroll
        for (int u = 0; u < STEP_REG; ++u)
            if (threadIdx.x + (int64_t)u * blockDim.x < d) pq += pv[u] * qv[u];
    } else {
        for (int64_t i = threadIdx.x; i < d; i += blockDim.x) pq += p[i * k + j] * q[i * k + j];
    }
    pq = block_sum(pq, sh);
    const double a = rr_old / pq;
    double ss = 0;
    if (reg) {
#pragma unroll
        for (int u = 0; u < STEP_REG; ++u) {
            const int64_t i = threadIdx.x + (int64_t)u * blockDim.x;
            if (i < d) {
                y[i * k + j] = yv[u] + a * pv[u];
                const double rn = rv[u] - a * qv[u];
                r[i * k + j] = rn;
                rv[u] = rn;
                ss += rn * rn;
            }
        }
    } else {
        for (int64_t i = threadIdx.x; i < d; i += blockDim.x) {
            y[i * k + j] += a * p[i * k + j];
            const double rn = r[i * k + j] - a * q[i * k + j];
            r[i * k + j] = rn;
            ss += rn * rn;
        }
    }
    const double rr_new = block_sum(ss, sh);
    const double bb = rr_new / rr_old;
    if (reg) {
#pragma unroll
        for (int u = 0; u < STEP_REG; ++u) {
            const int64_t i = threadIdx.x + (int64_t)u * blockDim.x;
            if (i < d) p[i * k + j] = rv[u] + bb * pv[u];
        }
    } else {
        for (int64_t i = threadIdx.x; i < d; i += blockDim.x)
            p[i * k + j] = r[i * k + j] + bb * p[i * k + j];
    }
    if (threadIdx.x == 0) {
        S.rr = rr_new;
        S.iters = iters_old + 1;
        S.rnorm = sqrt(rr_new);
        if (!isfinite(rr_new) || !isfinite(a)) {
            S.done = 1;
            S.status = SKI_EINVAL;
        } else if (rr_new <= stop2) {
            S.done = 1;
            S.status = SKI_OK;
        } else if (iters_old + 1 >= it_max) {
            S.done = 1;
            S.status = SKI_WNOCONV;
        }
    }
    if (cnt) post_all_done(stt, k, word, cnt);
}

// one wavefront: lane j reads column j's flag (64 columns per step), a vote ANDs them
__global__ __launch_bounds__(64) void k_all_done(const LsqrState* __restrict__ stt, int k,
                                                 int32_t* __restrict__ flag) {
    int all = 1;
    for (int j0 = 0; j0 < k; j0 += 64) {
        const int j = j0 + (int)threadIdx.x;
        const int dn = j < k ? (stt[j].done ? 1 : 0) : 1;
        all &= __all(dn) ? 1 : 0;
    }
    if (threadIdx.x == 0) *flag = all;
}

}  // namespace

// ---------------------------------------------------------------------------
hipError_t trtri_upper(const double* R, int64_t d, double* Rinv, double* RinvT,
                       const double* diag_add, double* tmp, GemmWs& ws, hipStream_t st) {
    const unsigned nblk = (unsigned)((d + DB - 1) / DB);
    // the recursion multiplies whole square blocks: the strictly lower part must be zero
    const int64_t tot = d * d;
    hipLaunchKernelGGL(k_fill_f64, dim3((unsigned)std::min<int64_t>((tot + 255) / 256, 65536)),
                       dim3(256), 0, st, Rinv, tot, 0.0);
    SKI_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_trtri_diag, dim3(nblk), dim3(256), 0, st, R, d, diag_add, Rinv);
    SKI_HIP(hipGetLastError());
    // the off-diagonal blocks use R with the same perturbed diagonal only through X11, X22
    SKI_HIP(trtri_rec(R, d, 0, d, Rinv, tmp, ws, st));
    hipLaunchKernelGGL(k_zero_lower_and_transpose, dim3(nblk, nblk), dim3(256), 0, st, Rinv, d,
                       RinvT);
    return hipGetLastError();
}

hipError_t launch_tri_gemv(const double* M, int64_t d, bool upper, const double* x, int64_t ldx,
                           double* y, int64_t ldy, double s, const int32_t* done, hipStream_t st,
                           const int32_t* perm) {
    if (d <= 0) return hipSuccess;
    const unsigned g = (unsigned)std::min<int64_t>((d + 1) / 2, 8192);
    if (perm)
        hipLaunchKernelGGL(k_tri_gemv<true>, dim3(g), dim3(TG), 0, st, M, d, upper ? 1 : 0, x, ldx,
                           y, ldy, s, done, perm);
    else
        hipLaunchKernelGGL(k_tri_gemv<false>, dim3(g), dim3(TG), 0, st, M, d, upper ? 1 : 0, x,
                           ldx, y, ldy, s, done, perm);
    return hipGetLastError();
}

hipError_t launch_permute_rows(const double* src, int64_t lds, double* dst, int64_t ldd,
                               const int32_t* perm, int64_t rows, int64_t cols, bool scatter,
                               hipStream_t st) {
    const int64_t tot = rows * cols;
    if (tot <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_permute_rows, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, src,
                       lds, dst, ldd, perm, rows, cols, scatter ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_fill_rows(double* y, int64_t rows, int64_t cols, int64_t ldy, double v,
                            hipStream_t st) {
    const int64_t tot = rows * cols;
    if (tot <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_rows, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, y, rows,
                       cols, ldy, v);
    return hipGetLastError();
}

int lsqr_pass_cpt(int64_t d) {
    const int64_t c = (d + 255) / 256;
    if (c <= 1) return 1;
    if (c <= 2) return 2;
    if (c <= 4) return 4;
    if (c <= 8) return 8;
    if (c <= 16) return 16;
    if (c <= 24) return 24;
    if (c <= 32) return 32;
    return 0;
}

hipError_t launch_pass_kernel(const double* A, int64_t lda, int64_t n, int64_t d, const double* z,
                              double* u, const LsqrState* stt, int64_t G, double* gpart,
                              double* upart, bool coef_m1, hipStream_t st) {
    const int64_t rpw = (n + G - 1) / G;
    const int cpt = lsqr_pass_cpt(d);
    const bool vec2 = (lda % 2 == 0) && (d % 2 == 0) && (((uintptr_t)A & 15) == 0) && cpt >= 2;
#define SKI_PASS(C, VV)                                                                            \
    hipLaunchKernelGGL((k_lsqr_pass<C, VV>), dim3((unsigned)G), dim3(256), 0, st, A, lda, n, d, z, \
                       u, stt, rpw, gpart, upart, coef_m1 ? 1 : 0)
    if (vec2) {
        switch (cpt) {
            case 2: SKI_PASS(2, 2); break;
            case 4: SKI_PASS(4, 2); break;
            case 8: SKI_PASS(8, 2); break;
            case 16: SKI_PASS(16, 2); break;
            case 24: SKI_PASS(24, 2); break;
            case 32: SKI_PASS(32, 2); break;
            default: return hipErrorInvalidValue;
        }
    } else {
        switch (cpt) {
            case 1: SKI_PASS(1, 1); break;
            case 2: SKI_PASS(2, 1); break;
            case 4: SKI_PASS(4, 1); break;
            case 8: SKI_PASS(8, 1); break;
            case 16: SKI_PASS(16, 1); break;
            case 24: SKI_PASS(24, 1); break;
            case 32: SKI_PASS(32, 1); break;
            default: return hipErrorInvalidValue;
        }
    }
#undef SKI_PASS
    return hipGetLastError();
}

hipError_t launch_pass_reduce(const double* gpart, const double* upart, int64_t G, int64_t d,
                              double* g, LsqrState* stt_w, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce_pass, dim3((unsigned)((d + RC - 1) / RC)), dim3(256), 0, st,
                       gpart, upart, G, d, g, stt_w);
    return hipGetLastError();
}

hipError_t launch_lsqr_pass(const double* A, int64_t lda, int64_t n, int64_t d, const double* z,
                            double* u, const LsqrState* stt, int64_t G, double* gpart,
                            double* upart, double* g, LsqrState* stt_w, bool coef_m1,
                            hipStream_t st) {
    SKI_HIP(launch_pass_kernel(A, lda, n, d, z, u, stt, G, gpart, upart, coef_m1, st));
    return launch_pass_reduce(gpart, upart, G, d, g, stt_w, st);
}

hipError_t launch_spmv_csr(const int64_t* rp, const int32_t* ci, const double* va, int64_t n, int k,
                           const double* z, double* u, LsqrState* stt, bool coef_m1,
                           double* upart, hipStream_t st) {
    const int64_t G = (n + SP_R - 1) / SP_R;
    hipLaunchKernelGGL(k_spmv_csr, dim3((unsigned)G), dim3(256), 0, st, rp, ci, va, n, k, z, u, stt,
                       coef_m1 ? 1 : 0, upart);
    SKI_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_reduce_upart, dim3((unsigned)k), dim3(1024), 0, st, upart, G, k, stt);
    return hipGetLastError();
}

int64_t spmv_csr_groups(int64_t n) { return (n + SP_R - 1) / SP_R; }

hipError_t launch_spmv_csrT(const int32_t* tp, const int32_t* ti, const double* tv, int64_t d, int k,
                            const double* u, double* g, const LsqrState* stt, hipStream_t st) {
    const unsigned G = (unsigned)((d + 3) / 4);
    hipLaunchKernelGGL(k_spmv_csrT, dim3(G), dim3(256), 0, st, tp, ti, tv, d, k, u, g, stt);
    return hipGetLastError();
}

hipError_t build_csrT(const int64_t* rp, const int32_t* ci, const double* va, int64_t n, int64_t d,
                      int64_t nnz, uint64_t* keys, uint64_t* keys_tmp, int32_t* table,
                      int32_t* tp, int32_t* payload, int32_t* ti, double* tv, hipStream_t st) {
    hipLaunchKernelGGL(k_csr_keys, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, rp, ci, n,
                       keys);
    SKI_HIP(hipGetLastError());
    SKI_HIP(launch_bucket_sort(keys, nnz, d, keys_tmp, table, tp, payload, st));
    if (nnz > 0)
        hipLaunchKernelGGL(k_csrT_fill, dim3((unsigned)((nnz + 255) / 256)), dim3(256), 0, st,
                           payload, nnz, rp, n, va, ti, tv);
    return hipGetLastError();
}

hipError_t launch_combine_u(const double* t, double* u, int64_t n, int k, const LsqrState* stt,
                            bool coef_m1, double* upart, int64_t G, LsqrState* stt_w,
                            hipStream_t st) {
    const int64_t rpw = (n + G - 1) / G;
    hipLaunchKernelGGL(k_combine_u, dim3((unsigned)G), dim3(256), 0, st, t, u, n, k, stt,
                       coef_m1 ? 1 : 0, upart, rpw);
    SKI_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_reduce_upart, dim3((unsigned)k), dim3(1024), 0, st, upart, G, k, stt_w);
    return hipGetLastError();
}

hipError_t launch_lsqr_init(LsqrState* stt, int64_t d, int k, const double* wp, double* v,
                            double* h, double* delta, double tau_a, hipStream_t st) {
    hipLaunchKernelGGL(k_lsqr_init, dim3((unsigned)k), dim3(1024), 0, st, stt, d, k, wp, v, h, delta,
                       tau_a);
    return hipGetLastError();
}

hipError_t launch_lsqr_step(LsqrState* stt, int64_t d, int k, const double* wp, double* v,
                            double* h, double* delta, double tau_r, int64_t it_max,
                            int32_t* hflag, uint32_t* cnt, hipStream_t st) {
    // 4 entries per thread in registers up to d = 4096, 8 up to 8192 (the same sums: only
    // the loads are batched differently), a loop beyond
    uint32_t* c = (k > 1 && hflag) ? cnt : nullptr;
    if (d > (int64_t)STEP_REG * 1024 && d <= (int64_t)2 * STEP_REG * 1024)
        hipLaunchKernelGGL(k_lsqr_step<2 * STEP_REG>, dim3((unsigned)k), dim3(1024), 0, st, stt, d, k,
                           wp, v, h, delta, tau_r, it_max, hflag, c);
    else
        hipLaunchKernelGGL(k_lsqr_step<STEP_REG>, dim3((unsigned)k), dim3(1024), 0, st, stt, d, k, wp,
                           v, h, delta, tau_r, it_max, hflag, c);
    return hipGetLastError();
}

hipError_t launch_final_y(const LsqrState* stt, int64_t d, int k, const double* c,
                          const double* delta, double* y, hipStream_t st) {
    const int64_t tot = d * k;
    if (tot <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_final_y, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, stt, d, k,
                       c, delta, y);
    return hipGetLastError();
}

hipError_t launch_scale_copy(const double* x, int64_t rows, int64_t cols, int64_t ldx, double s,
                             double* y, int64_t ldy, hipStream_t st) {
    const int64_t tot = rows * cols;
    if (tot == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scale_copy, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, x, rows,
                       cols, ldx, s, y, ldy);
    return hipGetLastError();
}

hipError_t launch_cg_init(LsqrState* stt, int64_t d, int k, const double* rhs, double* r, double* p,
                          double* y, double tol, hipStream_t st) {
    hipLaunchKernelGGL(k_cg_init, dim3((unsigned)k), dim3(1024), 0, st, stt, d, k, rhs, r, p, y, tol);
    return hipGetLastError();
}

hipError_t launch_cg_step(LsqrState* stt, int64_t d, int k, const double* q, double* r, double* p,
                          double* y, int64_t it_max, int32_t* word, uint32_t* cnt,
                          hipStream_t st) {
    hipLaunchKernelGGL(k_cg_step, dim3((unsigned)k), dim3(1024), 0, st, stt, d, k, q, r, p, y,
                       it_max, word, word ? cnt : nullptr);
    return hipGetLastError();
}

hipError_t launch_all_done(const LsqrState* stt, int k, int32_t* flag, hipStream_t st) {
    hipLaunchKernelGGL(k_all_done, dim3(1), dim3(64), 0, st, stt, k, flag);
    return hipGetLastError();
}

}  // namespace ski
