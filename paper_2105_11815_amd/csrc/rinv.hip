// R^-1 built alongside the factorisation of the sketch (Step 2 of Algorithm 1; the
// explicit inverse is the preconditioner of Steps 3-5).
//
// The QR leaves R_h = D R in its working copy (D = diag of the signs of R_h's diagonal;
// R has a non-negative diagonal).  Block column j of R_h (rows 0 .. j0 + nb) is final as
// soon as panel j is factored, so block column j of X = R_h^-1 can be formed then, on a
// stream of its own, while the next panels are factored (the right-looking order of a
// blocked triangular inversion):
//   X_jj = R_jj^-1                                 (one workgroup, LDS),
//   X(0:j0, j) = -X(0:j0, 0:j0) (R_h(0:j0, j) X_jj)  (the inner product on MFMA, then a
//                                                     narrow triangular GEMM).
// At the end R^-1 = X D: column c is scaled by the sign of r_cc, the strictly lower part is
// cleared, and the transpose is written for the R^-T products.
#include "ski_internal.h"
#include "tile64.h"

namespace ski {

namespace {

using namespace tile;

// x if keep, else +0.0, by integer masking (a conditional load would become a branch that
// waits for its own load; the loads below are clamped into the block and issued together)
__device__ __forceinline__ double keep_or_zero(double x, bool keep) {
    return __builtin_bit_cast(double, __builtin_bit_cast(uint64_t, x) & (keep ? ~0ull : 0ull));
}

// X_jj = inverse of the nb x nb diagonal block of R_h at (j0, j0), read from the column-major
// working copy (ld m); identity padding beyond nb; zeros below the diagonal are written too
__global__ __launch_bounds__(256) void k_rinv_diag(const double* __restrict__ Ac, int64_t m,
                                                   int64_t j0, int nb, double* __restrict__ X,
                                                   int64_t d) {
    __shared__ double Rs[PB][PP];
    const int t = threadIdx.x;
    {
        double v[PB * PB / 256];
#pragma unroll
        for (int q = 0; q < PB * PB / 256; ++q) {
            const int o = t + 256 * q, i = o % PB, j = o / PB;  // column-major walk
            const int jc = j < nb ? j : nb - 1, ic = i < jc ? i : jc;
            v[q] = Ac[(j0 + jc) * m + j0 + ic];
        }
#pragma unroll
        for (int q = 0; q < PB * PB / 256; ++q) {
            const int o = t + 256 * q, i = o % PB, j = o / PB;
            const bool in = i < nb && j < nb && i <= j;
            Rs[i][j] = keep_or_zero(v[q], in) + (!in && i == j ? 1.0 : 0.0);
        }
    }
    __syncthreads();
    tile_trinv(Rs, t, false);
    for (int o = t; o < PB * PB; o += 256) {
        const int i = o / PB, j = o % PB;
        if (i < nb && j < nb) X[(j0 + i) * d + j0 + j] = i <= j ? Rs[i][j] : 0.0;
    }
}

// Z(r, :) = R_h(r, j0 : j0 + nb) X_jj for the rows r < j0 (64 per workgroup); Z row-major,
// ld PB, columns from nb on are zero
__global__ __launch_bounds__(256) void k_rinv_panel(const double* __restrict__ Ac, int64_t m,
                                                    int64_t j0, int nb,
                                                    const double* __restrict__ X, int64_t d,
                                                    double* __restrict__ Z) {
    __shared__ double Ts[PB][PP];
    __shared__ double Xs[PB][PP];
    const int t = threadIdx.x;
    const int64_t r0 = (int64_t)blockIdx.x * PB;
    {
        double tv[PB * PB / 256], xv[PB * PB / 256];
#pragma unroll
        for (int q = 0; q < PB * PB / 256; ++q) {
            const int o = t + 256 * q;
            const int rr = o % PB, c = o / PB;  // R_h column-major: rows r0 + rr, column c
            const int64_t r = std::min<int64_t>(r0 + rr, j0 - 1);
            tv[q] = Ac[(j0 + (c < nb ? c : nb - 1)) * m + r];
            const int i = o / PB, j = o % PB;   // X_jj row-major
            xv[q] = X[(j0 + (i < nb ? i : nb - 1)) * d + j0 + (j < nb ? j : nb - 1)];
        }
#pragma unroll
        for (int q = 0; q < PB * PB / 256; ++q) {
            const int o = t + 256 * q;
            const int rr = o % PB, c = o / PB;
            Ts[rr][c] = keep_or_zero(tv[q], r0 + rr < j0 && c < nb);
            const int i = o / PB, j = o % PB;
            Xs[i][j] = keep_or_zero(xv[q], i < nb && j < nb);
        }
    }
    __syncthreads();
    tile_mma(Ts, t, [&](int i, int k) { return Ts[i][k]; }, [&](int k, int j) { return Xs[k][j]; },
             KFullUpper{}, [](int, int, double v) { return v; });
    for (int o = t; o < PB * PB; o += 256) {
        const int rr = o / PB, c = o % PB;
        if (r0 + rr < j0) Z[(r0 + rr) * PB + c] = Ts[rr][c];
    }
}

// X <- X D with the strictly lower triangle cleared, XT = X^T; 64 x 64 tiles through LDS
__global__ __launch_bounds__(256) void k_rinv_finish(const double* __restrict__ Ac, int64_t m,
                                                     double* __restrict__ X, int64_t d,
                                                     double* __restrict__ XT) {
    __shared__ double tl[64][65];
    __shared__ double sg[64];
    const int64_t r0 = (int64_t)blockIdx.y * 64, c0 = (int64_t)blockIdx.x * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    if (threadIdx.x < 64) {
        const int64_t c = c0 + threadIdx.x;
        sg[threadIdx.x] = (c < d && Ac[c * m + c] < 0) ? -1.0 : 1.0;
    }
    __syncthreads();
    for (int i = ty; i < 64; i += 4) {
        const int64_t r = r0 + i, c = c0 + tx;
        if (r < d && c < d) {
            const double v = c < r ? 0.0 : X[r * d + c] * sg[tx];
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

}  // namespace

size_t rinv_ws_bytes(int64_t d) { return (size_t)(2 * (4096 + d)) * PB * 8; }

hipError_t rinv_block(const double* Ac, int64_t m, int64_t j0, int nb, double* X, int64_t d,
                      double* Z, GemmWs& g, hipStream_t s) {
    if (nb < 1 || nb > PB || j0 + nb > d) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_rinv_diag, dim3(1), dim3(256), 0, s, Ac, m, j0, nb, X, d);
    SKI_HIP(hipGetLastError());
    if (j0 == 0) return hipSuccess;
    hipLaunchKernelGGL(k_rinv_panel, dim3((unsigned)((j0 + PB - 1) / PB)), dim3(256), 0, s, Ac, m,
                       j0, nb, X, d, Z);
    SKI_HIP(hipGetLastError());
    // X(0:j0, j0:j0+nb) = -X(0:j0, 0:j0) Z (X upper triangular; the product reads only the
    // columns below j0)
    return gemm_ts_f64(false, j0, nb, j0, -1.0, X, d, Z, PB, 0.0, X + j0, d, g, s, GEMM_A_UPPER);
}

hipError_t rinv_finish(const double* Ac, int64_t m, int64_t d, double* X, double* XT,
                       hipStream_t st) {
    if (d <= 0) return hipSuccess;
    const unsigned nblk = (unsigned)((d + 63) / 64);
    hipLaunchKernelGGL(k_rinv_finish, dim3(nblk, nblk), dim3(256), 0, st, Ac, m, X, d, XT);
    return hipGetLastError();
}

}  // namespace ski
