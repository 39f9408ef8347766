// FP64 products with a narrow right operand, for the multi-right-hand-side iterations
// (Algorithm 1 run on k columns at once, and CG on the normal equations for the adjoint):
//   nn: C[M x N] = alpha A B + beta C, A M x K, B K x N        (A Z, R^-1 V, R^-T G)
//   tn: C[M x N] = alpha A^T B + beta C, A stored K x M, B K x N  (A^T U)
// all row-major, N small (the number of right-hand sides).
//
// The general 64 x 64 GEMM tiles waste half their matrix-core work when N = 32 and give
// a 1000 x 1000 times 1000 x 32 product only 16 workgroups.  Here the output tile is
// 32 x 32 (nn) or 64 x 32 (tn), the four waves of a workgroup split the workgroup's
// range of K and sum their tiles through LDS in a fixed order, and a long K may also be
// split over workgroups (partials summed by a second kernel in a fixed order, so results
// are deterministic).  Operands go from global memory straight into the registers of
// v_mfma_f64_16x16x4f64 (lane l supplies row l%16 and k-index l/16 of the A block, k-index
// l/16 and column l%16 of the B block, and receives D[4 r + l/16][l%16] in accumulator
// element r), 32 (nn) or 16 (tn) values of K per step, the next step's loads issued
// before the current step's products.
#include "ski_internal.h"

namespace ski {

namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int TS_THR = 256;
constexpr int NN_KC = 32, NN_NJ = NN_KC / 4;  // K per step, 4-deep MFMA slices per step
constexpr int TN_KC = 16, TN_NJ = TN_KC / 4;

// Operands are read with raw buffer loads: a scalar base (the tile's first row), a
// 32-bit per-lane byte offset and a scalar offset per step, so the loads carry no 64-bit
// addresses; a read past the end of the buffer returns 0.  Rows of A beyond M and
// columns of B beyond N are never masked: they only feed outputs that are not stored.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const double* p, int64_t bytes) {
    const int32_t nr = (int32_t)std::min<int64_t>(std::max<int64_t>(bytes, 0), 0x7fffffff);
    return __builtin_amdgcn_make_buffer_rsrc((void*)p, (short)0, nr, 0x00020000);
}
__device__ __forceinline__ double bload(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}

__device__ __forceinline__ void store_out(int64_t M, int64_t N, int64_t i, int64_t j, double s,
                                          double alpha, double beta, double* C, int64_t ldc,
                                          double* part, int64_t z) {
    if (i >= M || j >= N) return;
    if (part) {
        part[(z * M + i) * N + j] = s;
    } else {
        double o = alpha * s;
        if (beta != 0.0) o += beta * C[i * ldc + j];
        C[i * ldc + j] = o;
    }
}

// the wave's chunks of the workgroup's nfull full chunks: contiguous quarters
__device__ __forceinline__ void wave_chunks(int64_t nfull, int w, int64_t& cs, int64_t& nch) {
    const int64_t per = (nfull + 3) / 4;
    cs = std::min(nfull, w * per);
    nch = std::min(nfull, cs + per) - cs;
}

__global__ __launch_bounds__(TS_THR) void k_ts_nn(int64_t M, int64_t N, int64_t K, int64_t kchunk,
                                                  double alpha, const double* __restrict__ A,
                                                  int64_t lda, const double* __restrict__ B,
                                                  int64_t ldb, double beta, double* __restrict__ C,
                                                  int64_t ldc, double* __restrict__ part, int tri) {
    __shared__ double red[4][16][64];
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int li = lane & 15, lk = lane >> 4;
    const int64_t m0 = (int64_t)blockIdx.x * 32, n0 = (int64_t)blockIdx.y * 32;
    int64_t kb = (int64_t)blockIdx.z * kchunk, ke = std::min(K, kb + kchunk);
    // A(i, k) = 0 for k < i (upper) or k > i (lower) over the tile's rows m0 .. m0 + 31
    if (tri & GEMM_A_UPPER) kb = std::max(kb, m0);
    if (tri & GEMM_A_LOWER) ke = std::min(ke, m0 + 32);
    const int64_t len = std::max<int64_t>(ke - kb, 0);
    const int64_t nfull = len / NN_KC;
    int64_t cs, nch;
    wave_chunks(nfull, w, cs, nch);

    dbl4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[a][b][r] = 0.0;

    // each buffer ends at the last element of its matrix
    const __amdgpu_buffer_rsrc_t ra =
        make_rsrc(A + m0 * lda + kb, ((M - 1 - m0) * lda + K - kb) * 8);
    const __amdgpu_buffer_rsrc_t rb =
        make_rsrc(B + kb * ldb + n0, ((K - 1 - kb) * ldb + N - n0) * 8);
    const uint32_t oa0 = (uint32_t)((li * lda + lk) * 8), oa1 = (uint32_t)(((16 + li) * lda + lk) * 8);
    const uint32_t ob0 = (uint32_t)((lk * ldb + li) * 8), ob1 = (uint32_t)((lk * ldb + 16 + li) * 8);
    double pa[2][NN_NJ], pb[2][NN_NJ], qa[2][NN_NJ], qb[2][NN_NJ];
    auto load = [&](int64_t c, double (&xa)[2][NN_NJ], double (&xb)[2][NN_NJ]) {
        const uint32_t sa = (uint32_t)(NN_KC * c * 8);
#pragma unroll
        for (int j = 0; j < NN_NJ; ++j) {
            const uint32_t sb = (uint32_t)((NN_KC * c + 4 * j) * ldb * 8);
            xa[0][j] = bload(ra, oa0 + 32 * j, sa);
            xa[1][j] = bload(ra, oa1 + 32 * j, sa);
            xb[0][j] = bload(rb, ob0, sb);
            xb[1][j] = bload(rb, ob1, sb);
        }
    };
    auto mma = [&](double (&ya)[2][NN_NJ], double (&yb)[2][NN_NJ]) {
#pragma unroll
        for (int j = 0; j < NN_NJ; ++j)
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ya[a][j], yb[b][j],
                                                                     acc[a][b], 0, 0, 0);
    };
    if (nch > 0) {
        // pa/pb hold chunk i, qa/qb chunk i + 1; the last pass reloads a chunk it does not use
        load(cs, pa, pb);
        int64_t i = 0;
        for (; i + 2 <= nch; i += 2) {
            load(cs + i + 1, qa, qb);
            mma(pa, pb);
            load(cs + std::min(i + 2, nch - 1), pa, pb);
            mma(qa, qb);
        }
        if (nch & 1) mma(pa, pb);
    }
    // the ragged end of the range (fewer than NN_KC values of K), by the last wave
    if (w == 3 && nfull * NN_KC < len) {
        const int64_t k = nfull * NN_KC;
#pragma unroll
        for (int j = 0; j < NN_NJ; ++j) {
            const bool kin = k + 4 * j + lk < len;
            const uint32_t sa = (uint32_t)((k + 4 * j) * 8), sb = (uint32_t)((k + 4 * j) * ldb * 8);
            const double a0 = bload(ra, oa0, sa), a1 = bload(ra, oa1, sa);
            const double b0 = bload(rb, ob0, sb), b1 = bload(rb, ob1, sb);
            pa[0][j] = kin ? a0 : 0.0;
            pa[1][j] = kin ? a1 : 0.0;
            pb[0][j] = kin ? b0 : 0.0;
            pb[1][j] = kin ? b1 : 0.0;
        }
        mma(pa, pb);
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) red[w][(a * 2 + b) * 4 + r][lane] = acc[a][b][r];
    __syncthreads();
    for (int e = tid; e < 16 * 64; e += TS_THR) {
        const int slot = e >> 6, ln = e & 63;
        const double s = ((red[0][slot][ln] + red[1][slot][ln]) + red[2][slot][ln]) +
                         red[3][slot][ln];
        const int a = slot >> 3, b = (slot >> 2) & 1, r = slot & 3;
        store_out(M, N, m0 + 16 * a + 4 * r + (ln >> 4), n0 + 16 * b + (ln & 15), s, alpha, beta,
                  C, ldc, part, blockIdx.z);
    }
}

__global__ __launch_bounds__(TS_THR) void k_ts_tn(int64_t M, int64_t N, int64_t K, int64_t kchunk,
                                                  double alpha, const double* __restrict__ A,
                                                  int64_t lda, const double* __restrict__ B,
                                                  int64_t ldb, double beta, double* __restrict__ C,
                                                  int64_t ldc, double* __restrict__ part) {
    __shared__ double red[2][32][64];
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int li = lane & 15, lk = lane >> 4;
    const int64_t m0 = (int64_t)blockIdx.x * 64, n0 = (int64_t)blockIdx.y * 32;
    const int64_t kb = (int64_t)blockIdx.z * kchunk, ke = std::min(K, kb + kchunk);
    const int64_t len = std::max<int64_t>(ke - kb, 0);
    const int64_t nfull = len / TN_KC;
    int64_t cs, nch;
    wave_chunks(nfull, w, cs, nch);

    dbl4 acc[4][2];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[a][b][r] = 0.0;

    const __amdgpu_buffer_rsrc_t ra =
        make_rsrc(A + kb * lda + m0, ((K - 1 - kb) * lda + M - m0) * 8);
    const __amdgpu_buffer_rsrc_t rb =
        make_rsrc(B + kb * ldb + n0, ((K - 1 - kb) * ldb + N - n0) * 8);
    uint32_t oa[4], ob[2];
#pragma unroll
    for (int a = 0; a < 4; ++a) oa[a] = (uint32_t)((lk * lda + 16 * a + li) * 8);
#pragma unroll
    for (int b = 0; b < 2; ++b) ob[b] = (uint32_t)((lk * ldb + 16 * b + li) * 8);
    double pa[4][TN_NJ], pb[2][TN_NJ], qa[4][TN_NJ], qb[2][TN_NJ];
    auto load = [&](int64_t c, double (&xa)[4][TN_NJ], double (&xb)[2][TN_NJ]) {
#pragma unroll
        for (int j = 0; j < TN_NJ; ++j) {
            const int64_t r = TN_KC * c + 4 * j;
            const uint32_t sa = (uint32_t)(r * lda * 8), sb = (uint32_t)(r * ldb * 8);
#pragma unroll
            for (int a = 0; a < 4; ++a) xa[a][j] = bload(ra, oa[a], sa);
#pragma unroll
            for (int b = 0; b < 2; ++b) xb[b][j] = bload(rb, ob[b], sb);
        }
    };
    auto mma = [&](double (&ya)[4][TN_NJ], double (&yb)[2][TN_NJ]) {
#pragma unroll
        for (int j = 0; j < TN_NJ; ++j)
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ya[a][j], yb[b][j],
                                                                     acc[a][b], 0, 0, 0);
    };
    if (nch > 0) {
        load(cs, pa, pb);
        int64_t i = 0;
        for (; i + 2 <= nch; i += 2) {
            load(cs + i + 1, qa, qb);
            mma(pa, pb);
            load(cs + std::min(i + 2, nch - 1), pa, pb);
            mma(qa, qb);
        }
        if (nch & 1) mma(pa, pb);
    }
    if (w == 3 && nfull * TN_KC < len) {
        const int64_t r0 = nfull * TN_KC;
#pragma unroll
        for (int j = 0; j < TN_NJ; ++j) {
            const int64_t r = r0 + 4 * j;
            const bool kin = r + lk < len;
            const uint32_t sa = (uint32_t)(r * lda * 8), sb = (uint32_t)(r * ldb * 8);
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                const double v = bload(ra, oa[a], sa);
                pa[a][j] = kin ? v : 0.0;
            }
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const double v = bload(rb, ob[b], sb);
                pb[b][j] = kin ? v : 0.0;
            }
        }
        mma(pa, pb);
    }
    // (w0 + w2) + (w1 + w3), through 32 KB of LDS in two rounds
    if (w >= 2) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r) red[w - 2][(a * 2 + b) * 4 + r][lane] = acc[a][b][r];
    }
    __syncthreads();
    if (w < 2) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[a][b][r] += red[w][(a * 2 + b) * 4 + r][lane];
    }
    __syncthreads();
    if (w == 1) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r) red[0][(a * 2 + b) * 4 + r][lane] = acc[a][b][r];
    }
    __syncthreads();
    if (w == 0) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const double s = acc[a][b][r] + red[0][(a * 2 + b) * 4 + r][lane];
                    store_out(M, N, m0 + 16 * a + 4 * r + lk, n0 + 16 * b + li, s, alpha, beta, C,
                              ldc, part, blockIdx.z);
                }
    }
}

// C = alpha sum_z part[z] + beta C, the splits in order
__global__ __launch_bounds__(256) void k_ts_reduce(int64_t M, int64_t N, int splits,
                                                   const double* __restrict__ part, double alpha,
                                                   double beta, double* __restrict__ C,
                                                   int64_t ldc) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= M * N) return;
    const int64_t i = idx / N, j = idx - i * N;
    // sixteen partials' loads at a time (indices clamped), summed in ascending order
    double s = 0.0;
    for (int z0 = 0; z0 < splits; z0 += 16) {
        double v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int z = z0 + u < splits ? z0 + u : splits - 1;
            v[u] = part[(int64_t)z * M * N + idx];
        }
#pragma unroll
        for (int u = 0; u < 16; ++u)
            if (z0 + u < splits) s += v[u];
    }
    double o = alpha * s;
    if (beta != 0.0) o += beta * C[i * ldc + j];
    C[i * ldc + j] = o;
}

// workgroups wanted per launch, and the least K per split (per workgroup)
constexpr int64_t TS_TARGET_WG = 256;
constexpr int64_t TS_MIN_KCHUNK = 128;

}  // namespace

bool gemm_ts_eligible(int64_t N) { return N >= 1 && N <= TS_MAX_N; }

hipError_t gemm_ts_f64(bool ta, int64_t M, int64_t N, int64_t K, double alpha, const double* A,
                       int64_t lda, const double* B, int64_t ldb, double beta, double* C,
                       int64_t ldc, GemmWs& ws, hipStream_t st, int tri) {
    if (M <= 0 || N <= 0) return hipSuccess;
    if (ta && tri) return hipErrorInvalidValue;
    // byte offsets inside a buffer are 32-bit: rows x leading dimension must stay below 2 GiB
    auto fits = [](int64_t rows, int64_t ld) { return rows * ld * 8 < ((int64_t)1 << 31) - 4096; };
    if (!ta && !fits(33, lda))
        return gemm_f64(false, false, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, ws, st, 0,
                        tri & GEMM_A_UPPER);
    const int64_t bm = ta ? 64 : 32;
    const int64_t tiles = ((M + bm - 1) / bm) * ((N + 31) / 32);
    int64_t splits = 1;
    if (tiles < TS_TARGET_WG && K > TS_MIN_KCHUNK)
        splits = std::min((TS_TARGET_WG + tiles - 1) / tiles, K / TS_MIN_KCHUNK);
    splits = std::max<int64_t>(1, std::min<int64_t>(splits, 256));
    int64_t kchunk = std::max<int64_t>(K, 0);
    auto chunk_of = [&](int64_t sp) { return ((K + sp - 1) / sp + 31) / 32 * 32; };
    if (splits > 1) kchunk = chunk_of(splits);
    // the offsets along K: rows of B (and of A for the transposed product) per workgroup
    const int64_t ldk = ta ? std::max(lda, ldb) : ldb;
    while (!fits(kchunk + 40, ldk) && kchunk > 32) kchunk = chunk_of(++splits);
    splits = K > 0 ? (K + kchunk - 1) / kchunk : 1;
    // past these limits (a leading dimension in the millions, or too little split-K space)
    // the general GEMM takes the product
    if (!fits(kchunk + 40, ldk) ||
        (splits > 1 && (size_t)splits * M * N * sizeof(double) > ws.bytes))
        return ta ? gemm_f64(true, false, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, ws, st)
                  : gemm_f64(false, false, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, ws, st, 0,
                             tri & GEMM_A_UPPER);
    double* part = splits > 1 ? (double*)ws.part : nullptr;
    const dim3 grid((unsigned)((M + bm - 1) / bm), (unsigned)((N + 31) / 32), (unsigned)splits);
    if (ta)
        hipLaunchKernelGGL(k_ts_tn, grid, dim3(TS_THR), 0, st, M, N, K, kchunk, alpha, A, lda, B,
                           ldb, beta, C, ldc, part);
    else
        hipLaunchKernelGGL(k_ts_nn, grid, dim3(TS_THR), 0, st, M, N, K, kchunk, alpha, A, lda, B,
                           ldb, beta, C, ldc, part, tri);
    SKI_HIP(hipGetLastError());
    if (part) {
        const int64_t tot = M * N;
        hipLaunchKernelGGL(k_ts_reduce, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, M, N,
                           (int)splits, part, alpha, beta, C, ldc);
        SKI_HIP(hipGetLastError());
    }
    return hipSuccess;
}

}  // namespace ski
