// Dense GEMM on CDNA4 matrix cores: C[MxN] = alpha op(A)[MxK] op(B)[KxN] + beta C, all
// row-major.  Used for the blocked Householder updates of the sketch's QR (the only
// dense contraction of the method), for the explicit inverse of R and for the
// multi-right-hand-side products of LSQR/CG.
//
// Tiles: 64 x 64 outputs per workgroup of four waves (2 x 2), 32 x 32 per wave as
// 2 x 2 blocks of the 16x16 MFMA; K is staged through LDS in slices of 16 (k-major
// layout, so each lane's operand is one conflict-free LDS read), with the next slice
// prefetched into registers while the current one is multiplied.
//   FP64: v_mfma_f64_16x16x4f64; FP32: v_mfma_f32_16x16x4f32;
//   BF16: FP32 storage, operands rounded to bf16, v_mfma_f32_16x16x16bf16_1k, FP32 sums.
// Operand lane layout (16x16xK, one block): lane l supplies A[l%16][k-group l/16] and
// B[k-group l/16][l%16]; it receives D[i][l%16] in its r-th accumulator element with
// i = 4*(l/16)+r for the FP32 and BF16 instructions and i = 4*r + l/16 for the FP64 one
// (checked on the device).
// Split-K: when the output has few tiles but K is long, slices of K go to separate
// workgroups that write partial products; a second kernel sums them in a fixed order
// (deterministic, no atomics) and applies alpha and beta.
#include "ski_internal.h"

namespace ski {

namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));
typedef short sht4 __attribute__((ext_vector_type(4)));

constexpr int BM = 64, BN = 64, BK = 16, GTHR = 256;
constexpr int PAD = 4;

enum class Mode { F64, F32, BF16 };

template <Mode MD>
struct MT;
template <>
struct MT<Mode::F64> {
    using T = double;
    using Acc = dbl4;
};
template <>
struct MT<Mode::F32> {
    using T = float;
    using Acc = flt4;
};
template <>
struct MT<Mode::BF16> {
    using T = float;
    using Acc = flt4;
};

__device__ __forceinline__ short f2bf_bits(float x) {
    __hip_bfloat16 h = __float2bfloat16(x);
    return *reinterpret_cast<short*>(&h);
}

template <Mode MD, bool TA, bool TB>
__global__ __launch_bounds__(GTHR) void k_gemm(int64_t M, int64_t N, int64_t K, int64_t kchunk,
                                               typename MT<MD>::T alpha,
                                               const typename MT<MD>::T* __restrict__ A,
                                               int64_t lda,
                                               const typename MT<MD>::T* __restrict__ B,
                                               int64_t ldb, typename MT<MD>::T beta,
                                               typename MT<MD>::T* __restrict__ C, int64_t ldc,
                                               typename MT<MD>::T* __restrict__ part, int unitA,
                                               int tri) {
    using T = typename MT<MD>::T;
    using Acc = typename MT<MD>::Acc;
    __shared__ T As[BK][BM + PAD];
    __shared__ T Bs[BK][BN + PAD];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int64_t m0 = (int64_t)blockIdx.y * BM, n0 = (int64_t)blockIdx.x * BN;
    int64_t kbeg = (int64_t)blockIdx.z * kchunk;
    int64_t kend = std::min(K, kbeg + kchunk);
    // triangular operands: A(i, k) = 0 for k < i, B(k, j) = 0 for k > j (m0, n0 are
    // multiples of BK, so the slices stay aligned)
    if (tri & GEMM_A_UPPER) kbeg = std::max(kbeg, m0);
    if (tri & GEMM_B_UPPER) kend = std::min(kend, n0 + BN);

    Acc acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[a][b][r] = 0;

    // register staging: 4 elements of the A slice and 4 of the B slice per thread
    // unitA: A holds Householder vectors stored in place (LAPACK style): the stored
    // matrix V has an implicit unit diagonal and zeros above it.
    T ra[4], rb[4];
    auto vget = [&](int64_t r, int64_t c, const T* p) -> T {
        if (unitA) {
            if (r < c) return (T)0;
            if (r == c) return (T)1;
        }
        return *p;
    };
    auto load_slices = [&](int64_t k0) {
        if (!TA) {  // A row-major M x K: row m0 + tid/4, k = k0 + 4*(tid%4) + u
            const int64_t i = m0 + (tid >> 2);
            const int64_t kk = k0 + 4 * (tid & 3);
#pragma unroll
            for (int u = 0; u < 4; ++u)
                ra[u] = (i < M && kk + u < kend) ? vget(i, kk + u, A + i * lda + kk + u) : (T)0;
        } else {  // A stored K x M: k = k0 + tid/16, i = m0 + 4*(tid%16) + u
            const int64_t kk = k0 + (tid >> 4);
            const int64_t i = m0 + 4 * (tid & 15);
#pragma unroll
            for (int u = 0; u < 4; ++u)
                ra[u] = (kk < kend && i + u < M) ? vget(kk, i + u, A + kk * lda + i + u) : (T)0;
        }
        if (!TB) {  // B row-major K x N
            const int64_t kk = k0 + (tid >> 4);
            const int64_t j = n0 + 4 * (tid & 15);
#pragma unroll
            for (int u = 0; u < 4; ++u)
                rb[u] = (kk < kend && j + u < N) ? B[kk * ldb + j + u] : (T)0;
        } else {  // B stored N x K
            const int64_t j = n0 + (tid >> 2);
            const int64_t kk = k0 + 4 * (tid & 3);
#pragma unroll
            for (int u = 0; u < 4; ++u)
                rb[u] = (j < N && kk + u < kend) ? B[j * ldb + kk + u] : (T)0;
        }
    };
    auto store_slices = [&]() {
        if (!TA) {
#pragma unroll
            for (int u = 0; u < 4; ++u) As[4 * (tid & 3) + u][tid >> 2] = ra[u];
        } else {
#pragma unroll
            for (int u = 0; u < 4; ++u) As[tid >> 4][4 * (tid & 15) + u] = ra[u];
        }
        if (!TB) {
#pragma unroll
            for (int u = 0; u < 4; ++u) Bs[tid >> 4][4 * (tid & 15) + u] = rb[u];
        } else {
#pragma unroll
            for (int u = 0; u < 4; ++u) Bs[4 * (tid & 3) + u][tid >> 2] = rb[u];
        }
    };

    const int li = lane & 15, lk = lane >> 4;
    if (kbeg < kend) {
        load_slices(kbeg);
        for (int64_t k0 = kbeg; k0 < kend; k0 += BK) {
            __syncthreads();
            store_slices();
            __syncthreads();
            if (k0 + BK < kend) load_slices(k0 + BK);
            if constexpr (MD == Mode::BF16) {
                sht4 af[2], bf[2];
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        af[a][r] = f2bf_bits(As[4 * lk + r][wm + 16 * a + li]);
                        bf[a][r] = f2bf_bits(Bs[4 * lk + r][wn + 16 * a + li]);
                    }
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b)
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af[a], bf[b],
                                                                               acc[a][b], 0, 0, 0);
            } else {
#pragma unroll
                for (int ks = 0; ks < BK; ks += 4) {
                    T af[2], bf[2];
#pragma unroll
                    for (int a = 0; a < 2; ++a) {
                        af[a] = As[ks + lk][wm + 16 * a + li];
                        bf[a] = Bs[ks + lk][wn + 16 * a + li];
                    }
#pragma unroll
                    for (int a = 0; a < 2; ++a)
#pragma unroll
                        for (int b = 0; b < 2; ++b) {
                            if constexpr (MD == Mode::F64)
                                acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bf[b],
                                                                                 acc[a][b], 0, 0, 0);
                            else
                                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[a], bf[b],
                                                                                 acc[a][b], 0, 0, 0);
                        }
                }
            }
        }
    }
    // epilogue
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                // output row inside the 16x16 block: FP64 MFMA interleaves (4 r + l/16),
                // FP32/BF16 MFMA stack (4 (l/16) + r)
                const int rr = (MD == Mode::F64) ? 4 * r + lk : 4 * lk + r;
                const int64_t i = m0 + wm + 16 * a + rr;
                const int64_t j = n0 + wn + 16 * b + li;
                if (i < M && j < N) {
                    T v = acc[a][b][r];
                    if (part) {
                        part[((int64_t)blockIdx.z * M + i) * N + j] = v;
                    } else {
                        T o = alpha * v;
                        if (beta != (T)0) o += beta * C[i * ldc + j];
                        C[i * ldc + j] = o;
                    }
                }
            }
}

template <typename T>
__global__ __launch_bounds__(256) void k_splitk_reduce(int64_t M, int64_t N, int splits,
                                                       const T* __restrict__ part, T alpha, T beta,
                                                       T* __restrict__ C, int64_t ldc) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= M * N) return;
    const int64_t i = idx / N, j = idx - i * N;
    // sixteen partials' loads at a time (indices clamped), summed in ascending order
    T s = 0;
    for (int z0 = 0; z0 < splits; z0 += 16) {
        T v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int z = z0 + u < splits ? z0 + u : splits - 1;
            v[u] = part[(int64_t)z * M * N + idx];
        }
#pragma unroll
        for (int u = 0; u < 16; ++u)
            if (z0 + u < splits) s += v[u];
    }
    T o = alpha * s;
    if (beta != (T)0) o += beta * C[i * ldc + j];
    C[i * ldc + j] = o;
}

// split-K for grids of few output tiles: enough splits for ~1280 workgroups (about five
// resident per CU), so that each works through a short K range.  The QR's W = C^T V
// products (64 output columns, K up to m) are latency-bound per 16-wide K step, and shorter
// ranges took the dense factorisation from ~13.0 to ~12.7 ms against a target of 384.
int choose_splits(int64_t M, int64_t N, int64_t K) {
    const int64_t tiles = ((M + BM - 1) / BM) * ((N + BN - 1) / BN);
    if (tiles >= 192 || K < 1024) return 1;
    int64_t s = (1280 + tiles - 1) / tiles;
    s = std::min<int64_t>(s, K / 256);
    return (int)std::max<int64_t>(1, std::min<int64_t>(s, 64));
}

template <Mode MD>
hipError_t gemm_impl(bool ta, bool tb, int64_t M, int64_t N, int64_t K, typename MT<MD>::T alpha,
                     const typename MT<MD>::T* A, int64_t lda, const typename MT<MD>::T* B,
                     int64_t ldb, typename MT<MD>::T beta, typename MT<MD>::T* C, int64_t ldc,
                     GemmWs& ws, hipStream_t st, int unitA, int tri) {
    using T = typename MT<MD>::T;
    if (M <= 0 || N <= 0) return hipSuccess;
    int splits = choose_splits(M, N, K);
    // as many splits as the workspace holds (none if it cannot hold two)
    if (splits > 1 && (size_t)splits * M * N * sizeof(T) > ws.bytes)
        splits = (int)std::max<size_t>(1, ws.bytes / ((size_t)M * N * sizeof(T)));
    int64_t kchunk = K;
    if (splits > 1) {
        kchunk = ((K + splits - 1) / splits + BK - 1) / BK * BK;
        splits = (int)((K + kchunk - 1) / kchunk);
    }
    T* part = splits > 1 ? (T*)ws.part : nullptr;
    dim3 grid((unsigned)((N + BN - 1) / BN), (unsigned)((M + BM - 1) / BM), (unsigned)splits);
    if (K <= 0) kchunk = 0;
#define SKI_GEMM_LAUNCH(TA_, TB_)                                                              \
    hipLaunchKernelGGL((k_gemm<MD, TA_, TB_>), grid, dim3(GTHR), 0, st, M, N, K, kchunk, alpha, \
                       A, lda, B, ldb, beta, C, ldc, part, unitA, tri)
    if (!ta && !tb)
        SKI_GEMM_LAUNCH(false, false);
    else if (ta && !tb)
        SKI_GEMM_LAUNCH(true, false);
    else if (!ta && tb)
        SKI_GEMM_LAUNCH(false, true);
    else
        SKI_GEMM_LAUNCH(true, true);
#undef SKI_GEMM_LAUNCH
    SKI_HIP(hipGetLastError());
    if (part) {
        const int64_t tot = M * N;
        hipLaunchKernelGGL((k_splitk_reduce<T>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0,
                           st, M, N, splits, part, alpha, beta, C, ldc);
        SKI_HIP(hipGetLastError());
    }
    return hipSuccess;
}

}  // namespace

size_t gemm_ws_bytes(int64_t M, int64_t N, int64_t K, size_t elem) {
    int s = choose_splits(M, N, K);
    return s > 1 ? (size_t)s * M * N * elem : 0;
}

hipError_t gemm_f64(bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha,
                    const double* A, int64_t lda, const double* B, int64_t ldb, double beta,
                    double* C, int64_t ldc, GemmWs& ws, hipStream_t st, int unitA, int tri) {
    return gemm_impl<Mode::F64>(ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, ws, st,
                                unitA, tri);
}

hipError_t gemm_f32(bool ta, bool tb, int64_t M, int64_t N, int64_t K, float alpha,
                    const float* A, int64_t lda, const float* B, int64_t ldb, float beta, float* C,
                    int64_t ldc, bool bf16_inputs, GemmWs& ws, hipStream_t st, int unitA) {
    if (bf16_inputs)
        return gemm_impl<Mode::BF16>(ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, ws, st,
                                     unitA, 0);
    return gemm_impl<Mode::F32>(ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, ws, st,
                                unitA, 0);
}

}  // namespace ski
