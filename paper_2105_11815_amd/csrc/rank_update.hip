// The trailing update of the blocked Householder QR (Step 2 of Algorithm 1):
//   C <- C - A B,  A: M x K,  B: K x N,  C: M x N,  K <= 64 (one panel's reflectors),
// all row-major with leading dimensions (the QR calls it on the transposed view of its
// column-major working copy: M = remaining columns, N = remaining rows).
//
// With K <= 64 the update reads and writes C once for 2K flops per entry: it is bound by
// moving C, not by the matrix cores.  A general GEMM walks K in slices with a barrier and a
// dependent load round trip per slice and reads C only in its epilogue, so for K = 64 it
// spends most of its time waiting on memory.  Here every load a tile needs is issued at
// once: the 64 x K block of A (into LDS, k-major so that each lane's MFMA operand is one
// conflict-free LDS read), this lane's B operands of the K/4 MFMA steps and its 16 entries
// of C (in the accumulator layout of the 16x16x4 MFMA).  In FP64 a workgroup owns a strip
// of four 64 x 64 tiles of C along N: A is loaded once for the strip, and the next tile's
// C is in flight while the current tile's MFMA steps run (B comes from L2); the register
// budget is two wavefronts per SIMD.  In FP32 a workgroup owns one tile with A and B both
// in LDS.  Addresses are clamped into the matrices and the values outside masked to zero,
// so no load waits behind a branch.  Each output is one fixed-order sum: the result is
// deterministic.
//
// The product that precedes the update, W = C V^T (M x K, K <= 64, the reduction over the
// N rows of the panel), walks N in tiles of 64: a workgroup owns 64 rows of W and one
// range of N, keeps the next tile's loads in flight while the current tile's 16 MFMA steps
// run, and writes its partial W; the partials are then summed in ascending range order.
// In FP64 the number of ranges is chosen so that the grid fills the 512 workgroup slots
// (two per CU) in as few rounds as possible.
#include "ski_internal.h"
#include "tile64.h"

#include <algorithm>
#include <climits>

namespace ski {

namespace {

constexpr int UT = 64;        // tile edge (M and N) and the largest K
constexpr int UP = UT + 1;    // LDS pitch

// ranges of N for W = C V^T.  FP32: about 640 workgroups in all, and at least 4 tiles per
// range.  FP64: the count s (at least 4 tiles per range, partials within 64 MiB) that
// minimises the rounds of 512 resident workgroups times the tiles per range, so that the
// last round is not a small remainder.
int rank_project_splits(int64_t M, int64_t N, size_t elem) {
    const int64_t gx = (M + UT - 1) / UT, tiles = (N + UT - 1) / UT;
    if (elem != 8) {
        int64_t s = (640 + gx - 1) / gx;
        s = std::min<int64_t>(s, std::max<int64_t>(1, tiles / 4));
        return (int)std::max<int64_t>(1, std::min<int64_t>(s, 64));
    }
    const int64_t smax =
        std::max<int64_t>(1, std::min<int64_t>({64, tiles / 4, ((int64_t)64 << 20) / (M * UT * 8)}));
    int64_t best = 1, bcost = INT64_MAX;
    for (int64_t s = 1; s <= smax; ++s) {
        const int64_t per = (tiles + s - 1) / s, ns = (tiles + per - 1) / per;
        const int64_t cost = 20 * ((gx * ns + 511) / 512) * per + ns;  // ties: fewer partials
        if (cost < bcost) {
            bcost = cost;
            best = s;
        }
    }
    return (int)best;
}

template <typename T>
__device__ __forceinline__ T mask_or_zero(T x, bool keep) {
    if constexpr (sizeof(T) == 8)
        return __builtin_bit_cast(T, __builtin_bit_cast(uint64_t, x) & (keep ? ~0ull : 0ull));
    else
        return __builtin_bit_cast(T, __builtin_bit_cast(uint32_t, x) & (keep ? ~0u : 0u));
}

template <typename T>
__global__ __launch_bounds__(256) void k_rank_update(int64_t M, int64_t N, int K,
                                                     const T* __restrict__ A, int64_t lda,
                                                     const T* __restrict__ B, int64_t ldb,
                                                     T* __restrict__ C, int64_t ldc) {
    using MF = tile::MF<T>;
    using A4 = typename MF::A4;
    __shared__ T At[UT][UP];  // At[q][j] = A(j0 + j, q)
    __shared__ T Bs[UT][UP];  // Bs[q][i] = B(q, i0 + i)
    const int t = threadIdx.x, l = t & 63, w = t >> 6, li = l & 15, lk = l >> 4;
    const int64_t i0 = (int64_t)blockIdx.x * UT, j0 = (int64_t)blockIdx.y * UT;
    const int wj = (w >> 1) * 32, wi = (w & 1) * 32;

    // every load of the tile at once: A and B blocks, and this lane's 16 entries of C
    T av[16], bv[16], cv[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int e = t + 256 * u;
        const int r = e >> 6, c = e & 63;  // A: row j0 + r, column c; B: row r, column i0 + c
        const int64_t ja = std::min<int64_t>(j0 + r, M - 1);
        const int qa = c < K ? c : K - 1;
        av[u] = A[ja * lda + qa];
        const int qb = r < K ? r : K - 1;
        const int64_t ib = std::min<int64_t>(i0 + c, N - 1);
        bv[u] = B[(int64_t)qb * ldb + ib];
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t j = std::min<int64_t>(j0 + wj + 16 * a + MF::row(r, l), M - 1);
                const int64_t i = std::min<int64_t>(i0 + wi + 16 * b + li, N - 1);
                cv[8 * a + 4 * b + r] = C[j * ldc + i];
            }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int e = t + 256 * u;
        const int r = e >> 6, c = e & 63;
        At[c][r] = mask_or_zero(av[u], c < K);
        Bs[r][c] = mask_or_zero(bv[u], r < K);
    }
    __syncthreads();

    A4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = (A4){0, 0, 0, 0};
    const int ksteps = (K + 3) >> 2;
    for (int s = 0; s < ksteps; ++s) {
        const int q = 4 * s + lk;
        T af[2], bf[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            af[a] = At[q][wj + 16 * a + li];
            bf[a] = Bs[q][wi + 16 * a + li];
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) acc[a][b] = MF::mma(af[a], bf[b], acc[a][b]);
    }

#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t j = j0 + wj + 16 * a + MF::row(r, l);
                const int64_t i = i0 + wi + 16 * b + li;
                if (j < M && i < N) C[j * ldc + i] = cv[8 * a + 4 * b + r] - acc[a][b][r];
            }
}


// FP64: C tiles per workgroup along N
constexpr int RU_STRIP = 4;

// C <- C - A B on a strip of RU_STRIP tiles along N (the FP64 form).  The A block goes to
// LDS once; each tile's B operands are loaded at the tile's start and the next tile's C
// entries while this tile's MFMA steps run.  The MFMA sequence per output is the one of
// k_rank_update.
template <typename T>
__global__ __launch_bounds__(256, 2) void k_rank_update_strip(int64_t M, int64_t N, int K,
                                                              const T* __restrict__ A,
                                                              int64_t lda,
                                                              const T* __restrict__ B,
                                                              int64_t ldb, T* __restrict__ C,
                                                              int64_t ldc) {
    using MF = tile::MF<T>;
    using A4 = typename MF::A4;
    __shared__ T At[UT][UP];  // At[q][j] = A(j0 + j, q)
    const int t = threadIdx.x, l = t & 63, w = t >> 6, li = l & 15, lk = l >> 4;
    const int64_t j0 = (int64_t)blockIdx.y * UT;
    const int64_t sbeg = (int64_t)blockIdx.x * UT * RU_STRIP;
    const int wj = (w >> 1) * 32, wi = (w & 1) * 32;
    const int ksteps = (K + 3) >> 2;
    T bf[32], cv0[16], cv1[16];  // B operands of the 16 k-steps (2 blocks each); C entries
    auto load_b = [&](int64_t i0) {
#pragma unroll
        for (int s = 0; s < 16; ++s)
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const int q = 4 * s + lk;
                const int64_t ib = std::min<int64_t>(i0 + wi + 16 * b + li, N - 1);
                bf[2 * s + b] = B[(int64_t)(q < K ? q : K - 1) * ldb + ib];
            }
    };
    auto load_c = [&](int64_t i0, T* cv) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t j = std::min<int64_t>(j0 + wj + 16 * a + MF::row(r, l), M - 1);
                    const int64_t i = std::min<int64_t>(i0 + wi + 16 * b + li, N - 1);
                    cv[8 * a + 4 * b + r] = C[j * ldc + i];
                }
    };
    auto update = [&](int64_t i0, const T* cv) {
        A4 acc[2][2];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) acc[a][b] = (A4){0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            if (s < ksteps) {
                const int q = 4 * s + lk;
                T af[2];
#pragma unroll
                for (int a = 0; a < 2; ++a) af[a] = At[q][wj + 16 * a + li];
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b)
                        acc[a][b] = MF::mma(af[a], mask_or_zero(bf[2 * s + b], q < K), acc[a][b]);
            }
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t j = j0 + wj + 16 * a + MF::row(r, l);
                    const int64_t i = i0 + wi + 16 * b + li;
                    if (j < M && i < N) C[j * ldc + i] = cv[8 * a + 4 * b + r] - acc[a][b][r];
                }
    };
    {
        T av[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int e = t + 256 * u;
            const int r = e >> 6, c = e & 63;  // A: row j0 + r, column c
            const int64_t ja = std::min<int64_t>(j0 + r, M - 1);
            av[u] = A[ja * lda + (c < K ? c : K - 1)];
        }
        load_b(sbeg);
        load_c(sbeg, cv0);
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int e = t + 256 * u;
            const int r = e >> 6, c = e & 63;
            At[c][r] = mask_or_zero(av[u], c < K);
        }
    }
    __syncthreads();
    // tiles of the strip inside N (the grid covers N, so there is at least one)
    const int nt = (int)std::min<int64_t>(RU_STRIP, (N - sbeg + UT - 1) / UT);
    for (int tt = 0; tt < nt; tt += 2) {  // two tiles per pass: the C buffers alternate
        const int64_t i0 = sbeg + (int64_t)tt * UT;
        if (tt + 1 < nt) load_c(i0 + UT, cv1);
        update(i0, cv0);
        if (tt + 1 >= nt) break;
        load_b(i0 + UT);
        if (tt + 2 < nt) load_c(i0 + 2 * UT, cv0);
        update(i0 + UT, cv1);
        if (tt + 2 < nt) load_b(i0 + 2 * UT);
    }
}

// W_s = C(j0:j0+64, n-range s) V(:, n-range s)^T: the partial product of range s.
// C: M x N (ldc), V: K x N (ldv); partial s of W at P + s * M * UT (row-major, ld UT).
template <typename T>
__global__ __launch_bounds__(256) void k_rank_project(int64_t M, int64_t N, int K, int64_t nrange,
                                                      const T* __restrict__ C, int64_t ldc,
                                                      const T* __restrict__ V, int64_t ldv,
                                                      T* __restrict__ P) {
    using MF = tile::MF<T>;
    using A4 = typename MF::A4;
    __shared__ T Cs[UT][UP];  // Cs[j][n] = C(j0 + j, nb + n)
    __shared__ T Vs[UT][UP];  // Vs[q][n] = V(q, nb + n)
    const int t = threadIdx.x, l = t & 63, w = t >> 6, li = l & 15, lk = l >> 4;
    const int64_t j0 = (int64_t)blockIdx.x * UT;
    const int64_t nbeg = (int64_t)blockIdx.y * nrange, nend = std::min<int64_t>(N, nbeg + nrange);
    const int wj = (w >> 1) * 32, wq = (w & 1) * 32;
    T cv[16], vv[16];
    auto load = [&](int64_t nb) {
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int e = t + 256 * u;
            const int r = e >> 6, c = e & 63;
            const int64_t n = std::min<int64_t>(nb + c, N - 1);
            cv[u] = C[std::min<int64_t>(j0 + r, M - 1) * ldc + n];
            vv[u] = V[(int64_t)(r < K ? r : K - 1) * ldv + n];
        }
    };
    A4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = (A4){0, 0, 0, 0};
    if (nbeg < nend) load(nbeg);
    for (int64_t nb = nbeg; nb < nend; nb += UT) {
        __syncthreads();  // the previous tile's MFMA reads are done
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int e = t + 256 * u;
            const int r = e >> 6, c = e & 63;
            const bool in = nb + c < nend;
            Cs[r][c] = mask_or_zero(cv[u], in);
            Vs[r][c] = mask_or_zero(vv[u], in && r < K);
        }
        __syncthreads();
        if (nb + UT < nend) load(nb + UT);
#pragma unroll 4
        for (int s = 0; s < UT / 4; ++s) {
            const int n = 4 * s + lk;
            T af[2], bf[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                af[a] = Cs[wj + 16 * a + li][n];
                bf[a] = Vs[wq + 16 * a + li][n];
            }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) acc[a][b] = MF::mma(af[a], bf[b], acc[a][b]);
        }
    }
    T* Ps = P + (int64_t)blockIdx.y * M * UT;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t j = j0 + wj + 16 * a + MF::row(r, l);
                const int q = wq + 16 * b + li;
                if (j < M && q < K) Ps[j * UT + q] = acc[a][b][r];
            }
}

// W (M x K, ldw) = the sum of the nsplit partials, in ascending order
template <typename T>
__global__ __launch_bounds__(256) void k_project_sum(int64_t M, int K, int nsplit,
                                                     const T* __restrict__ P, T* __restrict__ W,
                                                     int64_t ldw) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= M * UT) return;
    const int64_t j = e / UT;
    const int q = (int)(e % UT);
    if (q >= K) return;
    // sixteen partials' loads at a time (indices clamped), summed in ascending order
    T s = 0;
    for (int z0 = 0; z0 < nsplit; z0 += 16) {
        T v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int z = z0 + u < nsplit ? z0 + u : nsplit - 1;
            v[u] = P[(int64_t)z * M * UT + e];
        }
#pragma unroll
        for (int u = 0; u < 16; ++u)
            if (z0 + u < nsplit) s += v[u];
    }
    W[j * ldw + q] = s;
}

}  // namespace

template <typename T>
hipError_t launch_rank_update(int64_t M, int64_t N, int K, const T* A, int64_t lda, const T* B,
                              int64_t ldb, T* C, int64_t ldc, hipStream_t st) {
    if (M <= 0 || N <= 0 || K <= 0) return hipSuccess;
    if (K > UT) return hipErrorInvalidValue;
    const int64_t gx = (N + UT - 1) / UT, gy = (M + UT - 1) / UT;
    if (gy > 65535) return hipErrorInvalidValue;
    if constexpr (sizeof(T) == 8) {
        hipLaunchKernelGGL((k_rank_update_strip<T>), dim3((unsigned)((gx + RU_STRIP - 1) / RU_STRIP),
                           (unsigned)gy), dim3(256), 0, st, M, N, K, A, lda, B, ldb, C, ldc);
    } else {
        hipLaunchKernelGGL((k_rank_update<T>), dim3((unsigned)gx, (unsigned)gy), dim3(256), 0, st,
                           M, N, K, A, lda, B, ldb, C, ldc);
    }
    return hipGetLastError();
}

template hipError_t launch_rank_update<double>(int64_t, int64_t, int, const double*, int64_t,
                                               const double*, int64_t, double*, int64_t,
                                               hipStream_t);
template hipError_t launch_rank_update<float>(int64_t, int64_t, int, const float*, int64_t,
                                              const float*, int64_t, float*, int64_t,
                                              hipStream_t);

size_t rank_project_ws_bytes(int64_t M, int64_t N, size_t elem) {
    return (size_t)rank_project_splits(M, N, elem) * (size_t)M * UT * elem;
}

template <typename T>
hipError_t launch_rank_project(int64_t M, int64_t N, int K, const T* C, int64_t ldc, const T* V,
                               int64_t ldv, T* W, int64_t ldw, void* ws, size_t ws_bytes,
                               hipStream_t st) {
    if (M <= 0 || K <= 0) return hipSuccess;
    if (K > UT) return hipErrorInvalidValue;
    int ns = N > 0 ? rank_project_splits(M, N, sizeof(T)) : 1;
    if ((size_t)ns * M * UT * sizeof(T) > ws_bytes) return hipErrorInvalidValue;
    const int64_t tiles = N > 0 ? (N + UT - 1) / UT : 1;
    const int64_t per = (tiles + ns - 1) / ns;  // tiles of N per range
    const int64_t nrange = per * UT;
    ns = (int)((tiles + per - 1) / per);
    const int64_t gx = (M + UT - 1) / UT;
    T* P = (T*)ws;
    if (N > 0) {
        hipLaunchKernelGGL((k_rank_project<T>), dim3((unsigned)gx, (unsigned)ns), dim3(256), 0, st,
                           M, N, K, nrange, C, ldc, V, ldv, P);
        SKI_HIP(hipGetLastError());
    } else {
        ns = 0;
    }
    const int64_t tot = M * UT;
    hipLaunchKernelGGL((k_project_sum<T>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st,
                       M, K, ns, P, W, ldw);
    return hipGetLastError();
}

template hipError_t launch_rank_project<double>(int64_t, int64_t, int, const double*, int64_t,
                                                const double*, int64_t, double*, int64_t, void*,
                                                size_t, hipStream_t);
template hipError_t launch_rank_project<float>(int64_t, int64_t, int, const float*, int64_t,
                                               const float*, int64_t, float*, int64_t, void*,
                                               size_t, hipStream_t);

}  // namespace ski
