// Building blocks for 64 x 64 dense matrices held in LDS and worked on by one workgroup of
// 256 threads (four wavefronts): elementwise maps, products on the 16x16x4 MFMA, and
// blocked Cholesky, triangular inverse and sign-pivoted LU.  Used by the QR's panel
// factorisation and by the inversion of R's diagonal blocks.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ski {
namespace tile {

constexpr int PB = 64;       // tile size
constexpr int PP = PB + 1;   // LDS pitch of a PB x PB tile
constexpr int TB = 16;       // diagonal block of the Cholesky and LU factorisations
constexpr int TI = 8;        // diagonal block of the triangular inverse (8 x 8, 64 threads)

// compiler ordering point for LDS traffic between the lanes of one wavefront (a wavefront
// executes its LDS instructions in order)
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double bcast_lane(double x, int l) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), l),
                            __builtin_amdgcn_readlane(__double2loint(x), l));
}
__device__ __forceinline__ float bcast_lane(float x, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}

// 1/sqrt(x) and 1/x for x > 0: the hardware estimate refined by two Newton steps (each
// doubles the number of correct bits), accurate to a few units in the last place
__device__ __forceinline__ double rsqrt_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double e = fma(-x * y, y, 1.0);  // 1 - x y^2
        y = fma(0.5 * y, e, y);
    }
    return y;
}
__device__ __forceinline__ float rsqrt_nr(float x) {
    float y = __builtin_amdgcn_rsqf(x);
    const float e = fmaf(-x * y, y, 1.0f);
    return fmaf(0.5f * y, e, y);
}
__device__ __forceinline__ double rcp_nr(double x) {
    double y = __builtin_amdgcn_rcp(x);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double e = fma(-x, y, 1.0);  // 1 - x y
        y = fma(y, e, y);
    }
    return y;
}
__device__ __forceinline__ float rcp_nr(float x) {
    float y = __builtin_amdgcn_rcpf(x);
    const float e = fmaf(-x, y, 1.0f);
    return fmaf(y, e, y);
}

// 16x16x4 MFMA: lane l supplies A[l%16][l/16] and B[l/16][l%16] and holds D[row(r, l)][l%16]
// in accumulator element r (FP64: row 4r + l/16; FP32: row 4(l/16) + r)
template <typename T>
struct MF;
template <>
struct MF<double> {
    typedef double A4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ A4 mma(double a, double b, A4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int r, int l) { return 4 * r + (l >> 4); }
};
template <>
struct MF<float> {
    typedef float A4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ A4 mma(float a, float b, A4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int r, int l) { return 4 * (l >> 4) + r; }
};

// All are called by the 256 threads of a workgroup and end synchronised.

// X(i, j) = f(i, j) for every entry, through registers (dst may be read by f)
template <typename T, typename F>
__device__ __forceinline__ void tile_eval(T (*dst)[PP], int t, F f) {
    T v[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int o = t + 256 * q;
        v[q] = f(o / PB, o % PB);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int o = t + 256 * q;
        dst[o / PB][o % PB] = v[q];
    }
    __syncthreads();
}

// D(i, j) = fin(i, j, sum_k fa(i, k) fb(k, j)) on MFMA: wave w computes the 16-row tile
// row w; for output tile (w, q) the sum runs over the k-steps [s0, s1) of 4 given by
// kr(w, q) = (s0, s1).  The ranges must not depend on w: the k-loop is then the same on
// every wavefront, which the compiler pipelines (triangular factors are stored with
// explicit zeros, so a full x upper range is also right for upper x upper).  fin may read D.
template <typename T, typename FA, typename FB, typename KR, typename FIN>
__device__ __forceinline__ void tile_mma(T (*D)[PP], int t, FA fa, FB fb, KR kr, FIN fin) {
    using A4 = typename MF<T>::A4;
    const int l = t & 63, w = t >> 6, li = l & 15, lk = l >> 4;
    A4 acc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        acc[q] = (A4){0, 0, 0, 0};
        const int2 kk = kr(w, q);
        for (int u = kk.x; u < kk.y; ++u)
            acc[q] = MF<T>::mma(fa(16 * w + li, 4 * u + lk), fb(4 * u + lk, 16 * q + li), acc[q]);
    }
    T v[16];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) v[4 * q + r] = fin(16 * w + MF<T>::row(r, l), 16 * q + li, acc[q][r]);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) D[16 * w + MF<T>::row(r, l)][16 * q + li] = v[4 * q + r];
    __syncthreads();
}

// k-step ranges of products with triangular factors (tile row a, tile column b)
struct KFullUpper {  // full x upper: k in [0, 16b + 16)
    __device__ int2 operator()(int, int b) const { return make_int2(0, 4 * b + 4); }
};
struct KSlice {  // one slice [k0, k1) of k for every tile (the caller masks in fin)
    int k0, k1;
    __device__ int2 operator()(int, int) const { return make_int2(k0 / 4, k1 / 4); }
};
struct KSliceFrom {  // KSlice for the tile columns b >= bmin only (the others: no k-steps)
    int k0, k1, bmin;
    __device__ int2 operator()(int, int b) const {
        return b >= bmin ? make_int2(k0 / 4, k1 / 4) : make_int2(0, 0);
    }
};
struct KFull {
    __device__ int2 operator()(int, int) const { return make_int2(0, PB / 4); }
};
struct KLowerFull {  // lower x full: k in [0, 16a + 16)
    __device__ int2 operator()(int a, int) const { return make_int2(0, 4 * a + 4); }
};

// Cholesky of the symmetric positive definite A (upper triangle read): A <- R upper
// (A = R^T R), zero lower.  Blocks of TB rows: wavefront 0 eliminates the block row in
// registers (lane c holds rows k0..k0+TB-1 of column k0 + c, so the diagonal block and the
// block row R_kk^-T A(k0 block, :) come out of the same sweep), then the trailing update
// runs on MFMA.  Sets *bad if a pivot is not positive and finite.
template <typename T>
__device__ __forceinline__ void tile_chol(T (*A)[PP], int t, int* bad) {
    for (int k0 = 0; k0 < PB; k0 += TB) {
        if (t < PB - k0) {
            const int c = k0 + t;
            T col[TB];
#pragma unroll
            for (int i = 0; i < TB; ++i) col[i] = i <= t ? A[k0 + i][c] : (T)0;
            bool b = false;
#pragma unroll
            for (int k = 0; k < TB; ++k) {
                // row k of the block before scaling: the pivot and a_{k, k0+i}, i > k
                const T dkk = bcast_lane(col[k], k);
                T aki[TB];
#pragma unroll
                for (int i = k + 1; i < TB; ++i) aki[i] = bcast_lane(col[k], i);
                b = b || !(dkk > (T)0) || !isfinite(dkk);
                const T ip = rsqrt_nr(dkk), id = ip * ip;  // 1/sqrt(d), 1/d
                // a_ij -= r_ki r_kj = a_ki a_kj / d
                const T ck = col[k] * id;
#pragma unroll
                for (int i = k + 1; i < TB; ++i) col[i] -= aki[i] * ck;
                col[k] = t == k ? dkk * ip : (t > k ? col[k] * ip : (T)0);
            }
            // entries below the diagonal block's diagonal are cleared at the end
#pragma unroll
            for (int i = 0; i < TB; ++i) A[k0 + i][c] = col[i];
            if (b && t == 0) *bad = 1;
        }
        __syncthreads();
        if (k0 + TB == PB) break;
        const int lo = k0 + TB;
        // only the tile columns at or right of lo change (j >= i >= lo)
        tile_mma(A, t, [&](int i, int k) { return A[k][i]; }, [&](int k, int j) { return A[k][j]; },
                 KSliceFrom{k0, k0 + TB, lo / 16},
                 [&](int i, int j, T v) { return (i >= lo && j >= i) ? A[i][j] - v : A[i][j]; });
    }
    tile_eval(A, t, [&](int i, int j) { return i <= j ? A[i][j] : (T)0; });
}

// in-place inverse of the upper triangular A (unit: its diagonal is taken as 1) by
// recursive doubling: 8 x 8 diagonal blocks by back substitution, 16 x 16 blocks by one
// level on vector FMAs, then X12 = -X11 (A12 X22) on MFMA for blocks of 32 and 64
template <typename T>
__device__ __forceinline__ void tile_trinv(T (*A)[PP], int t, bool unit) {
    {
        T x[TI];
        const int b = t >> 3, j = t & 7, o = TI * b;
        if (t < PB) {
            T inv[TI];  // reciprocals of the diagonal, off the substitution's dependency chain
#pragma unroll
            for (int i = 0; i < TI; ++i) inv[i] = unit ? (T)1 : (T)1 / A[o + i][o + i];
#pragma unroll
            for (int i = TI - 1; i >= 0; --i) {
                T s = i == j ? (T)1 : (T)0;
#pragma unroll
                for (int l = i + 1; l < TI; ++l) s -= A[o + i][o + l] * x[l];
                x[i] = s * inv[i];
            }
        }
        __syncthreads();
        if (t < PB)
#pragma unroll
            for (int i = 0; i < TI; ++i)
                if (i <= j) A[o + i][o + j] = x[i];
        __syncthreads();
    }
    {
        // h = 8: four pairs of 8 x 8 blocks, one output of each product per thread
        const int base = 16 * (t >> 6), i = (t >> 3) & 7, jj = t & 7;
        T s = 0;
#pragma unroll
        for (int l = 0; l <= 7; ++l)
            if (l <= jj) s += A[base + i][base + 8 + l] * A[base + 8 + l][base + 8 + jj];
        __syncthreads();
        A[base + i][base + 8 + jj] = s;
        __syncthreads();
        s = 0;
#pragma unroll
        for (int l = 0; l <= 7; ++l)
            if (l >= i) s += A[base + i][base + l] * A[base + l][base + 8 + jj];
        __syncthreads();
        A[base + i][base + 8 + jj] = -s;
        __syncthreads();
    }
    // h = 16, 32: the off-diagonal blocks are whole tiles (tile row a, tile column b)
    for (int h = 16; h < PB; h *= 2) {
        const int hb = h / 16;  // block size in tiles
        auto in_pair = [=](int a, int b) {
            return (a / hb) % 2 == 0 && b / hb == a / hb + 1;
        };
        // Y = A12 X22: k over the X22 block
        tile_mma(A, t, [&](int i, int k) { return A[i][k]; }, [&](int k, int j) { return A[k][j]; },
                 [=](int, int b) {
                     const int s0 = 4 * hb * (b / hb);
                     return make_int2(s0, in_pair(0, b) || in_pair(2, b) ? 4 * b + 4 : s0);
                 },
                 [&](int i, int j, T v) { return in_pair(i / 16, j / 16) ? v : A[i][j]; });
        // X12 = -X11 Y: k over the X11 block (rows of Y), the same block as the row i
        tile_mma(A, t, [&](int i, int k) { return k / h == i / h ? A[i][k] : (T)0; },
                 [&](int k, int j) { return A[k][j]; },
                 [=](int, int b) { return make_int2(0, in_pair(0, b) || in_pair(2, b) ? 4 * b : 0); },
                 [&](int i, int j, T v) { return in_pair(i / 16, j / 16) ? -v : A[i][j]; });
    }
}

// LU without row exchanges of [I - C S] where the sign s_k = -sign(c_kk) is chosen at
// elimination step k (pivot 1 + |c_kk| >= 1).  The elimination runs on C itself:
// C <- [multipliers below the diagonal; eliminated C on and above it], sg <- s.
// Blocks of TB columns on wavefront 0: the panel with one row per lane, then the block row
// L11^-1 C(k0 block, :) with one column per lane; the trailing update on MFMA.
template <typename T>
__device__ __forceinline__ void tile_lu_signed(T (*C)[PP], T* sg, int t) {
    for (int k0 = 0; k0 < PB; k0 += TB) {
        const int nt = PB - k0 - TB;
        if (t < 64) {
            if (t < PB - k0) {
                const int i = k0 + t;
                T pr[TB];
#pragma unroll
                for (int c = 0; c < TB; ++c) pr[c] = C[i][k0 + c];
#pragma unroll
                for (int k = 0; k < TB; ++k) {
                    const T qkk = bcast_lane(pr[k], k);
                    T qk[TB];
#pragma unroll
                    for (int c = k + 1; c < TB; ++c) qk[c] = bcast_lane(pr[c], k);
                    const T s = qkk >= (T)0 ? (T)-1 : (T)1;
                    const T iu = rcp_nr((T)1 + fabs(qkk));
                    if (t == 0) sg[k0 + k] = s;
                    if (t > k) {
                        const T l = -s * pr[k] * iu;
#pragma unroll
                        for (int c = k + 1; c < TB; ++c) pr[c] -= l * qk[c];
                        pr[k] = l;
                    }
                }
#pragma unroll
                for (int c = 0; c < TB; ++c) C[i][k0 + c] = pr[c];
            }
            wave_sync();
            if (t < nt) {
                const int c = k0 + TB + t;
                T x[TB];
#pragma unroll
                for (int i = 0; i < TB; ++i) {
                    T s = C[k0 + i][c];
#pragma unroll
                    for (int l = 0; l < i; ++l) s -= C[k0 + i][k0 + l] * x[l];
                    x[i] = s;
                }
#pragma unroll
                for (int i = 0; i < TB; ++i) C[k0 + i][c] = x[i];
            }
        }
        __syncthreads();
        if (nt == 0) break;
        const int lo = k0 + TB;
        // only the tile columns at or right of lo change (j >= lo)
        tile_mma(C, t, [&](int i, int k) { return C[i][k]; }, [&](int k, int j) { return C[k][j]; },
                 KSliceFrom{k0, k0 + TB, lo / 16},
                 [&](int i, int j, T v) { return (i >= lo && j >= lo) ? C[i][j] - v : C[i][j]; });
    }
}

}  // namespace tile
}  // namespace ski
