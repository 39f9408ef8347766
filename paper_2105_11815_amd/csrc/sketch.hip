// Step 1 of Algorithm 1 on the GPU: T = H D [A B; 0] (dense, Definition of HRHT) by
// Walsh-Hadamard butterflies, then SA_aug[j, :] = scale * sum_{p in bucket j} (+-) T[src_p, :]
// (hashing, Definition of s-hashing), scale = 1/sqrt(n' s) (or 1/sqrt(s) without H).
//
// Layout: A is n x d row-major (lda), B n x k (ldb); T is n' x (d+k) row-major, n' the
// padded power of two.  A transform of length n' = 2^L runs as ceil(L/8) passes, each
// over 8 (or fewer, last) consecutive bits of the row index, lowest bits first, so the
// butterfly stages run over row bit 0, 1, 2, ... in order -- the order that makes the
// result reproducible bit for bit.  A pass over bits [p, p+R) treats every fixed pair
// (row bits above p+R, row bits below p) as one "line" of 2^R points.
//
// The 256-point pass keeps a 256 x 16 tile (one line, 16 columns) in registers and LDS:
// every thread owns 16 points of one column, runs the first four stages in registers,
// exchanges through LDS, and runs the last four stages in registers.  Rows >= n are
// zero and never read; in the first pass a line that holds no row < n produces zeros,
// is not written, and later passes treat those rows as zero.
//
// The hashing gather keeps the bucket order fixed (columns ascending inside a bucket,
// sum started at +0.0), so no atomics are needed and FP64 results are bit-identical to
// a sequential sum in that order.
#include "ski_internal.h"

namespace ski {

namespace {

constexpr int WT = 256;  // threads per workgroup
constexpr int WC = 16;   // columns per tile

__device__ __forceinline__ int64_t line_row(int64_t line, int p, int R, int64_t mid) {
    const int64_t lo_mask = ((int64_t)1 << p) - 1;
    return ((line >> p) << (p + R)) | (mid << p) | (line & lo_mask);
}

__device__ __forceinline__ bool dneg(const uint32_t* bits, int64_t row) {
    return (bits[row >> 5] >> (row & 31)) & 1u;
}

template <typename TIn, typename TAcc>
__device__ __forceinline__ TAcc load_as(const TIn* p) {
    if constexpr (sizeof(TAcc) == 8)
        return (TAcc)(*p);
    else
        return to_f(*p);
}

template <typename TAcc, typename TOut>
__device__ __forceinline__ TOut store_as(TAcc v) {
    if constexpr (sizeof(TAcc) == 8)
        return (TOut)v;
    else
        return from_f<TOut>(v);
}

// One 256-point pass over row bits [p, p+8).
template <typename TIn, typename TOut, typename TAcc>
__global__ __launch_bounds__(WT) void k_wht256(const TIn* __restrict__ in, int64_t ld_in,
                                               int64_t rows_valid, int64_t ncols_src,
                                               TOut* __restrict__ out, int64_t ld_out,
                                               int64_t out_col0, int p, int skip_zero_lines,
                                               const uint32_t* __restrict__ dbits) {
    __shared__ TAcc lds[256 * (WC + 1)];
    const int64_t line = blockIdx.x;
    const int64_t col = (int64_t)blockIdx.y * WC + (threadIdx.x & (WC - 1));
    const int q = threadIdx.x >> 4;  // 0..15
    const int c = threadIdx.x & (WC - 1);
    if (skip_zero_lines && line_row(line, p, 8, 0) >= rows_valid) return;  // p == 0 here
    const bool colok = col < ncols_src;
    TAcc v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        int64_t row = line_row(line, p, 8, 16 * q + i);
        TAcc x = 0;
        if (colok && row < rows_valid) {
            x = load_as<TIn, TAcc>(in + row * ld_in + col);
            if (dbits && dneg(dbits, row)) x = -x;
        }
        v[i] = x;
    }
#pragma unroll
    for (int h = 1; h < 16; h <<= 1) {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            if ((i & h) == 0) {
                TAcc a = v[i], b = v[i + h];
                v[i] = a + b;
                v[i + h] = a - b;
            }
        }
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) lds[(16 * q + i) * (WC + 1) + c] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = lds[(16 * i + q) * (WC + 1) + c];
#pragma unroll
    for (int h = 1; h < 16; h <<= 1) {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            if ((i & h) == 0) {
                TAcc a = v[i], b = v[i + h];
                v[i] = a + b;
                v[i + h] = a - b;
            }
        }
    }
    if (!colok) return;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        int64_t row = line_row(line, p, 8, 16 * i + q);
        out[row * ld_out + out_col0 + col] = store_as<TAcc, TOut>(v[i]);
    }
}

// A pass over R < 8 bits: 256/2^R lines of 2^R points per tile, stages in LDS.
template <typename TIn, typename TOut, typename TAcc>
__global__ __launch_bounds__(WT) void k_wht_small(const TIn* __restrict__ in, int64_t ld_in,
                                                  int64_t rows_valid, int64_t ncols_src,
                                                  TOut* __restrict__ out, int64_t ld_out,
                                                  int64_t out_col0, int p, int R,
                                                  int64_t nlines, int skip_zero_lines,
                                                  const uint32_t* __restrict__ dbits) {
    __shared__ TAcc lds[256 * (WC + 1)];
    const int lpt = 256 >> R;  // lines per tile
    const int64_t line0 = (int64_t)blockIdx.x * lpt;
    const int64_t col = (int64_t)blockIdx.y * WC + (threadIdx.x & (WC - 1));
    const int q = threadIdx.x >> 4;
    const int c = threadIdx.x & (WC - 1);
    const bool colok = col < ncols_src;
    const int pmask = (1 << R) - 1;
    if (skip_zero_lines && line_row(line0, p, R, 0) >= rows_valid) return;  // p == 0 here
    for (int i = 0; i < 16; ++i) {
        int e = 16 * q + i;
        int64_t line = line0 + (e >> R);
        TAcc x = 0;
        if (line < nlines) {
            int64_t row = line_row(line, p, R, e & pmask);
            if (colok && row < rows_valid) {
                x = load_as<TIn, TAcc>(in + row * ld_in + col);
                if (dbits && dneg(dbits, row)) x = -x;
            }
        }
        lds[e * (WC + 1) + c] = x;
    }
    __syncthreads();
    for (int lh = 0; lh < R; ++lh) {
        const int h = 1 << lh;
        for (int t = threadIdx.x; t < 128 * WC; t += WT) {
            int cc = t & (WC - 1);
            int pp = t >> 4;  // 0..127
            int e = ((pp >> lh) << (lh + 1)) | (pp & (h - 1));
            TAcc a = lds[e * (WC + 1) + cc], b = lds[(e + h) * (WC + 1) + cc];
            lds[e * (WC + 1) + cc] = a + b;
            lds[(e + h) * (WC + 1) + cc] = a - b;
        }
        __syncthreads();
    }
    if (!colok) return;
    for (int i = 0; i < 16; ++i) {
        int e = 16 * q + i;
        int64_t line = line0 + (e >> R);
        if (line >= nlines) continue;
        int64_t row = line_row(line, p, R, e & pmask);
        out[row * ld_out + out_col0 + col] = store_as<TAcc, TOut>(lds[e * (WC + 1) + c]);
    }
}

template <typename TIn, typename TOut, typename TAcc>
hipError_t run_pass(const TIn* in, int64_t ld_in, int64_t rows_valid, int64_t ncols_src, TOut* out,
                    int64_t ld_out, int64_t out_col0, int64_t npad, int p, int R, bool skip,
                    const uint32_t* dbits, hipStream_t st) {
    const int64_t nlines = npad >> R;
    dim3 blk(WT);
    const unsigned gy = (unsigned)((ncols_src + WC - 1) / WC);
    if (gy == 0) return hipSuccess;
    if (R == 8) {
        hipLaunchKernelGGL((k_wht256<TIn, TOut, TAcc>), dim3((unsigned)nlines, gy), blk, 0, st, in,
                           ld_in, rows_valid, ncols_src, out, ld_out, out_col0, p, skip ? 1 : 0,
                           dbits);
    } else {
        const int lpt = 256 >> R;
        const unsigned gx = (unsigned)((nlines + lpt - 1) / lpt);
        hipLaunchKernelGGL((k_wht_small<TIn, TOut, TAcc>), dim3(gx, gy), blk, 0, st, in, ld_in,
                           rows_valid, ncols_src, out, ld_out, out_col0, p, R, nlines,
                           skip ? 1 : 0, dbits);
    }
    return hipGetLastError();
}

template <typename TS, typename TAcc>
hipError_t wht_all(const double* A, int64_t lda, const double* B, int64_t ldb, int64_t n, int64_t d,
                   int64_t k, int64_t npad, const uint32_t* dbits, TS* T0, TS* T1, void** T_out,
                   hipStream_t st) {
    int L = 0;
    while (((int64_t)1 << L) < npad) ++L;
    const int64_t w = d + k;
    int p = 0;
    TS* cur_out = T0;
    TS* cur_in = nullptr;
    int64_t valid = n;
    bool first = true;
    if (L == 0) {  // n' = 1: T = D [A B]
        SKI_HIP((run_pass<double, TS, TAcc>(A, lda, n, d, T0, w, 0, 1, 0, 0, false, dbits, st)));
        SKI_HIP((run_pass<double, TS, TAcc>(B, ldb, n, k, T0, w, d, 1, 0, 0, false, dbits, st)));
        *T_out = T0;
        return hipSuccess;
    }
    while (p < L) {
        const int R = std::min(8, L - p);
        const bool last = (p + R == L);
        const bool skip = first && !last;
        if (first) {
            SKI_HIP((run_pass<double, TS, TAcc>(A, lda, valid, d, cur_out, w, 0, npad, p, R, skip,
                                                dbits, st)));
            SKI_HIP((run_pass<double, TS, TAcc>(B, ldb, valid, k, cur_out, w, d, npad, p, R, skip,
                                                dbits, st)));
            valid = last ? npad : std::min(npad, ((n + (1 << R) - 1) >> R) << R);
        } else {
            SKI_HIP((run_pass<TS, TS, TAcc>(cur_in, w, valid, w, cur_out, w, 0, npad, p, R, false,
                                            nullptr, st)));
            valid = npad;
        }
        first = false;
        p += R;
        cur_in = cur_out;
        cur_out = (cur_out == T0) ? T1 : T0;
    }
    *T_out = cur_in;
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// hashing gather over dense rows: out[j, c] = scale * sum (+-) X[src, c]
constexpr int GT = 256;
constexpr int GU = 4;  // columns per thread

template <typename TX, typename TAcc, typename TOut>
__global__ __launch_bounds__(GT) void k_gather_dense(const TX* __restrict__ X, int64_t ldx,
                                                     int64_t ncx, const double* __restrict__ Bx,
                                                     int64_t ldb, int64_t k,
                                                     const int32_t* __restrict__ ptr,
                                                     const int32_t* __restrict__ src, double scale,
                                                     TOut* __restrict__ out) {
    const int64_t j = blockIdx.x;
    const int64_t ncol = ncx + k;
    const int64_t c0 = (int64_t)blockIdx.y * (GT * GU) + threadIdx.x;
    const int32_t p0 = ptr[j], p1 = ptr[j + 1];
    TAcc acc[GU];
#pragma unroll
    for (int u = 0; u < GU; ++u) acc[u] = 0;
    for (int32_t pp = p0; pp < p1; ++pp) {
        const int32_t e = src[pp];
        const int64_t r = (int64_t)((uint32_t)e >> 1);
        const bool neg = e & 1;
#pragma unroll
        for (int u = 0; u < GU; ++u) {
            const int64_t c = c0 + (int64_t)u * GT;
            if (c < ncol) {
                TAcc x;
                if (c < ncx)
                    x = load_as<TX, TAcc>(X + r * ldx + c);
                else
                    x = (TAcc)Bx[r * ldb + (c - ncx)];
                acc[u] = neg ? acc[u] - x : acc[u] + x;
            }
        }
    }
#pragma unroll
    for (int u = 0; u < GU; ++u) {
        const int64_t c = c0 + (int64_t)u * GT;
        if (c < ncol) {
            if constexpr (sizeof(TAcc) == 8)
                out[j * ncol + c] = (TOut)(acc[u] * scale);
            else
                out[j * ncol + c] = from_f<TOut>(acc[u] * (float)scale);
        }
    }
}

// hashing gather over CSR rows: one wave per (bucket, column range), LDS accumulator
constexpr int CSR_RANGE = 8192;  // columns per range (64 KiB of FP64 accumulator)

template <typename TAcc, typename TOut>
__global__ __launch_bounds__(64) void k_gather_csr(const int64_t* __restrict__ row_ptr,
                                                   const int32_t* __restrict__ col,
                                                   const double* __restrict__ val,
                                                   const double* __restrict__ Bx, int64_t ldb,
                                                   int64_t d, int64_t k,
                                                   const int32_t* __restrict__ ptr,
                                                   const int32_t* __restrict__ src, double scale,
                                                   TOut* __restrict__ out) {
    __shared__ TAcc acc[CSR_RANGE];
    const int64_t j = blockIdx.x;
    const int64_t ncol = d + k;
    const int64_t c0 = (int64_t)blockIdx.y * CSR_RANGE;
    const int64_t c1 = std::min(ncol, c0 + CSR_RANGE);
    const int lane = threadIdx.x;
    for (int64_t c = c0 + lane; c < c1; c += 64) acc[c - c0] = 0;
    __syncthreads();
    const int32_t p0 = ptr[j], p1 = ptr[j + 1];
    for (int32_t pp = p0; pp < p1; ++pp) {
        const int32_t e = src[pp];
        const int64_t r = (int64_t)((uint32_t)e >> 1);
        const bool neg = e & 1;
        const int64_t e0 = row_ptr[r], e1 = row_ptr[r + 1];
        for (int64_t q = e0 + lane; q < e1; q += 64) {
            const int64_t c = col[q];
            if (c >= c0 && c < c1) {
                TAcc x = (TAcc)val[q];
                TAcc a = acc[c - c0];
                acc[c - c0] = neg ? a - x : a + x;
            }
        }
        for (int64_t t = lane; t < k; t += 64) {
            const int64_t c = d + t;
            if (c >= c0 && c < c1) {
                TAcc x = (TAcc)Bx[r * ldb + t];
                TAcc a = acc[c - c0];
                acc[c - c0] = neg ? a - x : a + x;
            }
        }
        __syncthreads();  // single wave: orders this entry's LDS updates before the next
    }
    for (int64_t c = c0 + lane; c < c1; c += 64) {
        if constexpr (sizeof(TAcc) == 8)
            out[j * ncol + c] = (TOut)(acc[c - c0] * scale);
        else
            out[j * ncol + c] = from_f<TOut>(acc[c - c0] * (float)scale);
    }
}

}  // namespace

hipError_t launch_wht_sketch_dense(const double* A, int64_t lda, const double* B, int64_t ldb,
                                   int64_t n, int64_t d, int64_t k, int64_t npad,
                                   const uint32_t* dbits, void* T0, void* T1, Prec prec,
                                   void** T_out, hipStream_t st) {
    switch (prec) {
        case Prec::F64:
            return wht_all<double, double>(A, lda, B, ldb, n, d, k, npad, dbits, (double*)T0,
                                           (double*)T1, T_out, st);
        case Prec::F32:
            return wht_all<float, float>(A, lda, B, ldb, n, d, k, npad, dbits, (float*)T0,
                                         (float*)T1, T_out, st);
        case Prec::BF16:
            return wht_all<__hip_bfloat16, float>(A, lda, B, ldb, n, d, k, npad, dbits,
                                                  (__hip_bfloat16*)T0, (__hip_bfloat16*)T1, T_out,
                                                  st);
    }
    return hipErrorInvalidValue;
}

// SA storage: FP64 for the FP64 form, FP32 for both mixed forms (the QR works in FP32)
hipError_t launch_gather_dense(const void* T, int64_t ncols, const int32_t* bucket_ptr,
                               const int32_t* src, int64_t m, double scale, Prec prec, void* SA,
                               hipStream_t st) {
    dim3 grid((unsigned)m, (unsigned)((ncols + GT * GU - 1) / (GT * GU)));
    switch (prec) {
        case Prec::F64:
            hipLaunchKernelGGL((k_gather_dense<double, double, double>), grid, dim3(GT), 0, st,
                               (const double*)T, ncols, ncols, nullptr, 0, 0, bucket_ptr, src,
                               scale, (double*)SA);
            break;
        case Prec::F32:
            hipLaunchKernelGGL((k_gather_dense<float, float, float>), grid, dim3(GT), 0, st,
                               (const float*)T, ncols, ncols, nullptr, 0, 0, bucket_ptr, src,
                               scale, (float*)SA);
            break;
        case Prec::BF16:
            hipLaunchKernelGGL((k_gather_dense<__hip_bfloat16, float, float>), grid, dim3(GT), 0,
                               st, (const __hip_bfloat16*)T, ncols, ncols, nullptr, 0, 0,
                               bucket_ptr, src, scale, (float*)SA);
            break;
    }
    return hipGetLastError();
}

hipError_t launch_gather_plain(const double* A, int64_t lda, const double* B, int64_t ldb,
                               int64_t d, int64_t k, const int32_t* bucket_ptr,
                               const int32_t* src, int64_t m, double scale, Prec prec, void* SA,
                               hipStream_t st) {
    const int64_t ncols = d + k;
    dim3 grid((unsigned)m, (unsigned)((ncols + GT * GU - 1) / (GT * GU)));
    if (prec == Prec::F64)
        hipLaunchKernelGGL((k_gather_dense<double, double, double>), grid, dim3(GT), 0, st, A, lda,
                           d, B, ldb, k, bucket_ptr, src, scale, (double*)SA);
    else
        hipLaunchKernelGGL((k_gather_dense<double, float, float>), grid, dim3(GT), 0, st, A, lda, d,
                           B, ldb, k, bucket_ptr, src, scale, (float*)SA);
    return hipGetLastError();
}

hipError_t launch_gather_csr(const int64_t* row_ptr, const int32_t* col, const double* val,
                             const double* B, int64_t ldb, int64_t d, int64_t k,
                             const int32_t* bucket_ptr, const int32_t* src, int64_t m,
                             double scale, Prec prec, void* SA, hipStream_t st) {
    const int64_t ncols = d + k;
    dim3 grid((unsigned)m, (unsigned)((ncols + CSR_RANGE - 1) / CSR_RANGE));
    if (prec == Prec::F64)
        hipLaunchKernelGGL((k_gather_csr<double, double>), grid, dim3(64), 0, st, row_ptr, col, val,
                           B, ldb, d, k, bucket_ptr, src, scale, (double*)SA);
    else
        hipLaunchKernelGGL((k_gather_csr<float, float>), grid, dim3(64), 0, st, row_ptr, col, val,
                           B, ldb, d, k, bucket_ptr, src, scale, (float*)SA);
    return hipGetLastError();
}

}  // namespace ski
