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

#include <type_traits>

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

// the data matrix is read once per sketch: non-temporal loads keep it from displacing the
// slab buffer in the caches
template <typename TIn, typename TAcc>
__device__ __forceinline__ TAcc load_in(const TIn* p) {
    if constexpr (std::is_same<TIn, double>::value) {
        const double x = __builtin_nontemporal_load(p);
        if constexpr (sizeof(TAcc) == 8)
            return x;
        else
            return (TAcc)x;
    } else {
        return load_as<TIn, TAcc>(p);
    }
}

template <typename TAcc, typename TOut>
__device__ __forceinline__ TOut store_as(TAcc v) {
    if constexpr (sizeof(TAcc) == 8)
        return (TOut)v;
    else
        return from_f<TOut>(v);
}

// x if keep, else +0.0, without a branch: a conditional load becomes a branch that waits
// for its load at once; clamped addresses and integer masking keep the loads together
template <typename TAcc>
__device__ __forceinline__ TAcc keep_or_zero(TAcc x, bool keep) {
    if constexpr (sizeof(TAcc) == 8) {
        return __builtin_bit_cast(TAcc, __builtin_bit_cast(uint64_t, x) & (keep ? ~0ull : 0ull));
    } else {
        return __builtin_bit_cast(TAcc, __builtin_bit_cast(uint32_t, x) & (keep ? ~0u : 0u));
    }
}

// One 256-point pass over row bits [p, p+8).
template <typename TIn, typename TOut, typename TAcc>
__global__ __launch_bounds__(WT) void k_wht256(const TIn* in, int64_t ld_in,
                                               int64_t rows_valid, int64_t ncols_src,
                                               TOut* out, int64_t ld_out,
                                               int64_t out_col0, int p, int skip_zero_lines,
                                               const uint32_t* __restrict__ dbits, int64_t nct) {
    __shared__ TAcc lds[256 * (WC + 1)];
    // the column tiles of one line are consecutive workgroups: together they read whole rows
    const int64_t line = (int64_t)blockIdx.x / nct;
    const int64_t col = ((int64_t)blockIdx.x % nct) * WC + (threadIdx.x & (WC - 1));
    const int q = threadIdx.x >> 4;  // 0..15
    const int c = threadIdx.x & (WC - 1);
    if (skip_zero_lines && line_row(line, p, 8, 0) >= rows_valid) return;  // p == 0 here
    const bool colok = col < ncols_src;
    const int64_t colc = colok ? col : ncols_src - 1;
    TAcc v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int64_t row = line_row(line, p, 8, 16 * q + i);
        const int64_t rc = row < rows_valid ? row : rows_valid - 1;
        v[i] = load_in<TIn, TAcc>(in + rc * ld_in + colc);
    }
    // the signs D come with the first pass only (p == 0): rows 16q .. 16q+15 of the line
    // share one 32-bit word
    const uint32_t sw = dbits ? dbits[line_row(line, p, 8, 16 * q) >> 5] : 0u;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int64_t row = line_row(line, p, 8, 16 * q + i);
        TAcc x = keep_or_zero(v[i], colok && row < rows_valid);
        if ((sw >> (row & 31)) & 1u) x = -x;
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
// Both passes may run in place (in == out): a workgroup reads all of its points before it
// writes any, and workgroups own disjoint points.
template <typename TIn, typename TOut, typename TAcc>
__global__ __launch_bounds__(WT) void k_wht_small(const TIn* in, int64_t ld_in,
                                                  int64_t rows_valid, int64_t ncols_src,
                                                  TOut* out, int64_t ld_out,
                                                  int64_t out_col0, int p, int R,
                                                  int64_t nlines, int skip_zero_lines,
                                                  const uint32_t* __restrict__ dbits,
                                                  int64_t nct) {
    __shared__ TAcc lds[256 * (WC + 1)];
    const int lpt = 256 >> R;  // lines per tile
    const int64_t line0 = ((int64_t)blockIdx.x / nct) * lpt;
    const int64_t col = ((int64_t)blockIdx.x % nct) * WC + (threadIdx.x & (WC - 1));
    const int q = threadIdx.x >> 4;
    const int c = threadIdx.x & (WC - 1);
    const bool colok = col < ncols_src;
    const int pmask = (1 << R) - 1;
    if (skip_zero_lines && line_row(line0, p, R, 0) >= rows_valid) return;  // p == 0 here
    {
        const int64_t colc = colok ? col : ncols_src - 1;
        TAcc v[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int e = 16 * q + i;
            const int64_t line = std::min(line0 + (e >> R), nlines - 1);
            const int64_t row = line_row(line, p, R, e & pmask);
            const int64_t rc = row < rows_valid ? row : rows_valid - 1;
            v[i] = load_in<TIn, TAcc>(in + rc * ld_in + colc);
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int e = 16 * q + i;
            const int64_t line = line0 + (e >> R);
            const int64_t row = line_row(std::min(line, nlines - 1), p, R, e & pmask);
            TAcc x = keep_or_zero(v[i], line < nlines && colok && row < rows_valid);
            if (dbits && dneg(dbits, row)) x = -x;
            lds[e * (WC + 1) + c] = x;
        }
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
    const int64_t nct = (ncols_src + WC - 1) / WC;
    if (nct == 0) return hipSuccess;
    if (R == 8) {
        hipLaunchKernelGGL((k_wht256<TIn, TOut, TAcc>), dim3((unsigned)(nlines * nct)), blk, 0, st,
                           in, ld_in, rows_valid, ncols_src, out, ld_out, out_col0, p,
                           skip ? 1 : 0, dbits, nct);
    } else {
        const int lpt = 256 >> R;
        const int64_t ntl = (nlines + lpt - 1) / lpt;
        hipLaunchKernelGGL((k_wht_small<TIn, TOut, TAcc>), dim3((unsigned)(ntl * nct)), blk, 0, st,
                           in, ld_in, rows_valid, ncols_src, out, ld_out, out_col0, p, R, nlines,
                           skip ? 1 : 0, dbits, nct);
    }
    return hipGetLastError();
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
                                                     TOut* __restrict__ out, int64_t ldo) {
    const int64_t j = blockIdx.x;
    const int64_t ncol = ncx + k;
    const int64_t c0 = (int64_t)blockIdx.y * (GT * GU) + threadIdx.x;
    const int32_t p0 = ptr[j], p1 = ptr[j + 1];
    TAcc acc[GU];
#pragma unroll
    for (int u = 0; u < GU; ++u) acc[u] = 0;
    auto value = [&](int32_t e, int64_t c) -> TAcc {
        const int64_t r = (int64_t)((uint32_t)e >> 1);
        if (c < ncx) return load_as<TX, TAcc>(X + r * ldx + c);
        return (TAcc)Bx[r * ldb + (c - ncx)];
    };
    // four bucket entries at a time: their loads are issued together, the sums still run
    // in bucket order
    int32_t pp = p0;
    for (; pp + 4 <= p1; pp += 4) {
        int32_t e[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) e[q] = src[pp + q];
#pragma unroll
        for (int u = 0; u < GU; ++u) {
            const int64_t c = c0 + (int64_t)u * GT;
            if (c < ncol) {
                TAcc x[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) x[q] = value(e[q], c);
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[u] = (e[q] & 1) ? acc[u] - x[q] : acc[u] + x[q];
            }
        }
    }
    for (; pp < p1; ++pp) {
        const int32_t e = src[pp];
#pragma unroll
        for (int u = 0; u < GU; ++u) {
            const int64_t c = c0 + (int64_t)u * GT;
            if (c < ncol) {
                const TAcc x = value(e, c);
                acc[u] = (e & 1) ? acc[u] - x : acc[u] + x;
            }
        }
    }
#pragma unroll
    for (int u = 0; u < GU; ++u) {
        const int64_t c = c0 + (int64_t)u * GT;
        if (c < ncol) {
            if constexpr (sizeof(TAcc) == 8)
                out[j * ldo + c] = (TOut)(acc[u] * scale);
            else
                out[j * ldo + c] = from_f<TOut>(acc[u] * (float)scale);
        }
    }
}

// hashing gather over CSR rows: one workgroup per (bucket, column range), LDS accumulator.
// The bucket's entries (its rows of A, then each row's k right-hand-side values, in bucket
// order) are first staged in LDS, all loads in flight together, GC_STAGE at a time; then
// one wave adds them row by row into the accumulator (a row's columns are distinct, so
// each column still receives its terms in bucket order: the sums are the same bits as a
// sequential loop), and the workgroup writes the range out.
constexpr int CSR_RANGE = 4096;  // columns per range (32 KiB of FP64 accumulator)
constexpr int GC_THREADS = 256;
constexpr int GC_STAGE = 2048;   // entries staged at a time
constexpr int GC_ROWS = 256;     // bucket rows described at a time

template <typename TAcc, typename TOut>
__global__ __launch_bounds__(GC_THREADS) void k_gather_csr(const int64_t* __restrict__ row_ptr,
                                                          const int32_t* __restrict__ col,
                                                          const double* __restrict__ val,
                                                          const double* __restrict__ Bx,
                                                          int64_t ldb, int64_t d, int64_t k,
                                                          const int32_t* __restrict__ ptr,
                                                          const int32_t* __restrict__ src,
                                                          double scale, TOut* __restrict__ out) {
    __shared__ TAcc acc[CSR_RANGE];
    __shared__ int32_t scol[GC_STAGE];   // column - c0, or -1 outside the range
    __shared__ TAcc sval[GC_STAGE];      // the signed term
    __shared__ int64_t roff[GC_ROWS + 1];  // flat offsets of the batch's rows
    __shared__ int64_t rbeg[GC_ROWS];    // row_ptr of each row
    __shared__ int32_t rlen[GC_ROWS];    // its stored entries
    __shared__ int32_t rrow[GC_ROWS];    // the row of A, sign in bit 31
    __shared__ int64_t wsum[GC_THREADS / 64];
    const int64_t j = blockIdx.x;
    const int64_t ncol = d + k;
    const int64_t c0 = (int64_t)blockIdx.y * CSR_RANGE;
    const int64_t c1 = std::min(ncol, c0 + CSR_RANGE);
    const int t = threadIdx.x, lane = t & 63;
    for (int64_t c = c0 + t; c < c1; c += GC_THREADS) acc[c - c0] = 0;
    const int32_t p0 = ptr[j], p1 = ptr[j + 1];
    for (int32_t b0 = p0; b0 < p1; b0 += GC_ROWS) {
        const int nb = (int)std::min<int32_t>(GC_ROWS, p1 - b0);
        int64_t v = 0;  // this row's entries: stored ones plus k
        if (t < nb) {
            const int32_t e = src[b0 + t];
            const int64_t r = (int64_t)((uint32_t)e >> 1);
            const int64_t e0 = row_ptr[r];
            const int32_t len = (int32_t)(row_ptr[r + 1] - e0);
            rbeg[t] = e0;
            rlen[t] = len;
            rrow[t] = (int32_t)r | (int32_t)((uint32_t)(e & 1) << 31);
            v = (int64_t)len + k;
        }
        // offsets: an inclusive scan in each wave, then the waves' totals in order
        for (int o = 1; o < 64; o <<= 1) {
            const int64_t y = __shfl_up(v, o);
            if (lane >= o) v += y;
        }
        if (lane == 63) wsum[t >> 6] = v;
        __syncthreads();
        int64_t base = 0;
        for (int w = 0; w < (t >> 6); ++w) base += wsum[w];
        if (t < nb) roff[t + 1] = base + v;
        if (t == 0) roff[0] = 0;
        __syncthreads();
        const int64_t tot = roff[nb];
        for (int64_t x0 = 0; x0 < tot; x0 += GC_STAGE) {
            const int32_t xn = (int32_t)std::min<int64_t>(GC_STAGE, tot - x0);
            // stage: entry i lies in the row whose offsets bracket it (binary search)
            for (int32_t u = t; u < xn; u += GC_THREADS) {
                const int64_t i = x0 + u;
                int lo = 0, hi = nb;  // roff[lo] <= i < roff[hi]
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (roff[mid] <= i)
                        lo = mid;
                    else
                        hi = mid;
                }
                const int64_t o = i - roff[lo];
                const int32_t rr = rrow[lo];
                const int64_t r = rr & 0x7fffffff;
                int64_t c;
                double x;
                if (o < rlen[lo]) {
                    c = col[rbeg[lo] + o];
                    x = val[rbeg[lo] + o];
                } else {
                    c = d + (o - rlen[lo]);
                    x = Bx[r * ldb + (o - rlen[lo])];
                }
                const bool in = c >= c0 && c < c1;
                const TAcc xv = (TAcc)x;
                scol[u] = in ? (int32_t)(c - c0) : -1;
                sval[u] = rr < 0 ? -xv : xv;
            }
            __syncthreads();
            // add, row by row, on one wave (program order keeps the rows in bucket order)
            if (t < 64) {
                for (int i = 0; i < nb; ++i) {
                    // row i's entries within this chunk, as chunk positions [a, z)
                    const int64_t a64 = std::max(roff[i], x0) - x0;
                    const int64_t z64 = std::min(roff[i + 1], x0 + (int64_t)xn) - x0;
                    if (z64 <= a64) continue;
                    const int32_t a = (int32_t)a64, z = (int32_t)z64;
                    for (int32_t u = a + lane; u < z; u += 64) {
                        const int32_t cc = scol[u];
                        if (cc >= 0) acc[cc] = acc[cc] + sval[u];
                    }
                }
            }
            __syncthreads();
        }
    }
    __syncthreads();
    for (int64_t c = c0 + t; c < c1; c += GC_THREADS) {
        if constexpr (sizeof(TAcc) == 8)
            out[j * ncol + c] = (TOut)(acc[c - c0] * scale);
        else
            out[j * ncol + c] = from_f<TOut>(acc[c - c0] * (float)scale);
    }
}

// the structure of a CSR matrix: *bad = 1 unless row_ptr[0] = 0, row_ptr[n] = nnz, the
// offsets never decrease and every column index lies in [0, d) (every writer writes 1)
__global__ __launch_bounds__(256) void k_check_csr(const int64_t* __restrict__ row_ptr,
                                                   const int32_t* __restrict__ col, int64_t n,
                                                   int64_t d, int64_t nnz, int* __restrict__ bad) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool ok = true;
    for (int64_t i = t0; i <= n; i += stride) {
        const int64_t v = row_ptr[i];
        ok = ok && v >= 0 && v <= nnz;
        if (i == 0) ok = ok && v == 0;
        if (i == n)
            ok = ok && v == nnz;
        else
            ok = ok && row_ptr[i + 1] >= v;
    }
    for (int64_t e = t0; e < nnz; e += stride) {
        const int64_t c = col[e];
        ok = ok && c >= 0 && c < d;
    }
    if (!ok) *bad = 1;
}

}  // namespace

namespace {

// Dense sketch by column slabs: for each slab of sc columns of [A B], the first pass
// reads A and B (with the signs D) into the slab buffer T (npad x sc, row-major), the later
// passes run in place, and the gather sums the slab's rows into SA's columns.  A slab
// buffer of ~128 MB stays in the 256 MB last-level cache between its passes, so HBM
// carries little more than A once and SA once.  Rows of T that the first pass skips (no
// row < n in their line) lie beyond the rows the later passes read.
template <typename TS, typename TAcc, typename TOut>
hipError_t sketch_slabs(const double* A, int64_t lda, const double* B, int64_t ldb, int64_t n,
                        int64_t d, int64_t k, int64_t npad, const uint32_t* dbits, TS* T,
                        int64_t sc, const int32_t* bucket_ptr, const int32_t* src, int64_t m,
                        double scale, TOut* SA, hipStream_t st) {
    int L = 0;
    while (((int64_t)1 << L) < npad) ++L;
    const int64_t w = d + k;
    for (int64_t c0 = 0; c0 < w; c0 += sc) {
        const int64_t c1 = std::min(w, c0 + sc), cw = c1 - c0;
        const int64_t a1 = std::min(c1, d), b0 = std::max(c0, d);
        int p = 0;
        int64_t valid = n;
        bool first = true;
        do {
            const int R = std::min(8, L - p);
            const bool last = (p + R >= L);
            if (first) {
                const bool skip = R > 0 && !last;
                if (a1 > c0)
                    SKI_HIP((run_pass<double, TS, TAcc>(A + c0, lda, valid, a1 - c0, T, sc, 0, npad,
                                                        p, R, skip, dbits, st)));
                if (c1 > b0)
                    SKI_HIP((run_pass<double, TS, TAcc>(B + (b0 - d), ldb, valid, c1 - b0, T, sc,
                                                        b0 - c0, npad, p, R, skip, dbits, st)));
                valid = last ? npad : std::min(npad, ((n + (1 << R) - 1) >> R) << R);
            } else {
                SKI_HIP((run_pass<TS, TS, TAcc>(T, sc, valid, cw, T, sc, 0, npad, p, R, false,
                                                nullptr, st)));
                valid = npad;
            }
            first = false;
            p += R;
        } while (p < L);
        dim3 grid((unsigned)m, (unsigned)((cw + GT * GU - 1) / (GT * GU)));
        hipLaunchKernelGGL((k_gather_dense<TS, TAcc, TOut>), grid, dim3(GT), 0, st, T, sc, cw,
                           nullptr, 0, 0, bucket_ptr, src, scale, SA + c0, w);
        SKI_HIP(hipGetLastError());
    }
    return hipSuccess;
}

}  // namespace

namespace {

// dst (n x d row-major, ld d) = src (n x d column-major, ld lds); 64 x 64 tiles through LDS so
// that both the reads (down columns) and the writes (along rows) are contiguous
__global__ __launch_bounds__(256) void k_colmajor_to_rowmajor(const double* __restrict__ src,
                                                              int64_t lds, int64_t n, int64_t d,
                                                              double* __restrict__ dst) {
    __shared__ double tl[64][65];
    const int64_t i0 = (int64_t)blockIdx.y * 64, j0 = (int64_t)blockIdx.x * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int c = ty; c < 64; c += 4) {
        const int64_t i = i0 + tx, j = j0 + c;
        if (i < n && j < d) tl[c][tx] = src[j * lds + i];
    }
    __syncthreads();
    for (int r = ty; r < 64; r += 4) {
        const int64_t i = i0 + r, j = j0 + tx;
        if (i < n && j < d) dst[i * d + j] = tl[tx][r];
    }
}

}  // namespace

hipError_t launch_colmajor_to_rowmajor(const double* src, int64_t lds, int64_t n, int64_t d,
                                       double* dst, hipStream_t st) {
    if (n <= 0 || d <= 0) return hipSuccess;
    const dim3 grid((unsigned)((d + 63) / 64), (unsigned)((n + 63) / 64));
    if (grid.y > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_colmajor_to_rowmajor, grid, dim3(256), 0, st, src, lds, n, d, dst);
    return hipGetLastError();
}

int64_t sketch_slab_cols(int64_t npad, int64_t ncols, Prec prec) {
    const int64_t te = prec == Prec::F64 ? 8 : (prec == Prec::F32 ? 4 : 2);
    int64_t sc = ((int64_t)128 << 20) / (npad * te);  // ~128 MB of slab
    sc = std::max<int64_t>(WC, sc / WC * WC);
    return std::min(sc, ncols);
}

hipError_t launch_sketch_dense(const double* A, int64_t lda, const double* B, int64_t ldb,
                               int64_t n, int64_t d, int64_t k, int64_t npad,
                               const uint32_t* dbits, void* T, int64_t sc,
                               const int32_t* bucket_ptr, const int32_t* src, int64_t m,
                               double scale, Prec prec, Prec out, void* SA, hipStream_t st) {
    switch (prec) {
        case Prec::F64:
            if (out == Prec::F64)
                return sketch_slabs<double, double, double>(A, lda, B, ldb, n, d, k, npad, dbits,
                                                            (double*)T, sc, bucket_ptr, src, m,
                                                            scale, (double*)SA, st);
            // FP64 transform and sums, the sketch rounded once to FP32 for an FP32/BF16 QR
            return sketch_slabs<double, double, float>(A, lda, B, ldb, n, d, k, npad, dbits,
                                                       (double*)T, sc, bucket_ptr, src, m, scale,
                                                       (float*)SA, st);
        case Prec::F32:
            return sketch_slabs<float, float, float>(A, lda, B, ldb, n, d, k, npad, dbits,
                                                     (float*)T, sc, bucket_ptr, src, m, scale,
                                                     (float*)SA, st);
        case Prec::BF16:
            return sketch_slabs<__hip_bfloat16, float, float>(A, lda, B, ldb, n, d, k, npad,
                                                              dbits, (__hip_bfloat16*)T, sc,
                                                              bucket_ptr, src, m, scale,
                                                              (float*)SA, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_gather_plain(const double* A, int64_t lda, const double* B, int64_t ldb,
                               int64_t d, int64_t k, const int32_t* bucket_ptr,
                               const int32_t* src, int64_t m, double scale, Prec prec, Prec out,
                               void* SA, hipStream_t st) {
    const int64_t ncols = d + k;
    dim3 grid((unsigned)m, (unsigned)((ncols + GT * GU - 1) / (GT * GU)));
    if (prec == Prec::F64 && out == Prec::F64)
        hipLaunchKernelGGL((k_gather_dense<double, double, double>), grid, dim3(GT), 0, st, A, lda,
                           d, B, ldb, k, bucket_ptr, src, scale, (double*)SA, ncols);
    else if (prec == Prec::F64)
        hipLaunchKernelGGL((k_gather_dense<double, double, float>), grid, dim3(GT), 0, st, A, lda,
                           d, B, ldb, k, bucket_ptr, src, scale, (float*)SA, ncols);
    else
        hipLaunchKernelGGL((k_gather_dense<double, float, float>), grid, dim3(GT), 0, st, A, lda, d,
                           B, ldb, k, bucket_ptr, src, scale, (float*)SA, ncols);
    return hipGetLastError();
}

hipError_t launch_check_csr(const int64_t* row_ptr, const int32_t* col, int64_t n, int64_t d,
                            int64_t nnz, int* bad, hipStream_t st) {
    const int64_t work = std::max<int64_t>(n + 1, nnz);
    const unsigned g = (unsigned)std::min<int64_t>((work + 255) / 256, 2048);
    hipLaunchKernelGGL(k_check_csr, dim3(g), dim3(256), 0, st, row_ptr, col, n, d, nnz, bad);
    return hipGetLastError();
}

hipError_t launch_gather_csr(const int64_t* row_ptr, const int32_t* col, const double* val,
                             const double* B, int64_t ldb, int64_t d, int64_t k,
                             const int32_t* bucket_ptr, const int32_t* src, int64_t m,
                             double scale, Prec prec, Prec out, void* SA, hipStream_t st) {
    const int64_t ncols = d + k;
    dim3 grid((unsigned)m, (unsigned)((ncols + CSR_RANGE - 1) / CSR_RANGE));
    if (prec == Prec::F64 && out == Prec::F64)
        hipLaunchKernelGGL((k_gather_csr<double, double>), grid, dim3(GC_THREADS), 0, st, row_ptr, col, val,
                           B, ldb, d, k, bucket_ptr, src, scale, (double*)SA);
    else if (prec == Prec::F64)
        hipLaunchKernelGGL((k_gather_csr<double, float>), grid, dim3(GC_THREADS), 0, st, row_ptr, col, val,
                           B, ldb, d, k, bucket_ptr, src, scale, (float*)SA);
    else
        hipLaunchKernelGGL((k_gather_csr<float, float>), grid, dim3(GC_THREADS), 0, st, row_ptr, col, val,
                           B, ldb, d, k, bucket_ptr, src, scale, (float*)SA);
    return hipGetLastError();
}

}  // namespace ski
