// The sparse QR of the sketch and its triangular solves (Section 6, the sparse solver);
// the structure comes from the symbolic phase (sparse_symbolic.cpp).
#include <algorithm>
#include <cmath>
#include <cstring>

#include "sparse_qr.h"

namespace ski {

namespace {

constexpr int SA_SORT_CAP = 2048;  // raw entries of a bucket sorted in LDS
constexpr int SA_RANGE = 2048;     // columns per pass of the wide-bucket path
constexpr int FT_ROWS = 128;       // rows of a front tile
constexpr int FT_LD = 65;          // leading dimension of the tile (64 columns + 1)
constexpr int FT_THREADS = 256;
constexpr int SOLVE_THREADS = 256;

// ---------------------------------------------------------------------------------------
// sketch: raw entry counts of every bucket (the lengths of its rows of A)
__global__ void k_sa_raw(const int32_t* __restrict__ bptr, const int32_t* __restrict__ src,
                         const int64_t* __restrict__ row_ptr, int64_t m,
                         int64_t* __restrict__ raw) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= m) return;
    int64_t s = 0;
    for (int32_t pp = bptr[b]; pp < bptr[b + 1]; ++pp) {
        const int64_t i = (int64_t)((uint32_t)src[pp] >> 1);
        s += row_ptr[i + 1] - row_ptr[i];
    }
    raw[b] = s;
}

// exclusive prefix sum of n int64 into out[0 .. n] (one workgroup of 1024 threads, each a
// contiguous chunk)
__global__ __launch_bounds__(1024) void k_scan_excl(const int64_t* __restrict__ in, int64_t n,
                                                    int64_t* __restrict__ out) {
    __shared__ int64_t part[1024];
    const int t = threadIdx.x;
    const int64_t chunk = (n + 1023) / 1024;
    const int64_t i0 = std::min<int64_t>(n, t * chunk), i1 = std::min<int64_t>(n, i0 + chunk);
    int64_t s = 0;
    for (int64_t i = i0; i < i1; ++i) s += in[i];
    part[t] = s;
    __syncthreads();
    if (t == 0) {
        int64_t run = 0;
        for (int u = 0; u < 1024; ++u) {
            const int64_t v = part[u];
            part[u] = run;
            run += v;
        }
        out[n] = run;
    }
    __syncthreads();
    int64_t run = part[t];
    for (int64_t i = i0; i < i1; ++i) {
        out[i] = run;
        run += in[i];
    }
}

// one bucket per wave: the bucket's rows of A merged by column, equal columns summed in
// bucket order (signed values; a + (-x) is a - x exactly), then scaled; and the bucket's
// right-hand-side sums
__global__ __launch_bounds__(64) void k_sa_build(
    const int32_t* __restrict__ bptr, const int32_t* __restrict__ src,
    const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
    const double* __restrict__ val, const double* __restrict__ B, int64_t ldb, int64_t k,
    int64_t d, double scale, const int64_t* __restrict__ rawoff, int32_t* __restrict__ ucnt,
    int32_t* __restrict__ sacol, double* __restrict__ saval, double* __restrict__ Sb) {
    __shared__ uint64_t keys[SA_SORT_CAP];
    __shared__ double vals[SA_SORT_CAP];
    __shared__ int32_t flag[SA_RANGE];
    const int64_t b = blockIdx.x;
    const int lane = threadIdx.x;
    const int32_t p0 = bptr[b], p1 = bptr[b + 1];
    const int64_t off = rawoff[b], raw = rawoff[b + 1] - off;
    // right-hand sides
    for (int64_t t = lane; t < k; t += 64) {
        double acc = 0.0;
        for (int32_t pp = p0; pp < p1; ++pp) {
            const int32_t e = src[pp];
            const int64_t i = (int64_t)((uint32_t)e >> 1);
            const double x = B[i * ldb + t];
            acc = (e & 1) ? acc - x : acc + x;
        }
        Sb[b * k + t] = acc * scale;
    }
    int64_t total = 0;
    if (raw <= SA_SORT_CAP) {
        int npow = 1;
        while (npow < raw) npow <<= 1;
        // gather (column << 32 | raw index), raw index in bucket order
        int64_t base = 0;
        for (int32_t pp = p0; pp < p1; ++pp) {
            const int32_t e = src[pp];
            const int64_t i = (int64_t)((uint32_t)e >> 1);
            const int64_t e0 = row_ptr[i], len = row_ptr[i + 1] - e0;
            for (int64_t q = lane; q < len; q += 64) {
                const int64_t ri = base + q;
                keys[ri] = ((uint64_t)(uint32_t)col[e0 + q] << 32) | (uint64_t)ri;
                const double x = val[e0 + q];
                vals[ri] = (e & 1) ? -x : x;
            }
            base += len;
        }
        for (int64_t q = raw + lane; q < npow; q += 64) keys[q] = ~0ull;
        __syncthreads();
        // bitonic sort of npow keys
        for (int size = 2; size <= npow; size <<= 1)
            for (int stride = size >> 1; stride > 0; stride >>= 1) {
                for (int i = lane; i < npow / 2; i += 64) {
                    const int lo = 2 * stride * (i / stride) + (i % stride), hi = lo + stride;
                    const bool up = (lo & size) == 0;
                    const uint64_t a = keys[lo], c = keys[hi];
                    if ((a > c) == up) {
                        keys[lo] = c;
                        keys[hi] = a;
                    }
                }
                __syncthreads();
            }
        // runs of equal column: the lane at a run's start sums it in raw order
        for (int64_t c0 = 0; c0 < raw; c0 += 64) {
            const int64_t i = c0 + lane;
            const uint32_t ci = i < raw ? (uint32_t)(keys[i] >> 32) : 0;
            const bool start = i < raw && (i == 0 || (uint32_t)(keys[i - 1] >> 32) != ci);
            const uint64_t mask = __ballot(start);
            if (start) {
                const int64_t slot = total + __popcll(mask & ((1ull << lane) - 1));
                double acc = 0.0;
                for (int64_t j = i; j < raw && (uint32_t)(keys[j] >> 32) == ci; ++j)
                    acc += vals[(uint32_t)keys[j]];
                sacol[off + slot] = (int32_t)ci;
                saval[off + slot] = acc * scale;
            }
            total += __popcll(mask);
        }
    } else {
        // wide bucket: column ranges of SA_RANGE, every row of the bucket read per range
        double* acc = (double*)vals;  // SA_RANGE <= SA_SORT_CAP doubles
        for (int64_t c0 = 0; c0 < d; c0 += SA_RANGE) {
            for (int q = lane; q < SA_RANGE; q += 64) {
                acc[q] = 0.0;
                flag[q] = 0;
            }
            __syncthreads();
            for (int32_t pp = p0; pp < p1; ++pp) {
                const int32_t e = src[pp];
                const int64_t i = (int64_t)((uint32_t)e >> 1);
                for (int64_t q = row_ptr[i] + lane; q < row_ptr[i + 1]; q += 64) {
                    const int64_t c = col[q];
                    if (c >= c0 && c < c0 + SA_RANGE) {
                        const double x = val[q];
                        acc[c - c0] = (e & 1) ? acc[c - c0] - x : acc[c - c0] + x;
                        flag[c - c0] = 1;
                    }
                }
                __syncthreads();  // single wave: this row's updates before the next row's
            }
            for (int q0 = 0; q0 < SA_RANGE; q0 += 64) {
                const bool on = flag[q0 + lane] != 0;
                const uint64_t mask = __ballot(on);
                if (on) {
                    const int64_t slot = total + __popcll(mask & ((1ull << lane) - 1));
                    sacol[off + slot] = (int32_t)(c0 + q0 + lane);
                    saval[off + slot] = acc[q0 + lane] * scale;
                }
                total += __popcll(mask);
            }
            __syncthreads();
        }
    }
    if (lane == 0) ucnt[b] = (int32_t)total;
}

// SA as a dense row-major m x (d + k) matrix (inspection)
__global__ void k_sa_dense(const int64_t* __restrict__ rawoff, const int32_t* __restrict__ ucnt,
                           const int32_t* __restrict__ sacol, const double* __restrict__ saval,
                           const double* __restrict__ Sb, int64_t d, int64_t k,
                           double* __restrict__ SA) {
    const int64_t b = blockIdx.x;
    const int64_t ld = d + k;
    for (int64_t c = threadIdx.x; c < ld; c += blockDim.x) SA[b * ld + c] = 0.0;
    __syncthreads();
    for (int64_t u = threadIdx.x; u < ucnt[b]; u += blockDim.x)
        SA[b * ld + sacol[rawoff[b] + u]] = saval[rawoff[b] + u];
    for (int64_t t = threadIdx.x; t < k; t += blockDim.x) SA[b * ld + d + t] = Sb[b * k + t];
}

// ---------------------------------------------------------------------------------------
// numeric factorisation of the leaf fronts
struct FrontArgs {
    const int64_t* lptr;
    const int32_t* relmap;
    const int64_t* srcptr;
    const int32_t* srca;
    const int32_t* srcb;
    const int64_t* cboff;
    const int32_t* entlc;
    const int64_t* rawoff;
    const int32_t* ucnt;
    const double* saval;
    const double* Sb;
    int64_t k;
    double* rdiag;
    double* rv;
    double* cleaf;
    double* cb;
    int* nonfinite;  // set to 1 when an assembled value is not finite
};

// tile row r <- its source: a sketch row (scattered by the entries' local columns, then the
// right-hand sides) or a contribution row of a child (through the child's column map)
__device__ __forceinline__ void front_fill_row(double* Trow, const FrontArgs& a, int64_t si, int ncA,
                                               int lane) {
    const int32_t s0 = a.srca[si], s1 = a.srcb[si];
    if (s1 < 0) {
        const int64_t o = a.rawoff[s0];
        const int32_t len = a.ucnt[s0];
        bool bad = false;
        for (int32_t u = lane; u < len; u += 64) {
            const double v = a.saval[o + u];
            bad = bad || !isfinite(v);
            Trow[a.entlc[o + u]] = v;
        }
        for (int64_t t = lane; t < a.k; t += 64) {
            const double v = a.Sb[(int64_t)s0 * a.k + t];
            bad = bad || !isfinite(v);
            Trow[ncA + t] = v;
        }
        if (bad) *a.nonfinite = 1;  // every writer writes the same value
    } else {
        const int64_t nlc = a.lptr[s0 + 1] - a.lptr[s0];
        const int64_t w = nlc + a.k;
        const double* cbr = a.cb + a.cboff[s0] + (int64_t)s1 * w;
        const int32_t* rm = a.relmap + a.lptr[s0];
        for (int64_t u = lane; u < w; u += 64) {
            const int lc = u < nlc ? rm[u] : (int)(ncA + (u - nlc));
            Trow[lc] = cbr[u];
        }
    }
}

// Householder QR of the tile's rows [0, rows) over its A columns [0, ncA), the reflections
// applied to all nct columns; below-diagonal entries are left at exact zero.  One wave forms
// each reflector (LAPACK's convention: beta = -sign(alpha) ||x||, tau = (beta - alpha) /
// beta, v = x / (alpha - beta), no reflection when x below the diagonal is zero); four
// threads per column form v^T T and update it, in a fixed order.
__device__ void front_qr(double* T, double* vs, double* wpart, double* sh, int rows, int ncA,
                         int nct) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int steps = min(rows, ncA);
    for (int p = 0; p < steps; ++p) {
        if (wave == 0) {
            double sg = 0.0;
            for (int i = p + 1 + lane; i < rows; i += 64) {
                const double x = T[i * FT_LD + p];
                sg += x * x;
            }
            for (int o = 32; o > 0; o >>= 1) sg += __shfl_xor(sg, o);
            const double alpha = T[p * FT_LD + p];
            double tau = 0.0, beta = alpha, scal = 0.0;
            if (sg > 0.0) {
                beta = -copysign(sqrt(alpha * alpha + sg), alpha);
                tau = (beta - alpha) / beta;
                scal = 1.0 / (alpha - beta);
            }
            for (int i = p + 1 + lane; i < rows; i += 64) {
                vs[i] = T[i * FT_LD + p] * scal;
                T[i * FT_LD + p] = 0.0;
            }
            if (lane == 0) {
                vs[p] = 1.0;
                T[p * FT_LD + p] = beta;
                sh[0] = tau;
            }
        }
        __syncthreads();
        const double tau = sh[0];
        const int ncol = nct - p - 1;
        if (tau != 0.0 && ncol > 0) {
            const int q = tid & 3, jj = tid >> 2;
            const int j = p + 1 + jj;
            if (jj < ncol) {
                double part = 0.0;
                for (int i = p + q; i < rows; i += 4) part += vs[i] * T[i * FT_LD + j];
                wpart[q * 64 + jj] = part;
            }
            __syncthreads();
            if (jj < ncol) {
                const double w = ((wpart[jj] + wpart[64 + jj]) + wpart[128 + jj]) + wpart[192 + jj];
                const double tw = tau * w;
                for (int i = p + q; i < rows; i += 4) T[i * FT_LD + j] -= vs[i] * tw;
            }
            __syncthreads();
        }
    }
}

__global__ __launch_bounds__(FT_THREADS) void k_front_level(const int32_t* __restrict__ fronts,
                                                             FrontArgs a) {
    __shared__ double T[FT_ROWS * FT_LD];
    __shared__ double vs[FT_ROWS];
    __shared__ double wpart[4 * 64];
    __shared__ double sh[2];
    const int32_t f = fronts[blockIdx.x];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nl = (int)(a.lptr[f + 1] - a.lptr[f]);
    const int ncA = 1 + nl;
    const int nct = ncA + (int)a.k;
    const int64_t s0 = a.srcptr[f];
    const int64_t total = a.srcptr[f + 1] - s0;
    int ra = 0;
    for (int64_t cur = 0; cur < total;) {
        const int cnt = (int)std::min<int64_t>(FT_ROWS - ra, total - cur);
        const int rows = ra + cnt;
        for (int idx = tid; idx < cnt * nct; idx += FT_THREADS)
            T[(ra + idx / nct) * FT_LD + idx % nct] = 0.0;
        __syncthreads();
        for (int r = ra + wave; r < rows; r += FT_THREADS / 64)
            front_fill_row(&T[r * FT_LD], a, s0 + cur + (r - ra), ncA, lane);
        __syncthreads();
        front_qr(T, vs, wpart, sh, rows, ncA, nct);
        ra = min(rows, ncA);
        cur += cnt;
        __syncthreads();
    }
    // the pivot row of R (diagonal made non-negative; c rides along), then the
    // contribution block: rows 1 .. ra-1, columns 1 .. nct-1
    const double sgn = (total > 0 && T[0] < 0.0) ? -1.0 : 1.0;
    if (tid == 0) a.rdiag[f] = total > 0 ? sgn * T[0] : 0.0;
    for (int u = tid; u < nl; u += FT_THREADS) a.rv[a.lptr[f] + u] = total > 0 ? sgn * T[1 + u] : 0.0;
    for (int t = tid; t < (int)a.k; t += FT_THREADS)
        a.cleaf[(int64_t)f * a.k + t] = total > 0 ? sgn * T[ncA + t] : 0.0;
    if (ra > 1) {
        double* cbf = a.cb + a.cboff[f];
        const int w = nct - 1;
        for (int idx = tid; idx < (ra - 1) * w; idx += FT_THREADS) {
            const int r = 1 + idx / w, c = 1 + idx % w;
            cbf[idx] = T[r * FT_LD + c];
        }
    }
}

// the root front: one wave per assembled row
__global__ void k_root_assemble(FrontArgs a, int64_t nleaf, int64_t nroot, int64_t rows,
                                double* __restrict__ root) {
    const int64_t r = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (r >= rows) return;
    const int64_t ld = nroot + a.k;
    front_fill_row(root + r * ld, a, a.srcptr[nleaf] + r, (int)nroot, lane);
}

__global__ void k_gather_tval(const int64_t* __restrict__ tent, const double* __restrict__ rv,
                              int64_t n, double* __restrict__ tval) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) tval[i] = rv[tent[i]];
}

__global__ void k_dense_R(const int64_t* __restrict__ lptr, const int32_t* __restrict__ lcol,
                          const double* __restrict__ rdiag, const double* __restrict__ rv,
                          const double* __restrict__ Rroot, int64_t nleaf, int64_t d,
                          double* __restrict__ R) {
    const int64_t q = blockIdx.x;
    for (int64_t c = threadIdx.x; c < d; c += blockDim.x) R[q * d + c] = 0.0;
    __syncthreads();
    if (q < nleaf) {
        if (threadIdx.x == 0) R[q * d + q] = rdiag[q];
        for (int64_t e = lptr[q] + threadIdx.x; e < lptr[q + 1]; e += blockDim.x)
            R[q * d + lcol[e]] = rv[e];
    } else {
        const int64_t nr = d - nleaf, i = q - nleaf;
        for (int64_t c = threadIdx.x; c < nr; c += blockDim.x)
            R[q * d + nleaf + c] = Rroot[i * nr + c];
    }
}

__global__ void k_copy_rows(const double* __restrict__ src, int64_t rows, int64_t cols,
                            double* __restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < rows * cols) dst[i] = src[i];
}

// ---------------------------------------------------------------------------------------
// triangular solves over the leaf forest: workgroup g walks its group's levels; row f of a
// level only needs values of earlier levels of the same trees (or of the root), written
// by this workgroup before the barrier that ends the level
struct SolveArgs {
    const int32_t* rows;
    const int64_t* gptr;
    const int64_t* lbptr;
    const int64_t* lb;
    int64_t G;
    const int64_t* ptr;  // lptr (upper) or tptr (lower)
    const int32_t* idx;  // lcol (upper) or trow (lower)
    const double* v;     // rv (upper) or tval (lower)
    const double* rdiag;
    const double* ladd;
    const int32_t* perm;
    int64_t nleaf, d;
};

// sum over the entries [e0, e1) of v[e] tmp[idx[e] k + t]: lanes take every 64th entry,
// then a butterfly over the wave (a fixed order, so the result is deterministic)
__device__ __forceinline__ double wave_dot(const SolveArgs& a, int64_t e0, int64_t e1,
                                           const double* tmp, int k, int t, int lane) {
    double part = 0.0;
    for (int64_t e = e0 + lane; e < e1; e += 64) part += a.v[e] * tmp[(int64_t)a.idx[e] * k + t];
    for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o);
    return part;
}

// One row of a level, for one right-hand side: what does not depend on earlier levels
// (the row's index, its entries' columns and values, its diagonal and right-hand side) is
// loaded before the level's barrier, so that only the values of tmp are read after it.
// Rows of up to 64 entries are held one entry per lane; longer ones loop.
struct RowPre {
    int64_t f, e0, e1;
    int32_t id;
    double v, dg, xv;
};

template <bool UPPER>
__device__ __forceinline__ void row_pre(const SolveArgs& a, const double* __restrict__ x, int64_t ldx,
                                        int64_t i, int lane, RowPre& p) {
    p.f = a.rows[i];
    p.e0 = a.ptr[p.f];
    p.e1 = a.ptr[p.f + 1];
    const int64_t e = p.e0 + lane;
    const bool has = e < p.e1;
    p.id = has ? a.idx[e] : 0;
    p.v = has ? a.v[e] : 0.0;
    p.dg = a.rdiag[p.f] + a.ladd[p.f];
    p.xv = UPPER ? x[p.f * ldx] : x[(int64_t)a.perm[p.f] * ldx];
}

// the row's sum after the barrier (k = 1): the held entry, the rest of a long row, then a
// butterfly over the wave
__device__ __forceinline__ double row_sum(const SolveArgs& a, const RowPre& p, const double* tmp,
                                          int lane) {
    double part = p.e0 + lane < p.e1 ? p.v * tmp[p.id] : 0.0;
    for (int64_t e = p.e0 + 64 + lane; e < p.e1; e += 64) part += a.v[e] * tmp[a.idx[e]];
    for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o);
    return part;
}

// upper: tmp[f] = (x[f] - sum_e R_f,lcol[e] tmp[lcol[e]]) / r_ff, y[perm[f]] = s tmp[f],
// one wave per row of a level; the workgroups past G scatter the root's values (already in
// tmp) to y
__global__ __launch_bounds__(SOLVE_THREADS) void k_leaf_upper(SolveArgs a, const double* __restrict__ x,
                                                              int64_t ldx, double* tmp,
                                                              double* __restrict__ y, int64_t ldy,
                                                              int k, double s,
                                                              const int32_t* __restrict__ done) {
    if (done && *done) return;
    const int64_t g = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int NW = SOLVE_THREADS / 64;
    if (g < a.G) {
        const int64_t l0 = a.lbptr[g], l1 = a.lbptr[g + 1];
        if (k == 1) {
            RowPre p;
            bool have = l0 + 1 < l1 && a.lb[l0] + wave < a.lb[l0 + 1];
            if (have) row_pre<true>(a, x, ldx, a.lb[l0] + wave, lane, p);
            for (int64_t l = l0; l + 1 < l1; ++l) {
                const int64_t r0 = a.lb[l], r1 = a.lb[l + 1];
                for (int64_t i = r0 + wave; i < r1; i += NW) {
                    if (i != r0 + wave) row_pre<true>(a, x, ldx, i, lane, p);
                    const double sum = row_sum(a, p, tmp, lane);
                    if (lane == 0) {
                        const double yv = (p.xv - sum) / p.dg;
                        tmp[p.f] = yv;
                        y[(int64_t)a.perm[p.f] * ldy] = s * yv;
                    }
                }
                // the next level's first row, loaded before the barrier
                have = l + 2 < l1 && a.lb[l + 1] + wave < a.lb[l + 2];
                if (have) row_pre<true>(a, x, ldx, a.lb[l + 1] + wave, lane, p);
                __syncthreads();
            }
            return;
        }
        for (int64_t l = l0; l + 1 < l1; ++l) {
            const int64_t r0 = a.lb[l], r1 = a.lb[l + 1];
            for (int64_t i = r0 + wave; i < r1; i += NW) {
                const int64_t f = a.rows[i];
                const int64_t e0 = a.ptr[f], e1 = a.ptr[f + 1];
                const double dg = a.rdiag[f] + a.ladd[f];
                for (int t = 0; t < k; ++t) {
                    const double sum = wave_dot(a, e0, e1, tmp, k, t, lane);
                    if (lane == 0) {
                        const double yv = (x[f * ldx + t] - sum) / dg;
                        tmp[f * k + t] = yv;
                        y[(int64_t)a.perm[f] * ldy + t] = s * yv;
                    }
                }
            }
            __syncthreads();
        }
        return;
    }
    const int64_t nr = a.d - a.nleaf;
    for (int64_t w = (g - a.G) * SOLVE_THREADS + threadIdx.x; w < nr * k;
         w += (gridDim.x - a.G) * SOLVE_THREADS) {
        const int64_t q = a.nleaf + w / k;
        const int t = (int)(w % k);
        y[(int64_t)a.perm[q] * ldy + t] = s * tmp[q * k + t];
    }
}

// lower: tmp[f] = (x[perm[f]] - sum over the rows i below f with f in L_i of R_if tmp[i])
// / r_ff, y[f] = s tmp[f], one wave per row of a level
__global__ __launch_bounds__(SOLVE_THREADS) void k_leaf_lower(SolveArgs a, const double* __restrict__ x,
                                                              int64_t ldx, double* tmp,
                                                              double* __restrict__ y, int64_t ldy,
                                                              int k, double s,
                                                              const int32_t* __restrict__ done) {
    if (done && *done) return;
    const int64_t g = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int NW = SOLVE_THREADS / 64;
    const int64_t l0 = a.lbptr[g], l1 = a.lbptr[g + 1];
    if (k == 1) {
        RowPre p;
        bool have = l0 + 1 < l1 && a.lb[l0] + wave < a.lb[l0 + 1];
        if (have) row_pre<false>(a, x, ldx, a.lb[l0] + wave, lane, p);
        for (int64_t l = l0; l + 1 < l1; ++l) {
            const int64_t r0 = a.lb[l], r1 = a.lb[l + 1];
            for (int64_t i = r0 + wave; i < r1; i += NW) {
                if (i != r0 + wave) row_pre<false>(a, x, ldx, i, lane, p);
                const double sum = row_sum(a, p, tmp, lane);
                if (lane == 0) {
                    const double yv = (p.xv - sum) / p.dg;
                    tmp[p.f] = yv;
                    y[p.f * ldy] = s * yv;
                }
            }
            have = l + 2 < l1 && a.lb[l + 1] + wave < a.lb[l + 2];
            if (have) row_pre<false>(a, x, ldx, a.lb[l + 1] + wave, lane, p);
            __syncthreads();
        }
        return;
    }
    for (int64_t l = l0; l + 1 < l1; ++l) {
        const int64_t r0 = a.lb[l], r1 = a.lb[l + 1];
        for (int64_t i = r0 + wave; i < r1; i += NW) {
            const int64_t f = a.rows[i];
            const int64_t e0 = a.ptr[f], e1 = a.ptr[f + 1];
            const double dg = a.rdiag[f] + a.ladd[f];
            for (int t = 0; t < k; ++t) {
                const double sum = wave_dot(a, e0, e1, tmp, k, t, lane);
                if (lane == 0) {
                    const double yv = (x[(int64_t)a.perm[f] * ldx + t] - sum) / dg;
                    tmp[f * k + t] = yv;
                    y[f * ldy + t] = s * yv;
                }
            }
        }
        __syncthreads();
    }
}

// the root's right-hand side: tmp[q] = x[perm[q]] - sum over leaf rows i with q in L_i of
// R_iq tmp[i], q >= nleaf, one wave per position
__global__ __launch_bounds__(SOLVE_THREADS) void k_root_rhs(SolveArgs a, const double* __restrict__ x,
                                                            int64_t ldx, double* tmp, int k,
                                                            const int32_t* __restrict__ done) {
    if (done && *done) return;
    const int lane = threadIdx.x & 63;
    const int64_t q = a.nleaf + (int64_t)blockIdx.x * (SOLVE_THREADS / 64) + (threadIdx.x >> 6);
    if (q >= a.d) return;
    const int64_t e0 = a.ptr[q], e1 = a.ptr[q + 1];
    for (int t = 0; t < k; ++t) {
        const double sum = wave_dot(a, e0, e1, tmp, k, t, lane);
        if (lane == 0) tmp[q * k + t] = x[(int64_t)a.perm[q] * ldx + t] - sum;
    }
}

__global__ void k_leaf_copy(const double* __restrict__ src, int64_t n, int64_t k, int64_t lds,
                            double* __restrict__ dst, int64_t ldd) {
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= n * k) return;
    dst[(w / k) * ldd + w % k] = src[(w / k) * lds + w % k];
}

unsigned blocks_for(int64_t n, int threads) { return (unsigned)std::max<int64_t>(1, (n + threads - 1) / threads); }

}  // namespace

// ---------------------------------------------------------------------------------------
SparseQR::~SparseQR() {
    Buf* all[] = {&rawoff_, &ucnt_, &sacol_, &saval_, &sb_, &scan_, &i64_, &i32_,
                  &rdiag_, &rv_, &cleaf_, &cb_, &tval_, &flag_};
    for (Buf* b : all)
        if (b->p) (void)hipFree(b->p);
}

hipError_t SparseQR::ensure(Buf& b, size_t bytes) {
    bytes = std::max<size_t>(bytes, 256);
    if (b.bytes >= bytes) return hipSuccess;
    if (b.p) {
        hipError_t e = hipFree(b.p);
        b.p = nullptr;
        b.bytes = 0;
        if (e != hipSuccess) return e;
    }
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) {
        b.p = nullptr;
        return e;
    }
    b.bytes = bytes;
    return hipSuccess;
}

hipError_t SparseQR::sketch(const int64_t* row_ptr, const int32_t* col, const double* val, int64_t n,
                            int64_t d, const double* B, int64_t ldb, int64_t k,
                            const int32_t* bucket_ptr, const int32_t* src, int64_t m, double scale,
                            hipStream_t st) {
    (void)n;
    m_ = m;
    d_ = d;
    k_ = k;
    hipError_t e;
    if ((e = ensure(scan_, m * 8)) != hipSuccess) return e;
    if ((e = ensure(rawoff_, (m + 1) * 8)) != hipSuccess) return e;
    if ((e = ensure(ucnt_, m * 4)) != hipSuccess) return e;
    if ((e = ensure(sb_, m * k * 8)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_sa_raw, dim3(blocks_for(m, 256)), dim3(256), 0, st, bucket_ptr, src, row_ptr, m,
                       ptr<int64_t>(scan_));
    hipLaunchKernelGGL(k_scan_excl, dim3(1), dim3(1024), 0, st, ptr<int64_t>(scan_), m,
                       ptr<int64_t>(rawoff_));
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // the raw total bounds the sketch's entries: read it to size the arrays
    int64_t raw = 0;
    if ((e = hipMemcpyAsync(&raw, ptr<int64_t>(rawoff_) + m, 8, hipMemcpyDeviceToHost, st)) !=
        hipSuccess)
        return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    nraw_ = raw;
    if ((e = ensure(sacol_, raw * 4)) != hipSuccess) return e;
    if ((e = ensure(saval_, raw * 8)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_sa_build, dim3((unsigned)m), dim3(64), 0, st, bucket_ptr, src, row_ptr, col,
                       val, B, ldb, k, d, scale, ptr<int64_t>(rawoff_), ptr<int32_t>(ucnt_),
                       ptr<int32_t>(sacol_), ptr<double>(saval_), ptr<double>(sb_));
    return hipGetLastError();
}

bool SparseQR::analyse(int dmax, hipStream_t st, std::string& err) {
    const int64_t m = m_, d = d_, k = k_;
    std::vector<int64_t> rawoff(m + 1);
    std::vector<int32_t> ucnt(m), cols(std::max<int64_t>(nraw_, 1));
    hipError_t e = hipMemcpyAsync(rawoff.data(), rawoff_.p, (m + 1) * 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(ucnt.data(), ucnt_.p, m * 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && nraw_ > 0)
        e = hipMemcpyAsync(cols.data(), sacol_.p, nraw_ * 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        err = std::string("sparse analysis: ") + hipGetErrorString(e);
        return false;
    }
    nnz_sa_ = 0;
    for (int64_t b = 0; b < m; ++b) nnz_sa_ += ucnt[b];
    if (!sparse_symbolic(m, d, k, rawoff.data(), ucnt.data(), cols.data(), std::max<int64_t>(nraw_, 1),
                         dmax, 1024, sym_, err))
        return false;
    const SparseSymbolic& S = sym_;
    // upload: int64 arrays then int32 arrays, each carved at 256-byte boundaries
    std::vector<std::pair<const void*, size_t>> a64 = {
        {S.lptr.data(), S.lptr.size()},     {S.src_ptr.data(), S.src_ptr.size()},
        {S.cboff.data(), S.cboff.size()},   {S.lev_ptr.data(), S.lev_ptr.size()},
        {S.up.gptr.data(), S.up.gptr.size()}, {S.up.lbptr.data(), S.up.lbptr.size()},
        {S.up.lb.data(), S.up.lb.size()},   {S.lo.gptr.data(), S.lo.gptr.size()},
        {S.lo.lbptr.data(), S.lo.lbptr.size()}, {S.lo.lb.data(), S.lo.lb.size()},
        {S.tptr.data(), S.tptr.size()},     {S.tent.data(), S.tent.size()}};
    std::vector<std::pair<const void*, size_t>> a32 = {
        {S.lcol.data(), S.lcol.size()},       {S.relmap.data(), S.relmap.size()},
        {S.src_a.data(), S.src_a.size()},     {S.src_b.data(), S.src_b.size()},
        {S.ent_lc.data(), S.ent_lc.size()},   {S.lev_front.data(), S.lev_front.size()},
        {S.up.rows.data(), S.up.rows.size()}, {S.lo.rows.data(), S.lo.rows.size()},
        {S.trow.data(), S.trow.size()},       {S.perm.data(), S.perm.size()},
        {S.cbrows.data(), S.cbrows.size()}};
    auto carve = [](const std::vector<std::pair<const void*, size_t>>& v, size_t es,
                    std::vector<size_t>& off) {
        size_t o = 0;
        for (auto& p : v) {
            off.push_back(o);
            o += (p.second * es + 255) & ~(size_t)255;
        }
        return o;
    };
    std::vector<size_t> o64, o32;
    const size_t b64 = carve(a64, 8, o64), b32 = carve(a32, 4, o32);
    if ((e = ensure(i64_, b64)) != hipSuccess || (e = ensure(i32_, b32)) != hipSuccess) {
        err = std::string("sparse analysis: ") + hipGetErrorString(e);
        return false;
    }
    std::vector<char> h64(b64), h32(b32);
    for (size_t i = 0; i < a64.size(); ++i)
        if (a64[i].second) memcpy(h64.data() + o64[i], a64[i].first, a64[i].second * 8);
    for (size_t i = 0; i < a32.size(); ++i)
        if (a32[i].second) memcpy(h32.data() + o32[i], a32[i].first, a32[i].second * 4);
    e = hipMemcpyAsync(i64_.p, h64.data(), b64, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(i32_.p, h32.data(), b32, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);  // the host staging is freed below
    if (e != hipSuccess) {
        err = std::string("sparse analysis: ") + hipGetErrorString(e);
        return false;
    }
    const char* p64 = (const char*)i64_.p;
    const char* p32 = (const char*)i32_.p;
    lptr_ = (const int64_t*)(p64 + o64[0]);
    srcptr_ = (const int64_t*)(p64 + o64[1]);
    cboff_ = (const int64_t*)(p64 + o64[2]);
    levptr_ = (const int64_t*)(p64 + o64[3]);
    upg_ = (const int64_t*)(p64 + o64[4]);
    uplbp_ = (const int64_t*)(p64 + o64[5]);
    uplb_ = (const int64_t*)(p64 + o64[6]);
    log_ = (const int64_t*)(p64 + o64[7]);
    lolbp_ = (const int64_t*)(p64 + o64[8]);
    lolb_ = (const int64_t*)(p64 + o64[9]);
    tptr_ = (const int64_t*)(p64 + o64[10]);
    tent_ = (const int64_t*)(p64 + o64[11]);
    lcol_ = (const int32_t*)(p32 + o32[0]);
    relmap_ = (const int32_t*)(p32 + o32[1]);
    srca_ = (const int32_t*)(p32 + o32[2]);
    srcb_ = (const int32_t*)(p32 + o32[3]);
    entlc_ = (const int32_t*)(p32 + o32[4]);
    levfront_ = (const int32_t*)(p32 + o32[5]);
    uprows_ = (const int32_t*)(p32 + o32[6]);
    lorows_ = (const int32_t*)(p32 + o32[7]);
    trow_ = (const int32_t*)(p32 + o32[8]);
    perm_ = (const int32_t*)(p32 + o32[9]);
    cbrows_ = (const int32_t*)(p32 + o32[10]);
    const int64_t nl = S.nleaf, nnzl = (int64_t)S.lcol.size();
    if ((e = ensure(rdiag_, nl * 8)) != hipSuccess || (e = ensure(rv_, nnzl * 8)) != hipSuccess ||
        (e = ensure(cleaf_, nl * k * 8)) != hipSuccess ||
        (e = ensure(cb_, S.cb_total * 8)) != hipSuccess ||
        (e = ensure(tval_, nnzl * 8)) != hipSuccess || (e = ensure(flag_, 4)) != hipSuccess) {
        err = std::string("sparse analysis: ") + hipGetErrorString(e);
        return false;
    }
    return true;
}

namespace {
FrontArgs front_args(const int64_t* lptr, const int32_t* relmap, const int64_t* srcptr,
                     const int32_t* srca, const int32_t* srcb, const int64_t* cboff,
                     const int32_t* entlc, const int64_t* rawoff, const int32_t* ucnt,
                     const double* saval, const double* Sb, int64_t k, double* rdiag, double* rv,
                     double* cleaf, double* cb, int* nonfinite) {
    FrontArgs a;
    a.nonfinite = nonfinite;
    a.lptr = lptr;
    a.relmap = relmap;
    a.srcptr = srcptr;
    a.srca = srca;
    a.srcb = srcb;
    a.cboff = cboff;
    a.entlc = entlc;
    a.rawoff = rawoff;
    a.ucnt = ucnt;
    a.saval = saval;
    a.Sb = Sb;
    a.k = k;
    a.rdiag = rdiag;
    a.rv = rv;
    a.cleaf = cleaf;
    a.cb = cb;
    return a;
}
}  // namespace

hipError_t SparseQR::factor_leaves(hipStream_t st) {
    const SparseSymbolic& S = sym_;
    hipError_t e0 = hipMemsetAsync(flag_.p, 0, sizeof(int), st);
    if (e0 != hipSuccess) return e0;
    FrontArgs a = front_args(lptr_, relmap_, srcptr_, srca_, srcb_, cboff_, entlc_,
                             ptr<int64_t>(rawoff_), ptr<int32_t>(ucnt_), ptr<double>(saval_),
                             ptr<double>(sb_), k_, ptr<double>(rdiag_), ptr<double>(rv_),
                             ptr<double>(cleaf_), ptr<double>(cb_), ptr<int>(flag_));
    const int nlev = (int)S.lev_ptr.size() - 1;
    for (int l = 0; l < nlev; ++l) {
        const int64_t nf = S.lev_ptr[l + 1] - S.lev_ptr[l];
        if (nf <= 0) continue;
        hipLaunchKernelGGL(k_front_level, dim3((unsigned)nf), dim3(FT_THREADS), 0, st,
                           levfront_ + S.lev_ptr[l], a);
    }
    return hipGetLastError();
}

int64_t SparseQR::root_rows_pad() const { return std::max<int64_t>(sym_.root_rows, sym_.nroot); }

hipError_t SparseQR::assemble_root(double* root, hipStream_t st) {
    const SparseSymbolic& S = sym_;
    const int64_t nr = S.nroot, ld = nr + k_, rows = S.root_rows;
    if (nr <= 0) return hipSuccess;
    hipError_t e = hipMemsetAsync(root, 0, (size_t)root_rows_pad() * ld * 8, st);
    if (e != hipSuccess) return e;
    FrontArgs a = front_args(lptr_, relmap_, srcptr_, srca_, srcb_, cboff_, entlc_,
                             ptr<int64_t>(rawoff_), ptr<int32_t>(ucnt_), ptr<double>(saval_),
                             ptr<double>(sb_), k_, ptr<double>(rdiag_), ptr<double>(rv_),
                             ptr<double>(cleaf_), ptr<double>(cb_), ptr<int>(flag_));
    if (rows > 0)
        hipLaunchKernelGGL(k_root_assemble, dim3(blocks_for(rows, 4)), dim3(256), 0, st, a, S.nleaf, nr,
                           rows, root);
    return hipGetLastError();
}

hipError_t SparseQR::finish_factor(hipStream_t st) {
    const int64_t n = (int64_t)sym_.tent.size();
    if (n > 0)
        hipLaunchKernelGGL(k_gather_tval, dim3(blocks_for(n, 256)), dim3(256), 0, st, tent_,
                           ptr<double>(rv_), n, ptr<double>(tval_));
    return hipGetLastError();
}

const int* SparseQR::nonfinite_dev() const { return ptr<int>(flag_); }

hipError_t SparseQR::leaf_diag(double* out, hipStream_t st) const {
    if (sym_.nleaf <= 0) return hipSuccess;
    return hipMemcpyAsync(out, rdiag_.p, sym_.nleaf * 8, hipMemcpyDeviceToDevice, st);
}

hipError_t SparseQR::leaf_c(double* c, hipStream_t st) const {
    const int64_t n = sym_.nleaf * k_;
    if (n > 0)
        hipLaunchKernelGGL(k_copy_rows, dim3(blocks_for(n, 256)), dim3(256), 0, st,
                           ptr<double>(cleaf_), sym_.nleaf, k_, c);
    return hipGetLastError();
}

hipError_t SparseQR::leaves_upper(const double* x, int64_t ldx, double* tmp, double* y, int64_t ldy,
                                  int k, double s, const int32_t* done, hipStream_t st) const {
    const SparseSymbolic& S = sym_;
    SolveArgs a;
    a.rows = uprows_;
    a.gptr = upg_;
    a.lbptr = uplbp_;
    a.lb = uplb_;
    a.G = S.nleaf > 0 ? (int64_t)S.up.gptr.size() - 1 : 0;
    a.ptr = lptr_;
    a.idx = lcol_;
    a.v = ptr<double>(rv_);
    a.rdiag = ptr<double>(rdiag_);
    a.ladd = ladd_;
    a.perm = perm_;
    a.nleaf = S.nleaf;
    a.d = S.d;
    const int64_t scatter = S.nroot > 0 ? std::min<int64_t>(64, blocks_for(S.nroot * k, SOLVE_THREADS)) : 0;
    const int64_t grid = a.G + scatter;
    if (grid > 0)
        hipLaunchKernelGGL(k_leaf_upper, dim3((unsigned)grid), dim3(SOLVE_THREADS), 0, st, a, x, ldx,
                           tmp, y, ldy, k, s, done);
    return hipGetLastError();
}

hipError_t SparseQR::leaves_lower(const double* x, int64_t ldx, double* tmp, double* y, int64_t ldy,
                                  int k, double s, const int32_t* done, hipStream_t st) const {
    const SparseSymbolic& S = sym_;
    SolveArgs a;
    a.rows = lorows_;
    a.gptr = log_;
    a.lbptr = lolbp_;
    a.lb = lolb_;
    a.G = S.nleaf > 0 ? (int64_t)S.lo.gptr.size() - 1 : 0;
    a.ptr = tptr_;
    a.idx = trow_;
    a.v = ptr<double>(tval_);
    a.rdiag = ptr<double>(rdiag_);
    a.ladd = ladd_;
    a.perm = perm_;
    a.nleaf = S.nleaf;
    a.d = S.d;
    if (a.G > 0)
        hipLaunchKernelGGL(k_leaf_lower, dim3((unsigned)a.G), dim3(SOLVE_THREADS), 0, st, a, x, ldx,
                           tmp, y, ldy, k, s, done);
    if (S.nroot > 0)
        hipLaunchKernelGGL(k_root_rhs, dim3(blocks_for(S.nroot, SOLVE_THREADS / 64)),
                           dim3(SOLVE_THREADS), 0, st, a, x, ldx, tmp, k, done);
    return hipGetLastError();
}

hipError_t SparseQR::dense_R(const double* Rroot, double* R, hipStream_t st) const {
    const int64_t d = sym_.d;
    if (d <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_dense_R, dim3((unsigned)d), dim3(256), 0, st, lptr_, lcol_, ptr<double>(rdiag_),
                       ptr<double>(rv_), Rroot, sym_.nleaf, d, R);
    return hipGetLastError();
}

hipError_t SparseQR::dense_SA(double* SA, hipStream_t st) const {
    if (m_ <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sa_dense, dim3((unsigned)m_), dim3(256), 0, st, ptr<int64_t>(rawoff_),
                       ptr<int32_t>(ucnt_), ptr<int32_t>(sacol_), ptr<double>(saval_),
                       ptr<double>(sb_), d_, k_, SA);
    return hipGetLastError();
}

}  // namespace ski
