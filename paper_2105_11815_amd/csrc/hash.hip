// s-hashing matrix S_h (Definition of s-hashing, Section 2.2) and the sign diagonal D
// (Definition of HRHT, Section 4.3), drawn from Philox4x64-10 with key (seed, 0):
//   column j of S_h: blocks at counter (j, blk, 0, 0), words in order; a word w
//     proposes row floor((w >> 32) * m / 2^32) with sign -1 iff bit 0 of w is set; a
//     row already taken by this column is rejected; the column stops at s rows.
//   d_i: bit (i mod 64) of word ((i >> 6) mod 4) of the block at counter
//     (i >> 8, 0, 1, 0); d_i = -1 iff the bit is set.
// The s-hashing variant (Section 4) takes the rows of the first s words without rejection
// (a row drawn twice gets both entries).  Row sampling (the sampled transform that
// Section 7 compares hashing against) gives sketch row i the row floor((w >> 32) n / 2^32)
// of the block at counter (i, 0, 2, 0), word 0, with sign +.
// The bucket-sorted form (CSR of S_h by sketch row) is built by a deterministic,
// atomic-free sort of the unique keys (row << 32 | (j << 1 | neg)): every workgroup
// sorts a chunk of keys in LDS and counts its runs per bucket; a column-wise scan
// over chunks gives each chunk's offset inside every bucket; a scatter places each
// key at bucket start + chunk offset + rank within the chunk's run.  The result is the
// sorted order of the keys (equal keys, from a row that a column of the variant drew
// twice with the same sign, are interchangeable): columns, then signs, ascend inside a
// bucket, which fixes the floating-point order of the hashing sums.
#include "ski_internal.h"

namespace ski {

namespace {

constexpr int HT = 256;  // threads per workgroup

__global__ __launch_bounds__(HT) void k_hash_keys(int64_t ncols, uint32_t m, int s, uint64_t seed,
                                                  int replace, int32_t* colrows, int8_t* colneg,
                                                  uint64_t* keys) {
    int64_t j = (int64_t)blockIdx.x * HT + threadIdx.x;
    if (j >= ncols) return;
    int32_t taken[32];
    int got = 0;
    for (uint64_t blk = 0; got < s; ++blk) {
        P4 w = philox4x64_10((uint64_t)j, blk, 0, 0, seed, 0);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            if (got < s) {
                uint64_t word = w.x[t];
                uint32_t row = (uint32_t)(((word >> 32) * (uint64_t)m) >> 32);
                bool dup = false;
                if (!replace)
                    for (int q = 0; q < got; ++q) dup |= (taken[q] == (int32_t)row);
                if (!dup) {
                    int neg = (int)(word & 1ull);
                    taken[got] = (int32_t)row;
                    colrows[j * s + got] = (int32_t)row;
                    colneg[j * s + got] = (int8_t)neg;
                    keys[j * s + got] = ((uint64_t)row << 32) | (uint64_t)(((uint64_t)j << 1) | neg);
                    ++got;
                }
            }
        }
    }
}

// row sampling: key (i << 32 | row << 1) for sketch row i
__global__ __launch_bounds__(HT) void k_sample_keys(int64_t m, uint64_t nrows, uint64_t seed,
                                                    int32_t* colrows, int8_t* colneg,
                                                    uint64_t* keys) {
    const int64_t i = (int64_t)blockIdx.x * HT + threadIdx.x;
    if (i >= m) return;
    const P4 w = philox4x64_10((uint64_t)i, 0, 2, 0, seed, 0);
    const uint64_t row = ((w.x[0] >> 32) * nrows) >> 32;
    colrows[i] = (int32_t)row;
    colneg[i] = 0;
    keys[i] = ((uint64_t)i << 32) | (row << 1);
}

__global__ __launch_bounds__(HT) void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
    int64_t i = (int64_t)blockIdx.x * HT + threadIdx.x;
    for (; i < n; i += (int64_t)gridDim.x * HT) p[i] = v;
}

__device__ __forceinline__ int lower_bound_bucket(const uint64_t* a, int n, uint32_t b) {
    // first index with (a[i] >> 32) >= b in the sorted array a[0..n)
    int lo = 0, hi = n;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if ((uint32_t)(a[mid] >> 32) < b)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// sort one chunk of SORT_CHUNK keys in LDS (bitonic), write it back, count runs
__global__ __launch_bounds__(HT) void k_chunk_sort(const uint64_t* keys, int64_t nkeys,
                                                   uint64_t* sorted, int32_t* table,
                                                   int64_t nbuckets) {
    __shared__ uint64_t sk[SORT_CHUNK];
    const int64_t base = (int64_t)blockIdx.x * SORT_CHUNK;
    const int nvalid = (int)min((int64_t)SORT_CHUNK, nkeys - base);
    for (int i = threadIdx.x; i < SORT_CHUNK; i += HT) sk[i] = i < nvalid ? keys[base + i] : ~0ull;
    __syncthreads();
    for (int size = 2; size <= SORT_CHUNK; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = threadIdx.x; t < SORT_CHUNK / 2; t += HT) {
                int i = 2 * t - (t & (stride - 1));
                int jx = i + stride;
                bool up = ((i & size) == 0);
                uint64_t a = sk[i], b = sk[jx];
                if ((a > b) == up) {
                    sk[i] = b;
                    sk[jx] = a;
                }
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < nvalid; i += HT) {
        uint64_t key = sk[i];
        sorted[base + i] = key;
        uint32_t b = (uint32_t)(key >> 32);
        bool last = (i == nvalid - 1) || ((uint32_t)(sk[i + 1] >> 32) != b);
        if (last) {
            int start = lower_bound_bucket(sk, nvalid, b);
            table[(int64_t)blockIdx.x * nbuckets + b] = i - start + 1;
        }
    }
}

// per bucket: exclusive prefix of the chunk counts (in place) and the bucket total
__global__ __launch_bounds__(HT) void k_bucket_offsets(int32_t* table, int64_t nchunks,
                                                       int64_t nbuckets, int32_t* totals) {
    int64_t b = (int64_t)blockIdx.x * HT + threadIdx.x;
    if (b >= nbuckets) return;
    int32_t run = 0;
    for (int64_t g = 0; g < nchunks; ++g) {
        int32_t t = table[g * nbuckets + b];
        table[g * nbuckets + b] = run;
        run += t;
    }
    totals[b] = run;
}

// exclusive scan of totals[0..n) into ptr[0..n], one workgroup
__global__ __launch_bounds__(1024) void k_scan_ptr(int32_t* ptr, int64_t n) {
    __shared__ int32_t part[1024];
    __shared__ int32_t carry_s;
    if (threadIdx.x == 0) carry_s = 0;
    __syncthreads();
    for (int64_t base = 0; base < n; base += 1024) {
        int64_t i = base + threadIdx.x;
        int32_t v = i < n ? ptr[i] : 0;
        part[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            int32_t add = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
            __syncthreads();
            part[threadIdx.x] += add;
            __syncthreads();
        }
        int32_t incl = part[threadIdx.x];
        int32_t carry = carry_s;
        if (i < n) ptr[i] = carry + incl - v;
        __syncthreads();
        if (threadIdx.x == 1023) carry_s = carry + incl;
        __syncthreads();
    }
    if (threadIdx.x == 0) ptr[n] = carry_s;
}

__global__ __launch_bounds__(HT) void k_scatter(const uint64_t* sorted, int64_t nkeys,
                                                const int32_t* table, int64_t nbuckets,
                                                const int32_t* ptr, int32_t* out) {
    const int64_t base = (int64_t)blockIdx.x * SORT_CHUNK;
    const int nvalid = (int)min((int64_t)SORT_CHUNK, nkeys - base);
    const uint64_t* sk = sorted + base;
    for (int i = threadIdx.x; i < nvalid; i += HT) {
        uint64_t key = sk[i];
        uint32_t b = (uint32_t)(key >> 32);
        int rank = i - lower_bound_bucket(sk, nvalid, b);
        int64_t pos = (int64_t)ptr[b] + table[(int64_t)blockIdx.x * nbuckets + b] + rank;
        out[pos] = (int32_t)(uint32_t)(key & 0xffffffffull);
    }
}

__global__ __launch_bounds__(HT) void k_dsign(int64_t nblocks, uint64_t seed, uint32_t* bits) {
    int64_t q = (int64_t)blockIdx.x * HT + threadIdx.x;
    if (q >= nblocks) return;
    P4 w = philox4x64_10((uint64_t)q, 0, 1, 0, seed, 0);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        bits[q * 8 + 2 * t] = (uint32_t)(w.x[t] & 0xffffffffull);
        bits[q * 8 + 2 * t + 1] = (uint32_t)(w.x[t] >> 32);
    }
}

inline unsigned grid_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

int64_t hash_num_chunks(int64_t nkeys) { return (nkeys + SORT_CHUNK - 1) / SORT_CHUNK; }

hipError_t launch_bucket_sort(const uint64_t* keys_unsorted, int64_t nkeys, int64_t nbuckets,
                              uint64_t* keys_tmp, int32_t* table, int32_t* bucket_ptr,
                              int32_t* out_payload, hipStream_t st) {
    const int64_t nch = hash_num_chunks(nkeys);
    const int64_t tsize = nch * nbuckets;
    if (nkeys == 0) {
        hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(nbuckets + 1, HT)), dim3(HT), 0, st,
                           bucket_ptr, nbuckets + 1, 0);
        return hipGetLastError();
    }
    unsigned gfill = (unsigned)std::min<int64_t>(grid_for(tsize, HT), 65536);
    hipLaunchKernelGGL(k_fill_i32, dim3(gfill), dim3(HT), 0, st, table, tsize, 0);
    hipLaunchKernelGGL(k_chunk_sort, dim3((unsigned)nch), dim3(HT), 0, st, keys_unsorted, nkeys,
                       keys_tmp, table, nbuckets);
    hipLaunchKernelGGL(k_bucket_offsets, dim3(grid_for(nbuckets, HT)), dim3(HT), 0, st, table, nch,
                       nbuckets, bucket_ptr);
    hipLaunchKernelGGL(k_scan_ptr, dim3(1), dim3(1024), 0, st, bucket_ptr, nbuckets);
    hipLaunchKernelGGL(k_scatter, dim3((unsigned)nch), dim3(HT), 0, st, keys_tmp, nkeys, table,
                       nbuckets, bucket_ptr, out_payload);
    return hipGetLastError();
}

int64_t hash_num_keys(int64_t ncols, int64_t m, int s, int kind) {
    return kind == SKI_SAMPLE_ROWS ? m : ncols * s;
}

hipError_t launch_hash_build(int64_t ncols, int64_t m, int s, uint64_t seed, int kind,
                             HashBuffers& hb, hipStream_t st) {
    const int64_t nkeys = hash_num_keys(ncols, m, s, kind);
    // the unsorted keys go to the tail half of hb.keys (sized 2 * nchunks * CHUNK)
    uint64_t* unsorted = hb.keys + hash_num_chunks(nkeys) * SORT_CHUNK;
    if (kind == SKI_SAMPLE_ROWS)
        hipLaunchKernelGGL(k_sample_keys, dim3(grid_for(m, HT)), dim3(HT), 0, st, m,
                           (uint64_t)ncols, seed, hb.colrows, hb.colneg, unsorted);
    else
        hipLaunchKernelGGL(k_hash_keys, dim3(grid_for(ncols, HT)), dim3(HT), 0, st, ncols,
                           (uint32_t)m, s, seed, kind == SKI_HASH_VARIANT ? 1 : 0, hb.colrows,
                           hb.colneg, unsorted);
    SKI_HIP(hipGetLastError());
    return launch_bucket_sort(unsorted, nkeys, m, hb.keys, hb.table, hb.bucket_ptr, hb.src, st);
}

hipError_t launch_dsign(int64_t npad, uint64_t seed, uint32_t* bits, hipStream_t st) {
    int64_t nblocks = (npad + 255) / 256;
    hipLaunchKernelGGL(k_dsign, dim3(grid_for(nblocks, HT)), dim3(HT), 0, st, nblocks, seed, bits);
    return hipGetLastError();
}

}  // namespace ski
