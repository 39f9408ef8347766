// ski_sketch_noalloc: Step 1 of Algorithm 1 (S [A B], the same kernels as ski_sketch) for
// callers that cannot allocate device memory.  Every buffer the kernels need beyond the
// caller's inputs and output (the hash keys and their bucket sort, the D sign bits and the
// transform's column slab) is carved out of one file-scope device array, `scratch`, of
// NOALLOC_SCRATCH_BYTES.  Host code never passes the array's name to a kernel: its device
// address is looked up once per device with hipGetSymbolAddress and kept.
#include <mutex>
#include <string>

#include "ski.h"
#include "ski_internal.h"

namespace ski {

constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;

// the scratch of every ski_sketch_noalloc call on a device (one copy per device)
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
constexpr int SLAB_ALIGN_COLS = 16;  // the transform passes work on 16-column tiles

std::mutex g_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};
thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = "ski_sketch_noalloc: " + msg;
    return code;
}

// device address of `scratch` on the current device, looked up on the first call there
hipError_t scratch_ptr(unsigned char** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = (unsigned char*)g_scratch_ptr[dev];
    return hipSuccess;
}

size_t up256(size_t b) { return (b + 255) & ~(size_t)255; }

// the scratch layout of one call: byte offsets of each buffer, and the slab width
struct Layout {
    size_t colrows, colneg, bucket_ptr, src, keys, table, dbits, slab, end;
    int64_t sc;
};

// Lays the buffers out from offset 0; the slab takes what is left (a multiple of 16
// columns, at most ncols).  Returns false when the hash buffers, or the narrowest slab,
// do not fit.
bool layout(int64_t nkeys, int64_t m, int64_t npad, int64_t ncols, bool had, Layout& L) {
    const int64_t nch = hash_num_chunks(nkeys);
    size_t o = 0;
    L.colrows = o;
    o += up256((size_t)nkeys * 4);
    L.colneg = o;
    o += up256((size_t)nkeys);
    L.bucket_ptr = o;
    o += up256((size_t)(m + 1) * 4);
    L.src = o;
    o += up256((size_t)nkeys * 4);
    L.keys = o;
    o += up256((size_t)2 * nch * SORT_CHUNK * 8);
    L.table = o;
    o += up256((size_t)nch * m * 4);
    L.dbits = o;
    L.slab = o;
    L.sc = 0;
    if (had) {
        o += up256((size_t)((npad + 255) / 256) * 32);
        L.slab = o;
        if (o >= NOALLOC_SCRATCH_BYTES) return false;
        const size_t col_bytes = (size_t)npad * 8;
        int64_t sc = (int64_t)((NOALLOC_SCRATCH_BYTES - o) / col_bytes);
        sc = std::min<int64_t>(sc / SLAB_ALIGN_COLS * SLAB_ALIGN_COLS, ncols);
        if (sc < std::min<int64_t>(SLAB_ALIGN_COLS, ncols)) return false;
        L.sc = sc;
        o += up256((size_t)sc * col_bytes);
    }
    L.end = o;
    return o <= NOALLOC_SCRATCH_BYTES;
}

int64_t next_pow2(int64_t n) {
    int64_t p = 1;
    while (p < n) p <<= 1;
    return p;
}

}  // namespace

const char* noalloc_last_error() { return g_err.c_str(); }

}  // namespace ski

using namespace ski;

extern "C" int ski_sketch_noalloc(const ski_matrix* A, const double* B, int32_t k, int64_t ldb,
                                  const ski_params* p, double* SA, void* stream) {
    g_err.clear();
    if (!A || !B || !p || !SA) return fail(SKI_EINVAL, "NULL argument");
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = A->n, d = A->d;
    if (d < 1 || n < d) return fail(SKI_EINVAL, "need n >= d >= 1");
    if (n > ((int64_t)1 << 30)) return fail(SKI_EINVAL, "n above 2^30 rows");
    if (k < 1 || ldb < k) return fail(SKI_EINVAL, "need k >= 1 and ldb >= k");
    if (A->kind != SKI_DENSE && A->kind != SKI_CSR)
        return fail(SKI_EINVAL, "A must be SKI_DENSE (row-major) or SKI_CSR");
    if (A->kind == SKI_DENSE && (!A->a || A->lda < d))
        return fail(SKI_EINVAL, "dense A needs a and lda >= d");
    if (A->kind == SKI_CSR && (!A->row_ptr || !A->col || !A->val || A->nnz < 0 ||
                               A->nnz >= ((int64_t)1 << 31)))
        return fail(SKI_EINVAL, "CSR A needs row_ptr, col, val, nnz < 2^31");
    if (p->hadamard != 0 && p->hadamard != 1)
        return fail(SKI_EINVAL, "hadamard must be 0 or 1 (the Hartley transform is not offered)");
    if (A->kind == SKI_CSR && p->hadamard)
        return fail(SKI_EINVAL, "the Hadamard transform is for dense A only");
    if (p->sketch_prec != SKI_FP64 || p->qr_prec != SKI_FP64)
        return fail(SKI_EINVAL, "the sketch is formed in FP64 only (sketch_prec, qr_prec)");
    if (p->s < 1 || p->s > 32) return fail(SKI_EINVAL, "need 1 <= s <= 32");
    if (p->hash_kind < SKI_HASH || p->hash_kind > SKI_SAMPLE_ROWS)
        return fail(SKI_EINVAL, "unknown hash_kind");
    if (p->hash_kind == SKI_SAMPLE_ROWS && p->s != 1)
        return fail(SKI_EINVAL, "row sampling needs s = 1");
    const int64_t m = p->m > 0 ? p->m : (int64_t)ceil(p->gamma * (double)d - 1e-9);
    const bool had = A->kind == SKI_DENSE && p->hadamard;
    const int64_t npad = had ? next_pow2(n) : n;
    if (m < d) return fail(SKI_EINVAL, "need m >= d");
    if (m > npad) return fail(SKI_EINVAL, "need m <= n (n' with Hadamard)");
    if (p->s > m) return fail(SKI_EINVAL, "need s <= m");
    if (m > ((int64_t)1 << 30)) return fail(SKI_EINVAL, "m above 2^30");
    const int64_t ncols = d + k;
    const int64_t nkeys = hash_num_keys(npad, m, p->s, p->hash_kind);
    Layout Lo;
    if (!layout(nkeys, m, npad, ncols, had, Lo))
        return fail(SKI_EINVAL,
                    "problem too large for the " + std::to_string(NOALLOC_SCRATCH_BYTES >> 20) +
                        " MiB scratch (hash buffers of 10 bytes per key plus 4 m bytes per 4096 "
                        "keys, and with the Hadamard transform a slab of at least 16 columns "
                        "of n' doubles)");

    unsigned char* base = nullptr;
    hipError_t e = scratch_ptr(&base);
    if (e != hipSuccess) return fail(SKI_EDEVICE, std::string("scratch lookup: ") + hipGetErrorString(e));

    HashBuffers hb;
    hb.colrows = (int32_t*)(base + Lo.colrows);
    hb.colneg = (int8_t*)(base + Lo.colneg);
    hb.bucket_ptr = (int32_t*)(base + Lo.bucket_ptr);
    hb.src = (int32_t*)(base + Lo.src);
    hb.keys = (uint64_t*)(base + Lo.keys);
    hb.table = (int32_t*)(base + Lo.table);
    e = launch_hash_build(npad, m, p->s, p->seed, p->hash_kind, hb, st);
    if (e != hipSuccess) return fail(SKI_EDEVICE, std::string("hash build: ") + hipGetErrorString(e));
    const double hscale = p->hash_kind == SKI_SAMPLE_ROWS ? 1.0 : 1.0 / sqrt((double)p->s);
    if (had) {
        uint32_t* dbits = (uint32_t*)(base + Lo.dbits);
        e = launch_dsign(npad, p->seed, dbits, st);
        if (e == hipSuccess)
            e = launch_sketch_dense(A->a, A->lda, B, ldb, n, d, k, npad, dbits, base + Lo.slab,
                                    Lo.sc, hb.bucket_ptr, hb.src, m, hscale / sqrt((double)npad),
                                    Prec::F64, Prec::F64, SA, st);
    } else if (A->kind == SKI_DENSE) {
        e = launch_gather_plain(A->a, A->lda, B, ldb, d, k, hb.bucket_ptr, hb.src, m, hscale,
                                Prec::F64, Prec::F64, SA, st);
    } else {
        e = launch_gather_csr(A->row_ptr, A->col, A->val, B, ldb, d, k, hb.bucket_ptr, hb.src, m,
                              hscale, Prec::F64, Prec::F64, SA, st);
    }
    if (e != hipSuccess) return fail(SKI_EDEVICE, std::string("sketch: ") + hipGetErrorString(e));
    return SKI_OK;
}
