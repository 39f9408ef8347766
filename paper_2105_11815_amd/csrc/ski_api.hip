// The C interface declared in include/ski.h: handle, device buffers, argument checks and
// the orchestration of Algorithm 1's steps on one HIP stream.  All arithmetic runs in the
// kernels of hash.hip, sketch.hip, qr.hip, gemm.hip and lsqr.hip.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <memory>
#include <string>
#include <vector>

#include "lsqr.h"
#include "ski_internal.h"
#include "sparse_qr.h"

using namespace ski;

namespace {

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

}  // namespace

struct ski_handle_s {
    std::string err;
    // problem description from ski_sketch
    int32_t kind = SKI_DENSE;
    int64_t n = 0, d = 0, k = 0, m = 0, npad = 0, ncols_hash = 0, nkeys = 0;
    int s = 1;
    bool had = false;
    ski_params p{};
    Prec sprec = Prec::F64, qprec = Prec::F64;
    const double* A = nullptr;
    int64_t lda = 0;
    const int64_t* rp = nullptr;
    const int32_t* ci = nullptr;
    const double* va = nullptr;
    int64_t nnz = 0;
    const double* Bsk = nullptr;
    int64_t ldb = 0;
    bool sketched = false, factored = false;
    double cond_est = 0.0;
    // device buffers
    DevBuf colrows, colneg, bucket_ptr, src, keys, table, dbits, T0, SA;
    DevBuf Arow;  // row-major copy of a column-major dense A
    DevBuf R, c, Rinv, RinvT, diag_add, tri_tmp, gemm_ws;
    DevBuf qr_part, qr_W, qr_T, qr_Y, qr_tau;
    DevBuf tkeys, tkeys_tmp, ttable, tp, tpay, ti, tv;
    DevBuf u, t, v, h, delta, z, wp, g, gpart, upart, y, st;
    DevBuf done_cnt;  // arrival counter of the step kernels' status word (zero between steps)
    DevBuf csr_bad;   // the CSR structure check's flag
    DevBuf cg_r, cg_p, cg_q, t2, dtmp, gemm_ws2, gemm_ws3;
    // column-pivoted factor: workspace, the permutation, compact R_11, p x k staging
    DevBuf piv_part, pivd, Rc, ptmp;
    int64_t rank = 0;      // p: columns kept (d without pivoting)
    int panels_cqr = 0;    // pivoted factor: panels factored by CholeskyQR2
    bool pivoted = false;  // the last ski_factor pivoted
    bool cod = false;      // ... and formed the minimal-norm P (d x p in cod_m)
    DevBuf cod_a, cod_m;   // Rtop^T and work, then P = Pi Rtop^T (L^T L)^-1
    // the sparse QR of the sketch (qr_panel = SKI_QR_SPARSE): its sketch, structure and
    // factor; sroot holds the dense root front, sptmp the solves' d x k scratch
    std::unique_ptr<SparseQR> sp;
    bool sparse = false;  // the last ski_factor was the sparse one
    DevBuf sroot, sptmp;
    hipStream_t st2 = nullptr;           // second stream of the QR's look-ahead
    hipEvent_t qev[4] = {};
    hipStream_t st3 = nullptr;           // third stream: R^-1 formed during the QR
    hipEvent_t rev[2] = {};
    double* hdiag = nullptr;  // pinned host copy of diag(R)
    HostFlag pflag;           // the pivoted QR's per-panel flag, written by the device
    int64_t hdiag_n = 0;
    hipEvent_t ev[6] = {};
    bool ev_ok = false;
    // kernel-class timing (ski_set_profiling)
    bool prof = false;
    std::vector<hipEvent_t> pool;
    std::vector<std::pair<int, int>> open_pairs;  // (class, index of the start event)
    size_t pool_used = 0;
    uint32_t prof_mask = 0;      // classes timed (bit c: class c)
    bool prof_recording = false;  // the last prof_begin recorded a start event
    double prof_ms[SKI_PROF_CLASSES] = {};
    int64_t prof_cnt[SKI_PROF_CLASSES] = {};
};

namespace {

int fail(ski_handle h, int code, const std::string& msg) {
    if (h) h->err = msg;
    return code;
}

int hip_fail(ski_handle h, hipError_t e, const char* where) {
    return fail(h, e == hipErrorOutOfMemory ? SKI_ENOMEM : SKI_EDEVICE,
                std::string(where) + ": " + hipGetErrorString(e));
}

hipError_t ensure(DevBuf& b, size_t bytes) {
    if (bytes == 0) bytes = 16;
    if (b.bytes >= bytes) return hipSuccess;
    if (b.p) {
        hipError_t e = hipFree(b.p);
        if (e != hipSuccess) return e;
        b.p = nullptr;
        b.bytes = 0;
    }
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) {
        b.p = nullptr;
        return e;
    }
    b.bytes = bytes;
    return hipSuccess;
}

void release(DevBuf& b) {
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
}

template <typename T>
T* P(DevBuf& b) {
    return (T*)b.p;
}

#define SKI_TRY(h, expr, where)                        \
    do {                                               \
        hipError_t e__ = (expr);                       \
        if (e__ != hipSuccess) return hip_fail(h, e__, where); \
    } while (0)

size_t elem_bytes(Prec p) { return p == Prec::F64 ? 8 : (p == Prec::F32 ? 4 : 2); }

int64_t next_pow2(int64_t n) {
    int64_t q = 1;
    while (q < n) q <<= 1;
    return q;
}

constexpr int64_t PASS_WG = 512;  // workgroups of the fused dense LSQR pass

enum ProfClass {
    PC_PASS = 0, PC_REDUCE = 1, PC_TRIGEMV = 2, PC_SPMV = 3, PC_SPMVT = 4, PC_STEP = 5,
    PC_HASH = 6, PC_WHT = 7, PC_GATHER = 8, PC_QR = 9, PC_TRTRI = 10, PC_QR_HH = 11,
    PC_QR_PIV = 12, PC_SPARSE_SKETCH = 13, PC_SPARSE_FRONTS = 14, PC_SPARSE_ROOT = 15
};

hipEvent_t pool_event(ski_handle h) {
    if (h->pool_used == h->pool.size()) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        h->pool.push_back(e);
    }
    return h->pool[h->pool_used++];
}

// bracket the launches between prof_begin and prof_end with an event pair
void prof_begin(ski_handle h, int cls, hipStream_t st) {
    h->prof_recording = false;
    if (!h->prof || !((h->prof_mask >> cls) & 1u)) return;
    hipEvent_t e = pool_event(h);
    if (!e) return;
    (void)hipEventRecord(e, st);
    h->open_pairs.push_back({cls, (int)h->pool_used - 1});
    h->prof_recording = true;
}
void prof_end(ski_handle h, hipStream_t st) {
    // the end event directly follows its start event in the pool (pairs never nest)
    if (!h->prof_recording) return;
    h->prof_recording = false;
    hipEvent_t e = pool_event(h);
    if (!e) return;
    (void)hipEventRecord(e, st);
}
// sum the recorded pairs (after the stream has been synchronised) and recycle the events
void prof_collect(ski_handle h) {
    if (!h->prof) return;
    for (auto& pr : h->open_pairs) {
        const int i0 = pr.second;
        if ((size_t)(i0 + 1) >= h->pool_used) continue;
        float ms = 0;
        if (hipEventSynchronize(h->pool[i0 + 1]) == hipSuccess &&
            hipEventElapsedTime(&ms, h->pool[i0], h->pool[i0 + 1]) == hipSuccess) {
            h->prof_ms[pr.first] += ms;
            h->prof_cnt[pr.first] += 1;
        }
    }
    h->open_pairs.clear();
    h->pool_used = 0;
}
constexpr int CHECK_EVERY = 8;    // LSQR iterations between status reads

}  // namespace

extern "C" {

int ski_create(ski_handle* h) {
    if (!h) return SKI_EINVAL;
    ski_handle_s* x = new (std::nothrow) ski_handle_s();
    if (!x) return SKI_ENOMEM;
    bool ok = true;
    for (auto& e : x->ev) ok = ok && hipEventCreate(&e) == hipSuccess;
    x->ev_ok = ok;
    *h = x;
    return ok ? SKI_OK : SKI_EDEVICE;
}

int ski_destroy(ski_handle h) {
    if (!h) return SKI_EINVAL;
    (void)hipDeviceSynchronize();
    DevBuf* all[] = {&h->colrows, &h->colneg, &h->bucket_ptr, &h->src, &h->keys, &h->table,
                     &h->dbits, &h->T0, &h->SA, &h->Arow, &h->R, &h->c, &h->Rinv, &h->RinvT,
                     &h->diag_add, &h->tri_tmp, &h->gemm_ws, &h->qr_part, &h->qr_W, &h->qr_T,
                     &h->qr_Y, &h->qr_tau, &h->tkeys, &h->tkeys_tmp, &h->ttable, &h->tp,
                     &h->tpay, &h->ti, &h->tv, &h->u, &h->t, &h->v, &h->h, &h->delta, &h->z,
                     &h->wp, &h->g, &h->gpart, &h->upart, &h->y, &h->st, &h->cg_r,
                     &h->cg_p, &h->cg_q, &h->t2, &h->dtmp, &h->gemm_ws2, &h->gemm_ws3,
                     &h->piv_part, &h->pivd, &h->Rc, &h->ptmp, &h->cod_a, &h->cod_m,
                     &h->done_cnt, &h->csr_bad, &h->sroot, &h->sptmp};
    for (DevBuf* b : all) release(*b);
    if (h->ev_ok)
        for (auto& e : h->ev) (void)hipEventDestroy(e);
    for (auto& e : h->pool) (void)hipEventDestroy(e);
    for (auto& e : h->qev)
        if (e) (void)hipEventDestroy(e);
    for (auto& e : h->rev)
        if (e) (void)hipEventDestroy(e);
    if (h->st2) (void)hipStreamDestroy(h->st2);
    if (h->st3) (void)hipStreamDestroy(h->st3);
    if (h->hdiag) (void)hipHostFree(h->hdiag);
    if (h->pflag.host) (void)hipHostFree((void*)h->pflag.host);
    delete h;
    return SKI_OK;
}

void ski_params_default(int32_t kind, ski_params* p) {
    if (!p) return;
    memset(p, 0, sizeof(*p));
    p->tau_a = 1e-8;
    p->tau_r = 1e-6;
    p->it_max = 10000;
    p->seed = 1;
    p->sketch_prec = SKI_FP64;
    p->qr_prec = SKI_FP64;
    if (kind == SKI_CSR) {
        p->gamma = 1.4;
        p->s = 2;
        p->hadamard = 0;
        p->rcond = 0.0;
        p->rcond_thres = 1e-10;
        p->perturb = 1e-10;
    } else {
        p->gamma = 1.7;
        p->s = 1;
        p->hadamard = 1;
        p->rcond = 1e-12;
        p->rcond_thres = 1e-10;
        p->perturb = 0.0;
    }
}

const char* ski_last_error(ski_handle h) {
    if (h) return h->err.c_str();
    const char* e = noalloc_last_error();  // the handle-free entry point reports here
    return e[0] ? e : "null handle";
}

int ski_sketch(ski_handle h, const ski_matrix* A, const double* B, int32_t k, int64_t ldb,
               const ski_params* p, void* stream) {
    if (!h) return SKI_EINVAL;
    if (!A || !p || !B) return fail(h, SKI_EINVAL, "ski_sketch: NULL argument");
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = A->n, d = A->d;
    if (d < 1 || n < d) return fail(h, SKI_EINVAL, "ski_sketch: need n >= d >= 1");
    if (n > ((int64_t)1 << 30)) return fail(h, SKI_EINVAL, "ski_sketch: n above 2^30 rows");
    if (k < 1 || ldb < k) return fail(h, SKI_EINVAL, "ski_sketch: need k >= 1 and ldb >= k");
    if (A->kind != SKI_DENSE && A->kind != SKI_DENSE_COLMAJOR && A->kind != SKI_CSR)
        return fail(h, SKI_EINVAL, "ski_sketch: unknown matrix kind");
    if (A->kind == SKI_DENSE && (!A->a || A->lda < d))
        return fail(h, SKI_EINVAL, "ski_sketch: dense A needs a and lda >= d");
    if (A->kind == SKI_DENSE_COLMAJOR && (!A->a || A->lda < n))
        return fail(h, SKI_EINVAL, "ski_sketch: column-major A needs a and lda >= n");
    if (A->kind == SKI_DENSE_COLMAJOR && n > (int64_t)64 * 65535)
        return fail(h, SKI_EINVAL, "ski_sketch: column-major A above 4194240 rows");
    // a column-major A is copied to row-major below; from here on it is dense
    const int32_t akind = A->kind == SKI_DENSE_COLMAJOR ? (int32_t)SKI_DENSE : A->kind;
    if (A->kind == SKI_CSR && (!A->row_ptr || !A->col || !A->val || A->nnz < 0 ||
                               A->nnz >= ((int64_t)1 << 31)))
        return fail(h, SKI_EINVAL, "ski_sketch: CSR A needs row_ptr, col, val, nnz < 2^31");
    if (p->hadamard < 0 || p->hadamard > 2)
        return fail(h, SKI_EINVAL, "ski_sketch: hadamard must be 0, 1 or 2");
    if (akind == SKI_CSR && p->hadamard)
        return fail(h, SKI_EINVAL, "ski_sketch: the Hadamard transform is for dense A only");
    if (p->s < 1 || p->s > 32) return fail(h, SKI_EINVAL, "ski_sketch: need 1 <= s <= 32");
    if (p->qr_panel < SKI_QR_AUTO || p->qr_panel > SKI_QR_SPARSE)
        return fail(h, SKI_EINVAL, "ski_sketch: unknown qr_panel");
    if (p->qr_panel == SKI_QR_SPARSE &&
        (akind != SKI_CSR || p->sketch_prec != SKI_FP64 || p->qr_prec != SKI_FP64 || k > 32))
        return fail(h, SKI_EINVAL,
                    "ski_sketch: the sparse QR (SKI_QR_SPARSE) needs CSR A, FP64 sketch and QR, "
                    "and k <= 32");
    if (p->hash_kind < SKI_HASH || p->hash_kind > SKI_SAMPLE_ROWS)
        return fail(h, SKI_EINVAL, "ski_sketch: unknown hash_kind");
    if (p->hash_kind == SKI_SAMPLE_ROWS && p->s != 1)
        return fail(h, SKI_EINVAL, "ski_sketch: row sampling needs s = 1");
    if (p->qr_panel >= SKI_QR_PIVOTED && p->qr_prec != SKI_FP64)
        return fail(h, SKI_EINVAL, "ski_sketch: the pivoted factorisation needs qr_prec = SKI_FP64");
    if (p->sketch_prec < 0 || p->sketch_prec > 2 || p->qr_prec < 0 || p->qr_prec > 2)
        return fail(h, SKI_EINVAL, "ski_sketch: unknown precision");
    if (!(p->tau_r >= 0) || !(p->tau_a >= 0) || p->it_max < 1)
        return fail(h, SKI_EINVAL, "ski_sketch: bad tolerances or it_max");
    int64_t m = p->m > 0 ? p->m : (int64_t)ceil(p->gamma * (double)d - 1e-9);
    const bool had = (akind == SKI_DENSE) && p->hadamard;
    const int64_t npad = had ? next_pow2(n) : n;
    if (m < d) return fail(h, SKI_EINVAL, "ski_sketch: need m >= d");
    if (m > npad) return fail(h, SKI_EINVAL, "ski_sketch: need m <= n (n' with Hadamard)");
    if (had && p->hadamard == 2 &&
        (!dht_supported(npad) || p->sketch_prec != SKI_FP64 || p->qr_prec != SKI_FP64))
        return fail(h, SKI_EINVAL,
                    "ski_sketch: the Hartley transform needs n' <= 2^24 and FP64 sketch and QR");
    if (p->s > m) return fail(h, SKI_EINVAL, "ski_sketch: need s <= m");
    // the dense QR keeps a column of up to 12288 rows in one workgroup's registers; the
    // sparse factorisation only sends its root front there (checked by ski_factor)
    if (m > 12288 && p->qr_panel != SKI_QR_SPARSE)
        return fail(h, SKI_EINVAL, "ski_sketch: m above 12288 is not supported");
    const int64_t ncols = d + k;
    Prec sprec = (Prec)p->sketch_prec, qprec = (Prec)p->qr_prec;
    // the sketch storage follows the QR precision: FP64 QR needs an FP64 sketch
    if (qprec == Prec::F64) sprec = Prec::F64;

    h->kind = akind;
    h->n = n;
    h->d = d;
    h->k = k;
    h->m = m;
    h->npad = npad;
    h->s = p->s;
    h->had = had;
    h->p = *p;
    h->p.m = m;
    h->sprec = sprec;
    h->qprec = qprec;
    h->A = A->a;
    h->lda = A->lda;
    if (A->kind == SKI_DENSE_COLMAJOR) {
        SKI_TRY(h, ensure(h->Arow, n * d * 8), "alloc");
        SKI_TRY(h, launch_colmajor_to_rowmajor(A->a, A->lda, n, d, P<double>(h->Arow), st),
                "transpose");
        h->A = P<double>(h->Arow);
        h->lda = d;
    }
    h->rp = A->row_ptr;
    h->ci = A->col;
    h->va = A->val;
    h->nnz = A->nnz;
    h->Bsk = B;
    h->ldb = ldb;
    h->sketched = h->factored = false;
    if (akind == SKI_CSR) {
        // the structure is checked before any kernel indexes with it
        int bad = 0;
        SKI_TRY(h, ensure(h->csr_bad, sizeof(int)), "alloc");
        SKI_TRY(h, hipMemsetAsync(h->csr_bad.p, 0, sizeof(int), st), "flag init");
        SKI_TRY(h, launch_check_csr(A->row_ptr, A->col, n, d, A->nnz, P<int>(h->csr_bad), st),
                "csr check");
        SKI_TRY(h, hipMemcpyAsync(&bad, h->csr_bad.p, sizeof(int), hipMemcpyDeviceToHost, st),
                "flag copy");
        SKI_TRY(h, hipStreamSynchronize(st), "sync");
        if (bad)
            return fail(h, SKI_EINVAL,
                        "ski_sketch: malformed CSR A (row offsets must rise from 0 to nnz and "
                        "column indices lie in [0, d))");
    }

    const int64_t nhc = npad;  // hashed columns of S_h
    h->ncols_hash = nhc;
    const int64_t nkeys = hash_num_keys(nhc, m, p->s, p->hash_kind);
    h->nkeys = nkeys;
    const int64_t nch = hash_num_chunks(nkeys);
    SKI_TRY(h, ensure(h->colrows, nkeys * 4), "alloc");
    SKI_TRY(h, ensure(h->colneg, nkeys), "alloc");
    SKI_TRY(h, ensure(h->bucket_ptr, (m + 1) * 4), "alloc");
    SKI_TRY(h, ensure(h->src, nkeys * 4), "alloc");
    SKI_TRY(h, ensure(h->keys, 2 * nch * SORT_CHUNK * 8), "alloc");
    SKI_TRY(h, ensure(h->table, (size_t)nch * m * 4), "alloc");
    // SA: FP64 in the FP64 form, FP32 in both mixed forms; the sparse QR keeps it sparse
    const bool sparse = p->qr_panel == SKI_QR_SPARSE;
    const size_t sa_e = qprec == Prec::F64 ? 8 : 4;
    if (!sparse) SKI_TRY(h, ensure(h->SA, (size_t)m * ncols * sa_e), "alloc");
    if (h->ev_ok) (void)hipEventRecord(h->ev[0], st);

    HashBuffers hb;
    hb.colrows = P<int32_t>(h->colrows);
    hb.colneg = P<int8_t>(h->colneg);
    hb.bucket_ptr = P<int32_t>(h->bucket_ptr);
    hb.src = P<int32_t>(h->src);
    hb.keys = P<uint64_t>(h->keys);
    hb.table = P<int32_t>(h->table);
    prof_begin(h, PC_HASH, st);
    SKI_TRY(h, launch_hash_build(nhc, m, p->s, p->seed, p->hash_kind, hb, st), "hash build");
    // the scalars of S: H's 1/sqrt(n') and the hashing's 1/sqrt(s) (sampling: value 1)
    const double hscale = p->hash_kind == SKI_SAMPLE_ROWS ? 1.0 : 1.0 / sqrt((double)p->s);
    prof_end(h, st);

    // gprec: the transform's arithmetic and slab type (sketch_prec); oprec: SA's storage,
    // FP64 for the FP64 QR, FP32 for the FP32 and BF16 QR forms (an FP64 sketch is then
    // rounded once, when it is written)
    const Prec gprec = sprec;
    const Prec oprec = qprec == Prec::F64 ? Prec::F64 : Prec::F32;
    // the hashing sums without a transform: FP64 for an FP64 sketch, else FP32
    const Prec hprec = sprec == Prec::F64 ? Prec::F64 : Prec::F32;
    if (akind == SKI_DENSE && had) {
        const size_t te = elem_bytes(gprec);
        SKI_TRY(h, ensure(h->dbits, ((npad + 255) / 256) * 32), "alloc");
        const int64_t sc = sketch_slab_cols(npad, ncols, gprec);
        SKI_TRY(h, ensure(h->T0, (size_t)npad * sc * te), "alloc");
        prof_begin(h, PC_WHT, st);
        SKI_TRY(h, launch_dsign(npad, p->seed, P<uint32_t>(h->dbits), st), "dsign");
        const double scale = hscale / sqrt((double)npad);
        if (p->hadamard == 2)
            SKI_TRY(h, launch_sketch_dht(h->A, h->lda, B, ldb, n, d, k, npad,
                                         P<uint32_t>(h->dbits), P<double>(h->T0), sc,
                                         P<int32_t>(h->bucket_ptr), P<int32_t>(h->src), m, scale,
                                         P<double>(h->SA), st),
                    "sketch (Hartley)");
        else
            SKI_TRY(h, launch_sketch_dense(h->A, h->lda, B, ldb, n, d, k, npad,
                                           P<uint32_t>(h->dbits), h->T0.p, sc,
                                           P<int32_t>(h->bucket_ptr), P<int32_t>(h->src), m, scale,
                                           gprec, oprec, h->SA.p, st),
                    "sketch");
        prof_end(h, st);
    } else if (akind == SKI_DENSE) {
        const double scale = hscale;
        SKI_TRY(h, launch_gather_plain(h->A, h->lda, B, ldb, d, k, P<int32_t>(h->bucket_ptr),
                                       P<int32_t>(h->src), m, scale, hprec, oprec, h->SA.p, st),
                "gather");
    } else {
        const double scale = hscale;
        if (sparse) {
            if (!h->sp) h->sp.reset(new (std::nothrow) SparseQR());
            if (!h->sp) return fail(h, SKI_ENOMEM, "ski_sketch: out of host memory");
            prof_begin(h, PC_SPARSE_SKETCH, st);
            SKI_TRY(h, h->sp->sketch(A->row_ptr, A->col, A->val, n, d, B, ldb, k,
                                     P<int32_t>(h->bucket_ptr), P<int32_t>(h->src), m, scale, st),
                    "sparse sketch");
            prof_end(h, st);
        } else {
            SKI_TRY(h, launch_gather_csr(A->row_ptr, A->col, A->val, B, ldb, d, k,
                                         P<int32_t>(h->bucket_ptr), P<int32_t>(h->src), m, scale,
                                         hprec, oprec, h->SA.p, st),
                    "gather csr");
        }
        // CSR of A^T for the transposed products of LSQR
        const int64_t nnz = A->nnz;
        const int64_t tch = hash_num_chunks(nnz);
        SKI_TRY(h, ensure(h->tkeys, nnz * 8), "alloc");
        SKI_TRY(h, ensure(h->tkeys_tmp, tch * SORT_CHUNK * 8), "alloc");
        SKI_TRY(h, ensure(h->ttable, (size_t)tch * d * 4), "alloc");
        SKI_TRY(h, ensure(h->tp, (d + 1) * 4), "alloc");
        SKI_TRY(h, ensure(h->tpay, nnz * 4), "alloc");
        SKI_TRY(h, ensure(h->ti, nnz * 4), "alloc");
        SKI_TRY(h, ensure(h->tv, nnz * 8), "alloc");
        SKI_TRY(h, build_csrT(A->row_ptr, A->col, A->val, n, d, nnz, P<uint64_t>(h->tkeys),
                              P<uint64_t>(h->tkeys_tmp), P<int32_t>(h->ttable), P<int32_t>(h->tp),
                              P<int32_t>(h->tpay), P<int32_t>(h->ti), P<double>(h->tv), st),
                "csr transpose");
    }
    if (h->ev_ok) (void)hipEventRecord(h->ev[1], st);
    h->sketched = true;
    return SKI_OK;
}

}  // extern "C"

namespace {

// The minimal-norm form of Step 2, after the pivoted factorisation truncated at p:
//   Rtop^T (d x p) = the transpose of R's first p rows (pivoted column order);
//   Rtop^T = Y L by the same QR (CholeskyQR2 panels, column-by-column if a panel fails),
//   L^-1 formed during it on the third stream, L^-T alongside;
//   P = Pi (Rtop^T L^-1) L^-T, rows scattered by the pivots, into cod_m (d x p).
// Rinv / RinvT then hold L^-1 / L^-T (p x p).  Uses the QR workspace of the sketch (the
// d x p factorisation needs less).
int cod_factor(ski_handle h, QrWs& ws, int64_t p, int* hflag, GemmWs& gw, hipStream_t st) {
    const int64_t d = h->d;
    SKI_TRY(h, ensure(h->cod_a, d * p * 8), "alloc");
    SKI_TRY(h, ensure(h->cod_m, d * p * 8), "alloc");
    double* Rt = P<double>(h->cod_a);
    double* Mw = P<double>(h->cod_m);
    // R (d x d row-major): its first p rows, read as a d x p column-major matrix (ld d)
    SKI_TRY(h, launch_colmajor_to_rowmajor(P<double>(h->R), d, d, p, Rt, st), "transpose");
    QrWs w2;
    qr_ws_carve(Prec::F64, h->qr_part.p, d, p, w2);
    w2.g = ws.g;
    w2.g2 = ws.g2;
    w2.st2 = ws.st2;
    w2.evF[0] = ws.evF[0];
    w2.evF[1] = ws.evF[1];
    w2.evE[0] = ws.evE[0];
    w2.evE[1] = ws.evE[1];
    SKI_TRY(h, ensure(h->gemm_ws3, rinv_ws_bytes(p)), "alloc");
    w2.Xinv = P<double>(h->Rinv);
    w2.Zinv = P<double>(h->tri_tmp);
    w2.g3.part = h->gemm_ws3.p;
    w2.g3.bytes = h->gemm_ws3.bytes;
    w2.st3 = h->st3;
    w2.evP = h->rev[0];
    w2.evI = h->rev[1];
    for (bool cqr = true;;) {
        w2.cqr_panels = cqr;
        SKI_TRY(h, qr_factor(Prec::F64, Rt, d, p, p, w2, st), "qr of Rtop^T");
        if (!cqr) break;
        SKI_TRY(h, hipMemcpyAsync(hflag, w2.cqr.flag, sizeof(int), hipMemcpyDeviceToHost, st),
                "flag copy");
        SKI_TRY(h, hipStreamSynchronize(st), "sync");
        if (*hflag == 0) break;
        cqr = false;  // a panel too ill-conditioned for CholeskyQR2: column by column
    }
    double* Li = P<double>(h->Rinv);
    double* LiT = P<double>(h->RinvT);
    SKI_TRY(h, rinv_finish((const double*)w2.Ac, d, p, Li, LiT, st), "L inverse");
    // Rt still holds Rtop^T (the QR copied it into its working copy)
    SKI_TRY(h, gemm_f64(false, false, d, p, p, 1.0, Rt, p, Li, p, 0.0, Mw, p, gw, st, 0,
                        GEMM_B_UPPER),
            "Rtop^T L^-1");
    SKI_TRY(h, gemm_f64(false, false, d, p, p, 1.0, Mw, p, LiT, p, 0.0, Rt, p, gw, st), "(.) L^-T");
    SKI_TRY(h, launch_permute_rows(Rt, p, Mw, p, P<int32_t>(h->pivd), d, p, true, st), "Pi");
    return SKI_OK;
}

// Step 2 in the sparse form of Section 6: the multifrontal QR of the sparse sketch
// (sparse_qr.h).  The leaf fronts give the leaf rows of R; the root front, assembled
// densely, is factored by the dense QR of the sketch (CholeskyQR2 panels, falling back to
// Householder columns), and its R^-1 is formed explicitly.  The guards of the dense path
// (rank, perturbation) apply to the whole diagonal.
int sparse_factor(ski_handle h, hipStream_t st) {
    const int64_t d = h->d, k = h->k;
    SparseQR& S = *h->sp;
    if (h->ev_ok) (void)hipEventRecord(h->ev[2], st);
    h->factored = false;
    h->sparse = false;
    std::string err;
    prof_begin(h, PC_SPARSE_FRONTS, st);
    if (!S.analyse((int)(63 - k), st, err)) return fail(h, SKI_EINVAL, "ski_factor: " + err);
    SKI_TRY(h, S.factor_leaves(st), "leaf fronts");
    prof_end(h, st);
    const int64_t nl = S.nleaf(), nr = S.nroot();
    SKI_TRY(h, ensure(h->c, d * k * 8), "alloc");
    SKI_TRY(h, ensure(h->dtmp, d * 8), "alloc");
    SKI_TRY(h, ensure(h->diag_add, d * 8), "alloc");
    SKI_TRY(h, ensure(h->pivd, d * 4), "alloc");
    SKI_TRY(h, ensure(h->sptmp, d * std::max<int64_t>(k, 1) * 8), "alloc");
    SKI_TRY(h, ensure(h->gemm_ws, (size_t)64 << 20), "alloc");
    if (h->hdiag_n < d) {
        if (h->hdiag) (void)hipHostFree(h->hdiag);
        h->hdiag = nullptr;
        h->hdiag_n = 0;
        SKI_TRY(h, hipHostMalloc((void**)&h->hdiag, (2 * d + 2) * 8, hipHostMallocDefault),
                "pinned");
        h->hdiag_n = d;
    }
    int* hflag = (int*)(h->hdiag + 2 * d);
    int* hnonfinite = (int*)(h->hdiag + 2 * d + 1);
    SKI_TRY(h, S.leaf_diag(P<double>(h->dtmp), st), "leaf diag");
    SKI_TRY(h, S.leaf_c(P<double>(h->c), st), "leaf c");
    SKI_TRY(h, hipMemcpyAsync(h->pivd.p, S.perm_dev(), d * 4, hipMemcpyDeviceToDevice, st),
            "perm copy");
    *hflag = 0;
    const int* root_nonfinite = nullptr;  // the root QR's own check of its front
    const void* root_ac = nullptr;  // the root's factored working copy (for R_h^-1)
    int64_t root_rows = 0;
    if (nr > 0 && S.root_rows_pad() > 12288) {
        char buf[240];
        snprintf(buf, sizeof buf,
                 "ski_factor: the root front of the sparse factorisation has %lld rows; its "
                 "dense QR takes at most 12288 (a larger gamma or a sparser A shrinks it)",
                 (long long)S.root_rows_pad());
        return fail(h, SKI_EINVAL, buf);
    }
    if (nr > 0) {
        prof_begin(h, PC_SPARSE_ROOT, st);
        const int64_t rows = S.root_rows_pad(), ncols = nr + k;
        SKI_TRY(h, ensure(h->sroot, (size_t)rows * ncols * 8), "alloc");
        SKI_TRY(h, S.assemble_root(P<double>(h->sroot), st), "root assembly");
        size_t gb = 0;
        SKI_TRY(h, ensure(h->qr_part, qr_ws_bytes(Prec::F64, rows, ncols, &gb)), "alloc");
        SKI_TRY(h, ensure(h->gemm_ws, std::max<size_t>(gb, (size_t)64 << 20)), "alloc");
        SKI_TRY(h, ensure(h->gemm_ws2, std::max<size_t>(gb, (size_t)64 << 20)), "alloc");
        if (!h->st2) {
            SKI_TRY(h, hipStreamCreateWithFlags(&h->st2, hipStreamNonBlocking), "stream");
            for (auto& e : h->qev) SKI_TRY(h, hipEventCreateWithFlags(&e, hipEventDisableTiming), "event");
            SKI_TRY(h, hipStreamCreateWithFlags(&h->st3, hipStreamNonBlocking), "stream");
            for (auto& e : h->rev) SKI_TRY(h, hipEventCreateWithFlags(&e, hipEventDisableTiming), "event");
        }
        SKI_TRY(h, ensure(h->R, nr * nr * 8), "alloc");
        SKI_TRY(h, ensure(h->Rinv, nr * nr * 8), "alloc");
        SKI_TRY(h, ensure(h->RinvT, nr * nr * 8), "alloc");
        SKI_TRY(h, ensure(h->tri_tmp, ((nr + 1) / 2 + 64) * ((nr + 1) / 2 + 64) * 8), "alloc");
        QrWs ws;
        qr_ws_carve(Prec::F64, h->qr_part.p, rows, ncols, ws);
        ws.g.part = h->gemm_ws.p;
        ws.g.bytes = h->gemm_ws.bytes;
        ws.g2.part = h->gemm_ws2.p;
        ws.g2.bytes = h->gemm_ws2.bytes;
        ws.st2 = h->st2;
        ws.evF[0] = h->qev[0];
        ws.evF[1] = h->qev[1];
        ws.evE[0] = h->qev[2];
        ws.evE[1] = h->qev[3];
        // the root's R_h^-1 formed block by block on the third stream during its QR, as in
        // the dense factorisation (used unless the perturbation applies)
        SKI_TRY(h, ensure(h->gemm_ws3, rinv_ws_bytes(nr)), "alloc");
        ws.Xinv = P<double>(h->Rinv);
        ws.Zinv = P<double>(h->tri_tmp);
        ws.g3.part = h->gemm_ws3.p;
        ws.g3.bytes = h->gemm_ws3.bytes;
        ws.st3 = h->st3;
        ws.evP = h->rev[0];
        ws.evI = h->rev[1];
        for (bool cqr = true;;) {
            ws.cqr_panels = cqr;
            SKI_TRY(h, qr_factor(Prec::F64, h->sroot.p, rows, ncols, nr, ws, st), "root qr");
            SKI_TRY(h, launch_extract_Rc(Prec::F64, ws, rows, nr, k, P<double>(h->R),
                                         P<double>(h->c) + nl * k, st),
                    "extract R");
            if (!cqr) break;
            SKI_TRY(h, hipMemcpyAsync(hflag, ws.cqr.flag, sizeof(int), hipMemcpyDeviceToHost, st),
                    "flag copy");
            SKI_TRY(h, hipStreamSynchronize(st), "sync");
            if (*hflag == 0) break;
            cqr = false;  // a panel too ill-conditioned for CholeskyQR2: column by column
        }
        SKI_TRY(h, launch_scale_copy(P<double>(h->R), nr, 1, nr + 1, 1.0, P<double>(h->dtmp) + nl,
                                     1, st),
                "diag gather");
        prof_end(h, st);
        root_ac = ws.Ac;
        root_rows = rows;
        root_nonfinite = ws.nonfinite;
    }
    // the fronts' and the root assembly's non-finite flag (set by both), then the root QR's
    SKI_TRY(h, hipMemcpyAsync(hnonfinite, S.nonfinite_dev(), sizeof(int), hipMemcpyDeviceToHost, st),
            "flag copy");
    if (root_nonfinite)
        SKI_TRY(h, hipMemcpyAsync(hflag, root_nonfinite, sizeof(int), hipMemcpyDeviceToHost, st),
                "flag copy");
    SKI_TRY(h, hipMemcpyAsync(h->hdiag, h->dtmp.p, d * 8, hipMemcpyDeviceToHost, st), "diag copy");
    SKI_TRY(h, hipStreamSynchronize(st), "sync");
    if (*hnonfinite || (root_nonfinite && *hflag))
        return fail(h, SKI_EINVAL, "ski_factor: the sketch holds a non-finite entry (A or B is not finite)");
    const double* Rd = h->hdiag;
    bool finite = true;
    for (int64_t i = 0; i < d; ++i) finite = finite && std::isfinite(Rd[i]);
    if (!finite) return fail(h, SKI_EINVAL, "ski_factor: non-finite R (overflow in the QR)");
    double amax = 0, amin = INFINITY;
    for (int64_t i = 0; i < d; ++i) {
        amax = std::max(amax, fabs(Rd[i]));
        amin = std::min(amin, fabs(Rd[i]));
    }
    h->cond_est = amin > 0 ? amax / amin : INFINITY;
    if (h->p.rcond > 0) {
        const double r11 = fabs(Rd[0]);
        for (int64_t i = 0; i < d; ++i)
            if (!(r11 > 0) || fabs(Rd[i]) < h->p.rcond * r11) {
                char buf[200];
                snprintf(buf, sizeof buf,
                         "rank guard failed at position %lld: |r_qq| = %.3e < rcond |r_11| "
                         "(r_11 = %.3e)",
                         (long long)i, fabs(Rd[i]), r11);
                return fail(h, SKI_ERANK, buf);
            }
    }
    double* add = h->hdiag + d;
    const bool pert = h->p.perturb > 0 && h->p.rcond_thres > 0 &&
                      h->cond_est >= 1.0 / h->p.rcond_thres;
    for (int64_t i = 0; i < d; ++i) add[i] = pert ? copysign(h->p.perturb, Rd[i]) : 0.0;
    SKI_TRY(h, hipMemcpyAsync(h->diag_add.p, add, d * 8, hipMemcpyHostToDevice, st), "perturb copy");
    if (nr > 0) {
        GemmWs gw;
        gw.part = h->gemm_ws.p;
        gw.bytes = h->gemm_ws.bytes;
        prof_begin(h, PC_TRTRI, st);
        if (!pert) {
            // the blocks of R_h^-1 are done (the QR's stream waited for them): R^-1 = R_h^-1 D
            SKI_TRY(h, rinv_finish((const double*)root_ac, root_rows, nr, P<double>(h->Rinv),
                                   P<double>(h->RinvT), st),
                    "root inverse");
        } else {
            SKI_TRY(h, trtri_upper(P<double>(h->R), nr, P<double>(h->Rinv), P<double>(h->RinvT),
                                   P<double>(h->diag_add) + nl, P<double>(h->tri_tmp), gw, st),
                    "root inverse");
        }
        prof_end(h, st);
    }
    S.set_root(P<double>(h->Rinv), P<double>(h->RinvT), P<double>(h->diag_add));
    SKI_TRY(h, S.finish_factor(st), "transposed values");
    h->sparse = true;
    h->pivoted = true;  // LSQR works in position order: z and x are scattered by perm
    h->cod = false;
    h->rank = d;
    if (h->ev_ok) (void)hipEventRecord(h->ev[3], st);
    SKI_TRY(h, hipStreamSynchronize(st), "sync");
    prof_collect(h);
    h->factored = true;
    return SKI_OK;
}

}  // namespace

extern "C" {

int ski_factor(ski_handle h, void* stream) {
    if (!h) return SKI_EINVAL;
    if (!h->sketched) return fail(h, SKI_ESTATE, "ski_factor: call ski_sketch first");
    hipStream_t st = (hipStream_t)stream;
    if (h->p.qr_panel == SKI_QR_SPARSE) return sparse_factor(h, st);
    h->sparse = false;
    const int64_t m = h->m, d = h->d, k = h->k, ncols = d + k;
    size_t gb = 0;
    const size_t qrb = qr_ws_bytes(h->qprec, m, ncols, &gb);
    SKI_TRY(h, ensure(h->qr_part, qrb), "alloc");
    const size_t gws = std::max<size_t>(gb, (size_t)64 << 20);
    SKI_TRY(h, ensure(h->gemm_ws, gws), "alloc");
    SKI_TRY(h, ensure(h->R, d * d * 8), "alloc");
    SKI_TRY(h, ensure(h->c, d * k * 8), "alloc");
    SKI_TRY(h, ensure(h->Rinv, d * d * 8), "alloc");
    SKI_TRY(h, ensure(h->RinvT, d * d * 8), "alloc");
    SKI_TRY(h, ensure(h->diag_add, d * 8), "alloc");
    SKI_TRY(h, ensure(h->tri_tmp, ((d + 1) / 2 + 64) * ((d + 1) / 2 + 64) * 8), "alloc");
    if (h->ev_ok) (void)hipEventRecord(h->ev[2], st);
    SKI_TRY(h, ensure(h->gemm_ws2, gws), "alloc");
    if (!h->st2) {
        // default priority (no priority argument), non-blocking with respect to stream 0
        SKI_TRY(h, hipStreamCreateWithFlags(&h->st2, hipStreamNonBlocking), "stream");
        for (auto& e : h->qev) SKI_TRY(h, hipEventCreateWithFlags(&e, hipEventDisableTiming), "event");
        SKI_TRY(h, hipStreamCreateWithFlags(&h->st3, hipStreamNonBlocking), "stream");
        for (auto& e : h->rev) SKI_TRY(h, hipEventCreateWithFlags(&e, hipEventDisableTiming), "event");
    }
    QrWs ws;
    qr_ws_carve(h->qprec, h->qr_part.p, m, ncols, ws);
    ws.g.part = h->gemm_ws.p;
    ws.g.bytes = h->gemm_ws.bytes;
    ws.g2.part = h->gemm_ws2.p;
    ws.g2.bytes = h->gemm_ws2.bytes;
    ws.st2 = h->st2;
    ws.evF[0] = h->qev[0];
    ws.evF[1] = h->qev[1];
    ws.evE[0] = h->qev[2];
    ws.evE[1] = h->qev[3];
    SKI_TRY(h, ensure(h->dtmp, d * 8), "alloc");
    if (h->hdiag_n < d) {
        if (h->hdiag) (void)hipHostFree(h->hdiag);
        h->hdiag = nullptr;
        h->hdiag_n = 0;
        // 2d doubles: diag(R), then the perturbation; then the panel flag and the
        // non-finite flag (one slot each)
        SKI_TRY(h, hipHostMalloc((void**)&h->hdiag, (2 * d + 2) * 8, hipHostMallocDefault),
                "pinned");
        h->hdiag_n = d;
    }
    int* hflag = (int*)(h->hdiag + 2 * d);
    int* hnonfinite = (int*)(h->hdiag + 2 * d + 1);
    const char* nonfinite_msg =
        "ski_factor: the sketch holds a non-finite entry (A or B is not finite)";
    const bool cod = h->p.qr_panel == SKI_QR_PIVOTED_COD;
    const bool piv = h->p.qr_panel == SKI_QR_PIVOTED ||
                     h->p.qr_panel == SKI_QR_PIVOTED_HOUSEHOLDER || cod;
    h->cod = false;
    h->pivoted = false;
    h->rank = d;
    if (piv) {
        if (!h->pflag.host) {
            int32_t* w = nullptr;
            SKI_TRY(h, hipHostMalloc((void**)&w, 256, hipHostMallocMapped | hipHostMallocCoherent),
                    "pinned");
            w[0] = 0;
            h->pflag.host = w;
            h->pflag.seq = 0;
            SKI_TRY(h, hipHostGetDevicePointer((void**)&h->pflag.dev, w, 0), "device pointer");
        }
        SKI_TRY(h, ensure(h->piv_part, piv_ws_bytes(m, d)), "alloc");
        SKI_TRY(h, ensure(h->pivd, d * 4), "alloc");
        SKI_TRY(h, ensure(h->Rc, d * d * 8), "alloc");
        PivWs pw;
        piv_ws_carve(h->piv_part.p, m, d, pw);
        prof_begin(h, PC_QR_PIV, st);
        SKI_TRY(h, qr_factor_pivoted((const double*)h->SA.p, m, ncols, d, ws, pw, h->p.seed,
                                     h->p.qr_panel != SKI_QR_PIVOTED_HOUSEHOLDER, h->pflag,
                                     &h->panels_cqr, st),
                "pivoted qr");
        prof_end(h, st);
        SKI_TRY(h, launch_extract_Rc(h->qprec, ws, m, d, k, P<double>(h->R), P<double>(h->c), st),
                "extract R");
        SKI_TRY(h, launch_scale_copy(P<double>(h->R), d, 1, d + 1, 1.0, P<double>(h->dtmp), 1, st),
                "diag gather");
        SKI_TRY(h, hipMemcpyAsync(h->hdiag, h->dtmp.p, d * 8, hipMemcpyDeviceToHost, st),
                "diag copy");
        SKI_TRY(h, hipMemcpyAsync(h->pivd.p, pw.perm, d * 4, hipMemcpyDeviceToDevice, st),
                "perm copy");
        SKI_TRY(h, hipMemcpyAsync(hnonfinite, ws.nonfinite, sizeof(int), hipMemcpyDeviceToHost, st),
                "flag copy");
        SKI_TRY(h, hipStreamSynchronize(st), "sync");
        if (*hnonfinite) return fail(h, SKI_EINVAL, nonfinite_msg);
    }
    bool cqr = h->p.qr_panel == SKI_QR_AUTO;
    // without pivoting, in FP64, R_h^-1 is formed block by block on a third stream while the
    // panels are factored (the Rinv buffer holds it until the signs are applied)
    if (!piv && h->qprec == Prec::F64 && d > 0) {
        SKI_TRY(h, ensure(h->gemm_ws3, rinv_ws_bytes(d)), "alloc");
        ws.Xinv = P<double>(h->Rinv);
        ws.Zinv = P<double>(h->tri_tmp);
        ws.g3.part = h->gemm_ws3.p;
        ws.g3.bytes = h->gemm_ws3.bytes;
        ws.st3 = h->st3;
        ws.evP = h->rev[0];
        ws.evI = h->rev[1];
    }
    for (; !piv;) {
        ws.cqr_panels = cqr;
        prof_begin(h, cqr ? PC_QR : PC_QR_HH, st);
        SKI_TRY(h, qr_factor(h->qprec, h->SA.p, m, ncols, d, ws, st), "qr");
        prof_end(h, st);
        SKI_TRY(h, launch_extract_Rc(h->qprec, ws, m, d, k, P<double>(h->R), P<double>(h->c), st),
                "extract R");
        // guards on diag(R): gather the diagonal on the device, copy it to pinned host memory
        SKI_TRY(h, launch_scale_copy(P<double>(h->R), d, 1, d + 1, 1.0, P<double>(h->dtmp), 1, st),
                "diag gather");
        SKI_TRY(h, hipMemcpyAsync(h->hdiag, h->dtmp.p, d * 8, hipMemcpyDeviceToHost, st),
                "diag copy");
        if (cqr)
            SKI_TRY(h, hipMemcpyAsync(hflag, ws.cqr.flag, sizeof(int), hipMemcpyDeviceToHost, st),
                    "flag copy");
        SKI_TRY(h, hipMemcpyAsync(hnonfinite, ws.nonfinite, sizeof(int), hipMemcpyDeviceToHost, st),
                "flag copy");
        SKI_TRY(h, hipStreamSynchronize(st), "sync");
        if (*hnonfinite) return fail(h, SKI_EINVAL, nonfinite_msg);
        if (cqr && *hflag != 0) {
            // a panel was too ill-conditioned for CholeskyQR2: factor again column by column
            cqr = false;
            continue;
        }
        break;
    }
    const double* Rd = h->hdiag;
    bool finite = true;
    for (int64_t i = 0; i < d; ++i) finite = finite && std::isfinite(Rd[i]);
    if (!finite) return fail(h, SKI_EINVAL, "ski_factor: non-finite R (overflow in the QR)");
    if (piv) {
        // p = the leading diagonal entries with |r_qq| >= rcond |r_11| (all non-zero ones
        // when rcond = 0): R_11 ends at the first entry below the threshold
        const double r11 = fabs(Rd[0]);
        const double thr = h->p.rcond > 0 ? h->p.rcond * r11 : 0.0;
        int64_t p = 0;
        if (r11 > 0)
            while (p < d && fabs(Rd[p]) > 0 && fabs(Rd[p]) >= thr) ++p;
        h->rank = p;
    }
    const int64_t dp = h->rank;
    double amax = 0, amin = INFINITY;
    for (int64_t i = 0; i < dp; ++i) {
        const double a = fabs(Rd[i]);
        amax = std::max(amax, a);
        amin = std::min(amin, a);
    }
    h->cond_est = amin > 0 ? amax / amin : INFINITY;
    if (!piv && h->p.rcond > 0) {
        const double r11 = fabs(Rd[0]);
        for (int64_t i = 0; i < d; ++i)
            if (!(r11 > 0) || fabs(Rd[i]) < h->p.rcond * r11) {
                h->factored = false;
                char buf[200];
                snprintf(buf, sizeof buf,
                         "rank guard failed at column %lld: |r_qq| = %.3e < rcond |r_11| "
                         "(r_11 = %.3e)",
                         (long long)i, fabs(Rd[i]), r11);
                return fail(h, SKI_ERANK, buf);
            }
    }
    double* add = h->hdiag + d;  // pinned
    const bool pert = h->p.perturb > 0 && h->p.rcond_thres > 0 &&
                      h->cond_est >= 1.0 / h->p.rcond_thres;
    for (int64_t i = 0; i < dp; ++i) add[i] = pert ? copysign(h->p.perturb, Rd[i]) : 0.0;
    if (dp > 0)
        SKI_TRY(h, hipMemcpyAsync(h->diag_add.p, add, dp * 8, hipMemcpyHostToDevice, st),
                "perturb copy");
    GemmWs gw;
    gw.part = h->gemm_ws.p;
    gw.bytes = h->gemm_ws.bytes;
    // R_11 (the leading p x p block; all of R without pivoting) and its inverse
    const double* R11 = P<double>(h->R);
    if (piv) {
        SKI_TRY(h, launch_scale_copy(P<double>(h->R), dp, dp, d, 1.0, P<double>(h->Rc), dp, st),
                "R11 copy");
        R11 = P<double>(h->Rc);
    }
    if (cod && dp > 0) {
        // the minimal-norm P = Pi Rtop^T (L^T L)^-1 from the QR Rtop^T = Y L of the top p rows
        // of R (Rtop = [R_11 R_12], pivoted column order); L^-1 is formed during that QR
        const int rc = cod_factor(h, ws, dp, hflag, gw, st);
        if (rc != SKI_OK) return rc;
        h->cod = true;
    } else {
    prof_begin(h, PC_TRTRI, st);
    if (ws.Xinv && !pert) {
        // the blocks of R_h^-1 are done (the QR's stream waited for them): R^-1 = R_h^-1 D
        SKI_TRY(h, rinv_finish((const double*)ws.Ac, m, d, P<double>(h->Rinv), P<double>(h->RinvT),
                               st),
                "R inverse");
    } else if (dp > 0) {
        SKI_TRY(h, trtri_upper(R11, dp, P<double>(h->Rinv), P<double>(h->RinvT),
                               P<double>(h->diag_add), P<double>(h->tri_tmp), gw, st),
                "R inverse");
    }
    prof_end(h, st);
    }
    h->pivoted = piv;
    if (h->ev_ok) (void)hipEventRecord(h->ev[3], st);
    SKI_TRY(h, hipStreamSynchronize(st), "sync");
    prof_collect(h);
    h->factored = true;
    return SKI_OK;
}

}  // extern "C"

namespace {

// W v products for the multi-RHS dense path through the GEMM
hipError_t dense_AZ(ski_handle h, const double* Zm, int k, double* out, GemmWs& gw,
                    hipStream_t st) {
    if (gemm_ts_eligible(k))
        return gemm_ts_f64(false, h->n, k, h->d, 1.0, h->A, h->lda, Zm, k, 0.0, out, k, gw, st);
    return gemm_f64(false, false, h->n, k, h->d, 1.0, h->A, h->lda, Zm, k, 0.0, out, k, gw, st);
}
hipError_t dense_ATU(ski_handle h, const double* U, int k, double* out, GemmWs& gw,
                     hipStream_t st) {
    if (gemm_ts_eligible(k))
        return gemm_ts_f64(true, h->d, k, h->n, 1.0, h->A, h->lda, U, k, 0.0, out, k, gw, st);
    return gemm_f64(true, false, h->d, k, h->n, 1.0, h->A, h->lda, U, k, 0.0, out, k, gw, st);
}

// y = s M x for the p x p triangle M (R_11^-1 upper, R_11^-T lower) and k > 1 columns
hipError_t tri_products(const double* Mtx, int64_t dp, bool upper, const double* x, double* y,
                        int64_t ldy, int k, double s, GemmWs& gw, hipStream_t st) {
    if (gemm_ts_eligible(k))
        return gemm_ts_f64(false, dp, k, dp, s, Mtx, dp, x, k, 0.0, y, ldy, gw, st,
                           upper ? GEMM_A_UPPER : GEMM_A_LOWER);
    return gemm_f64(false, false, dp, k, dp, s, Mtx, dp, x, k, 0.0, y, ldy, gw, st);
}

// y = s R^-1 x (upper: x in position order, y scattered to column order) or y = s R^-T x
// (x in column order, y in position order) through the sparse factor: the root block by
// its explicit inverse, the leaf rows by substitution over the leaf forest
hipError_t sparse_apply(ski_handle h, bool upper, const double* x, int64_t ldx, double* y,
                        int64_t ldy, int k, double s, const int32_t* done, GemmWs& gw,
                        hipStream_t st) {
    const SparseQR& S = *h->sp;
    const int64_t nl = S.nleaf(), nr = S.nroot();
    double* tmp = P<double>(h->sptmp);
    const double* Ri = P<double>(h->Rinv);
    const double* RiT = P<double>(h->RinvT);
    if (upper) {
        if (nr > 0) {
            // tmp[nl ..] = R_root^-1 x[nl ..]
            if (k == 1) {
                SKI_HIP(launch_tri_gemv(Ri, nr, true, x + nl * ldx, ldx, tmp + nl, 1, 1.0, done, st));
            } else {
                if (ldx != k) return hipErrorInvalidValue;
                SKI_HIP(tri_products(Ri, nr, true, x + nl * ldx, tmp + nl * k, k, k, 1.0, gw, st));
            }
        }
        return S.leaves_upper(x, ldx, tmp, y, ldy, k, s, done, st);
    }
    SKI_HIP(S.leaves_lower(x, ldx, tmp, y, ldy, k, s, done, st));
    if (nr > 0) {
        // y[nl ..] = s R_root^-T tmp[nl ..]
        if (k == 1) return launch_tri_gemv(RiT, nr, false, tmp + nl, 1, y + nl * ldy, ldy, s, done, st);
        return tri_products(RiT, nr, false, tmp + nl * k, y + nl * ldy, ldy, k, s, gw, st);
    }
    return hipSuccess;
}

int alloc_solve_ws(ski_handle h, int k) {
    const int64_t n = h->n, d = h->d;
    SKI_TRY(h, ensure(h->u, n * k * 8), "alloc");
    SKI_TRY(h, ensure(h->t, n * k * 8), "alloc");
    SKI_TRY(h, ensure(h->v, d * k * 8), "alloc");
    SKI_TRY(h, ensure(h->h, d * k * 8), "alloc");
    SKI_TRY(h, ensure(h->delta, d * k * 8), "alloc");
    SKI_TRY(h, ensure(h->z, d * k * 8), "alloc");
    SKI_TRY(h, ensure(h->wp, d * k * 8), "alloc");
    SKI_TRY(h, ensure(h->g, d * k * 8), "alloc");
    SKI_TRY(h, ensure(h->y, d * k * 8), "alloc");
    SKI_TRY(h, ensure(h->gpart, PASS_WG * d * 8), "alloc");
    const int64_t G = std::max<int64_t>({PASS_WG, spmv_csr_groups(n), 1});
    SKI_TRY(h, ensure(h->upart, G * k * 8), "alloc");
    SKI_TRY(h, ensure(h->st, k * sizeof(LsqrState)), "alloc");
    // the arrival counter of the step kernels' status word: every step that uses it leaves
    // it at zero; it is cleared again here (on the solve's stream) so that a solve never
    // depends on how an earlier one ended
    SKI_TRY(h, ensure(h->done_cnt, 256), "alloc");
    if (h->pivoted) SKI_TRY(h, ensure(h->ptmp, d * k * 8), "alloc");
    return SKI_OK;
}

// y = s R_11^-1 x (upper, Mtx = R_11^-1) or y = s R_11^-T x (Mtx = R_11^-T), leading
// dimension k.  Without pivoting both are d x k.  With pivoting (p = rank columns kept),
// the upper product takes a compact p x k x and scatters row i of the result to row
// perm[i] of the d x k y (whose other rows the caller keeps at zero); the transposed
// product gathers rows perm[i] of the d x k x and writes a compact p x k y.
hipError_t apply_Rinv(ski_handle h, const double* Mtx, bool upper, const double* x, double* y, int k,
                      double s, const int32_t* done, GemmWs& gw, hipStream_t st) {
    const int64_t dp = h->rank;
    if (dp <= 0) return hipSuccess;
    if (h->sparse) return sparse_apply(h, upper, x, k, y, k, k, s, done, gw, st);
    if (h->cod) {
        // P = cod_m (d x p): upper: y (d x k) = s P x (p x k); lower: y (p x k) = s P^T x
        const double* Pm = (const double*)h->cod_m.p;
        const int64_t d = h->d;
        if (upper)
            return gemm_ts_eligible(k)
                       ? gemm_ts_f64(false, d, k, dp, s, Pm, dp, x, k, 0.0, y, k, gw, st)
                       : gemm_f64(false, false, d, k, dp, s, Pm, dp, x, k, 0.0, y, k, gw, st);
        return gemm_ts_eligible(k)
                   ? gemm_ts_f64(true, dp, k, d, s, Pm, dp, x, k, 0.0, y, k, gw, st)
                   : gemm_f64(true, false, dp, k, d, s, Pm, dp, x, k, 0.0, y, k, gw, st);
    }
    const int32_t* perm = h->pivoted ? (const int32_t*)h->pivd.p : nullptr;
    if (k == 1) return launch_tri_gemv(Mtx, dp, upper, x, 1, y, 1, s, done, st, perm);
    if (!perm) return tri_products(Mtx, dp, upper, x, y, k, k, s, gw, st);
    double* t = (double*)h->ptmp.p;
    if (upper) {
        SKI_HIP(tri_products(Mtx, dp, upper, x, t, k, k, s, gw, st));
        return launch_permute_rows(t, k, y, k, perm, dp, k, true, st);
    }
    SKI_HIP(launch_permute_rows(x, k, t, k, perm, dp, k, false, st));
    return tri_products(Mtx, dp, upper, t, y, k, k, s, gw, st);
}

// out (d x k, ld ldo) = P y for the minimal-norm P = cod_m (d x p), y p x k (ld k)
hipError_t apply_P_out(ski_handle h, const double* y, double* out, int64_t ldo, int k,
                       GemmWs& gw, hipStream_t st) {
    const double* Pm = (const double*)h->cod_m.p;
    const int64_t d = h->d, p = h->rank;
    if (gemm_ts_eligible(k)) return gemm_ts_f64(false, d, k, p, 1.0, Pm, p, y, k, 0.0, out, ldo, gw, st);
    return gemm_f64(false, false, d, k, p, 1.0, Pm, p, y, k, 0.0, out, ldo, gw, st);
}

// Convergence status read back with a one-iteration lag: after iteration i the all-done
// word is copied to pinned host memory and an event recorded; the host waits on the event
// of iteration i-1 only, so at most one idle iteration is ever launched.
// The host learns that the iterations have stopped through a status word in pinned host
// memory mapped for the device: the iteration's scalar step writes it (for several
// right-hand sides, the last of its workgroups to finish; before the first iteration a
// one-wave kernel), an event marks the iteration, and the host reads the word one
// iteration later, so the device always has the next iteration queued.
struct LagFlag {
    volatile int32_t* host = nullptr;  // [2], one slot per iteration parity
    int32_t* dev = nullptr;            // the same words, device address
    hipEvent_t ev[2] = {nullptr, nullptr};
    bool stop = false;
    int init(ski_handle h) {
        int32_t* p = nullptr;
        SKI_TRY(h, hipHostMalloc((void**)&p, 2 * sizeof(int32_t),
                                 hipHostMallocMapped | hipHostMallocCoherent),
                "pinned");
        host = p;
        host[0] = host[1] = 0;
        SKI_TRY(h, hipHostGetDevicePointer((void**)&dev, p, 0), "device pointer");
        for (auto& e : ev) SKI_TRY(h, hipEventCreateWithFlags(&e, hipEventDisableTiming), "event");
        return SKI_OK;
    }
    // the slot that the step kernel of iteration it (counted from 1) writes
    int32_t* slot_dev(int64_t it) const { return dev + (it & 1); }
    // written: the iteration's step kernel already wrote the slot
    int post(ski_handle h, int k, hipStream_t st, int64_t it, bool written) {
        const int slot = (int)(it & 1);
        if (!written)
            SKI_TRY(h, launch_all_done(P<LsqrState>(h->st), k, dev + slot, st), "flag");
        SKI_TRY(h, hipEventRecord(ev[slot], st), "event");
        return SKI_OK;
    }
    // 1 if every column had stopped after iteration it, 0 if not, < 0 on error
    int wait(ski_handle h, int64_t it) {
        const int slot = (int)(it & 1);
        SKI_TRY(h, hipEventSynchronize(ev[slot]), "event sync");
        return host[slot] ? 1 : 0;
    }
    void release() {
        for (auto& e : ev)
            if (e) (void)hipEventDestroy(e);
        if (host) (void)hipHostFree((void*)host);
        host = nullptr;
    }
};

int finish_info(ski_handle h, int k, ski_info* info, float ms_solve, bool cg, hipStream_t st) {
    std::vector<LsqrState> S(k);
    SKI_TRY(h, hipMemcpyAsync(S.data(), h->st.p, k * sizeof(LsqrState), hipMemcpyDeviceToHost, st),
            "state copy");
    SKI_TRY(h, hipStreamSynchronize(st), "sync");
    float ms_sk = 0, ms_f = 0;
    if (h->ev_ok) {
        (void)hipEventElapsedTime(&ms_sk, h->ev[0], h->ev[1]);
        (void)hipEventElapsedTime(&ms_f, h->ev[2], h->ev[3]);
    }
    int worst = SKI_OK;
    bool nonfinite = false;
    for (int j = 0; j < k; ++j) {
        const int stj = S[j].done ? S[j].status : SKI_WNOCONV;
        if (stj == SKI_EINVAL)
            nonfinite = true;
        else if (stj == SKI_WNOCONV)
            worst = SKI_WNOCONV;
        else if (stj == SKI_WEARLY && worst == SKI_OK)
            worst = SKI_WEARLY;
        if (info) {
            ski_info& I = info[j];
            I.iters = S[j].iters;
            I.status = stj;
            I.early_exit = S[j].early;
            I.rnorm = S[j].rnorm;
            I.arnorm = cg ? 0.0 : S[j].arnorm;
            I.wnorm_est = cg ? 0.0 : sqrt(S[j].anorm2);
            I.tc = cg ? 0.0 : S[j].tc;
            I.cond_est = h->cond_est;
            I.ms_sketch = ms_sk;
            I.ms_factor = ms_f;
            I.ms_solve = ms_solve;
        }
    }
    if (worst == SKI_WEARLY && k > 1) {
        bool all_early = true;
        for (int j = 0; j < k; ++j) all_early = all_early && S[j].early;
        if (!all_early) worst = SKI_OK;
    }
    if (nonfinite)
        return fail(h, SKI_EINVAL,
                    cg ? "ski_solve: a non-finite value in the iteration (G is not finite)"
                       : "ski_solve: a non-finite value in the iteration (B is not finite)");
    return worst;
}

int solve_lls(ski_handle h, const double* B, int k, int64_t ldb, double* X, int64_t ldx,
              ski_info* info, hipStream_t st) {
    const int64_t n = h->n, d = h->d;
    int rc = alloc_solve_ws(h, k);
    if (rc != SKI_OK) return rc;
    GemmWs gw;
    gw.part = h->gemm_ws.p;
    gw.bytes = h->gemm_ws.bytes;
    LsqrState* S = P<LsqrState>(h->st);
    double *u = P<double>(h->u), *t = P<double>(h->t), *v = P<double>(h->v), *hh = P<double>(h->h);
    double *dl = P<double>(h->delta), *z = P<double>(h->z), *wp = P<double>(h->wp);
    double *g = P<double>(h->g), *y = P<double>(h->y);
    const double* Rinv = P<double>(h->Rinv);
    const double* RinvT = P<double>(h->RinvT);
    const double* c = P<double>(h->c);
    const bool fused = (h->kind == SKI_DENSE && k == 1 && lsqr_pass_cpt(d) > 0);
    const bool csr = (h->kind == SKI_CSR);
    hipEvent_t e0 = h->ev[4], e1 = h->ev[5];
    if (h->ev_ok) (void)hipEventRecord(e0, st);
    const int64_t dp = h->rank;  // the LSQR vectors v, h, delta, y live in R^p
    SKI_TRY(h, hipMemsetAsync(S, 0, k * sizeof(LsqrState), st), "state init");
    SKI_TRY(h, hipMemsetAsync(h->done_cnt.p, 0, 256, st), "counter init");
    // with pivoting z = V_1 (...) is zero outside the kept columns
    if (h->pivoted) SKI_TRY(h, launch_fill_rows(z, d, k, k, 0.0, st), "zero z");
    // u = B (the residual is formed in place), z = -x_s
    SKI_TRY(h, launch_scale_copy(B, n, k, ldb, 1.0, u, k, st), "copy b");
    SKI_TRY(h, apply_Rinv(h, Rinv, true, c, z, k, -1.0, nullptr, gw, st), "x_s");
    // r_0 = b - A x_s ; g = A^T r_0
    if (fused) {
        SKI_TRY(h, launch_lsqr_pass(h->A, h->lda, n, d, z, u, S, PASS_WG, P<double>(h->gpart),
                                    P<double>(h->upart), g, S, true, st),
                "pass");
    } else if (csr) {
        SKI_TRY(h, launch_spmv_csr(h->rp, h->ci, h->va, n, k, z, u, S, true, P<double>(h->upart), st),
                "spmv");
        SKI_TRY(h, launch_spmv_csrT(P<int32_t>(h->tp), P<int32_t>(h->ti), P<double>(h->tv), d, k, u,
                                    g, S, st),
                "spmvT");
    } else {
        SKI_TRY(h, dense_AZ(h, z, k, t, gw, st), "AZ");
        SKI_TRY(h, launch_combine_u(t, u, n, k, S, true, P<double>(h->upart), PASS_WG, S, st),
                "combine");
        SKI_TRY(h, dense_ATU(h, u, k, g, gw, st), "ATU");
    }
    SKI_TRY(h, apply_Rinv(h, RinvT, false, g, wp, k, 1.0, nullptr, gw, st), "R^-T g");
    SKI_TRY(h, launch_lsqr_init(S, dp, k, wp, v, hh, dl, h->p.tau_a, st), "init");
    const int32_t* done1 = (k == 1) ? &S[0].done : nullptr;
    LagFlag lf;
    int out = lf.init(h);
    if (out == SKI_OK) out = lf.post(h, k, st, 0, false);
    if (out == SKI_OK && lf.wait(h, 0) == 1) lf.stop = true;
    int64_t it = 0;
    while (out == SKI_OK && !lf.stop && it < h->p.it_max) {
        {
            prof_begin(h, PC_TRIGEMV, st);
            hipError_t e = apply_Rinv(h, Rinv, true, v, z, k, 1.0, done1, gw, st);
            prof_end(h, st);
            if (e == hipSuccess) {
                if (fused) {
                    prof_begin(h, PC_PASS, st);
                    e = launch_pass_kernel(h->A, h->lda, n, d, z, u, S, PASS_WG,
                                           P<double>(h->gpart), P<double>(h->upart), false, st);
                    prof_end(h, st);
                    prof_begin(h, PC_REDUCE, st);
                    if (e == hipSuccess)
                        e = launch_pass_reduce(P<double>(h->gpart), P<double>(h->upart), PASS_WG,
                                               d, g, S, st);
                    prof_end(h, st);
                } else if (csr) {
                    prof_begin(h, PC_SPMV, st);
                    e = launch_spmv_csr(h->rp, h->ci, h->va, n, k, z, u, S, false,
                                        P<double>(h->upart), st);
                    prof_end(h, st);
                    prof_begin(h, PC_SPMVT, st);
                    if (e == hipSuccess)
                        e = launch_spmv_csrT(P<int32_t>(h->tp), P<int32_t>(h->ti), P<double>(h->tv),
                                             d, k, u, g, S, st);
                    prof_end(h, st);
                } else {
                    e = dense_AZ(h, z, k, t, gw, st);
                    if (e == hipSuccess)
                        e = launch_combine_u(t, u, n, k, S, false, P<double>(h->upart), PASS_WG, S,
                                             st);
                    if (e == hipSuccess) e = dense_ATU(h, u, k, g, gw, st);
                }
            }
            prof_begin(h, PC_TRIGEMV, st);
            if (e == hipSuccess) e = apply_Rinv(h, RinvT, false, g, wp, k, 1.0, done1, gw, st);
            prof_end(h, st);
            prof_begin(h, PC_STEP, st);
            if (e == hipSuccess)
                e = launch_lsqr_step(S, dp, k, wp, v, hh, dl, h->p.tau_r, h->p.it_max,
                                     lf.slot_dev(it + 1), P<uint32_t>(h->done_cnt), st);
            prof_end(h, st);
            if (e != hipSuccess) {
                out = hip_fail(h, e, "lsqr iteration");
                break;
            }
        }
        ++it;
        // status of this iteration is posted now and read one iteration later, so the
        // device always has the next iteration queued while the host checks
        out = lf.post(h, k, st, it, true);
        if (out == SKI_OK && it >= 2 && lf.wait(h, it - 1) == 1) break;
    }
    lf.release();
    if (out != SKI_OK) return out;
    // x = R^-1 (c + delta); with pivoting x = V_1 R_11^-1 (c + delta), zero elsewhere
    SKI_TRY(h, launch_final_y(S, dp, k, c, dl, y, st), "final y");
    if (h->sparse) {
        // x = P R^-1 (c + delta), every row of X written through perm
        SKI_TRY(h, sparse_apply(h, true, y, k, X, ldx, k, 1.0, nullptr, gw, st), "x");
    } else if (h->cod) {
        // x = P (c + delta), P = cod_m (d x p)
        if (dp > 0) SKI_TRY(h, apply_P_out(h, y, X, ldx, k, gw, st), "x");
    } else if (h->pivoted) {
        SKI_TRY(h, launch_fill_rows(X, d, k, ldx, 0.0, st), "zero x");
        if (k == 1) {
            SKI_TRY(h, launch_tri_gemv(Rinv, dp, true, y, 1, X, ldx, 1.0, nullptr, st,
                                       P<int32_t>(h->pivd)),
                    "x");
        } else if (dp > 0) {
            SKI_TRY(h, tri_products(Rinv, dp, true, y, P<double>(h->ptmp), k, k, 1.0, gw, st),
                    "x");
            SKI_TRY(h, launch_permute_rows(P<double>(h->ptmp), k, X, ldx, P<int32_t>(h->pivd), dp,
                                           k, true, st),
                    "x scatter");
        }
    } else if (k == 1) {
        SKI_TRY(h, launch_tri_gemv(Rinv, d, true, y, 1, X, ldx, 1.0, nullptr, st), "x");
    } else {
        SKI_TRY(h, tri_products(Rinv, d, true, y, X, ldx, k, 1.0, gw, st), "x");
    }
    float ms = 0;
    if (h->ev_ok) {
        (void)hipEventRecord(e1, st);
        (void)hipEventSynchronize(e1);
        (void)hipEventElapsedTime(&ms, e0, e1);
    }
    const int rcf = finish_info(h, k, info, ms, false, st);
    prof_collect(h);
    return rcf;
}

// Z = (A^T A)^-1 G by CG on R^-T A^T A R^-1 (dense A)
int solve_normal(ski_handle h, const double* G, int k, int64_t ldg, double* Z, int64_t ldz,
                 ski_info* info, hipStream_t st) {
    const int64_t n = h->n, d = h->d;
    int rc = alloc_solve_ws(h, k);
    if (rc != SKI_OK) return rc;
    SKI_TRY(h, ensure(h->cg_r, d * k * 8), "alloc");
    SKI_TRY(h, ensure(h->cg_p, d * k * 8), "alloc");
    SKI_TRY(h, ensure(h->cg_q, d * k * 8), "alloc");
    GemmWs gw;
    gw.part = h->gemm_ws.p;
    gw.bytes = h->gemm_ws.bytes;
    LsqrState* S = P<LsqrState>(h->st);
    double *t = P<double>(h->t), *z = P<double>(h->z), *g = P<double>(h->g), *y = P<double>(h->y);
    double *r = P<double>(h->cg_r), *pp = P<double>(h->cg_p), *q = P<double>(h->cg_q);
    double* wp = P<double>(h->wp);
    const double* Rinv = P<double>(h->Rinv);
    const double* RinvT = P<double>(h->RinvT);
    hipEvent_t e0 = h->ev[4], e1 = h->ev[5];
    if (h->ev_ok) (void)hipEventRecord(e0, st);
    const int64_t dp = h->rank;  // CG runs in R^p (p = d without pivoting)
    SKI_TRY(h, hipMemsetAsync(S, 0, k * sizeof(LsqrState), st), "state init");
    SKI_TRY(h, hipMemsetAsync(h->done_cnt.p, 0, 256, st), "counter init");
    if (h->pivoted) SKI_TRY(h, launch_fill_rows(z, d, k, k, 0.0, st), "zero z");
    // rhs = R^-T G (into wp, compact leading dimension k)
    SKI_TRY(h, launch_scale_copy(G, d, k, ldg, 1.0, g, k, st), "copy g");
    SKI_TRY(h, apply_Rinv(h, RinvT, false, g, wp, k, 1.0, nullptr, gw, st), "rhs");
    SKI_TRY(h, launch_cg_init(S, dp, k, wp, r, pp, y, h->p.tau_r, st), "cg init");
    LagFlag lf;
    int out = lf.init(h);
    if (out == SKI_OK) out = lf.post(h, k, st, 0, false);
    if (out == SKI_OK && lf.wait(h, 0) == 1) lf.stop = true;
    int64_t it = 0;
    while (out == SKI_OK && !lf.stop && it < h->p.it_max) {
        hipError_t e = apply_Rinv(h, Rinv, true, pp, z, k, 1.0, nullptr, gw, st);
        if (e == hipSuccess) e = dense_AZ(h, z, k, t, gw, st);
        if (e == hipSuccess) e = dense_ATU(h, t, k, g, gw, st);
        if (e == hipSuccess) e = apply_Rinv(h, RinvT, false, g, q, k, 1.0, nullptr, gw, st);
        if (e == hipSuccess)
            e = launch_cg_step(S, dp, k, q, r, pp, y, h->p.it_max, lf.slot_dev(it + 1),
                               P<uint32_t>(h->done_cnt), st);
        if (e != hipSuccess) {
            out = hip_fail(h, e, "cg iteration");
            break;
        }
        ++it;
        out = lf.post(h, k, st, it, true);
        if (out == SKI_OK && it >= 2 && lf.wait(h, it - 1) == 1) break;
    }
    lf.release();
    if (out != SKI_OK) return out;
    if (h->cod) {
        if (dp > 0) SKI_TRY(h, apply_P_out(h, y, Z, ldz, k, gw, st), "z");
    } else if (h->pivoted) {
        SKI_TRY(h, launch_fill_rows(Z, d, k, ldz, 0.0, st), "zero Z");
        if (dp > 0) {
            SKI_TRY(h, tri_products(Rinv, dp, true, y, P<double>(h->ptmp), k, k, 1.0, gw, st),
                    "z");
            SKI_TRY(h, launch_permute_rows(P<double>(h->ptmp), k, Z, ldz, P<int32_t>(h->pivd), dp,
                                           k, true, st),
                    "z scatter");
        }
    } else {
        SKI_TRY(h, tri_products(Rinv, d, true, y, Z, ldz, k, 1.0, gw, st), "z");
    }
    float ms = 0;
    if (h->ev_ok) {
        (void)hipEventRecord(e1, st);
        (void)hipEventSynchronize(e1);
        (void)hipEventElapsedTime(&ms, e0, e1);
    }
    (void)n;
    return finish_info(h, k, info, ms, true, st);
}

}  // namespace

extern "C" {

int ski_solve(ski_handle h, int32_t op, const double* B, int32_t k, int64_t ldb, double* X,
              int64_t ldx, ski_info* info, void* stream) {
    if (!h) return SKI_EINVAL;
    if (!h->factored) return fail(h, SKI_ESTATE, "ski_solve: call ski_sketch and ski_factor first");
    if (!B || !X) return fail(h, SKI_EINVAL, "ski_solve: NULL B or X");
    if (k < 1 || ldb < k || ldx < k) return fail(h, SKI_EINVAL, "ski_solve: bad k or leading dims");
    hipStream_t st = (hipStream_t)stream;
    if (op == SKI_OP_LLS) {
        if (k != h->k)
            return fail(h, SKI_EINVAL,
                        "ski_solve: B must be the k right-hand sides given to ski_sketch");
        return solve_lls(h, B, k, ldb, X, ldx, info, st);
    }
    if (op == SKI_OP_NORMAL) {
        if (h->kind != SKI_DENSE) return fail(h, SKI_EINVAL, "ski_solve: NORMAL needs dense A");
        return solve_normal(h, B, k, ldb, X, ldx, info, st);
    }
    return fail(h, SKI_EINVAL, "ski_solve: unknown op");
}

int ski_gradients(ski_handle h, const double* X, int64_t ldx, const double* B, int64_t ldb,
                  const double* Z, int64_t ldz, int32_t k, double* grad_A, int64_t ldga,
                  double* grad_B, int64_t ldgb, void* stream) {
    if (!h) return SKI_EINVAL;
    if (!h->sketched) return fail(h, SKI_ESTATE, "ski_gradients: no matrix (call ski_sketch)");
    if (h->kind != SKI_DENSE) return fail(h, SKI_EINVAL, "ski_gradients: dense A only");
    if (!X || !B || !Z || k < 1 || ldx < k || ldb < k || ldz < k)
        return fail(h, SKI_EINVAL, "ski_gradients: bad arguments");
    if ((grad_A && ldga < h->d) || (grad_B && ldgb < k))
        return fail(h, SKI_EINVAL, "ski_gradients: bad output leading dimensions");
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = h->n, d = h->d;
    SKI_TRY(h, ensure(h->gemm_ws, (size_t)64 << 20), "alloc");
    SKI_TRY(h, ensure(h->t, n * k * 8), "alloc");
    SKI_TRY(h, ensure(h->t2, n * k * 8), "alloc");
    GemmWs gw;
    gw.part = h->gemm_ws.p;
    gw.bytes = h->gemm_ws.bytes;
    double* AZ = P<double>(h->t);
    double* Res = P<double>(h->t2);
    SKI_TRY(h, gemm_f64(false, false, n, k, d, 1.0, h->A, h->lda, Z, ldz, 0.0, AZ, k, gw, st), "AZ");
    if (grad_B) SKI_TRY(h, launch_scale_copy(AZ, n, k, k, 1.0, grad_B, ldgb, st), "grad_B");
    if (grad_A) {
        SKI_TRY(h, launch_scale_copy(B, n, k, ldb, 1.0, Res, k, st), "copy B");
        SKI_TRY(h, gemm_f64(false, false, n, k, d, -1.0, h->A, h->lda, X, ldx, 1.0, Res, k, gw, st),
                "residual");
        SKI_TRY(h, gemm_f64(false, true, n, d, k, 1.0, Res, k, Z, ldz, 0.0, grad_A, ldga, gw, st),
                "r Z^T");
        SKI_TRY(h, gemm_f64(false, true, n, d, k, -1.0, AZ, k, X, ldx, 1.0, grad_A, ldga, gw, st),
                "(AZ) X^T");
    }
    return SKI_OK;
}

int ski_set_profiling(ski_handle h, int32_t on) {
    return ski_set_profiling_mask(h, on ? 0xffffffffu : 0u);
}

int ski_set_profiling_mask(ski_handle h, uint32_t mask) {
    if (!h) return SKI_EINVAL;
    if (h->prof) {
        (void)hipDeviceSynchronize();
        prof_collect(h);
    }
    h->prof = mask != 0;
    h->prof_mask = mask;
    for (int c = 0; c < SKI_PROF_CLASSES; ++c) {
        h->prof_ms[c] = 0;
        h->prof_cnt[c] = 0;
    }
    return SKI_OK;
}

int ski_get_profile(ski_handle h, double* ms, int64_t* count) {
    if (!h || !ms || !count) return SKI_EINVAL;
    prof_collect(h);
    for (int c = 0; c < SKI_PROF_CLASSES; ++c) {
        ms[c] = h->prof_ms[c];
        count[c] = h->prof_cnt[c];
    }
    return SKI_OK;
}

int ski_get_dims(ski_handle h, int64_t dims[6]) {
    if (!h || !dims) return SKI_EINVAL;
    dims[0] = h->n;
    dims[1] = h->d;
    dims[2] = h->k;
    dims[3] = h->m;
    dims[4] = h->npad;
    dims[5] = h->s;
    return SKI_OK;
}

int ski_get_hash(ski_handle h, int32_t* rows, int8_t* neg, int64_t* bucket_ptr, int32_t* src,
                 int8_t* src_neg) {
    if (!h) return SKI_EINVAL;
    if (!h->sketched) return fail(h, SKI_ESTATE, "ski_get_hash: nothing sketched");
    const int64_t nk = h->nkeys;
    if (hipDeviceSynchronize() != hipSuccess) return fail(h, SKI_EDEVICE, "sync");
    if (rows && hipMemcpy(rows, h->colrows.p, nk * 4, hipMemcpyDeviceToHost) != hipSuccess)
        return fail(h, SKI_EDEVICE, "copy");
    if (neg && hipMemcpy(neg, h->colneg.p, nk, hipMemcpyDeviceToHost) != hipSuccess)
        return fail(h, SKI_EDEVICE, "copy");
    if (bucket_ptr) {
        std::vector<int32_t> bp(h->m + 1);
        if (hipMemcpy(bp.data(), h->bucket_ptr.p, (h->m + 1) * 4, hipMemcpyDeviceToHost) !=
            hipSuccess)
            return fail(h, SKI_EDEVICE, "copy");
        for (int64_t i = 0; i <= h->m; ++i) bucket_ptr[i] = bp[i];
    }
    if (src || src_neg) {
        std::vector<int32_t> sv(nk);
        if (hipMemcpy(sv.data(), h->src.p, nk * 4, hipMemcpyDeviceToHost) != hipSuccess)
            return fail(h, SKI_EDEVICE, "copy");
        for (int64_t i = 0; i < nk; ++i) {
            if (src) src[i] = (int32_t)((uint32_t)sv[i] >> 1);
            if (src_neg) src_neg[i] = (int8_t)(sv[i] & 1);
        }
    }
    return SKI_OK;
}

int ski_get_dsign(ski_handle h, int8_t* dsign) {
    if (!h || !dsign) return SKI_EINVAL;
    if (!h->sketched || !h->had) return fail(h, SKI_ESTATE, "ski_get_dsign: no Hadamard sketch");
    std::vector<uint32_t> bits((h->npad + 31) / 32);
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(bits.data(), h->dbits.p, bits.size() * 4, hipMemcpyDeviceToHost) != hipSuccess)
        return fail(h, SKI_EDEVICE, "copy");
    for (int64_t i = 0; i < h->npad; ++i) dsign[i] = ((bits[i >> 5] >> (i & 31)) & 1u) ? -1 : 1;
    return SKI_OK;
}

int ski_get_SA(ski_handle h, double* SA) {
    if (!h || !SA) return SKI_EINVAL;
    if (!h->sketched) return fail(h, SKI_ESTATE, "ski_get_SA: nothing sketched");
    const int64_t cnt = h->m * (h->d + h->k);
    if (hipDeviceSynchronize() != hipSuccess) return fail(h, SKI_EDEVICE, "sync");
    if (h->p.qr_panel == SKI_QR_SPARSE) {
        DevBuf tmp;
        if (ensure(tmp, cnt * 8) != hipSuccess) return fail(h, SKI_ENOMEM, "ski_get_SA: alloc");
        const bool ok = h->sp->dense_SA(P<double>(tmp), nullptr) == hipSuccess &&
                        hipMemcpy(SA, tmp.p, cnt * 8, hipMemcpyDeviceToHost) == hipSuccess;
        release(tmp);
        return ok ? SKI_OK : fail(h, SKI_EDEVICE, "ski_get_SA: copy");
    }
    if (h->qprec == Prec::F64) {
        if (hipMemcpy(SA, h->SA.p, cnt * 8, hipMemcpyDeviceToHost) != hipSuccess)
            return fail(h, SKI_EDEVICE, "copy");
    } else {
        std::vector<float> f(cnt);
        if (hipMemcpy(f.data(), h->SA.p, cnt * 4, hipMemcpyDeviceToHost) != hipSuccess)
            return fail(h, SKI_EDEVICE, "copy");
        for (int64_t i = 0; i < cnt; ++i) SA[i] = f[i];
    }
    return SKI_OK;
}

int ski_get_R(ski_handle h, double* R, double* c, double* Rinv) {
    if (!h) return SKI_EINVAL;
    const int64_t d = h->d;
    if (h->sparse && h->factored) {
        if (Rinv) return fail(h, SKI_ESTATE, "ski_get_R: the sparse factor forms no R^-1");
        if (hipDeviceSynchronize() != hipSuccess) return fail(h, SKI_EDEVICE, "sync");
        if (R) {
            DevBuf tmp;
            if (ensure(tmp, d * d * 8) != hipSuccess) return fail(h, SKI_ENOMEM, "ski_get_R: alloc");
            const bool ok = h->sp->dense_R(P<double>(h->R), P<double>(tmp), nullptr) == hipSuccess &&
                            hipMemcpy(R, tmp.p, d * d * 8, hipMemcpyDeviceToHost) == hipSuccess;
            release(tmp);
            if (!ok) return fail(h, SKI_EDEVICE, "ski_get_R: copy");
        }
        if (c && hipMemcpy(c, h->c.p, d * h->k * 8, hipMemcpyDeviceToHost) != hipSuccess)
            return fail(h, SKI_EDEVICE, "copy");
        return SKI_OK;
    }
    if (!h->R.p || !h->sketched) return fail(h, SKI_ESTATE, "ski_get_R: not factored");
    if (hipDeviceSynchronize() != hipSuccess) return fail(h, SKI_EDEVICE, "sync");
    if (R && hipMemcpy(R, h->R.p, d * d * 8, hipMemcpyDeviceToHost) != hipSuccess)
        return fail(h, SKI_EDEVICE, "copy");
    if (c && hipMemcpy(c, h->c.p, d * h->k * 8, hipMemcpyDeviceToHost) != hipSuccess)
        return fail(h, SKI_EDEVICE, "copy");
    if (Rinv && h->factored && h->rank > 0 &&
        hipMemcpy(Rinv, h->Rinv.p, h->rank * h->rank * 8, hipMemcpyDeviceToHost) != hipSuccess)
        return fail(h, SKI_EDEVICE, "copy");
    return SKI_OK;
}

int ski_get_factor_stats(ski_handle h, int64_t stats[4]) {
    if (!h || !stats) return SKI_EINVAL;
    if (!h->factored) return fail(h, SKI_ESTATE, "ski_get_factor_stats: not factored");
    stats[0] = h->rank;
    if (h->sparse) {
        stats[1] = h->sp->nleaf();
        stats[2] = h->sp->nroot();
        stats[3] = 2;
        return SKI_OK;
    }
    stats[1] = (h->d + 63) / 64;
    stats[2] = h->pivoted ? h->panels_cqr : -1;
    stats[3] = h->pivoted ? 1 : 0;
    return SKI_OK;
}

int ski_get_pivots(ski_handle h, int32_t* perm, int64_t* rank) {
    if (!h) return SKI_EINVAL;
    if (!h->factored) return fail(h, SKI_ESTATE, "ski_get_pivots: not factored");
    const int64_t d = h->d;
    if (rank) *rank = h->rank;
    if (perm) {
        if (h->pivoted) {
            if (hipDeviceSynchronize() != hipSuccess ||
                hipMemcpy(perm, h->pivd.p, d * 4, hipMemcpyDeviceToHost) != hipSuccess)
                return fail(h, SKI_EDEVICE, "copy");
        } else {
            for (int64_t j = 0; j < d; ++j) perm[j] = (int32_t)j;
        }
    }
    return SKI_OK;
}

}  // extern "C"
