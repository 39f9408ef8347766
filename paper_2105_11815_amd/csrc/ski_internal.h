// Internal declarations shared by the HIP sources of the solver library.
// Host-side launchers are declared here; kernels live in the .hip files.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/ski.h"

namespace ski {

// ---------------------------------------------------------------------------
// error plumbing: launchers return hipError_t; the API layer maps it to a status
#define SKI_HIP(expr)                                   \
    do {                                                \
        hipError_t e_ = (expr);                         \
        if (e_ != hipSuccess) return e_;                \
    } while (0)

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon et al., SC'11): ten rounds of the 4x64 bijection with the
// key bumped by the Weyl constants between rounds.
struct P4 {
    uint64_t x[4];
};

__device__ __forceinline__ P4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                             uint64_t k0, uint64_t k1) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
        uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
        uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    P4 o;
    o.x[0] = c0;
    o.x[1] = c1;
    o.x[2] = c2;
    o.x[3] = c3;
    return o;
}

// ---------------------------------------------------------------------------
// wave64 sum with DPP lane moves (CDNA, gfx9 family): pairs and quads by quad_perm,
// 16-lane rows by row_ror 4 and 8, then row_bcast 15 and 31 carry the row sums up to
// lane 63, whose value is broadcast.  The order of the additions is fixed, so the
// result is the same on every run.  Lanes other than 63 may hold partial garbage
// before the final broadcast.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double x) {
    int lo = __double2loint(x), hi = __double2hiint(x);
    lo = __builtin_amdgcn_mov_dpp(lo, CTRL, 0xf, 0xf, false);
    hi = __builtin_amdgcn_mov_dpp(hi, CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_move(float x) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, 0xf, 0xf, false));
}
__device__ __forceinline__ double lane63(double x) {
    int lo = __builtin_amdgcn_readlane(__double2loint(x), 63);
    int hi = __builtin_amdgcn_readlane(__double2hiint(x), 63);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float lane63(float x) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
}
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
    v += dpp_move<0xb1>(v);   // quad_perm [1,0,3,2]
    v += dpp_move<0x4e>(v);   // quad_perm [2,3,0,1]
    v += dpp_move<0x124>(v);  // row_ror 4
    v += dpp_move<0x128>(v);  // row_ror 8
    v += dpp_move<0x142>(v);  // row_bcast 15
    v += dpp_move<0x143>(v);  // row_bcast 31
    return lane63(v);
}

// ---------------------------------------------------------------------------
// storage types for the mixed-precision forms
__device__ __forceinline__ float to_f(float x) { return x; }
__device__ __forceinline__ float to_f(double x) { return (float)x; }
__device__ __forceinline__ float to_f(__hip_bfloat16 x) { return __bfloat162float(x); }
template <typename T>
__device__ __forceinline__ T from_f(float x);
template <>
__device__ __forceinline__ float from_f<float>(float x) { return x; }
template <>
__device__ __forceinline__ double from_f<double>(float x) { return (double)x; }
template <>
__device__ __forceinline__ __hip_bfloat16 from_f<__hip_bfloat16>(float x) { return __float2bfloat16(x); }

// ---------------------------------------------------------------------------
// launchers (all asynchronous on `st`)

// hashing: per-column rows/signs and the bucket-sorted CSR of S_h
struct HashBuffers {
    int32_t* colrows = nullptr;   // [ncols*s]
    int8_t* colneg = nullptr;     // [ncols*s]
    int32_t* bucket_ptr = nullptr;  // [m+1]
    int32_t* src = nullptr;       // [ncols*s]  column index | sign bit 31
    uint64_t* keys = nullptr;     // [nchunks*CHUNK] sorted keys per chunk
    int32_t* table = nullptr;     // [nchunks*m] per-chunk bucket counts -> bases
};
constexpr int SORT_CHUNK = 4096;  // keys sorted per workgroup in LDS
int64_t hash_num_chunks(int64_t nkeys);
// keys of the sketch's sparse factor: ncols * s for the two hashings, m for row sampling
int64_t hash_num_keys(int64_t ncols, int64_t m, int s, int kind);
// kind: SKI_HASH (s-hashing), SKI_HASH_VARIANT (rows with replacement), SKI_SAMPLE_ROWS
// (one of the ncols rows per sketch row; colrows[i] = that row)
hipError_t launch_hash_build(int64_t ncols, int64_t m, int s, uint64_t seed, int kind,
                             HashBuffers& hb, hipStream_t st);
// generic deterministic bucket sort of nkeys (bucket << 32 | payload) keys already in
// `keys_unsorted` (payloads unique): writes bucket_ptr[nb+1] and out_payload[nkeys]
hipError_t launch_bucket_sort(const uint64_t* keys_unsorted, int64_t nkeys, int64_t nbuckets,
                              uint64_t* keys_tmp, int32_t* table, int32_t* bucket_ptr,
                              int32_t* out_payload, hipStream_t st);
hipError_t launch_dsign(int64_t npad, uint64_t seed, uint32_t* bits, hipStream_t st);

// Walsh-Hadamard passes and the hashing gathers
enum class Prec { F64 = 0, F32 = 1, BF16 = 2 };
// dense sketch with the Hadamard row mix, by column slabs of sc columns through the slab
// buffer T (npad x sc elements of the storage type), into SA (m x (d+k)).  prec: the
// transform's arithmetic and slab type (F64, F32, or BF16 storage with F32 arithmetic);
// out: SA's type (F64 only with prec F64; otherwise F32)
int64_t sketch_slab_cols(int64_t npad, int64_t ncols, Prec prec);
hipError_t launch_sketch_dense(const double* A, int64_t lda, const double* B, int64_t ldb,
                               int64_t n, int64_t d, int64_t k, int64_t npad,
                               const uint32_t* dbits, void* T, int64_t sc,
                               const int32_t* bucket_ptr, const int32_t* src, int64_t m,
                               double scale, Prec prec, Prec out, void* SA, hipStream_t st);
// dense sketch with the randomised Hartley transform (FP64; n' <= 2^24), through the
// same slab buffer T (npad x sc doubles, sc a multiple of 16) into SA (m x (d+k))
bool dht_supported(int64_t npad);
hipError_t launch_sketch_dht(const double* A, int64_t lda, const double* B, int64_t ldb,
                             int64_t n, int64_t d, int64_t k, int64_t npad,
                             const uint32_t* dbits, double* T, int64_t sc,
                             const int32_t* bucket_ptr, const int32_t* src, int64_t m,
                             double scale, double* SA, hipStream_t st);
hipError_t launch_gather_plain(const double* A, int64_t lda, const double* B, int64_t ldb,
                               int64_t d, int64_t k, const int32_t* bucket_ptr,
                               const int32_t* src, int64_t m, double scale, Prec prec, Prec out,
                               void* SA, hipStream_t st);
// dst (n x d row-major) = the column-major src (ld lds >= n); n <= 64 * 65535
hipError_t launch_colmajor_to_rowmajor(const double* src, int64_t lds, int64_t n, int64_t d,
                                       double* dst, hipStream_t st);
// message of the last failed ski_sketch_noalloc call on this host thread ("" if none)
const char* noalloc_last_error();
// *bad = 1 (it is not cleared here) unless row_ptr[0] = 0, row_ptr[n] = nnz, the row offsets
// never decrease and every column index lies in [0, d); reads row_ptr[0 .. n] and col[0 .. nnz)
hipError_t launch_check_csr(const int64_t* row_ptr, const int32_t* col, int64_t n, int64_t d,
                            int64_t nnz, int* bad, hipStream_t st);
hipError_t launch_gather_csr(const int64_t* row_ptr, const int32_t* col, const double* val,
                             const double* B, int64_t ldb, int64_t d, int64_t k,
                             const int32_t* bucket_ptr, const int32_t* src, int64_t m,
                             double scale, Prec prec, Prec out, void* SA, hipStream_t st);

// GEMM: C[MxN] = alpha op(A) op(B) + beta C, row-major, on MFMA.
//   T = double (FP64 MFMA), float (FP32 MFMA), or float with bf16 MFMA inputs.
struct GemmWs {
    void* part = nullptr;   // split-K partials
    size_t bytes = 0;
};
// tri: GEMM_A_UPPER when op(A) is upper triangular (A(i, k) = 0 for k < i), GEMM_B_UPPER
// when op(B) is (B(k, j) = 0 for k > j), GEMM_A_LOWER (narrow products only) when
// A(i, k) = 0 for k > i; each output tile then skips the zero part of K
enum { GEMM_A_UPPER = 1, GEMM_B_UPPER = 2, GEMM_A_LOWER = 4 };
hipError_t gemm_f64(bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha,
                    const double* A, int64_t lda, const double* B, int64_t ldb, double beta,
                    double* C, int64_t ldc, GemmWs& ws, hipStream_t st, int unitA = 0,
                    int tri = 0);
hipError_t gemm_f32(bool ta, bool tb, int64_t M, int64_t N, int64_t K, float alpha,
                    const float* A, int64_t lda, const float* B, int64_t ldb, float beta, float* C,
                    int64_t ldc, bool bf16_inputs, GemmWs& ws, hipStream_t st, int unitA = 0);
size_t gemm_ws_bytes(int64_t M, int64_t N, int64_t K, size_t elem);
// FP64 products with a narrow right operand (tsgemm.hip): C = alpha op(A) B + beta C with
// op(A) = A (M x K) or, with ta, A^T (A stored K x M); B K x N; N <= TS_MAX_N is where they
// beat the general GEMM.  Split-K partials go to ws (fewer splits when it is small).
constexpr int64_t TS_MAX_N = 64;
bool gemm_ts_eligible(int64_t N);
hipError_t gemm_ts_f64(bool ta, int64_t M, int64_t N, int64_t K, double alpha, const double* A,
                       int64_t lda, const double* B, int64_t ldb, double beta, double* C,
                       int64_t ldc, GemmWs& ws, hipStream_t st, int tri = 0);

// C -= A B (row-major, leading dimensions) for K <= 64: the QR's trailing update
// (rank_update.hip); FP64 or FP32
template <typename T>
hipError_t launch_rank_update(int64_t M, int64_t N, int K, const T* A, int64_t lda, const T* B,
                              int64_t ldb, T* C, int64_t ldc, hipStream_t st);

// W = C V^T (W: M x K, ldw) for K <= 64, C: M x N (ldc), V: K x N (ldv), with partial sums
// over ranges of N in ws (rank_project_ws_bytes(M, N, elem) bytes); FP64 or FP32
size_t rank_project_ws_bytes(int64_t M, int64_t N, size_t elem);
template <typename T>
hipError_t launch_rank_project(int64_t M, int64_t N, int K, const T* C, int64_t ldc, const T* V,
                               int64_t ldv, T* W, int64_t ldw, void* ws, size_t ws_bytes,
                               hipStream_t st);

// panel factorisation by CholeskyQR2 and Householder reconstruction (qr_panel.hip)
struct CqrWs {
    void* Q1 = nullptr;   // m x 64 column-major, the first orthonormalised panel
    void* Gp = nullptr;   // cqr_num_chunks(m) Gram partials of 64 x 64
    void* G = nullptr;    // reduced Gram matrix, 64 x 64
    void* R1 = nullptr;   // first Cholesky factor and its inverse, 64 x 64 each
    void* R1i = nullptr;
    void* Mx = nullptr;   // -R2^-1 S U'^-1, 64 x 64
    void* Tx = nullptr;   // the panels' T (compact WY), two alternating 64 x 64 row-major
    void* W = nullptr;    // V^T C_next of the last finished panel, 64 x 64
    void* tau = nullptr;  // the QR's taus (indexed by global column)
    int* flag = nullptr;  // set to 1 when a panel is too ill-conditioned for CholeskyQR2
    int* one_pass = nullptr;  // per panel, set by the first Cholesky: 1 when one pass suffices
};
int64_t cqr_num_chunks(int64_t m);
// Gram matrix of the panel [j0, j0+nb) into w.G; with jq >= 0 the previous panel's block
// reflector (explicit V over the rows [jq, m), column-major; T; w.W = V^T C) is applied to
// the panel's columns first
template <typename T>
hipError_t cqr_gram_update(T* Ac, int64_t m, int64_t jq, int64_t j0, int nb, const T* V,
                           const T* Tq, const CqrWs& w, hipStream_t st);
// CholeskyQR2 and the reconstruction of the panel: R and the reflectors' top block in place,
// the taus, M and the panel's T into Tout
template <typename T>
hipError_t cqr_factor_panel(T* Ac, int64_t m, int64_t j0, int nb, const CqrWs& w, T* Tout,
                            hipStream_t st);
// the rest of the reflectors in place, the explicit V (column-major, ld m - j0) into Vout,
// and with a next panel of nbn columns w.W = V^T C_next
template <typename T>
hipError_t cqr_finish_panel(T* Ac, int64_t m, int64_t j0, int nb, int nbn, const CqrWs& w,
                            T* Vout, hipStream_t st);
hipError_t cqr_clear_flag(int* flag, hipStream_t st);

// column pivoting on a sketch of the trailing columns (rcpqr.hip)
constexpr int PIV_YL = 72;  // rows of the pivot sketch: panel width + 8
struct PivWs {
    double* Om = nullptr;        // PIV_YL x m random signs
    double* Yt = nullptr;        // the pivot sketch, transposed: row j = sketch of column j
    double* Bt = nullptr;        // 64 x PIV_YL, R_11^-T Y_1^T of the last panel
    int32_t* cand[2] = {};       // tournament winners per group, 64 slots each
    int32_t* cnt[2] = {};        // winners per group
    int32_t* sel = nullptr;      // the panel's pivots (positions), in the order chosen
    double* nu = nullptr;        // remaining sketch norm at each choice
    int32_t* mv = nullptr;       // column moves: sources, destinations, count
    double* tA = nullptr;        // staging of the moved columns, 128 x m
    double* tY = nullptr;        // staging of their sketch rows
    int32_t* tP = nullptr;       // staging of their permutation entries
    int32_t* perm = nullptr;     // perm[j] = column of A now at position j
};
int64_t piv_groups(int64_t d);
size_t piv_ws_bytes(int64_t m, int64_t d);
void piv_ws_carve(void* base, int64_t m, int64_t d, PivWs& w);
// Omega, the sketch Y^T = (S A)^T Omega^T of the column-major Ac and perm = identity
hipError_t piv_init(double* Ac, int64_t m, int64_t d, uint64_t seed, PivWs& w, GemmWs& g,
                    hipStream_t st);
// nb pivots among the positions j0 .. d-1 into w.sel
hipError_t piv_select(int64_t j0, int64_t d, int nb, PivWs& w, hipStream_t st);
// move the pivots to positions j0 .. j0+nb-1 (columns of Ac, sketch rows, perm)
hipError_t piv_apply(double* Ac, int64_t m, int64_t j0, int nb, PivWs& w, hipStream_t st);
// Y_2 <- Y_2 - (Y_1 R_11^-1) R_12 after the panel at j0 and its trailing update
hipError_t piv_update_sketch(const double* Ac, int64_t m, int64_t j0, int nb, int64_t d,
                             PivWs& w, GemmWs& g, hipStream_t st);

// Householder QR of the m x (d+k) sketch on a column-major working copy
struct QrWs {
    void* Ac = nullptr;   // column-major copy of the sketch (ld = m), factored in place
    void* Vt = nullptr;   // [V^T; C_next^T] of a panel, explicit reflectors (two, alternating)
    void* Vt2 = nullptr;
    void* Wt = nullptr;   // products of the look-ahead update (caller's stream)
    void* W2t = nullptr;
    void* Wt2 = nullptr;  // products of the remaining-columns update (second stream)
    void* W2t2 = nullptr;
    void* Tp = nullptr;   // [V^T V; W_next^T] of a panel (two, alternating)
    void* Tp2 = nullptr;
    void* Tl = nullptr;   // the current leaf's T
    void* tau = nullptr;
    int* nonfinite = nullptr;  // set to 1 when the sketch holds a non-finite entry
    CqrWs cqr;            // panel factorisation by CholeskyQR2 (when cqr_panels)
    bool cqr_panels = true;
    GemmWs g;             // split-K partials, caller's stream
    GemmWs g2;            // split-K partials, second stream
    hipStream_t st2 = nullptr;
    hipEvent_t evF[2] = {nullptr, nullptr};  // panel's V^T V and reflectors ready
    hipEvent_t evE[2] = {nullptr, nullptr};  // remaining-columns update done
    // R_h^-1 formed alongside (FP64 without pivoting; rinv.hip): when Xinv is set, block
    // column j of X = R_h^-1 (row-major d x d) is formed on st3 once panel j is factored
    double* Xinv = nullptr;
    double* Zinv = nullptr;  // d x 64 scratch
    GemmWs g3;               // split-K partials, third stream
    hipStream_t st3 = nullptr;
    hipEvent_t evP = nullptr;  // panel factored
    hipEvent_t evI = nullptr;  // inverse blocks done
};
// R_h^-1 block by block (rinv.hip): block column [j0, j0 + nb) of X from the factored
// working copy Ac (column-major, ld m) and the blocks of X left of it; then R^-1 = X D with
// D the signs of R_h's diagonal, the lower triangle cleared, and XT = (R^-1)^T
size_t rinv_ws_bytes(int64_t d);
hipError_t rinv_block(const double* Ac, int64_t m, int64_t j0, int nb, double* X, int64_t d,
                      double* Z, GemmWs& g, hipStream_t s);
hipError_t rinv_finish(const double* Ac, int64_t m, int64_t d, double* X, double* XT,
                       hipStream_t st);
size_t qr_ws_bytes(Prec prec, int64_t m, int64_t ncols, size_t* gemm_bytes);
void qr_ws_carve(Prec prec, void* base, int64_t m, int64_t ncols, QrWs& ws);
hipError_t qr_factor(Prec prec, const void* SA, int64_t m, int64_t ncols, int64_t d, QrWs& ws,
                     hipStream_t st);
// A word of mapped, coherent pinned host memory that a kernel writes and the host polls:
// the host learns a device flag without a copy and a stream synchronisation.  host and dev
// are the two addresses of the same word (zero when allocated); seq counts publications.
struct HostFlag {
    volatile int32_t* host = nullptr;
    int32_t* dev = nullptr;
    int32_t seq = 0;
};
// after the work queued on st so far: word <- (seq << 1) | (*src != 0), with seq advanced
hipError_t launch_publish_flag(const int* src, HostFlag& f, hipStream_t st);
// polls the word until it carries the last published seq and returns its flag bit in *flag.
// The stream is queried while waiting, so an error on st (or st running dry without the
// word appearing) ends the wait with an error instead of a hang.
hipError_t wait_flag(HostFlag& f, hipStream_t st, int* flag);
// FP64 QR with column pivoting of the first d columns (the last ncols - d ride along),
// pivots chosen on the sketch of rcpqr.hip, the permutation in pw.perm.  Panels by
// CholeskyQR2 (cqr) with a per-panel fallback to Householder columns, or Householder
// columns only; pf: the host word through which each panel's flag is read (the host waits
// for it once per panel when cqr is set); panels_cqr (may be null) receives the number of
// panels that CholeskyQR2 factored.
hipError_t qr_factor_pivoted(const double* SA, int64_t m, int64_t ncols, int64_t d, QrWs& ws,
                             PivWs& pw, uint64_t seed, bool cqr, HostFlag& pf, int* panels_cqr,
                             hipStream_t st);
// copy R (d x d) and c (d x k) out of the factored copy into FP64 row-major, flipping
// rows so that diag(R) >= 0
hipError_t launch_extract_Rc(Prec prec, const QrWs& ws, int64_t m, int64_t d, int64_t k, double* R,
                             double* c, hipStream_t st);

}  // namespace ski
