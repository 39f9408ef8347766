// Device-side state of the LSQR and CG recurrences (one entry per right-hand side)
// and the launchers of the solve kernels.
#pragma once

#include "ski_internal.h"

namespace ski {

struct LsqrState {
    double alpha, beta, beta2, rhobar, phibar, anorm2, coef;
    double rnorm, arnorm, tc;
    double rr, stop2;  // CG
    int64_t iters;
    int32_t done, status, early, pad;
};

hipError_t trtri_upper(const double* R, int64_t d, double* Rinv, double* RinvT,
                       const double* diag_add, double* tmp, GemmWs& ws, hipStream_t st);
// y = s M x over the triangle of the d x d M; with perm, an upper product writes row i to
// y[perm[i]] and a lower one reads x[perm[j]]
hipError_t launch_tri_gemv(const double* M, int64_t d, bool upper, const double* x, int64_t ldx,
                           double* y, int64_t ldy, double s, const int32_t* done, hipStream_t st,
                           const int32_t* perm = nullptr);
// scatter dst[perm[i], :] = src[i, :] or gather dst[i, :] = src[perm[i], :]
hipError_t launch_permute_rows(const double* src, int64_t lds, double* dst, int64_t ldd,
                               const int32_t* perm, int64_t rows, int64_t cols, bool scatter,
                               hipStream_t st);
hipError_t launch_fill_rows(double* y, int64_t rows, int64_t cols, int64_t ldy, double v,
                            hipStream_t st);
int lsqr_pass_cpt(int64_t d);
hipError_t launch_lsqr_pass(const double* A, int64_t lda, int64_t n, int64_t d, const double* z,
                            double* u, const LsqrState* stt, int64_t G, double* gpart,
                            double* upart, double* g, LsqrState* stt_w, bool coef_m1,
                            hipStream_t st);
hipError_t launch_pass_kernel(const double* A, int64_t lda, int64_t n, int64_t d, const double* z,
                              double* u, const LsqrState* stt, int64_t G, double* gpart,
                              double* upart, bool coef_m1, hipStream_t st);
hipError_t launch_pass_reduce(const double* gpart, const double* upart, int64_t G, int64_t d,
                              double* g, LsqrState* stt_w, hipStream_t st);
hipError_t launch_spmv_csr(const int64_t* rp, const int32_t* ci, const double* va, int64_t n, int k,
                           const double* z, double* u, LsqrState* stt, bool coef_m1,
                           double* upart, hipStream_t st);
int64_t spmv_csr_groups(int64_t n);
hipError_t launch_spmv_csrT(const int32_t* tp, const int32_t* ti, const double* tv, int64_t d, int k,
                            const double* u, double* g, const LsqrState* stt, hipStream_t st);
hipError_t build_csrT(const int64_t* rp, const int32_t* ci, const double* va, int64_t n, int64_t d,
                      int64_t nnz, uint64_t* keys, uint64_t* keys_tmp, int32_t* table,
                      int32_t* tp, int32_t* payload, int32_t* ti, double* tv, hipStream_t st);
hipError_t launch_combine_u(const double* t, double* u, int64_t n, int k, const LsqrState* stt,
                            bool coef_m1, double* upart, int64_t G, LsqrState* stt_w,
                            hipStream_t st);
hipError_t launch_lsqr_init(LsqrState* stt, int64_t d, int k, const double* wp, double* v,
                            double* h, double* delta, double tau_a, hipStream_t st);
// hflag: the status word (1 once every column has stopped), written by the step itself:
// directly when k == 1, through the counter cnt (one uint32, zero between launches) when
// k > 1; with hflag null nothing is written
hipError_t launch_lsqr_step(LsqrState* stt, int64_t d, int k, const double* wp, double* v,
                            double* h, double* delta, double tau_r, int64_t it_max,
                            int32_t* hflag, uint32_t* cnt, hipStream_t st);
hipError_t launch_final_y(const LsqrState* stt, int64_t d, int k, const double* c,
                          const double* delta, double* y, hipStream_t st);
hipError_t launch_scale_copy(const double* x, int64_t rows, int64_t cols, int64_t ldx, double s,
                             double* y, int64_t ldy, hipStream_t st);
hipError_t launch_cg_init(LsqrState* stt, int64_t d, int k, const double* rhs, double* r, double* p,
                          double* y, double tol, hipStream_t st);
// word: the status word as for the LSQR step, through cnt (any k); null writes nothing
hipError_t launch_cg_step(LsqrState* stt, int64_t d, int k, const double* q, double* r, double* p,
                          double* y, int64_t it_max, int32_t* word, uint32_t* cnt,
                          hipStream_t st);
// flag <- 1 if every column has stopped (flag may be host memory mapped for the device)
hipError_t launch_all_done(const LsqrState* stt, int k, int32_t* flag, hipStream_t st);

}  // namespace ski
