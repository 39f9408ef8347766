// The sparse QR of the sketch (Section 6, the sparse solver: S A is factored by a sparse
// QR after a fill-reducing column ordering, and every product with R^-1 is a sparse
// back-substitution).  Multifrontal: the columns eliminated by the minimum-degree order
// (sparse_symbolic.h) are factored one front each, a Householder QR in LDS per front and
// one launch per elimination-tree level; the columns left form one dense root front that
// the dense QR of the sketch factors.  R is held as the leaf rows (sparse) and the root
// block (dense, with its explicit inverse); R^-1 x and R^-T x walk the leaf forest level by
// level inside one launch, a workgroup per group of whole trees.
#pragma once

#include <string>
#include <vector>

#include "ski_internal.h"
#include "sparse_symbolic.h"

namespace ski {

class SparseQR {
   public:
    SparseQR() = default;
    SparseQR(const SparseQR&) = delete;
    SparseQR& operator=(const SparseQR&) = delete;
    ~SparseQR();

    // Step 1: SA = scale S_h A as rows of ascending columns (row b at rawoff[b], ucnt[b]
    // entries; the sums run over the bucket's entries in order from +0.0, as the dense
    // gather's do) and Sb = scale S_h B (m x k).  CSR A (row_ptr int64, col int32
    // ascending within a row).
    hipError_t sketch(const int64_t* row_ptr, const int32_t* col, const double* val, int64_t n,
                      int64_t d, const double* B, int64_t ldb, int64_t k, const int32_t* bucket_ptr,
                      const int32_t* src, int64_t m, double scale, hipStream_t st);
    // symbolic phase on the host (synchronises st): copies the pattern of SA, orders it
    // (degree cap dmax <= 63 - k) and uploads the structure.  false: message in err.
    bool analyse(int dmax, hipStream_t st, std::string& err);
    // numeric leaf fronts, level by level: the leaf rows of R (diag, off-diagonal values,
    // c) and the contribution blocks; clears the non-finite flag first
    hipError_t factor_leaves(hipStream_t st);
    // device int set to 1 when the fronts or the root assembly met a non-finite value
    const int* nonfinite_dev() const;
    // the root front (root_rows_pad() x (nroot + k), row-major) assembled from the sketch
    // rows and the contribution blocks that reach it; rows beyond root_rows() are zero
    int64_t root_rows_pad() const;
    hipError_t assemble_root(double* root, hipStream_t st);
    // after the root's QR: the leaf diagonal perturbation (nleaf entries, device) and the
    // root inverses (nroot x nroot, row-major: Rinv upper, RinvT = its transpose)
    void set_root(const double* Rinv, const double* RinvT, const double* leaf_add) {
        rinv_ = Rinv;
        rinvT_ = RinvT;
        ladd_ = leaf_add;
    }
    hipError_t finish_factor(hipStream_t st);  // transposed values for R^-T
    // diag(R) in position order (device, d doubles: leaf rows; the root's is filled by the
    // caller from its dense R)
    hipError_t leaf_diag(double* out, hipStream_t st) const;
    // c of the leaf rows (position order, ld k) into c (d x k)
    hipError_t leaf_c(double* c, hipStream_t st) const;
    // y = s R^-1 x: x in position order (ld ldx), y in column order (row perm[p], ld ldy).
    // tmp: d x k doubles.  The root part through root_upper (computes tmp[nleaf ..] =
    // R_root^-1 x[nleaf ..]) supplied by the caller.
    hipError_t leaves_upper(const double* x, int64_t ldx, double* tmp, double* y, int64_t ldy,
                            int k, double s, const int32_t* done, hipStream_t st) const;
    // y = s R^-T x, part one: x in column order (ld ldx); the leaf part of y (position
    // order, ld ldy) and tmp (d x k, the unscaled leaf values, then at nleaf .. the root's
    // right-hand side x_root - R_leaf,root^T y_leaf) for the caller's root product
    hipError_t leaves_lower(const double* x, int64_t ldx, double* tmp, double* y, int64_t ldy,
                            int k, double s, const int32_t* done, hipStream_t st) const;
    // dense R (position space, d x d row-major, root block included from Rroot) for
    // inspection
    hipError_t dense_R(const double* Rroot, double* R, hipStream_t st) const;

    const SparseSymbolic& sym() const { return sym_; }
    const int32_t* perm_dev() const { return perm_; }
    int64_t nleaf() const { return sym_.nleaf; }
    int64_t nroot() const { return sym_.nroot; }
    int64_t m() const { return m_; }
    int64_t k() const { return k_; }
    int64_t nnz_sa() const { return nnz_sa_; }
    int64_t root_rows() const { return sym_.root_rows; }
    // SA as the dense m x (d + k) row-major sketch, for inspection
    hipError_t dense_SA(double* SA, hipStream_t st) const;

   private:
    struct Buf {
        void* p = nullptr;
        size_t bytes = 0;
    };
    hipError_t ensure(Buf& b, size_t bytes);
    template <typename T>
    T* ptr(const Buf& b) const {
        return (T*)b.p;
    }

    int64_t m_ = 0, d_ = 0, k_ = 0, nraw_ = 0, nnz_sa_ = 0;
    Buf rawoff_, ucnt_, sacol_, saval_, sb_, scan_;
    SparseSymbolic sym_;
    // device structure (one int64 buffer, one int32 buffer, carved)
    Buf i64_, i32_;
    const int64_t *lptr_ = nullptr, *srcptr_ = nullptr, *cboff_ = nullptr, *levptr_ = nullptr,
                  *upg_ = nullptr, *uplbp_ = nullptr, *uplb_ = nullptr, *log_ = nullptr,
                  *lolbp_ = nullptr, *lolb_ = nullptr, *tptr_ = nullptr, *tent_ = nullptr;
    const int32_t *lcol_ = nullptr, *relmap_ = nullptr, *srca_ = nullptr, *srcb_ = nullptr,
                  *entlc_ = nullptr, *levfront_ = nullptr, *uprows_ = nullptr, *lorows_ = nullptr,
                  *trow_ = nullptr, *perm_ = nullptr, *cbrows_ = nullptr;
    // numeric factor
    Buf rdiag_, rv_, cleaf_, cb_, tval_, flag_;
    const double *rinv_ = nullptr, *rinvT_ = nullptr, *ladd_ = nullptr;
};

}  // namespace ski
