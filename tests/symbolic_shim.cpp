// C entry points for testing the host symbolic phase of the sparse QR of the sketch
// (sparse_symbolic.cpp) on the CPU, without a GPU: run it on given row patterns and copy
// its arrays out.  Built by tests/test_host_symbolic.py with the host compiler.
#include <cstring>
#include <string>

#include "sparse_symbolic.h"

namespace {
ski::SparseSymbolic g_sym;
std::string g_err;

template <typename T>
void copy_out(T* dst, const std::vector<T>& src) {
    if (dst && !src.empty()) std::memcpy(dst, src.data(), src.size() * sizeof(T));
}
}  // namespace

extern "C" {

int sym_run(int64_t m, int64_t d, int64_t k, const int64_t* rstart, const int32_t* rlen,
            const int32_t* col, int64_t nvals, int dmax, int groups_target) {
    g_err.clear();
    return ski::sparse_symbolic(m, d, k, rstart, rlen, col, nvals, dmax, groups_target, g_sym,
                                g_err)
               ? 0
               : -1;
}

const char* sym_error() { return g_err.c_str(); }

// nleaf, nnz of the leaf rows (lcol), total sources, cb_total, root_rows, levels,
// transposed entries, up rows, lo rows, up lb entries, lo lb entries
void sym_sizes(int64_t* out) {
    const ski::SparseSymbolic& S = g_sym;
    out[0] = S.nleaf;
    out[1] = (int64_t)S.lcol.size();
    out[2] = (int64_t)S.src_a.size();
    out[3] = S.cb_total;
    out[4] = S.root_rows;
    out[5] = (int64_t)S.lev_ptr.size();
    out[6] = (int64_t)S.trow.size();
    out[7] = (int64_t)S.up.rows.size();
    out[8] = (int64_t)S.lo.rows.size();
    out[9] = (int64_t)S.up.gptr.size();
    out[10] = (int64_t)S.lo.gptr.size();
    out[11] = (int64_t)S.up.lb.size();
    out[12] = (int64_t)S.lo.lb.size();
}

void sym_get(int32_t* perm, int64_t* lptr, int32_t* lcol, int32_t* relmap, int32_t* parent,
             int32_t* nrows, int32_t* cbrows, int64_t* cboff, int64_t* src_ptr, int32_t* src_a,
             int32_t* src_b, int32_t* ent_lc, int64_t* lev_ptr, int32_t* lev_front,
             int64_t* tptr, int32_t* trow, int64_t* tent) {
    const ski::SparseSymbolic& S = g_sym;
    copy_out(perm, S.perm);
    copy_out(lptr, S.lptr);
    copy_out(lcol, S.lcol);
    copy_out(relmap, S.relmap);
    copy_out(parent, S.parent);
    copy_out(nrows, S.nrows);
    copy_out(cbrows, S.cbrows);
    copy_out(cboff, S.cboff);
    copy_out(src_ptr, S.src_ptr);
    copy_out(src_a, S.src_a);
    copy_out(src_b, S.src_b);
    copy_out(ent_lc, S.ent_lc);
    copy_out(lev_ptr, S.lev_ptr);
    copy_out(lev_front, S.lev_front);
    copy_out(tptr, S.tptr);
    copy_out(trow, S.trow);
    copy_out(tent, S.tent);
}

// the two solve schedules: rows, group pointers, level-boundary pointers and boundaries
void sym_sched(int upper, int32_t* rows, int64_t* gptr, int64_t* lbptr, int64_t* lb) {
    const ski::SparseSymbolic::Sched& s = upper ? g_sym.up : g_sym.lo;
    copy_out(rows, s.rows);
    copy_out(gptr, s.gptr);
    copy_out(lbptr, s.lbptr);
    copy_out(lb, s.lb);
}

}  // extern "C"
