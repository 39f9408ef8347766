// Symbolic phase of the sparse QR of the sketch (Section 6, the sparse solver: the sketch
// S A of a sparse A is factored by a sparse QR after a fill-reducing column ordering).
// Host code only: the ordering, the elimination tree, the fronts of the multifrontal
// factorisation with their assembly maps, and the level schedules of the factorisation
// and of the triangular solves.  The numeric work runs on the GPU (sparse_qr.hip).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace ski {

// The factorisation: positions 0 .. nleaf-1 hold the eliminated columns in elimination
// order (one leaf front each); positions nleaf .. d-1 hold the root, the columns whose
// degree exceeded the cap, in increasing column index, factored as one dense front.
// Row q < nleaf of R is non-zero at q and at lcol[lptr[q] .. lptr[q+1]) (ascending
// positions > q).  Front q's local columns are: 0 = q, 1 .. |L_q| = lcol of row q, then
// the k right-hand-side columns.  The root front's local columns are position - nleaf,
// then the k right-hand sides.  Fronts are indexed 0 .. nleaf, nleaf being the root.
struct SparseSymbolic {
    int64_t d = 0, m = 0, k = 0;
    int64_t nleaf = 0, nroot = 0;
    int dmax = 0;
    std::vector<int32_t> perm;    // [d] position -> column
    std::vector<int64_t> lptr;    // [nleaf+1]
    std::vector<int32_t> lcol;    // positions
    std::vector<int32_t> relmap;  // [lcol.size()] local column in the parent front of
                                  // the child's CB column (the parent's root index when the
                                  // parent is the root)
    std::vector<int32_t> parent;  // [nleaf] parent position (>= nleaf: the root), -1: none
    // fronts 0 .. nleaf
    std::vector<int32_t> nrows;   // [nleaf+1] rows assembled into the front
    std::vector<int32_t> cbrows;  // [nleaf] contribution rows passed to the parent
    std::vector<int64_t> cboff;   // [nleaf] offset (doubles) of the contribution block,
                                  // cbrows x (|L_q| + k), row-major
    int64_t cb_total = 0;
    // row sources of each front, in assembly order: sa rows (src_a = SA row, src_b = -1)
    // ascending, then each child's contribution rows (src_a = child, src_b = row)
    std::vector<int64_t> src_ptr;  // [nleaf+2]
    std::vector<int32_t> src_a, src_b;
    // local column of every stored entry of SA within the front its row is assembled
    // into (indexed like the SA values; -1 for rows with no stored entry)
    std::vector<int32_t> ent_lc;
    // factorisation levels: fronts of equal height (children before parents)
    std::vector<int64_t> lev_ptr;
    std::vector<int32_t> lev_front;
    // the triangular solves: groups of whole trees of the leaf forest, each walked level
    // by level by one workgroup; rows of group g in [gptr[g], gptr[g+1]) sorted by level,
    // its level boundaries (absolute offsets) in lb[lbptr[g] .. lbptr[g+1]]
    struct Sched {
        std::vector<int32_t> rows;
        std::vector<int64_t> gptr, lbptr, lb;
    } up, lo;  // up: R^-1 (top-down by depth); lo: R^-T (bottom-up by height)
    // R^-T: for each position q, the leaf rows f with q in L_f (ascending f) and the index
    // of R_fq among the leaf rows' stored entries
    std::vector<int64_t> tptr;  // [d+1]
    std::vector<int32_t> trow;
    std::vector<int64_t> tent;
    int64_t root_rows = 0;  // rows assembled into the root front
    int max_height = 0, max_depth = 0;
};

// SA given by rows: row r holds rlen[r] ascending columns at col[rstart[r] ..) (nvals:
// the length of the value array those offsets index).  dmax: the degree cap, at most
// 63 - k so that a front holds at most 64 columns (-1 puts every column in the root).
// Returns false (message in err) if the problem does not fit the limits (k <= 32).
bool sparse_symbolic(int64_t m, int64_t d, int64_t k, const int64_t* rstart, const int32_t* rlen,
                     const int32_t* col, int64_t nvals, int dmax, int groups_target,
                     SparseSymbolic& S, std::string& err);

}  // namespace ski
