// Symbolic phase of the sparse QR of the sketch (Section 6, the sparse solver).
//
// Ordering: exact minimum degree on the column graph of (SA)^T (SA), kept as a quotient
// graph: the rows of SA are the initial elements (each a clique of its columns);
// eliminating column j absorbs every element that holds j into one new element holding
// j's live neighbours.  The degree of a column is the number of distinct other live
// columns in its live elements, which equals its degree in the elimination graph, so the
// order is the one the plain elimination-graph rule gives: smallest degree first, ties by
// smallest column index.  Elimination stops as soon as the smallest degree exceeds the
// cap (at most 63 - k, so that a front holds at most 64 columns); the rest is the root.
#include "sparse_symbolic.h"

#include <algorithm>
#include <climits>
#include <numeric>
#include <queue>
#include <utility>

namespace ski {

namespace {

// Columns by degree (0 .. cap, cap = dmax + 1 for every column above the cap): one
// two-level bitset per degree, so that the smallest column index of the smallest degree
// is found by scanning d/4096 summary words and one word.
class DegreeBuckets {
   public:
    DegreeBuckets(int64_t d, int ndeg)
        : nw_((d + 63) / 64), ns_((nw_ + 63) / 64), w_((size_t)ndeg * nw_, 0),
          s_((size_t)ndeg * ns_, 0), ndeg_(ndeg) {}
    void insert(int deg, int64_t v) {
        uint64_t* w = &w_[(size_t)deg * nw_];
        w[v >> 6] |= 1ull << (v & 63);
        s_[(size_t)deg * ns_ + (v >> 12)] |= 1ull << ((v >> 6) & 63);
    }
    void erase(int deg, int64_t v) {
        uint64_t* w = &w_[(size_t)deg * nw_];
        w[v >> 6] &= ~(1ull << (v & 63));
        if (!w[v >> 6]) s_[(size_t)deg * ns_ + (v >> 12)] &= ~(1ull << ((v >> 6) & 63));
    }
    // smallest (degree, column) with degree < limit; false if none
    bool first(int limit, int& deg, int64_t& v) const {
        for (int g = 0; g < std::min(limit, ndeg_); ++g) {
            const uint64_t* s = &s_[(size_t)g * ns_];
            for (int64_t i = 0; i < ns_; ++i)
                if (s[i]) {
                    const int64_t wi = i * 64 + __builtin_ctzll(s[i]);
                    const uint64_t wv = w_[(size_t)g * nw_ + wi];
                    deg = g;
                    v = wi * 64 + __builtin_ctzll(wv);
                    return true;
                }
        }
        return false;
    }

   private:
    int64_t nw_, ns_;
    std::vector<uint64_t> w_, s_;
    int ndeg_;
};

// the level schedule of the triangular solves: trees of the leaf forest packed into
// groups (heaviest tree first, each to the lightest group), rows sorted by level
void build_sched(const SparseSymbolic& S, const std::vector<int32_t>& top,
                 const std::vector<int32_t>& level, int groups_target,
                 SparseSymbolic::Sched& out) {
    const int64_t nl = S.nleaf;
    out = SparseSymbolic::Sched();
    std::vector<int64_t> weight(nl, 0);
    std::vector<int32_t> tops;
    for (int64_t q = 0; q < nl; ++q) {
        weight[top[q]] += 1 + (S.lptr[q + 1] - S.lptr[q]);
        if (top[q] == q) tops.push_back((int32_t)q);
    }
    const int64_t G = std::max<int64_t>(1, std::min<int64_t>((int64_t)tops.size(), groups_target));
    std::vector<int32_t> order = tops;
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b) { return weight[a] > weight[b]; });
    using Slot = std::pair<int64_t, int64_t>;  // (load, group)
    std::priority_queue<Slot, std::vector<Slot>, std::greater<Slot>> pq;
    for (int64_t g = 0; g < G; ++g) pq.push({0, g});
    std::vector<int32_t> group_of_top(nl, -1);
    for (int32_t t : order) {
        Slot s = pq.top();
        pq.pop();
        group_of_top[t] = (int32_t)s.second;
        pq.push({s.first + weight[t], s.second});
    }
    std::vector<std::vector<int32_t>> rows(G);
    for (int64_t q = 0; q < nl; ++q) rows[group_of_top[top[q]]].push_back((int32_t)q);
    out.gptr.push_back(0);
    out.lbptr.push_back(0);
    for (int64_t g = 0; g < G; ++g) {
        auto& r = rows[g];
        std::stable_sort(r.begin(), r.end(),
                         [&](int32_t a, int32_t b) { return level[a] < level[b]; });
        const int64_t base = (int64_t)out.rows.size();
        for (size_t i = 0; i < r.size(); ++i) {
            if (i == 0 || level[r[i]] != level[r[i - 1]]) out.lb.push_back(base + (int64_t)i);
            out.rows.push_back(r[i]);
        }
        out.lb.push_back(base + (int64_t)r.size());
        out.gptr.push_back((int64_t)out.rows.size());
        out.lbptr.push_back((int64_t)out.lb.size());
    }
}

}  // namespace

bool sparse_symbolic(int64_t m, int64_t d, int64_t k, const int64_t* rstart, const int32_t* rlen,
                     const int32_t* col, int64_t nvals, int dmax, int groups_target,
                     SparseSymbolic& S, std::string& err) {
    if (k < 1 || k > 32) {
        err = "the sparse factorisation takes 1 <= k <= 32 right-hand sides";
        return false;
    }
    if (dmax < -1 || dmax > 63 - k) {
        err = "the degree cap must lie in [-1, 63 - k]";
        return false;
    }
    if (d > ((int64_t)1 << 30) || m > ((int64_t)1 << 30)) {
        err = "the sparse factorisation takes m, d <= 2^30";
        return false;
    }
    S = SparseSymbolic();
    S.d = d;
    S.m = m;
    S.k = k;
    S.dmax = dmax;

    // ---- minimum degree on the quotient graph
    // element e's columns: ev[eoff[e] .. eoff[e + 1]) in one append-only array (the rows of
    // SA first, then one new element per elimination)
    std::vector<int32_t> ev;
    std::vector<int64_t> eoff{0};
    std::vector<std::vector<int32_t>> vel(d);  // elements holding each column (may list dead)
    // the rows must lie in the value array and hold strictly ascending columns in [0, d)
    // (the sketch merges equal columns, so only a column index of A outside [0, d) can
    // break this; it would otherwise index past the arrays below)
    for (int64_t r = 0; r < m; ++r) {
        if (rlen[r] <= 0) continue;
        if (rstart[r] < 0 || rstart[r] + rlen[r] > nvals) {
            err = "the sketch's row offsets run past its entries";
            return false;
        }
        int64_t prev = -1;
        for (int32_t u = 0; u < rlen[r]; ++u) {
            const int64_t c = col[rstart[r] + u];
            if (c <= prev || c >= d) {
                err = "a column index of A lies outside [0, d)";
                return false;
            }
            prev = c;
        }
    }
    {
        int64_t tot = 0;
        for (int64_t r = 0; r < m; ++r) tot += std::max<int32_t>(rlen[r], 0);
        ev.reserve(tot + (size_t)d * 16);
        eoff.reserve(m + d + 1);
        std::vector<int32_t> cnt(d, 0);
        for (int64_t r = 0; r < m; ++r)
            for (int32_t u = 0; u < rlen[r]; ++u) ++cnt[col[rstart[r] + u]];
        for (int64_t v = 0; v < d; ++v) vel[v].reserve(cnt[v] + 4);
    }
    for (int64_t r = 0; r < m; ++r) {
        if (rlen[r] <= 0) continue;
        const int32_t e = (int32_t)(eoff.size() - 1);
        ev.insert(ev.end(), col + rstart[r], col + rstart[r] + rlen[r]);
        eoff.push_back((int64_t)ev.size());
        for (int32_t u = 0; u < rlen[r]; ++u) vel[col[rstart[r] + u]].push_back(e);
    }
    std::vector<char> edead(eoff.size() - 1, 0);
    std::vector<char> elim(d, 0);
    std::vector<int32_t> mark(d, -1);  // 4-byte stamps: d = 8000 columns stay in L1
    int32_t stamp = 0;
    // The degree, counted only up to CNT_CAP: a column above the cap dmax is never chosen,
    // and eliminating a neighbour lowers a column's degree by at most one (it loses that
    // neighbour and keeps the others), while a non-neighbour's degree does not change.  So
    // lb[v], the count (a lower bound once it reached CNT_CAP), minus one per eliminated
    // neighbour, stays a lower bound, and v is counted again only once lb[v] - 1 could be
    // <= dmax; from there on it is counted exactly.  The order is the uncapped rule's.
    const int64_t CNT_CAP = (int64_t)dmax + 65;
    // a fresh stamp; room for `need` more is made first (the marks are cleared when the
    // stamps would run out), so that the stamps of one elimination stay valid together
    auto next_stamp = [&](int need = 1) {
        if (stamp > INT32_MAX - 1 - need) {
            std::fill(mark.begin(), mark.end(), -1);
            stamp = 0;
        }
        return ++stamp;
    };
    auto degree = [&](int32_t v) {
        const int32_t sv = next_stamp();
        mark[v] = sv;  // v itself is not counted
        int64_t cnt = 0;
        for (int32_t e : vel[v]) {
            if (edead[e]) continue;
            for (int64_t q = eoff[e]; q < eoff[e + 1]; ++q) {
                const int32_t u = ev[q];
                const bool fresh = mark[u] != sv;
                mark[u] = sv;
                cnt += fresh;
            }
            if (cnt >= CNT_CAP) break;  // a lower bound from here (checked per element)
        }
        return cnt;
    };
    // the same count for a neighbour v of the column just eliminated, whose members Lj carry
    // the stamp s0 (v among them), before the new element joins v's list: |Lj| - 1, plus the
    // members of v's other live elements outside Lj.  Every absorbed element lay inside Lj
    // and j, so this is v's degree; Lj is marked once per elimination instead of once per
    // neighbour.  The same pass drops the absorbed elements from v's list, and absorbs any
    // element found to lie inside Lj: each of its members holds Lj too, so no degree changes.
    auto degree_after = [&](int32_t v, int32_t s0, int64_t nlj) {
        const int32_t sv = next_stamp();
        int64_t cnt = nlj - 1;
        auto& L = vel[v];
        size_t w = 0;
        for (size_t i = 0; i < L.size(); ++i) {
            const int32_t e = L[i];
            if (edead[e]) continue;
            if (cnt >= CNT_CAP) {
                L[w++] = e;
                continue;
            }
            // branch-free over the members (their marks follow no pattern); the cap is
            // checked per element, so the count can pass it by less than one element
            bool inside = true;
            for (int64_t q = eoff[e]; q < eoff[e + 1]; ++q) {
                const int32_t u = ev[q];
                const int32_t mu = mark[u];
                const bool in_lj = mu == s0, fresh = !in_lj & (mu != sv);
                inside &= in_lj;
                mark[u] = fresh ? sv : mu;
                cnt += fresh;
            }
            if (inside)
                edead[e] = 1;
            else
                L[w++] = e;
        }
        L.resize(w);
        return cnt;
    };
    std::vector<int64_t> lb(d);
    const int ndeg = dmax + 2;  // degrees 0 .. dmax, and dmax + 1 for every capped column
    std::vector<int> deg(d);
    DegreeBuckets pq(d, ndeg);
    for (int64_t v = 0; v < d; ++v) {
        lb[v] = degree((int32_t)v);
        deg[v] = (int)std::min<int64_t>(lb[v], dmax + 1);
        pq.insert(deg[v], v);
    }
    std::vector<int32_t> order;
    std::vector<int64_t> lptr_c{0};
    std::vector<int32_t> lcol_c;  // neighbours as column ids
    std::vector<int32_t> Lj;
    for (;;) {
        int bdeg = 0;
        int64_t bv = 0;
        if (!pq.first(dmax + 1, bdeg, bv)) break;  // the smallest degree exceeds the cap
        pq.erase(bdeg, bv);
        const int32_t j = (int32_t)bv;
        // j's live neighbours: the union of its live elements (which hold live columns only:
        // every element holding an eliminated column was absorbed when it was eliminated).
        // Their stamp s0 stays valid through this elimination: one stamp per neighbour follows.
        const int32_t s0 = next_stamp(64);
        Lj.clear();
        for (int32_t e : vel[j]) {
            if (edead[e]) continue;
            for (int64_t q = eoff[e]; q < eoff[e + 1]; ++q) {
                const int32_t u = ev[q];
                if (u != j && mark[u] != s0) {
                    mark[u] = s0;
                    Lj.push_back(u);
                }
            }
            edead[e] = 1;  // absorbed into the new element
        }
        std::sort(Lj.begin(), Lj.end());
        elim[j] = 1;
        order.push_back(j);
        lcol_c.insert(lcol_c.end(), Lj.begin(), Lj.end());
        lptr_c.push_back((int64_t)lcol_c.size());
        std::vector<int32_t>().swap(vel[j]);
        const int32_t ne = (int32_t)(eoff.size() - 1);
        ev.insert(ev.end(), Lj.begin(), Lj.end());
        eoff.push_back((int64_t)ev.size());
        edead.push_back(0);
        for (int32_t v : Lj) {
            if (lb[v] - 1 > dmax) {
                // still above the cap: its bucket (dmax + 1) is unchanged, and its list keeps
                // the absorbed elements until it is counted again (they are skipped)
                --lb[v];
                vel[v].push_back(ne);
                continue;
            }
            pq.erase(deg[v], v);
            lb[v] = degree_after(v, s0, (int64_t)Lj.size());
            vel[v].push_back(ne);
            deg[v] = (int)std::min<int64_t>(lb[v], dmax + 1);
            pq.insert(deg[v], v);
        }
    }
    const int64_t nl = (int64_t)order.size();
    S.nleaf = nl;
    S.nroot = d - nl;
    S.perm = order;
    for (int64_t v = 0; v < d; ++v)
        if (!elim[v]) S.perm.push_back((int32_t)v);
    std::vector<int32_t> pos(d);
    for (int64_t q = 0; q < d; ++q) pos[S.perm[q]] = (int32_t)q;

    // ---- rows of R (positions), elimination tree
    S.lptr = lptr_c;
    S.lcol.resize(lcol_c.size());
    S.parent.assign(nl, -1);
    for (int64_t q = 0; q < nl; ++q) {
        for (int64_t e = S.lptr[q]; e < S.lptr[q + 1]; ++e) S.lcol[e] = pos[lcol_c[e]];
        std::sort(S.lcol.begin() + S.lptr[q], S.lcol.begin() + S.lptr[q + 1]);
        if (S.lptr[q + 1] > S.lptr[q]) S.parent[q] = S.lcol[S.lptr[q]];
    }
    const int64_t ROOT = nl;  // front index of the root
    auto front_of_parent = [&](int64_t q) -> int64_t {
        const int32_t p = S.parent[q];
        return p < 0 ? -1 : (p < nl ? p : ROOT);
    };
    // lcmap[pq] = the local column of position pq in the front being visited, -1 elsewhere:
    // set from a leaf front's columns, used, then cleared (each front costs |L_f| + 1)
    std::vector<int32_t> lcmap(d, -1);
    auto map_front = [&](int64_t f, bool on) {
        lcmap[f] = on ? 0 : -1;
        for (int64_t e = S.lptr[f]; e < S.lptr[f + 1]; ++e)
            lcmap[S.lcol[e]] = on ? (int32_t)(1 + (e - S.lptr[f])) : -1;
    };

    // ---- row assignment: each non-empty row of SA goes to the front of its first position;
    // the rows of front f, ascending, are orows[optr[f] .. optr[f + 1])
    std::vector<int32_t> rfront(m, -1);
    std::vector<int64_t> optr(nl + 2, 0);
    for (int64_t r = 0; r < m; ++r) {
        if (rlen[r] <= 0) continue;
        int32_t first = INT32_MAX;
        for (int32_t u = 0; u < rlen[r]; ++u) first = std::min(first, pos[col[rstart[r] + u]]);
        rfront[r] = first < nl ? first : (int32_t)ROOT;
        ++optr[rfront[r] + 1];
    }
    for (int64_t f = 0; f <= nl; ++f) optr[f + 1] += optr[f];
    std::vector<int32_t> orows(optr[nl + 1]);
    {
        std::vector<int64_t> fill(optr.begin(), optr.end() - 1);
        for (int64_t r = 0; r < m; ++r)
            if (rfront[r] >= 0) orows[fill[rfront[r]]++] = (int32_t)r;
    }
    S.ent_lc.assign(nvals, -1);
    for (int64_t f = 0; f <= nl; ++f) {
        if (optr[f] == optr[f + 1]) continue;
        if (f < nl) map_front(f, true);
        for (int64_t i = optr[f]; i < optr[f + 1]; ++i) {
            const int32_t r = orows[i];
            for (int32_t u = 0; u < rlen[r]; ++u) {
                const int32_t pq = pos[col[rstart[r] + u]];
                const int32_t lc = f == ROOT ? (int32_t)(pq - nl) : lcmap[pq];
                if (lc < 0) {
                    err = "internal: a row of the sketch does not fit its front";
                    return false;
                }
                S.ent_lc[rstart[r] + u] = lc;
            }
        }
        if (f < nl) map_front(f, false);
    }
    // ---- children (ascending, kid[kptr[f] .. kptr[f + 1])), front sizes, contribution blocks
    std::vector<int64_t> kptr(nl + 2, 0);
    for (int64_t q = 0; q < nl; ++q) {
        const int64_t pf = front_of_parent(q);
        if (pf >= 0) ++kptr[pf + 1];
    }
    for (int64_t f = 0; f <= nl; ++f) kptr[f + 1] += kptr[f];
    std::vector<int32_t> kid(kptr[nl + 1]);
    {
        std::vector<int64_t> fill(kptr.begin(), kptr.end() - 1);
        for (int64_t q = 0; q < nl; ++q) {
            const int64_t pf = front_of_parent(q);
            if (pf >= 0) kid[fill[pf]++] = (int32_t)q;
        }
    }
    S.nrows.assign(nl + 1, 0);
    S.cbrows.assign(nl, 0);
    S.cboff.assign(nl, 0);
    for (int64_t q = 0; q <= nl; ++q) {
        int64_t rows = optr[q + 1] - optr[q];
        for (int64_t i = kptr[q]; i < kptr[q + 1]; ++i) rows += S.cbrows[kid[i]];
        if (rows > INT32_MAX) {
            err = "a front holds more than 2^31 rows";
            return false;
        }
        S.nrows[q] = (int32_t)rows;
        if (q < nl) {
            const int64_t ncA = 1 + (S.lptr[q + 1] - S.lptr[q]);
            S.cbrows[q] = (int32_t)std::max<int64_t>(0, std::min<int64_t>(rows, ncA) - 1);
            S.cboff[q] = S.cb_total;
            S.cb_total += (int64_t)S.cbrows[q] * ((S.lptr[q + 1] - S.lptr[q]) + k);
        }
    }
    S.root_rows = S.nrows[nl];
    S.src_ptr.assign(nl + 2, 0);
    S.src_a.reserve(optr[nl + 1] + (size_t)S.cb_total);
    for (int64_t q = 0; q <= nl; ++q) {
        for (int64_t i = optr[q]; i < optr[q + 1]; ++i) {
            S.src_a.push_back(orows[i]);
            S.src_b.push_back(-1);
        }
        for (int64_t i = kptr[q]; i < kptr[q + 1]; ++i) {
            const int32_t c = kid[i];
            for (int32_t t = 0; t < S.cbrows[c]; ++t) {
                S.src_a.push_back(c);
                S.src_b.push_back(t);
            }
        }
        S.src_ptr[q + 1] = (int64_t)S.src_a.size();
    }
    // ---- where each child's contribution columns land in its parent
    S.relmap.assign(S.lcol.size(), -1);
    for (int64_t f = 0; f <= nl; ++f) {
        if (kptr[f] == kptr[f + 1]) continue;
        if (f < nl) map_front(f, true);
        for (int64_t i = kptr[f]; i < kptr[f + 1]; ++i) {
            const int32_t q = kid[i];
            for (int64_t e = S.lptr[q]; e < S.lptr[q + 1]; ++e) {
                const int32_t lc = f == ROOT ? (int32_t)(S.lcol[e] - nl) : lcmap[S.lcol[e]];
                if (lc < 0) {
                    err = "internal: a contribution column is missing from its parent front";
                    return false;
                }
                S.relmap[e] = lc;
            }
        }
        if (f < nl) map_front(f, false);
    }
    // ---- heights (factorisation levels), depths, trees
    std::vector<int32_t> height(nl, 0), depth(nl, 0), top(nl, 0);
    for (int64_t q = 0; q < nl; ++q) {
        const int32_t p = S.parent[q];
        if (p >= 0 && p < nl) height[p] = std::max(height[p], height[q] + 1);
    }
    for (int64_t q = nl - 1; q >= 0; --q) {
        const int32_t p = S.parent[q];
        const bool inner = p >= 0 && p < nl;
        depth[q] = inner ? depth[p] + 1 : 0;
        top[q] = inner ? top[p] : (int32_t)q;
    }
    for (int64_t q = 0; q < nl; ++q) {
        S.max_height = std::max(S.max_height, height[q]);
        S.max_depth = std::max(S.max_depth, depth[q]);
    }
    const int nlev = nl ? S.max_height + 1 : 0;
    S.lev_ptr.assign(nlev + 1, 0);
    for (int64_t q = 0; q < nl; ++q) ++S.lev_ptr[height[q] + 1];
    for (int l = 0; l < nlev; ++l) S.lev_ptr[l + 1] += S.lev_ptr[l];
    S.lev_front.resize(nl);
    {
        std::vector<int64_t> fill(S.lev_ptr.begin(), S.lev_ptr.end() - (nlev ? 1 : 0));
        for (int64_t q = 0; q < nl; ++q) S.lev_front[fill[height[q]]++] = (int32_t)q;
    }
    build_sched(S, top, depth, groups_target, S.up);
    build_sched(S, top, height, groups_target, S.lo);
    // ---- transposed lists for R^-T
    S.tptr.assign(d + 1, 0);
    for (int32_t q : S.lcol) ++S.tptr[q + 1];
    for (int64_t q = 0; q < d; ++q) S.tptr[q + 1] += S.tptr[q];
    S.trow.resize(S.lcol.size());
    S.tent.resize(S.lcol.size());
    {
        std::vector<int64_t> fill(S.tptr.begin(), S.tptr.end() - 1);
        for (int64_t f = 0; f < nl; ++f)
            for (int64_t e = S.lptr[f]; e < S.lptr[f + 1]; ++e) {
                const int64_t slot = fill[S.lcol[e]]++;
                S.trow[slot] = (int32_t)f;
                S.tent[slot] = e;
            }
    }
    return true;
}

}  // namespace ski
