// Column pivoting for the rank-revealing factorisation of the sketch (Step 2 of Algorithm 1
// in the form S A V-hat = Q R; Section 6 names randomised column-pivoted QR as the default
// dense factorisation).  The pivots of each 64-column panel are chosen on a small random
// sketch of the trailing columns, Y = Omega [S A] (Omega: 72 rows of random signs), as in
// the blocked randomised QRCP of Martinsson et al. (2017) and Duersch and Gu (2017):
//
//   * selection: greedy column pivoting on Y (the column with the largest remaining norm,
//     then its direction projected out of every other column), arranged as a tournament
//     (Demmel, Grigori, Gu and Xiang 2015) so that it runs on many workgroups: groups of
//     up to 512 columns each choose 64 with the sketch held in registers, then the
//     winners of up to 8 groups meet in one group, until one group is left;
//   * the chosen columns are moved to the front of the trailing matrix, whole columns
//     (rows above the panel hold R entries and move with them), as are their sketch rows
//     and their entries of the permutation;
//   * after the panel's Householder QR and the trailing update, the sketch of the
//     trailing columns is brought up to date without touching [S A] again:
//     Y_2 <- Y_2 - (Y_1 R_11^-1) R_12.
//
// The panel itself is factored by Householder reflections in FP64 (qr.hip), so the
// diagonal of R that decides the rank is that of a backward-stable QR of S A P.  The
// random signs come from Philox4x64-10 keyed by the caller's seed: the pivots are
// deterministic.  Ties in the selection go to the lower candidate slot.
#include "ski_internal.h"
#include "tile64.h"

namespace ski {

namespace {

constexpr int TN = 512;        // threads of a tournament workgroup
constexpr int TC = 512;        // candidate columns per workgroup (two per lane pair)
constexpr int YH = PIV_YL / 2; // sketch rows per lane
constexpr int NBP = 64;

// Omega (yl x m, row-major) of random signs: entry (i, j) is bit j % 64 of the first word
// of Philox4x64-10 at counter (i, j / 64, 0x52435051, 0) under the key (seed, ~seed)
__global__ __launch_bounds__(256) void k_omega(double* __restrict__ Om, int yl, int64_t m,
                                               uint64_t seed) {
    const int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (o >= (int64_t)yl * m) return;
    const int64_t i = o / m, j = o - i * m;
    const P4 w = philox4x64_10((uint64_t)i, (uint64_t)(j >> 6), 0x52435051ull, 0ull, seed, ~seed);
    Om[o] = ((w.x[0] >> (j & 63)) & 1ull) ? -1.0 : 1.0;
}

__global__ __launch_bounds__(256) void k_iota(int32_t* __restrict__ p, int64_t n) {
    const int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (o < n) p[o] = (int32_t)o;
}

// the better of (key, idx) and its value in the lane that the DPP control selects: larger
// key, then lower index (lanes without a source keep their own value)
template <int CTRL>
__device__ __forceinline__ void dpp_best(double& key, int& idx) {
    const int lo = __double2loint(key), hi = __double2hiint(key);
    const int olo = __builtin_amdgcn_update_dpp(lo, lo, CTRL, 0xf, 0xf, false);
    const int ohi = __builtin_amdgcn_update_dpp(hi, hi, CTRL, 0xf, 0xf, false);
    const int oi = __builtin_amdgcn_update_dpp(idx, idx, CTRL, 0xf, 0xf, false);
    const double ok = __hiloint2double(ohi, olo);
    if (ok > key || (ok == key && oi < idx)) {
        key = ok;
        idx = oi;
    }
}
// argmax over the wave with the lane moves of wave_sum; lane 63 ends with the best, which
// is broadcast
__device__ __forceinline__ void wave_best(double& key, int& idx) {
    dpp_best<0xb1>(key, idx);   // quad_perm [1,0,3,2]
    dpp_best<0x4e>(key, idx);   // quad_perm [2,3,0,1]
    dpp_best<0x124>(key, idx);  // row_ror 4
    dpp_best<0x128>(key, idx);  // row_ror 8
    dpp_best<0x142>(key, idx);  // row_bcast 15
    dpp_best<0x143>(key, idx);  // row_bcast 31
    key = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(key), 63),
                           __builtin_amdgcn_readlane(__double2loint(key), 63));
    idx = __builtin_amdgcn_readlane(idx, 63);
}

// One round of the tournament.  Group g owns up to TC candidate slots: on the first round
// the positions first + g*TC + c (c < TC, within the nrem trailing columns); later, slot
// c = 64 q' + i holds the i-th winner of input group q = 8 g + q' (i < nin[q]).  The group
// picks min(nsel, #candidates) of them by greedy pivoting on their sketch columns and
// writes the chosen positions in order to cout[g*64 ..], their number to nout[g], and,
// when nu is given, the remaining sketch norm at each choice to nu.
//
// Layout: 8 waves; wave w holds rows 36 h .. 36 h + 35 (h = w / 4) of the two columns
// 128 (w % 4) + lane and 128 (w % 4) + 64 + lane in registers.  Every lane of a wave needs
// the same 36 entries of the chosen column: one LDS read per lane, then scalar registers.
// The two halves of a column exchange partial sums through LDS (two buffers, alternating
// by step); every sum has four accumulators added in a fixed order.  The squared norms are
// recomputed after every projection (no downdating: the norms of a 72-row sketch collapse
// by design as the selection proceeds).  The choices stay in LDS until the end (a global
// store inside the loop would make every later barrier wait for it).
__global__ __launch_bounds__(TN) void k_tourney(const double* __restrict__ Yt, int64_t first,
                                                int64_t nrem, const int32_t* __restrict__ cin,
                                                const int32_t* __restrict__ nin, int nin_groups,
                                                int nsel, int32_t* __restrict__ cout,
                                                int32_t* __restrict__ nout,
                                                double* __restrict__ nu) {
    constexpr int NW = TN / 64;
    constexpr int NWH = NW / 2;
    __shared__ double pn[2][2][TC];   // [parity][half][slot]
    __shared__ double skey[NWH];
    __shared__ int sidx[NWH];
    __shared__ __align__(16) double qv[PIV_YL];
    __shared__ int spos[TC];
    __shared__ int ssel[NBP];
    __shared__ double snu[NBP];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int h = wv / NWH;
    const int c0 = ((wv % NWH) << 7) | lane, c1 = c0 + 64;
    const int g = blockIdx.x;
    auto slot_pos = [&](int c) -> int {
        if (cin == nullptr) {
            const int64_t off = (int64_t)g * TC + c;
            return off < nrem ? (int)(first + off) : -1;
        }
        const int q = 8 * g + (c >> 6), i = c & 63;
        return (q < nin_groups && i < nin[q]) ? cin[q * 64 + i] : -1;
    };
    const int pos0 = slot_pos(c0), pos1 = slot_pos(c1);
    if (h == 0) {
        spos[c0] = pos0;
        spos[c1] = pos1;
    }
    double y0[YH], y1[YH];
    auto load = [&](int pos, double (&y)[YH]) {
        if (pos >= 0) {
            const double2* src =
                reinterpret_cast<const double2*>(Yt + (int64_t)pos * PIV_YL + h * YH);
#pragma unroll
            for (int r = 0; r < YH / 2; ++r) {
                const double2 v = src[r];
                y[2 * r] = v.x;
                y[2 * r + 1] = v.y;
            }
        } else {
#pragma unroll
            for (int r = 0; r < YH; ++r) y[r] = 0.0;
        }
    };
    load(pos0, y0);
    load(pos1, y1);
    bool taken0 = pos0 < 0, taken1 = pos1 < 0;
    // partial squared norms, four accumulators each, summed in a fixed order
    auto partial_norms = [&](int par) {
        double a[4] = {0, 0, 0, 0}, b[4] = {0, 0, 0, 0};
#pragma unroll
        for (int r = 0; r < YH; ++r) {
            a[r & 3] += y0[r] * y0[r];
            b[r & 3] += y1[r] * y1[r];
        }
        pn[par][h][c0] = (a[0] + a[1]) + (a[2] + a[3]);
        pn[par][h][c1] = (b[0] + b[1]) + (b[2] + b[3]);
    };
    const int ncand = __syncthreads_count(h == 0 && pos0 >= 0) +
                      __syncthreads_count(h == 0 && pos1 >= 0);
    const int steps = min(nsel, ncand);
    partial_norms(0);
    __syncthreads();
    for (int s = 0; s < steps; ++s) {
        const int par = s & 1;
        if (h == 0) {
            const double n20 = pn[par][0][c0] + pn[par][1][c0];
            const double n21 = pn[par][0][c1] + pn[par][1][c1];
            const double k0 = taken0 ? -1.0 : (n20 >= 0.0 && n20 <= 1.7e308 ? n20 : 0.0);
            const double k1 = taken1 ? -1.0 : (n21 >= 0.0 && n21 <= 1.7e308 ? n21 : 0.0);
            double key = k0;
            int idx = c0;
            if (k1 > k0) {
                key = k1;
                idx = c1;
            }
            wave_best(key, idx);
            if (lane == 0) {
                skey[wv] = key;
                sidx[wv] = idx;
            }
        }
        __syncthreads();
        double bkey = skey[0];
        int bidx = sidx[0];
#pragma unroll
        for (int w = 1; w < NWH; ++w) {
            const double k2 = skey[w];
            const int i2 = sidx[w];
            if (k2 > bkey || (k2 == bkey && i2 < bidx)) {
                bkey = k2;
                bidx = i2;
            }
        }
        if (c0 == bidx) {
            taken0 = true;
#pragma unroll
            for (int r = 0; r < YH; ++r) qv[h * YH + r] = y0[r];
        } else if (c1 == bidx) {
            taken1 = true;
#pragma unroll
            for (int r = 0; r < YH; ++r) qv[h * YH + r] = y1[r];
        }
        if (tid == 0) {
            ssel[s] = spos[bidx];
            snu[s] = sqrt(bkey);
        }
        __syncthreads();
        if (bkey > 0.0) {
            // this half's 36 entries of the chosen column: one LDS read per lane, then
            // broadcast into scalar registers
            const double qsrc = lane < YH ? qv[h * YH + lane] : 0.0;
            double q[YH];
#pragma unroll
            for (int r = 0; r < YH; ++r)
                q[r] = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(qsrc), r),
                                        __builtin_amdgcn_readlane(__double2loint(qsrc), r));
            double a[4] = {0, 0, 0, 0}, b[4] = {0, 0, 0, 0};
#pragma unroll
            for (int r = 0; r < YH; ++r) {
                a[r & 3] += q[r] * y0[r];
                b[r & 3] += q[r] * y1[r];
            }
            pn[par ^ 1][h][c0] = (a[0] + a[1]) + (a[2] + a[3]);
            pn[par ^ 1][h][c1] = (b[0] + b[1]) + (b[2] + b[3]);
            __syncthreads();
            const double inv = 1.0 / bkey;
            const double f0 = (pn[par ^ 1][0][c0] + pn[par ^ 1][1][c0]) * inv;
            const double f1 = (pn[par ^ 1][0][c1] + pn[par ^ 1][1][c1]) * inv;
            __syncthreads();
#pragma unroll
            for (int r = 0; r < YH; ++r) {
                y0[r] -= f0 * q[r];
                y1[r] -= f1 * q[r];
            }
            partial_norms(par ^ 1);
        } else {
            // nothing left to project: carry the norms to the next parity
            pn[par ^ 1][h][c0] = pn[par][h][c0];
            pn[par ^ 1][h][c1] = pn[par][h][c1];
        }
        __syncthreads();
    }
    __syncthreads();
    if (tid < steps) {
        cout[g * 64 + tid] = ssel[tid];
        if (nu) nu[tid] = snu[tid];
    }
    if (tid == 0) nout[g] = steps;
}

// The moves that bring the chosen positions sel[0..nb) (all >= j0) to j0 .. j0+nb-1:
// move k (k < nb) takes sel[k] to j0 + k; the columns displaced from j0 .. j0+nb-1 (those
// not chosen) go, in ascending order, to the vacated positions sel[k] >= j0 + nb in
// ascending order.  mv[0..2*NBP) = sources, mv[2*NBP..4*NBP) = destinations,
// mv[4*NBP] = number of moves.  One wave.
__global__ __launch_bounds__(64) void k_pivot_plan(const int32_t* __restrict__ sel, int64_t j0,
                                                   int nb, int32_t* __restrict__ mv) {
    __shared__ int inT[NBP];
    __shared__ int svac[NBP];
    __shared__ int dpos[NBP];
    const int k = threadIdx.x;
    inT[k] = 0;
    __syncthreads();
    const int s = k < nb ? sel[k] : -1;
    const int hi = (int)(j0 + nb);
    if (k < nb && s < hi) inT[s - (int)j0] = 1;
    svac[k] = (k < nb && s >= hi) ? s : -1;
    __syncthreads();
    if (k < nb) {
        mv[k] = s;
        mv[2 * NBP + k] = (int)j0 + k;
    }
    // rank of this lane's displaced target position and of its vacated position
    if (k < nb && inT[k] == 0) {
        int r = 0;
        for (int q = 0; q < k; ++q) r += (inT[q] == 0);
        dpos[r] = (int)j0 + k;
    }
    __syncthreads();
    int nvac = 0;
    for (int q = 0; q < nb; ++q) nvac += (svac[q] >= 0);
    if (svac[k] >= 0) {
        int r = 0;
        for (int q = 0; q < nb; ++q) r += (svac[q] >= 0 && svac[q] < svac[k]);
        mv[nb + r] = dpos[r];
        mv[2 * NBP + nb + r] = svac[k];
    }
    if (k == 0) mv[4 * NBP] = nb + nvac;
}

// gather (dir 0) the moved columns of Ac (all m rows), their sketch rows and permutation
// entries into the staging buffers, or scatter (dir 1) them to their destinations;
// grid (2*NBP, row chunks)
__global__ __launch_bounds__(256) void k_pivot_move(double* __restrict__ Ac, int64_t m,
                                                    double* __restrict__ Yt,
                                                    int32_t* __restrict__ perm,
                                                    const int32_t* __restrict__ mv,
                                                    double* __restrict__ tA,
                                                    double* __restrict__ tY,
                                                    int32_t* __restrict__ tP, int dir) {
    const int i = blockIdx.x;
    if (i >= mv[4 * NBP]) return;
    const int src = mv[i], dst = mv[2 * NBP + i];
    if (src == dst) return;
    const int col = dir == 0 ? src : dst;
    double* a = Ac + (int64_t)col * m;
    double* t = tA + (int64_t)i * m;
    const double* from = dir == 0 ? a : t;
    double* to = dir == 0 ? t : a;
    // four rows per thread per step, their loads issued together (clamped into the column;
    // only rows < m are stored)
    const int64_t stride = (int64_t)gridDim.y * 256;
    for (int64_t r0 = (int64_t)blockIdx.y * 256 + threadIdx.x; r0 < m; r0 += 4 * stride) {
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = from[std::min(r0 + u * stride, m - 1)];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (r0 + u * stride < m) to[r0 + u * stride] = v[u];
    }
    if (blockIdx.y == 0) {
        double* yr = Yt + (int64_t)col * PIV_YL;
        for (int r = threadIdx.x; r < PIV_YL; r += 256) {
            if (dir == 0)
                tY[i * PIV_YL + r] = yr[r];
            else
                yr[r] = tY[i * PIV_YL + r];
        }
        if (threadIdx.x == 0) {
            if (dir == 0)
                tP[i] = perm[col];
            else
                perm[col] = tP[i];
        }
    }
}

// Bt = R_11^-T Y_1^T (nb x yl) for the sketch update, with the panel's R_11 (upper, rows and
// columns j0 .. j0+nb-1 of Ac).  A diagonal entry at or below 1e-13 of the panel's largest
// one leaves its direction in the sketch: its column of R_11 is replaced by the unit vector
// and its row of Y_1^T by zeros, which gives a zero row of Bt (what forward substitution
// that skips the entry gives).  R_11 is inverted in LDS (padded to 64 with the identity),
// then multiplied.
__global__ __launch_bounds__(256) void k_sketch_bt(const double* __restrict__ Ac, int64_t m,
                                                   int64_t j0, int nb,
                                                   const double* __restrict__ Yt,
                                                   double* __restrict__ Bt) {
    __shared__ double R[NBP][tile::PP];
    __shared__ double Ys[NBP][PIV_YL];
    __shared__ int skip[NBP];
    const int t = threadIdx.x;
    // every load is issued before the first one is used
    constexpr int NR = NBP * NBP / 256, NY = NBP * PIV_YL / 256;
    double ra[NR], ya[NY];
    // (addresses clamped into the panel and the unused values masked: a conditional load
    // becomes a branch that waits for its own load)
    auto keep = [](double x, bool k) {
        return __builtin_bit_cast(double, __builtin_bit_cast(uint64_t, x) & (k ? ~0ull : 0ull));
    };
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        const int o = t + 256 * q, i = o / NBP, k = o - i * NBP;  // column i, row k
        const int ic = i < nb ? i : nb - 1, kc = k < ic ? k : ic;
        ra[q] = Ac[(j0 + ic) * m + j0 + kc];
    }
#pragma unroll
    for (int q = 0; q < NY; ++q) {
        const int o = t + 256 * q, i = o / PIV_YL, u = o - i * PIV_YL;
        ya[q] = Yt[(j0 + (i < nb ? i : nb - 1)) * PIV_YL + u];
    }
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        const int o = t + 256 * q, i = o / NBP, k = o - i * NBP;
        const bool in = i < nb && k <= i;
        ra[q] = keep(ra[q], in) + (!in && k == i ? 1.0 : 0.0);
    }
#pragma unroll
    for (int q = 0; q < NY; ++q) {
        const int o = t + 256 * q, i = o / PIV_YL;
        ya[q] = keep(ya[q], i < nb);
    }
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        const int o = t + 256 * q;
        R[o % NBP][o / NBP] = ra[q];
    }
#pragma unroll
    for (int q = 0; q < NY; ++q) {
        const int o = t + 256 * q;
        Ys[o / PIV_YL][o % PIV_YL] = ya[q];
    }
    __syncthreads();
    if (t < NBP) {
        double dmax = 0.0;
        for (int i = 0; i < nb; ++i) dmax = fmax(dmax, fabs(R[i][i]));
        skip[t] = !(fabs(R[t][t]) > 1e-13 * dmax);
    }
    __syncthreads();
    for (int o = t; o < NBP * NBP; o += 256) {
        const int i = o / NBP, k = o - i * NBP;
        if (skip[i]) R[k][i] = k == i ? 1.0 : 0.0;
    }
    for (int o = t; o < NBP * PIV_YL; o += 256) {
        const int i = o / PIV_YL, u = o - i * PIV_YL;
        if (skip[i]) Ys[i][u] = 0.0;
    }
    __syncthreads();
    tile::tile_trinv(R, t, false);
    // Bt(i, u) = sum_{k <= i} R^-1(k, i) Y(k, u)
    for (int o = t; o < nb * PIV_YL; o += 256) {
        const int i = o / PIV_YL, u = o - i * PIV_YL;
        double a = 0.0;
        for (int k = 0; k <= i; ++k) a += R[k][i] * Ys[k][u];
        Bt[i * PIV_YL + u] = a;
    }
}

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace

int64_t piv_groups(int64_t d) { return std::max<int64_t>(1, ceil_div(d, TC)); }

size_t piv_ws_bytes(int64_t m, int64_t d) {
    const int64_t G = piv_groups(d);
    const size_t al = 256;
    auto r = [&](size_t b) { return ((b + al - 1) / al) * al; };
    return r((size_t)PIV_YL * m * 8) + r((size_t)d * PIV_YL * 8) + r((size_t)NBP * PIV_YL * 8) +
           2 * r((size_t)G * 64 * 4) + 2 * r((size_t)G * 4) + r(NBP * 4) + r(NBP * 8) +
           r((4 * NBP + 1) * 4) + r((size_t)2 * NBP * m * 8) + r((size_t)2 * NBP * PIV_YL * 8) +
           r(2 * NBP * 4) + r((size_t)d * 4);
}

void piv_ws_carve(void* base, int64_t m, int64_t d, PivWs& w) {
    const int64_t G = piv_groups(d);
    char* p = (char*)base;
    auto take = [&](size_t b) {
        void* q = p;
        p += ((b + 255) / 256) * 256;
        return q;
    };
    w.Om = (double*)take((size_t)PIV_YL * m * 8);
    w.Yt = (double*)take((size_t)d * PIV_YL * 8);
    w.Bt = (double*)take((size_t)NBP * PIV_YL * 8);
    w.cand[0] = (int32_t*)take((size_t)G * 64 * 4);
    w.cand[1] = (int32_t*)take((size_t)G * 64 * 4);
    w.cnt[0] = (int32_t*)take((size_t)G * 4);
    w.cnt[1] = (int32_t*)take((size_t)G * 4);
    w.sel = (int32_t*)take(NBP * 4);
    w.nu = (double*)take(NBP * 8);
    w.mv = (int32_t*)take((4 * NBP + 1) * 4);
    w.tA = (double*)take((size_t)2 * NBP * m * 8);
    w.tY = (double*)take((size_t)2 * NBP * PIV_YL * 8);
    w.tP = (int32_t*)take(2 * NBP * 4);
    w.perm = (int32_t*)take((size_t)d * 4);
}

hipError_t piv_init(double* Ac, int64_t m, int64_t d, uint64_t seed, PivWs& w, GemmWs& g,
                    hipStream_t st) {
    hipLaunchKernelGGL(k_omega, dim3((unsigned)ceil_div((int64_t)PIV_YL * m, 256)), dim3(256), 0,
                       st, w.Om, PIV_YL, m, seed);
    SKI_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_iota, dim3((unsigned)ceil_div(d, 256)), dim3(256), 0, st, w.perm, d);
    SKI_HIP(hipGetLastError());
    // Y^T (d x yl) = (S A)^T Omega^T; Ac is column-major, i.e. (S A)^T row-major with ld m
    return gemm_f64(false, true, d, PIV_YL, m, 1.0, Ac, m, w.Om, m, 0.0, w.Yt, PIV_YL, g, st);
}

hipError_t piv_select(int64_t j0, int64_t d, int nb, PivWs& w, hipStream_t st) {
    const int64_t nrem = d - j0;
    int ng = (int)piv_groups(nrem);
    int cur = 0;
    const bool last = ng == 1;
    hipLaunchKernelGGL(k_tourney, dim3((unsigned)ng), dim3(TN), 0, st, (const double*)w.Yt, j0,
                       nrem, (const int32_t*)nullptr, (const int32_t*)nullptr, 0, nb,
                       last ? w.sel : w.cand[cur], w.cnt[cur], last ? w.nu : (double*)nullptr);
    SKI_HIP(hipGetLastError());
    while (ng > 1) {
        const int ng2 = (int)ceil_div(ng, 8);
        const bool fin = ng2 == 1;
        hipLaunchKernelGGL(k_tourney, dim3((unsigned)ng2), dim3(TN), 0, st, (const double*)w.Yt,
                           j0, nrem, (const int32_t*)w.cand[cur], (const int32_t*)w.cnt[cur], ng,
                           nb, fin ? w.sel : w.cand[cur ^ 1], w.cnt[cur ^ 1],
                           fin ? w.nu : (double*)nullptr);
        SKI_HIP(hipGetLastError());
        cur ^= 1;
        ng = ng2;
    }
    return hipSuccess;
}

hipError_t piv_apply(double* Ac, int64_t m, int64_t j0, int nb, PivWs& w, hipStream_t st) {
    hipLaunchKernelGGL(k_pivot_plan, dim3(1), dim3(64), 0, st, (const int32_t*)w.sel, j0, nb,
                       w.mv);
    SKI_HIP(hipGetLastError());
    const unsigned ych = (unsigned)std::min<int64_t>(ceil_div(m, 1024), 16);
    for (int dir = 0; dir < 2; ++dir) {
        hipLaunchKernelGGL(k_pivot_move, dim3(2 * NBP, ych), dim3(256), 0, st, Ac, m, w.Yt, w.perm,
                           (const int32_t*)w.mv, w.tA, w.tY, w.tP, dir);
        SKI_HIP(hipGetLastError());
    }
    return hipSuccess;
}

hipError_t piv_update_sketch(const double* Ac, int64_t m, int64_t j0, int nb, int64_t d,
                             PivWs& w, GemmWs& g, hipStream_t st) {
    const int64_t n2 = d - j0 - nb;
    if (n2 <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sketch_bt, dim3(1), dim3(256), 0, st, Ac, m, j0, nb,
                       (const double*)w.Yt, w.Bt);
    SKI_HIP(hipGetLastError());
    // Y_2^T -= R_12^T Bt; R_12^T (n2 x nb) is row-major with ld m inside the column-major Ac
    return gemm_f64(false, false, n2, PIV_YL, nb, -1.0, Ac + (j0 + nb) * m + j0, m, w.Bt, PIV_YL,
                    1.0, w.Yt + (j0 + nb) * PIV_YL, PIV_YL, g, st);
}

}  // namespace ski
