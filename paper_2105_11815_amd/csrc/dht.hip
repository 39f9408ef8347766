// The randomised Hartley transform of the paper's dense software (Section 6, HR-DHT):
// S = S_h F D with F the discrete Hartley transform, F_kj = n'^-1/2 cas(2 pi k j / n'),
// applied to the zero-padded n' rows of [A b] (n' a power of two, at most 2^24).
//
// F is computed through the discrete Fourier transform: for real x, DHT(x)_k = Re X_k -
// Im X_k with X = DFT(x).  Two real columns a, b ride in one complex column z = a + i b;
// with Z = DFT(z), the Hartley values of both come from Z_k and Z_{n'-k}:
//   H_a[k] = ((P + P') - (Q - Q')) / 2,  H_b[k] = ((Q + Q') + (P - P')) / 2,
// where Z_k = P + iQ and Z_{n'-k} = P' + iQ'.
// The DFT of length N = N1 N2 (N1 = min(N, 256)) is taken in two passes over a slab of
// columns held in the last-level cache, as in Cooley and Tukey's four-step method:
//   pass A: for each j1 < N1, the N2-point DFT over j2 of z[j1 + N1 j2] (D applied on
//           load), times the twiddle e^{-2 pi i j1 k2 / N}, stored at slab row k2 N1 + j1;
//   pass B: for each k2 < N2, the N1-point DFT over j1 of those rows, in place: slab row
//           k2 N1 + k1 then holds Z_{k2 + N2 k1}.
// When N2 > 256 (n' > 65536), pass A is itself split the same way, N2 = Na Nb (Na = 256),
// with j2 = ja + Na jb and k2 = kb + Nb ka:
//   pass A1: for each (j1, ja), the Nb-point DFT over jb of z[j1 + N1 (ja + Na jb)] (D on
//            load), times e^{-2 pi i ja kb / N2}, stored at slab row (kb + Nb ja) N1 + j1;
//   pass A2: for each (j1, kb), the Na-point DFT over ja of those rows, times the twiddle
//            e^{-2 pi i j1 k2 / N}, written back in place at row (kb + Nb ka) N1 + j1 =
//            k2 N1 + j1, the layout pass A leaves; pass B and the gather are unchanged.
// Each short DFT is radix-2 decimation in time in LDS, with its input in bit-reversed
// order and twiddles from sincospi.  The hashing gather then forms H from the two rows
// k and n' - k of every bucket entry and sums the bucket's entries in the same fixed
// order as the Walsh-Hadamard gather.  The rounding differs from any other FFT, so this
// sketch matches a reference DHT to rounding, not to the bit.
#include "ski_internal.h"

namespace ski {

namespace {

constexpr int FT = 256;   // threads of the transform and gather kernels
constexpr int QW = 8;     // complex columns (column pairs) per workgroup
constexpr int LMAX = 256; // longest short DFT
constexpr int GB = FT / QW;  // buckets per gather workgroup

__device__ __forceinline__ int bitrev(int v, int bits) {
    return (int)(__builtin_bitreverse32((uint32_t)v) >> (32 - bits));
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// W[t] = e^{-2 pi i t / L} for t < L/2
__device__ __forceinline__ void twiddles(double2* W, int L, int tid) {
    for (int t = tid; t < L / 2; t += FT) {
        double s, c;
        sincospi(-2.0 * (double)t / (double)L, &s, &c);
        W[t] = make_double2(c, s);
    }
}

// in-place radix-2 DFT of length L along the first index of X (input in bit-reversed
// order, output in natural order), for the QW columns; ends synchronised
__device__ __forceinline__ void dft_lds(double2 (*X)[QW], int L, const double2* W, int tid) {
    for (int h = 1; h < L; h <<= 1) {
        const int tstep = L / (2 * h);
        for (int o = tid; o < (L / 2) * QW; o += FT) {
            const int i = o / QW, q = o - i * QW;
            const int blk = i / h, off = i - blk * h;
            const int i0 = blk * 2 * h + off, i1 = i0 + h;
            const double2 w = W[off * tstep];
            const double2 a = X[i0][q];
            const double2 b = cmul(X[i1][q], w);
            X[i0][q] = make_double2(a.x + b.x, a.y + b.y);
            X[i1][q] = make_double2(a.x - b.x, a.y - b.y);
        }
        __syncthreads();
    }
}

// column c of [A b] at row j (zero past the n rows and past the d + k columns)
__device__ __forceinline__ double aug(const double* A, int64_t lda, const double* B, int64_t ldb,
                                      int64_t n, int64_t d, int64_t w, int64_t j, int64_t c) {
    if (j >= n || c >= w) return 0.0;
    return c < d ? A[j * lda + c] : B[j * ldb + (c - d)];
}

__global__ __launch_bounds__(FT) void k_dht_pass_a(const double* __restrict__ A, int64_t lda,
                                                   const double* __restrict__ B, int64_t ldb,
                                                   int64_t n, int64_t d, int64_t w, int64_t c0,
                                                   int64_t c1, const uint32_t* __restrict__ dbits,
                                                   int N1, int N2, int lg2, int64_t N,
                                                   double2* __restrict__ T, int64_t sq) {
    __shared__ double2 X[LMAX][QW];
    __shared__ double2 W[LMAX / 2];
    const int tid = threadIdx.x;
    const int j1 = blockIdx.x;
    const int64_t qb = (int64_t)blockIdx.y * QW;
    twiddles(W, N2, tid);
    for (int o = tid; o < N2 * QW; o += FT) {
        const int j2 = o / QW, q = o - j2 * QW;
        const int64_t j = j1 + (int64_t)N1 * j2;
        const int64_t ca = c0 + 2 * (qb + q), cb = ca + 1;
        const double sg = ((dbits[j >> 5] >> (j & 31)) & 1u) ? -1.0 : 1.0;
        const bool qok = qb + q < sq;
        const double va = (qok && ca < c1) ? aug(A, lda, B, ldb, n, d, w, j, ca) : 0.0;
        const double vb = (qok && cb < c1) ? aug(A, lda, B, ldb, n, d, w, j, cb) : 0.0;
        X[lg2 ? bitrev(j2, lg2) : 0][q] = make_double2(sg * va, sg * vb);
    }
    __syncthreads();
    dft_lds(X, N2, W, tid);
    for (int o = tid; o < N2 * QW; o += FT) {
        const int k2 = o / QW, q = o - k2 * QW;
        if (qb + q >= sq) continue;
        const int64_t t = ((int64_t)j1 * k2) % N;
        double s, c;
        sincospi(-2.0 * (double)t / (double)N, &s, &c);
        T[((int64_t)k2 * N1 + j1) * sq + qb + q] = cmul(X[k2][q], make_double2(c, s));
    }
}

// pass A1 (N2 = Na Nb > 256): block x = j1 + N1 ja
__global__ __launch_bounds__(FT) void k_dht_pass_a1(const double* __restrict__ A, int64_t lda,
                                                    const double* __restrict__ B, int64_t ldb,
                                                    int64_t n, int64_t d, int64_t w, int64_t c0,
                                                    int64_t c1, const uint32_t* __restrict__ dbits,
                                                    int N1, int Na, int Nb, int lgb, int64_t N2,
                                                    double2* __restrict__ T, int64_t sq) {
    __shared__ double2 X[LMAX][QW];
    __shared__ double2 W[LMAX / 2];
    const int tid = threadIdx.x;
    const int j1 = (int)(blockIdx.x % (unsigned)N1), ja = (int)(blockIdx.x / (unsigned)N1);
    const int64_t qb = (int64_t)blockIdx.y * QW;
    twiddles(W, Nb, tid);
    for (int o = tid; o < Nb * QW; o += FT) {
        const int jb = o / QW, q = o - jb * QW;
        const int64_t j = j1 + (int64_t)N1 * (ja + (int64_t)Na * jb);
        const int64_t ca = c0 + 2 * (qb + q), cb = ca + 1;
        const double sg = ((dbits[j >> 5] >> (j & 31)) & 1u) ? -1.0 : 1.0;
        const bool qok = qb + q < sq;
        const double va = (qok && ca < c1) ? aug(A, lda, B, ldb, n, d, w, j, ca) : 0.0;
        const double vb = (qok && cb < c1) ? aug(A, lda, B, ldb, n, d, w, j, cb) : 0.0;
        X[bitrev(jb, lgb)][q] = make_double2(sg * va, sg * vb);
    }
    __syncthreads();
    dft_lds(X, Nb, W, tid);
    for (int o = tid; o < Nb * QW; o += FT) {
        const int kb = o / QW, q = o - kb * QW;
        if (qb + q >= sq) continue;
        const int64_t t = ((int64_t)ja * kb) % N2;
        double s, c;
        sincospi(-2.0 * (double)t / (double)N2, &s, &c);
        T[((int64_t)(kb + (int64_t)Nb * ja) * N1 + j1) * sq + qb + q] =
            cmul(X[kb][q], make_double2(c, s));
    }
}

// pass A2 (N2 = Na Nb > 256), in place: block x = j1 + N1 kb
__global__ __launch_bounds__(FT) void k_dht_pass_a2(double2* __restrict__ T, int64_t sq, int N1,
                                                    int Na, int Nb, int lga, int64_t N) {
    __shared__ double2 X[LMAX][QW];
    __shared__ double2 W[LMAX / 2];
    const int tid = threadIdx.x;
    const int j1 = (int)(blockIdx.x % (unsigned)N1), kb = (int)(blockIdx.x / (unsigned)N1);
    const int64_t qb = (int64_t)blockIdx.y * QW;
    twiddles(W, Na, tid);
    for (int o = tid; o < Na * QW; o += FT) {
        const int ja = o / QW, q = o - ja * QW;
        const int64_t row = (kb + (int64_t)Nb * ja) * N1 + j1;
        X[bitrev(ja, lga)][q] = qb + q < sq ? T[row * sq + qb + q] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    dft_lds(X, Na, W, tid);
    for (int o = tid; o < Na * QW; o += FT) {
        const int ka = o / QW, q = o - ka * QW;
        if (qb + q >= sq) continue;
        const int64_t k2 = kb + (int64_t)Nb * ka;
        const int64_t t = ((int64_t)j1 * k2) % N;
        double s, c;
        sincospi(-2.0 * (double)t / (double)N, &s, &c);
        T[(k2 * N1 + j1) * sq + qb + q] = cmul(X[ka][q], make_double2(c, s));
    }
}

__global__ __launch_bounds__(FT) void k_dht_pass_b(double2* __restrict__ T, int64_t sq, int N1,
                                                   int lg1) {
    __shared__ double2 X[LMAX][QW];
    __shared__ double2 W[LMAX / 2];
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * N1;
    const int64_t qb = (int64_t)blockIdx.y * QW;
    twiddles(W, N1, tid);
    for (int o = tid; o < N1 * QW; o += FT) {
        const int j1 = o / QW, q = o - j1 * QW;
        X[lg1 ? bitrev(j1, lg1) : 0][q] =
            qb + q < sq ? T[(base + j1) * sq + qb + q] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    dft_lds(X, N1, W, tid);
    for (int o = tid; o < N1 * QW; o += FT) {
        const int k1 = o / QW, q = o - k1 * QW;
        if (qb + q < sq) T[(base + k1) * sq + qb + q] = X[k1][q];
    }
}

// SA[b][c0 + 2 qq + {0,1}] = scale/2 * sum over the bucket's entries (row r, sign) of
// +-H[r], H from the slab rows of Z_r and Z_{N-r}
__global__ __launch_bounds__(FT) void k_dht_gather(const double2* __restrict__ T, int64_t sq,
                                                   int64_t cw, const int32_t* __restrict__ bptr,
                                                   const int32_t* __restrict__ src, int64_t m,
                                                   int N1, int N2, int64_t N, double scale,
                                                   double* __restrict__ SA, int64_t ldsa,
                                                   int64_t c0) {
    const int tid = threadIdx.x;
    const int q = tid % QW;
    const int64_t b = (int64_t)blockIdx.x * GB + tid / QW;
    const int64_t qq = (int64_t)blockIdx.y * QW + q;
    if (b >= m || 2 * qq >= cw) return;
    double acc_a = 0.0, acc_b = 0.0;
    const int e1 = bptr[b + 1];
    for (int e = bptr[b]; e < e1; ++e) {
        const uint32_t v = (uint32_t)src[e];
        const int64_t r = v >> 1;
        const int64_t rr = (N - r) & (N - 1);
        const int64_t pr = (r % N2) * N1 + r / N2;
        const int64_t prr = (rr % N2) * N1 + rr / N2;
        const double2 z = T[pr * sq + qq];
        const double2 zp = T[prr * sq + qq];
        const double ha = (z.x + zp.x) - (z.y - zp.y);
        const double hb = (z.y + zp.y) + (z.x - zp.x);
        if (v & 1u) {
            acc_a -= ha;
            acc_b -= hb;
        } else {
            acc_a += ha;
            acc_b += hb;
        }
    }
    const double f = 0.5 * scale;
    SA[b * ldsa + c0 + 2 * qq] = acc_a * f;
    if (2 * qq + 1 < cw) SA[b * ldsa + c0 + 2 * qq + 1] = acc_b * f;
}

}  // namespace

bool dht_supported(int64_t npad) { return npad >= 1 && npad <= (int64_t)LMAX * LMAX * LMAX; }

hipError_t launch_sketch_dht(const double* A, int64_t lda, const double* B, int64_t ldb,
                             int64_t n, int64_t d, int64_t k, int64_t npad,
                             const uint32_t* dbits, double* T, int64_t sc,
                             const int32_t* bucket_ptr, const int32_t* src, int64_t m,
                             double scale, double* SA, hipStream_t st) {
    // complex slab columns: sq pairs of real columns per slab (the buffer holds npad x sc)
    const int64_t sq = sc / 2;
    if (!dht_supported(npad) || sq < 1) return hipErrorInvalidValue;
    int lg = 0;
    while (((int64_t)1 << lg) < npad) ++lg;
    const int lg1 = std::min(lg, 8), lg2 = lg - lg1;
    const int N1 = 1 << lg1, N2 = 1 << lg2;
    const int64_t w = d + k;
    double2* Tc = reinterpret_cast<double2*>(T);
    for (int64_t c0 = 0; c0 < w; c0 += 2 * sq) {
        const int64_t c1 = std::min(w, c0 + 2 * sq), cw = c1 - c0;
        const unsigned gq = (unsigned)(((cw + 1) / 2 + QW - 1) / QW);
        if (lg2 <= 8) {
            hipLaunchKernelGGL(k_dht_pass_a, dim3((unsigned)N1, gq), dim3(FT), 0, st, A, lda, B,
                               ldb, n, d, w, c0, c1, dbits, N1, N2, lg2, npad, Tc, sq);
        } else {
            // N2 = Na Nb with Na = 256 and Nb = N2 / 256 <= 256
            const int lga = 8, lgb = lg2 - 8, Na = 1 << lga, Nb = 1 << lgb;
            hipLaunchKernelGGL(k_dht_pass_a1, dim3((unsigned)(N1 * Na), gq), dim3(FT), 0, st, A,
                               lda, B, ldb, n, d, w, c0, c1, dbits, N1, Na, Nb, lgb, (int64_t)N2,
                               Tc, sq);
            SKI_HIP(hipGetLastError());
            hipLaunchKernelGGL(k_dht_pass_a2, dim3((unsigned)(N1 * Nb), gq), dim3(FT), 0, st, Tc,
                               sq, N1, Na, Nb, lga, npad);
        }
        SKI_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_dht_pass_b, dim3((unsigned)N2, gq), dim3(FT), 0, st, Tc, sq, N1, lg1);
        SKI_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_dht_gather, dim3((unsigned)((m + GB - 1) / GB), gq), dim3(FT), 0, st,
                           (const double2*)Tc, sq, cw, bucket_ptr, src, m, N1, N2, npad, scale, SA,
                           w, c0);
        SKI_HIP(hipGetLastError());
    }
    return hipSuccess;
}

}  // namespace ski
