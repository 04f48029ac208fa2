// Device helpers shared by the forward (approx.hip) and adjoint (grad.hip)
// kernels of the order-j estimate: block reductions, the principal complex
// inverse square root, the LDS layout of M(w) per contour point, the radix-2
// FFT and the per-sector max-entropy fit.
#pragma once
#include "cplx.h"
#include "internal.h"

#define CONT_THREADS 512
#define FIT_THREADS 256
// Rounding of a contour value relative to the largest value of its transform:
// fp64 throughout (a few units of 2^-53), and the cluster sums of the mixed
// precision tier, whose eliminations run in fp32 (a few units of 2^-24).
#define ROUND_FP64 2e-16
#define ROUND_FP32 2e-7
// Mixed precision: a row whose estimated error exceeds the tier's target is
// run again in fp64 (GBS_PS_ESCALATED).
#ifndef MIXED_BOUND
#define MIXED_BOUND 1e-5
#endif
#define FIT_MAXIT 100
// largest odd factor of a contour size (K = r 2^a, r odd <= DFT_RMAX)
#ifndef DFT_RMAX
#define DFT_RMAX 15
#endif
#define FIT_KPT (GBS_KMAX / FIT_THREADS)

namespace {

__device__ double block_sum(double v, double *red)
{
    const int tid = threadIdx.x;
    red[tid] = v;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
    }
    double r = red[0];
    __syncthreads();
    return r;
}

__device__ double block_max(double v, double *red)
{
    const int tid = threadIdx.x;
    red[tid] = v;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (tid < s) red[tid] = fmax(red[tid], red[tid + s]);
        __syncthreads();
    }
    double r = red[0];
    __syncthreads();
    return r;
}

__device__ __forceinline__ cplx warp_csum(cplx v)
{
    for (int m = 32; m > 0; m >>= 1) {
        v.re += __shfl_xor(v.re, m);
        v.im += __shfl_xor(v.im, m);
    }
    return v;
}

// product over the 64 lanes of a wavefront (butterfly; every lane gets it)
__device__ __forceinline__ cplx warp_cprod(cplx v)
{
    for (int m = 32; m > 0; m >>= 1) {
        const cplx o = cplx{__shfl_xor(v.re, m), __shfl_xor(v.im, m)};
        v = cplx{fma(v.re, o.re, -v.im * o.im), fma(v.re, o.im, v.im * o.re)};
    }
    return v;
}

// z^{-1/2} on the principal branch, from |z| and the half-angle: with
// r = |z|, A = (|Re z| + r)/2, sqrt(z) = (sqrt A, Im z/(2 sqrt A)) for Re z >= 0
// and (|Im z|/(2 sqrt A), sign(Im z) sqrt A) otherwise; 1/sqrt(z) = conj(sqrt z)/r.
__device__ __forceinline__ cplx crsqrt_p(cplx z)
{
    const double s2 = fma(z.re, z.re, z.im * z.im);
    const double q = rsqrt(s2);          // 1/r
    const double r = s2 * q;
    const double A = 0.5 * (fabs(z.re) + r);
    const double w = rsqrt(A);
    const double big = A * w, small = 0.5 * fabs(z.im) * w;
    double sr, si;
    if (z.re >= 0.0) { sr = big; si = copysign(small, z.im); }
    else { sr = small; si = copysign(big, z.im); }
    return cmk(sr * q, -si * q);
}

// the same in fp32
__device__ __forceinline__ cplxf crsqrt_p(cplxf z)
{
    const float s2 = fmaf(z.re, z.re, z.im * z.im);
    const float q = rsqrtf(s2);
    const float r = s2 * q;
    const float A = 0.5f * (fabsf(z.re) + r);
    const float w = rsqrtf(A);
    const float big = A * w, small = 0.5f * fabsf(z.im) * w;
    float sr, si;
    if (z.re >= 0.0f) { sr = big; si = copysignf(small, z.im); }
    else { sr = small; si = copysignf(big, z.im); }
    return cmkf(sr * q, -si * q);
}

constexpr int CONT_MAXG = 8;
static_assert(CONT_MAXG <= CONT_THREADS / 64, "one wavefront per contour point of a pass");

// 2n rounded up to whole 16-wide tiles: rows kept in LDS hold V zero-padded to
// cont_tp x cont_tp (row stride cont_tp + 1) and d zero-padded to cont_tp
// entries, so that the M(w) tiles fetch their operands without masks
__host__ __device__ __forceinline__ int cont_tp(int n) { return 16 * ((2 * n + 15) / 16); }
// V (padded) and alpha (2n)
__host__ __device__ __forceinline__ int cont_vbytes(int n)
{
    return 8 * (cont_tp(n) * (cont_tp(n) + 1) + 2 * n);
}
// bytes of one slot: d (fp64 complex, cont_tp entries), z^{-1/2} (2n) and the
// 2x2 mode blocks of M(w) (3n + 4 n(n-1)/2 entries of the block type C),
// 16-byte aligned
template <class C = cplx>
__host__ __device__ __forceinline__ int cont_mbytes(int n)
{
    return 16 * (cont_tp(n) + 2 * n) + (((int)sizeof(C) * (2 * n * n + n) + 15) & ~15);
}
__host__ __device__ __forceinline__ int cont_fixed() { return 16 * (CONT_THREADS / 64) * 4 + 16 * CONT_MAXG; }

// Contour plan of one row from the spectrum alpha of A (entry i at
// alpha[i * astride]), run by one thread: log P_vac(Cbar), and unless the plan is
// frozen the radius rho (the saddle point of the photon-number generating
// function at n photons, capped at 0.98 of the convergence radius
// 1/max|alpha - 1|) and the size K (the smallest r 2^a, r odd <= DFT_RMAX,
// a >= 1, that is >= 2n + 32 and whose aliasing factor (rho/R_b)^K is below
// 1e-16, at most GBS_KMAX); then log G_0(rho).
// (The radius thus tilts towards max(n, untilted mean).)
// A frozen radius is kept only while it still lies inside the current
// convergence disc with an aliasing factor (rho max|alpha - 1|)^K <= 1e-14 (the
// rule above with a margin, so that small changes of the model keep the plan);
// otherwise the row is planned afresh and flagged GBS_PS_CONTOUR.
// With target > 0 the tilted mean is set to target instead (the re-tilt of a
// row whose estimate lies in sectors far from the first target); the target
// used is kept in kbar.
__device__ __forceinline__ void row_plan(RowPlan &rp, int n, const double *alpha, int astride,
                                         double logdetQ, double logdetA, double amin, double dev,
                                         bool nonpd, int frozen, bool whole = false, double target_in = 0.0)
{
    const int N = 2 * n;
    rp.status = 0;
    rp.flags = 0;
    rp.logdet_a = logdetA;
    rp.log_pvac = -0.5 * (logdetQ + logdetA);
    if (!(amin > 0.0) || nonpd) {
        rp.status = GBS_PS_PIVOT;
        return;
    }
    if (frozen) {
        const double x = rp.rho * dev;
        if (!(rp.K > 0 && rp.K <= GBS_KMAX) || !(x < 1.0) || (x > 0.0 && rp.K * log(x) > log(1e-14))) {
            frozen = 0;
            rp.flags = GBS_PS_CONTOUR;
        }
    }
    if (!frozen) {
        const double rb = dev > 1e-300 ? 1.0 / dev : 1e300;
        double hi = 0.98 * rb;
        auto mfun = [&](double rho) {
            double s = 0.0;
            for (int i = 0; i < N; ++i) {
                const double a = alpha[i * astride];
                s += 0.5 * rho * (1.0 - a) / (1.0 + rho * (a - 1.0));
            }
            return s;
        };
        // the tilted mean photon number is set to n (the sectors of a click
        // pattern of n detectors start at n), or to the untilted mean where that
        // is larger (then the sectors that carry the estimate lie at and above
        // the untilted mean, and a radius below 1 would push them under the
        // transform's rounding floor); for the whole distribution, to the
        // untilted mean: rho = 1, every sector at its own weight
        const double target = target_in > 0.0 ? target_in : whole ? mfun(1.0) : fmax((double)n, mfun(1.0));
        double rho;
        if (dev < 1e-300) rho = 1.0;
        else if (mfun(hi) <= target) rho = hi;
        else {
            // (bisection to the last few bits of rho; at most 200 halvings)
            double lo = 0.0;
            for (int it = 0; it < 200 && hi - lo > 4e-16 * hi; ++it) {
                const double mid = 0.5 * (lo + hi);
                if (mfun(mid) < target) lo = mid;
                else hi = mid;
            }
            rho = 0.5 * (lo + hi);
        }
        double kneed = 2.0 * n + 32.0;
        if (dev >= 1e-300) kneed = fmax(kneed, log(1e-16) / log(rho / rb));
        // the smallest r 2^a (r odd <= DFT_RMAX, a >= 1; the sizes dft_lds
        // takes) >= kneed
        int K = GBS_KMAX;
        for (int r = 1; r <= DFT_RMAX; r += 2) {
            int k = 2 * r;
            while (k < kneed && k < GBS_KMAX) k *= 2;
            if (k >= kneed && k < K) K = k;
        }
        rp.rho = rho;
        rp.kbar = target;
        rp.rconv = rb;
        rp.K = K;
        rp.log_rho = log(rho);
    }
    double s = 0.0;
    for (int i = 0; i < N; ++i) s += log1p(rp.rho * (alpha[i * astride] - 1.0));
    rp.log_g_rho = 0.5 * logdetA - 0.5 * s;
}

typedef double dbl4 __attribute__((ext_vector_type(4)));
// One 16x16x4 fp64 MFMA step, D += A B.  Lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; element e of D sits at row 4e + l/16, column l%16.
__device__ __forceinline__ dbl4 mfma4(double a, double b, dbl4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Position of the pair (a, b), a < b, inside one plane of pair blocks.  Column
// layout (DIAG false): b(b-1)/2 + a, so that pairs sharing b are adjacent.
// Diagonal layout (DIAG true): the pairs of each distance b - a in turn, so
// that (a, b), (a+1, b+1), ... are adjacent.
template <bool DIAG>
__device__ __forceinline__ int pair_pos(int n, int a, int b)
{
    if (!DIAG) return b * (b - 1) / 2 + a;
    const int d = b - a;
    return (d - 1) * n - (((d - 1) * d) >> 1) + a;
}

// Store one 16x16 tile (it <= jt) of M(w) (2n x 2n, quadrature-major rows
// x_0..x_{n-1}, p_0..p_{n-1}) from the MFMA layout into the 2x2 mode-block
// layout at blk: every entry i <= j of the upper triangle is one block entry,
// diagonal blocks (x_a x_a, x_a p_a, p_a p_a) at a, n + a, 2n + a, pair blocks
// a < b (x_a x_b, x_a p_b, p_a x_b, p_a p_b) at 3n + t np + pair_pos(a, b).
// With FIX the arrays sit at the strides of a GBS_NSMALL-click row instead
// (GBS_NSMALL for the diagonal-block arrays, its pair count for the others).
template <class C, bool DIAG = false, bool FIX = false>
__device__ __forceinline__ void m_store(int n, int it, int jt, const dbl4 &mre, const dbl4 &mim,
                                        C *blk, int lane)
{
    const int N = 2 * n;
    const int ds = FIX ? GBS_NSMALL : n, np = FIX ? GBS_NSMALL * (GBS_NSMALL - 1) / 2 : n * (n - 1) / 2;
    const int l16 = lane & 15, lq = lane >> 4;
    const int j = jt * 16 + l16;
    if (j >= N) return;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int ii = it * 16 + 4 * e + lq;
        if (ii > j) continue;
        int off;
        if (j < n) {
            off = ii == j ? ii : 3 * ds + pair_pos<DIAG>(n, ii, j);
        } else if (ii < n) {
            const int a = ii, b = j - n;
            off = a == b ? ds + a : (a < b ? 3 * ds + np + pair_pos<DIAG>(n, a, b)
                                           : 3 * ds + 2 * np + pair_pos<DIAG>(n, b, a));
        } else {
            const int a = ii - n, b = j - n;
            off = a == b ? 2 * ds + a : 3 * ds + 3 * np + pair_pos<DIAG>(n, a, b);
        }
        blk[off] = from_d<C>(cmk(mre[e], mim[e]));
    }
}

// A BS x BS block of 16x16 tiles of M(w) = V diag(d) V^T on the matrix cores, by
// one wavefront: tiles (BS ib + s, BS jb + t), those with it <= jt stored.  Vt
// holds the eigenvectors as rows (entry i of eigenvector k at k*vs + i).  Each
// operand fetched per k-step serves BS tiles (BS = 2 halves the loads per MFMA
// where V is read from L2).
// With PAD, Vt and d are zero beyond 2n up to the tile edge, and no fetch is
// masked; FIX selects the fixed-stride block layout of m_store.
template <int BS, class C = cplx, bool DIAG = false, bool PAD = false, bool FIX = false>
__device__ __forceinline__ void m_block_mfma(int n, int ib, int jb, const double *Vt, int vs,
                                             const cplx *d, C *blk, int lane)
{
    const int N = 2 * n, KS = (N + 3) >> 2;
    const int l16 = lane & 15, lq = lane >> 4;
    int iv[BS], jv[BS];
#pragma unroll
    for (int s = 0; s < BS; ++s) {
        iv[s] = (BS * ib + s) * 16 + l16;
        jv[s] = (BS * jb + s) * 16 + l16;
    }
    dbl4 mre[BS][BS], mim[BS][BS];
#pragma unroll
    for (int s = 0; s < BS; ++s)
#pragma unroll
        for (int t = 0; t < BS; ++t) mre[s][t] = mim[s][t] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 2
    for (int ks = 0; ks < KS; ++ks) {
        const int k = ks * 4 + lq;
        const bool kok = PAD || k < N;
        const cplx dl = d[kok ? k : 0];
        double ar[BS], ai[BS], bv[BS];
#pragma unroll
        for (int s = 0; s < BS; ++s) {
            const bool aok = PAD || (kok && iv[s] < N), bok = PAD || (kok && jv[s] < N);
            const double va = Vt[aok ? k * vs + iv[s] : 0], vb = Vt[bok ? k * vs + jv[s] : 0];
            ar[s] = aok ? va * dl.re : 0.0;
            ai[s] = aok ? va * dl.im : 0.0;
            bv[s] = bok ? vb : 0.0;
        }
#pragma unroll
        for (int s = 0; s < BS; ++s)
#pragma unroll
            for (int t = 0; t < BS; ++t) {
                mre[s][t] = mfma4(ar[s], bv[t], mre[s][t]);
                mim[s][t] = mfma4(ai[s], bv[t], mim[s][t]);
            }
    }
#pragma unroll
    for (int s = 0; s < BS; ++s)
#pragma unroll
        for (int t = 0; t < BS; ++t)
            if (BS * ib + s <= BS * jb + t)
                m_store<C, DIAG, FIX>(n, BS * ib + s, BS * jb + t, mre[s][t], mim[s][t], blk, lane);
}

template <class C = cplx>
__device__ __forceinline__ void m_tile_mfma(int n, int it, int jt, const double *Vt, int vs,
                                            const cplx *d, C *blk, int lane)
{
    m_block_mfma<1, C>(n, it, jt, Vt, vs, d, blk, lane);
}

// tile u of the column-major list of upper tiles (it <= jt)
__device__ __forceinline__ void upper_tile(int u, int &it, int &jt)
{
    jt = 0;
    while ((jt + 1) * (jt + 2) / 2 <= u) ++jt;
    it = u - jt * (jt + 1) / 2;
}

template <class C>
struct SlotMT {
    cplx *d, *rz;
    C *d0, *d1, *d2, *o0, *o1, *o2, *o3;
};
using SlotM = SlotMT<cplx>;

template <class C = cplx>
__device__ __forceinline__ SlotMT<C> slot_view(cplx *base, int n)
{
    const int N = 2 * n, np = n * (n - 1) / 2;
    SlotMT<C> m;
    m.d = base;
    m.rz = base + cont_tp(n);
    m.d0 = (C *)(m.rz + N);
    m.d1 = m.d0 + n;
    m.d2 = m.d1 + n;
    m.o0 = m.d2 + n;
    m.o1 = m.o0 + np;
    m.o2 = m.o1 + np;
    m.o3 = m.o2 + np;
    return m;
}

// Log-partition sum of the exp-polynomial on n' = 1..n - v0 (v = n - n' empty modes,
// basis phi_t = C(v, t) ib[t]) and, with WANT_E, the mean E[phi] and the
// second moments E2 (upper triangle, row-major) of its JP features.  JP is a
// template argument so that every array index is static (kept in registers).
template <int JP, bool WANT_E>
__device__ __forceinline__ void fit_eval(int n, int v0, const double *ib, const double *c, double *lse,
                                         double *E, double *E2)
{
    double zmax = -1e300;
    for (int v = v0; v < n; ++v) {
        const double f[4] = {v * ib[0], 0.5 * v * (v - 1) * ib[1], v * (v - 1.0) * (v - 2.0) / 6.0 * ib[2],
                             v * (v - 1.0) * (v - 2.0) * (v - 3.0) / 24.0 * ib[3]};
        double z = 0.0;
#pragma unroll
        for (int t = 0; t < JP; ++t) z -= c[t] * f[t];
        zmax = fmax(zmax, z);
    }
    double s = 0.0, e[4] = {0, 0, 0, 0}, e2[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int v = v0; v < n; ++v) {
        const double f[4] = {v * ib[0], 0.5 * v * (v - 1) * ib[1], v * (v - 1.0) * (v - 2.0) / 6.0 * ib[2],
                             v * (v - 1.0) * (v - 2.0) * (v - 3.0) / 24.0 * ib[3]};
        double z = 0.0;
#pragma unroll
        for (int t = 0; t < JP; ++t) z -= c[t] * f[t];
        const double wgt = exp(z - zmax);
        s += wgt;
        if (WANT_E) {
#pragma unroll
            for (int t = 0; t < JP; ++t) e[t] += wgt * f[t];
            int k = 0;
#pragma unroll
            for (int t = 0; t < JP; ++t)
#pragma unroll
                for (int u = t; u < JP; ++u) e2[k++] += wgt * f[t] * f[u];
        }
    }
    *lse = zmax + log(s);
    if (WANT_E) {
#pragma unroll
        for (int t = 0; t < JP; ++t) E[t] = e[t] / s;
#pragma unroll
        for (int k = 0; k < JP * (JP + 1) / 2; ++k) E2[k] = e2[k] / s;
    }
}

// Cholesky solve of the JP x JP system H x = r (H from E, E2 as the covariance
// of the features, damped by 1e-14 of its trace); false if H is not positive.
template <int JP>
__device__ __forceinline__ bool fit_solve(const double *E, const double *E2, const double *r, double *x)
{
    double Hm[4][4];
    int k = 0;
#pragma unroll
    for (int t = 0; t < JP; ++t)
#pragma unroll
        for (int u = t; u < JP; ++u) Hm[t][u] = Hm[u][t] = E2[k++] - E[t] * E[u];
    double tr = 0.0;
#pragma unroll
    for (int t = 0; t < JP; ++t) tr += Hm[t][t];
#pragma unroll
    for (int t = 0; t < JP; ++t) Hm[t][t] += 1e-14 * tr;
    if (!(tr > 0.0)) return false;
    double L[4][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
#pragma unroll
    for (int j = 0; j < JP; ++j) {
        double d = Hm[j][j];
#pragma unroll
        for (int l = 0; l < j; ++l) d -= L[j][l] * L[j][l];
        if (!(d > 0.0)) return false;
        L[j][j] = sqrt(d);
#pragma unroll
        for (int i = j + 1; i < JP; ++i) {
            double sv = Hm[i][j];
#pragma unroll
            for (int l = 0; l < j; ++l) sv -= L[i][l] * L[j][l];
            L[i][j] = sv / L[j][j];
        }
    }
    double y[4];
#pragma unroll
    for (int i = 0; i < JP; ++i) {
        double sv = r[i];
#pragma unroll
        for (int l = 0; l < i; ++l) sv -= L[i][l] * y[l];
        y[i] = sv / L[i][i];
    }
#pragma unroll
    for (int i = JP - 1; i >= 0; --i) {
        double sv = y[i];
#pragma unroll
        for (int l = i + 1; l < JP; ++l) sv -= L[l][i] * x[l];
        x[i] = sv / L[i][i];
    }
    return true;
}

// Max-entropy fit on n' = 1..n - v0 (v = n - n' empty modes, v >= v0) of the JP
// moments m[]; returns 0, minus the log-partition sum (log q(n) when v0 = 0)
// and the parameters in c_out on success.
template <int JP>
__device__ __forceinline__ int fit_last_point(int n, int v0, const double *m, double *logq, double *c_out)
{
    double ib[4] = {0, 0, 0, 0};
    ib[0] = 1.0 / (n - 1.0);
    if (JP > 1) ib[1] = 2.0 / ((n - 1.0) * (n - 2.0));
    if (JP > 2) ib[2] = 6.0 / ((n - 1.0) * (n - 2.0) * (n - 3.0));
    if (JP > 3) ib[3] = 24.0 / ((n - 1.0) * (n - 2.0) * (n - 3.0) * (n - 4.0));
    double c[4] = {0, 0, 0, 0};
    for (int it = 0; it <= FIT_MAXIT; ++it) {
        double lse, E[4], E2[10];
        fit_eval<JP, true>(n, v0, ib, c, &lse, E, E2);
        double g[4] = {0, 0, 0, 0}, mg[4] = {0, 0, 0, 0};
        bool conv = true;
#pragma unroll
        for (int t = 0; t < JP; ++t) {
            g[t] = m[t] - E[t];
            mg[t] = -g[t];
            if (!(fabs(g[t]) <= 1e-15 + 1e-12 * fabs(m[t]))) conv = false;
        }
        // Newton step H x = -g, H the covariance of the features
        double x[4] = {0, 0, 0, 0};
        if (!fit_solve<JP>(E, E2, mg, x)) return 1;
        if (conv) {
            double cn[4] = {0, 0, 0, 0};
#pragma unroll
            for (int t = 0; t < JP; ++t) cn[t] = c[t] + x[t];
            double l2;
            fit_eval<JP, false>(n, v0, ib, cn, &l2, nullptr, nullptr);
            *logq = -l2;
            if (c_out)
#pragma unroll
                for (int t = 0; t < JP; ++t) c_out[t] = cn[t];
            return 0;
        }
        double L0 = lse, slope = 0.0;
#pragma unroll
        for (int t = 0; t < JP; ++t) {
            L0 += c[t] * m[t];
            slope += g[t] * x[t];
        }
        double st = 1.0;
        if (-slope > 1e-13 * fmax(1.0, fabs(L0))) {
            while (st > 1e-12) {
                double cn[4] = {0, 0, 0, 0};
#pragma unroll
                for (int t = 0; t < JP; ++t) cn[t] = c[t] + st * x[t];
                double l2;
                fit_eval<JP, false>(n, v0, ib, cn, &l2, nullptr, nullptr);
#pragma unroll
                for (int t = 0; t < JP; ++t) l2 += cn[t] * m[t];
                if (l2 <= L0 + 1e-4 * st * slope) break;
                st *= 0.5;
            }
        }
#pragma unroll
        for (int t = 0; t < JP; ++t) c[t] += st * x[t];
    }
    return 1;
}

__device__ __forceinline__ void lse_add(double &mx, double &s, double v)
{
    if (v == -INFINITY) return;
    if (v > mx) {
        s = s * exp(mx - v) + 1.0;
        mx = v;
    } else {
        s += exp(v - mx);
    }
}

// exp(2 pi i q / K), q >= 0, with the angle reduced to the nearest quarter
// turn in integers first: 2q/K = k/2 + x, k = round(4q/K), x = (4q - kK)/(2K)
// in [-1/4, 1/4], so that the only rounding is that of x.  Points near -1 (on
// a contour, w = -rho, next to the generating function's singularity on the
// negative axis) and near +-1, +-i then carry phase errors of ~1e-17 rad for
// every K, where rounding 2q/K itself would cost ~3e-16 rad whenever K is not
// a power of two.
__device__ __forceinline__ cplx unit_root(long long q, int K)
{
    const long long k = (4 * q + K / 2) / K;
    const double x = (double)(4 * q - k * K) / (2.0 * (double)K);
    double s, c;
    sincospi(x, &s, &c);
    switch ((int)(k & 3)) {
    case 0: return cplx{c, s};
    case 1: return cplx{-s, c};
    case 2: return cplx{-c, -s};
    default: return cplx{s, -c};
    }
}

// Sector transforms.  A contour has K = r 2^a points, r odd and at most
// DFT_RMAX, a >= 1 (the smallest such K that meets the aliasing rule, so that
// fewer points are evaluated than with powers of two alone).  The forward DFT
// X[k] = sum_q x[q] W^{qk}, W = exp(-2 pi i / K), runs in LDS by decimation in
// time: the r interleaved subsequences x[j + r m] (j < r) are transformed by
// radix-2 stages, each in its own block of L = K / r entries, and combined by
// r-point DFTs: X[m + s L] = sum_j W^{j m} F_j[m] W^{j s L} (s < r).
struct DftShape {
    int K, r, L, lgL;
};
__device__ __forceinline__ DftShape dft_shape(int K)
{
    DftShape d;
    d.K = K;
    d.r = K >> __builtin_ctz((unsigned)K);  // the odd part
    d.L = K / d.r;
    d.lgL = 0;
    while ((1 << d.lgL) < d.L) ++d.lgL;
    return d;
}
// Where input sample q goes: block q mod r, bit-reversed position q div r.
__device__ __forceinline__ int dft_pos(const DftShape &d, int q)
{
    const int j = q % d.r, m = q / d.r;
    return j * d.L + (int)(__brev((unsigned)m) >> (32 - d.lgL));
}
// W^e for 0 <= e < K from the half table W[m] = exp(-2 pi i m / K), m < K/2.
__device__ __forceinline__ cplx dft_tw(const cplx *W, int K, int e)
{
    return e < K / 2 ? W[e] : cneg(W[e - K / 2]);
}
// In-place forward DFT of X[0..K) in LDS, input placed by dft_pos, output in
// natural order.  All threads of the block take part.
__device__ void dft_lds(cplx *X, const cplx *W, const DftShape &d)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    const int K = d.K, L = d.L, hl = L / 2;
    for (int half = 1; half < L; half <<= 1) {
        // W_L^{pos L / (2 half)} = W^{pos r L / (2 half)}
        const int tstep = d.r * (L / (2 * half));
        for (int b = tid; b < K / 2; b += nt) {
            const int blk = b / hl, bb = b - blk * hl;
            const int grp = bb / half, pos = bb - grp * half;
            const int i = blk * L + grp * 2 * half + pos, j = i + half;
            const cplx w = W[pos * tstep];
            const cplx u = X[i], v = cmul(w, X[j]);
            X[i] = cadd(u, v);
            X[j] = csub(u, v);
        }
        __syncthreads();
    }
    if (d.r > 1) {
        for (int m = tid; m < L; m += nt) {
            cplx f[DFT_RMAX];
#pragma unroll
            for (int j = 0; j < DFT_RMAX; ++j)
                if (j < d.r) f[j] = j == 0 ? X[m] : cmul(dft_tw(W, K, j * m), X[j * L + m]);
            for (int s2 = 0; s2 < d.r; ++s2) {
                cplx acc = f[0];
                int e = 0;  // (j s2 mod r) L, stepped by s2 L
#pragma unroll
                for (int j = 1; j < DFT_RMAX; ++j) {
                    if (j >= d.r) continue;
                    e += s2 * L;
                    if (e >= K) e -= K;
                    acc = cadd(acc, cmul(dft_tw(W, K, e), f[j]));
                }
                X[s2 * L + m] = acc;
            }
        }
        __syncthreads();
    }
}


// Result of one sector fit with at most JM moments: log q(n), the fitted
// parameters and the moments (zero past the ones used), how many moments were
// used, and bad != 0 if no fit succeeded.
template <int JM>
struct SectorFitT {
    double lq;
    double c[JM];
    double m[JM];
    int jr, bad;
};
using SectorFit = SectorFitT<3>;

// Fit one sector from its tilted moments t0..t4 (t0 > 0; moments past JM are
// ignored) on n' = 1..n - v0 (v0 > 0: a sector with fewer photons than
// modes): the moments m_t = tau_t / (tau_0 C(n-1,t)) are used up to the
// longest feasible prefix (0 < m_t < 1, decreasing in t, since
// 0 <= phi_{t+1} <= phi_t <= 1).  A moment whose true value lies below the
// transform's rounding floor can come out infeasible; it is then dropped, and
// so is the next one if the fit fails.  With m_1 <= 0 every clicked mode
// fires: q(n) = 1.  The moments arrive by value and the fit runs out of line,
// so that callers index nothing at run time.
template <int JM>
__device__ __noinline__ SectorFitT<JM> fit_sector(int n, int v0, int jp, double t0, double t1, double t2,
                                                  double t3, double t4)
{
    SectorFitT<JM> r;
    const double binv[4] = {1.0 / (n - 1.0), 2.0 / ((n - 1.0) * (n - 2.0)),
                            6.0 / ((n - 1.0) * (n - 2.0) * (n - 3.0)),
                            24.0 / ((n - 1.0) * (n - 2.0) * (n - 3.0) * (n - 4.0))};
    const double tau[4] = {t1, t2, t3, t4};
#pragma unroll
    for (int t = 0; t < JM; ++t) {
        r.m[t] = t < jp ? tau[t] / t0 * binv[t] : 0.0;
        r.c[t] = 0.0;
    }
    int jr = 0;
#pragma unroll
    for (int t = 1; t <= JM; ++t)
        if (jr == t - 1 && t <= jp && r.m[t - 1] > 0.0 && r.m[t - 1] < 1.0 &&
            (t == 1 || r.m[t - 1] < r.m[t - 2]))
            jr = t;
    r.lq = 0.0;
    if (jp == 0) {
        r.jr = 0;
        r.bad = 0;
        return r;
    }
    int bad = 1;
    while (jr >= 1 && bad) {
        switch (jr) {
        case 1: bad = fit_last_point<1>(n, v0, r.m, &r.lq, r.c); break;
        case 2: bad = fit_last_point<2>(n, v0, r.m, &r.lq, r.c); break;
        case 3: bad = fit_last_point<JM >= 3 ? 3 : 1>(n, v0, r.m, &r.lq, r.c); break;
        default: bad = fit_last_point<JM >= 4 ? 4 : 1>(n, v0, r.m, &r.lq, r.c); break;
        }
        if (bad) --jr;
    }
    if (jr == 0) {
        bad = r.m[0] <= 0.0 ? 0 : 1;
        r.lq = 0.0;
#pragma unroll
        for (int t = 0; t < JM; ++t) r.c[t] = 0.0;
    }
    r.jr = jr;
    r.bad = bad;
    return r;
}

// Sensitivity of a fitted sector's log q(n) to its moments: d log q / d m_t =
// -u_t with u = H^{-1} m, H the covariance of the basis under the fitted
// distribution (t < jr; zero for the moments the fit did not use).
template <int JM>
__device__ __noinline__ void fit_sensitivity(int n, const SectorFitT<JM> &f, double *u)
{
    const double binv[4] = {1.0 / (n - 1.0), 2.0 / ((n - 1.0) * (n - 2.0)),
                            6.0 / ((n - 1.0) * (n - 2.0) * (n - 3.0)),
                            24.0 / ((n - 1.0) * (n - 2.0) * (n - 3.0) * (n - 4.0))};
    double lse, E[4], E2[10];
    bool ok = true;
#pragma unroll
    for (int t = 0; t < 4; ++t) u[t] = 0.0;
    switch (f.jr) {
    case 0: return;
    case 1: fit_eval<1, true>(n, 0, binv, f.c, &lse, E, E2); ok = fit_solve<1>(E, E2, f.m, u); break;
    case 2: fit_eval<2, true>(n, 0, binv, f.c, &lse, E, E2); ok = fit_solve<2>(E, E2, f.m, u); break;
    case 3:
        fit_eval<JM >= 3 ? 3 : 1, true>(n, 0, binv, f.c, &lse, E, E2);
        ok = fit_solve<JM >= 3 ? 3 : 1>(E, E2, f.m, u);
        break;
    default:
        fit_eval<JM >= 4 ? 4 : 1, true>(n, 0, binv, f.c, &lse, E, E2);
        ok = fit_solve<JM >= 4 ? 4 : 1>(E, E2, f.m, u);
        break;
    }
    if (!ok)
#pragma unroll
        for (int t = 0; t < 4; ++t) u[t] = 1e300;
}

}  // namespace
