// Adjoint of the order-j estimate: gradient of L = sum_p w_p log p_hat_p with
// respect to the squeezing parameters r and the transmissions eta, with the
// contour radius rho, the contour size K, the sector set and the number of
// moments each sector fit uses held at their forward values.
//
// Every determinant enters through d log det X = tr(X^{-1} dX).  With
// N(w) = (1-w)I + wA, M(w) = N^{-1} and dM = -w M dA M, the forward quantities
//   S_t(w) = g(w) C_t(w),  g(w) = G_0(w)/G_0(rho),  C_t = sum_{|T|=t} det(M_TT)^{-1/2}
// give, for a cotangent alpha_t(w) (dL = Re sum alpha dS),
//   dL = Re[ (w/2) tr(M Z M dA) - (w/2) beta tr(M dA) + (rho/2) beta tr(M(rho) dA) ]
// with gamma_t = alpha_t g, Z = sum_T gamma_|T| det(M_TT)^{-1/2} E_T M_TT^{-1} E_T^T
// and beta = sum_t gamma_t C_t.  In A's eigenbasis (A = V diag(alpha) V^T,
// M = V diag(d) V^T) this is A_bar = V R V^T with
//   R += Re[(w/2) d_i d_j (V^T Z V)_ij] + delta_ij Re[beta (rho dr_i - w d_i)/2],
// dr_i = 1/(1 + rho(alpha_i - 1)).  Kernels:
//   k_adj_fit      per row: the sector transform and fits again; the log-sum and
//                  each fit differentiated (implicitly: d log q / dm = -H^{-1} m,
//                  H the covariance of the fitted basis); the sector cotangents
//                  pushed back through the FFT to alpha_t(w_q)
//   k_adj_contour  per (row, 64 contour points): M(w) and the clusters again
//                  (the same work units as the forward, in an order that spreads
//                  neighbouring lanes over different blocks of Z(w)),
//                  Z(w) by LDS atomics, V^T Z V on the matrix cores (rows up to
//                  40 clicks: column units, each wavefront's share of R in
//                  registers over the item; larger rows at orders 1, 3, 4:
//                  Y = Z V into an HBM panel, then X = V^T Y, R
//                  read-modified-written per point)
//   k_adj_pairs_big  larger rows at order 2: M(w) never stored, each pair's
//                  block of Z(w) written once, R's tiles formed from 16-row
//                  blocks of Z with Z V kept in the accumulators
//                  (k_v_transpose first lays out V's transposed copy)
//   k_adj_reduce   per row: sum of the items' R in a fixed order, the
//                  contour-independent terms, A_bar = V R V^T, added into the
//                  adjoint of Q^{-1} at the row's mode pairs (global atomics)
//   k_adj_model    Q_bar = -(sum w)/2 Q^{-1} - Q^{-1} Psi Q^{-1}, then sigma_bar,
//                  and the chain to r and eta through the model build
#include "contour_common.h"

#include <algorithm>
#include <cfloat>
#include <type_traits>

#define ADJ_QCHUNK GBS_ADJ_CHUNK
static_assert(GBS_ADJ_CHUNK_BIG <= ADJ_QCHUNK, "one pass of points per item fits s_wq");

namespace {

// ---------------------------------------------------------------------------
// k_adj_fit
// ---------------------------------------------------------------------------
template <int ORDER>
__global__ __launch_bounds__(FIT_THREADS) void k_adj_fit(const int *__restrict__ offsets,
                                                         const RowPlan *__restrict__ rows,
                                                         const cplx *__restrict__ sw,
                                                         const double *__restrict__ dl,
                                                         const int *__restrict__ status,
                                                         cplx *__restrict__ asw)
{
    extern __shared__ __attribute__((aligned(16))) double sh[];
    __shared__ double red[FIT_THREADS];
    const int p = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
    const int n = offsets[p + 1] - offsets[p];
    const RowPlan rp = rows[p];
    const double wp = dl[p];
    // (rows without a forward result take no part)
    if (n == 0 || rp.status != 0 || (status[p] & GBS_PS_FAILED) || wp == 0.0 || !isfinite(wp)) {
        for (int i = tid; i < (ORDER + 1) * GBS_QCAP; i += nt)
            asw[(long)p * (ORDER + 1) * GBS_QCAP + i] = cmk(0.0, 0.0);
        return;
    }
    const int K = rp.K, Q = K / 2 + 1, jp = min(ORDER, n - 1);
    const DftShape dsh = dft_shape(K);
    cplx *X = (cplx *)sh;
    cplx *W = X + K;
    for (int m = tid; m < K / 2; m += nt) {
        const cplx u = unit_root(m, K);
        W[m] = cmk(u.re, -u.im);
    }
    // (loops over t and j unrolled: every index into the per-thread arrays is static)
    constexpr int NT = ORDER >= 4 ? 5 : 4;  // moments held per sector
    constexpr int JM = ORDER >= 4 ? 4 : 3;  // most moments a fit uses
    double tau[FIT_KPT][NT];
    const double invK = 1.0 / K;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        if (t <= ORDER && t <= jp) {
            const cplx *src = sw + ((long)p * (ORDER + 1) + t) * GBS_QCAP;
            for (int q = tid; q < K; q += nt) {
                const cplx v = q < Q ? src[q] : cmk(src[K - q].re, -src[K - q].im);
                X[dft_pos(dsh, q)] = v;
            }
            __syncthreads();
            dft_lds(X, W, dsh);
#pragma unroll
            for (int j = 0; j < FIT_KPT; ++j) {
                const int kap = n + tid + nt * j;
                tau[j][t] = kap < K ? X[kap].re * invK : 0.0;
            }
            __syncthreads();
        } else {
#pragma unroll
            for (int j = 0; j < FIT_KPT; ++j) tau[j][t] = 0.0;
        }
    }
    double tmax = 0.0;
#pragma unroll
    for (int j = 0; j < FIT_KPT; ++j)
        if (n + tid + nt * j < K) tmax = fmax(tmax, tau[j][0]);
    tmax = block_max(tmax, red);
    const double thr = 1e-14 * tmax;
    // forward pass again: which sectors are fitted, their log p_hat and fits
    double ell[FIT_KPT];
    SectorFitT<JM> fits[FIT_KPT];
    double fm = -INFINITY, fs = 0.0, lower = -INFINITY;
#pragma unroll
    for (int j = 0; j < FIT_KPT; ++j) {
        if (j == 1) {
            double mx = block_max(fm, red);
            double sm = block_sum(fm == -INFINITY ? 0.0 : fs * exp(fm - mx), red);
            lower = sm > 0.0 ? mx + log(sm) : -INFINITY;
        }
        ell[j] = -INFINITY;
        fits[j].jr = -1;
        const int kap = n + tid + nt * j;
        if (kap >= K) continue;
        const double t0 = tau[j][0];
        if (!(t0 >= thr) || !(t0 > 0.0)) continue;
        const double lw = log(t0) + rp.log_g_rho - kap * rp.log_rho;
        if (lw < lower + log(1e-17)) continue;
        const SectorFitT<JM> f = fit_sector<JM>(n, 0, jp, t0, tau[j][1], tau[j][2], tau[j][3],
                                                 ORDER >= 4 ? tau[j][NT - 1] : 0.0);
        if (f.bad) continue;
        fits[j] = f;
        ell[j] = lw + f.lq;
        lse_add(fm, fs, ell[j]);
    }
    const double fmx = block_max(fm, red);
    const double fsum = block_sum(fm == -INFINITY ? 0.0 : fs * exp(fm - fmx), red);
    const double total = fmx + log(fsum);
    // sector cotangents: pi_kappa w_p d ell / d tau_t
    const double binv[4] = {1.0 / (n - 1.0), 2.0 / ((n - 1.0) * (n - 2.0)),
                            6.0 / ((n - 1.0) * (n - 2.0) * (n - 3.0)),
                            24.0 / ((n - 1.0) * (n - 2.0) * (n - 3.0) * (n - 4.0))};
    double tbar[FIT_KPT][NT];
#pragma unroll
    for (int j = 0; j < FIT_KPT; ++j) {
#pragma unroll
        for (int t = 0; t < NT; ++t) tbar[j][t] = 0.0;
        const int jr = fits[j].jr;
        if (jr < 0 || !(fsum > 0.0)) continue;
        const double pi = wp * exp(ell[j] - total);
        const double t0 = tau[j][0];
        const double *m = fits[j].m;
        // H = Cov_c[phi] at the fitted c; u = H^{-1} m (zero if H is singular)
        double u[4];
        fit_sensitivity<JM>(n, fits[j], u);
        if (!(fabs(u[0]) < 1e299))
#pragma unroll
            for (int t = 0; t < 4; ++t) u[t] = 0.0;
        double um = 0.0;
#pragma unroll
        for (int t = 0; t < JM; ++t)
            if (t < jr) um += u[t] * m[t];
        tbar[j][0] = pi * (1.0 + um) / t0;
#pragma unroll
        for (int t = 1; t <= JM; ++t)
            if (t <= jr) tbar[j][t] = -pi * u[t - 1] * binv[t - 1] / t0;
    }
    // alpha_t(w_q) = c_q FFT(tbar_t)[q], c_q = 1/K at q = 0, K/2 and 2/K otherwise
#pragma unroll
    for (int t = 0; t <= ORDER; ++t) {
        cplx *dst = asw + ((long)p * (ORDER + 1) + t) * GBS_QCAP;
        if (t > jp) {
            for (int q = tid; q < Q; q += nt) dst[q] = cmk(0.0, 0.0);
            continue;
        }
        for (int k = tid; k < K; k += nt) X[k] = cmk(0.0, 0.0);
        __syncthreads();
#pragma unroll
        for (int j = 0; j < FIT_KPT; ++j) {
            const int kap = n + tid + nt * j;
            if (kap < K) X[dft_pos(dsh, kap)] = cmk(tbar[j][t], 0.0);
        }
        __syncthreads();
        dft_lds(X, W, dsh);
        for (int q = tid; q < Q; q += nt) {
            const double cq = (q == 0 || q == K / 2) ? invK : 2.0 * invK;
            dst[q] = cscale(X[q], cq);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// k_adj_contour
// ---------------------------------------------------------------------------
// Rows up to 40 clicks keep V in LDS zero-padded to ADJ_TP x ADJ_TP (row stride
// ADJ_VS, a compile-time constant) and d_k zero-padded to ADJ_TP entries, so
// that no MFMA operand fetch needs a bounds mask.
#define ADJ_TMAX 5
#define ADJ_TP (16 * ADJ_TMAX)
#define ADJ_VS (ADJ_TP + 1)
static_assert(2 * GBS_NSMALL <= ADJ_TP, "padded V must hold the rows kept in LDS");
// After the cluster sums, Z(w) is copied into the M(w) region as the packed
// upper triangle of a 16T x 16T matrix (T = ceil(2n/16) tiles, zero beyond
// 2n), the A operand layout of Z V.
// The M(w) and Z(w) blocks of these rows sit at the strides of a 40-click row
// (ADJ_DS for the diagonal-block arrays, ADJ_OS for the pair-block arrays), so
// that the arrays of one block are compile-time offsets of each other.
#define ADJ_DS GBS_NSMALL
#define ADJ_OS (GBS_NSMALL * (GBS_NSMALL - 1) / 2)
#define ADJ_MREG (3 * ADJ_DS + 4 * ADJ_OS)
static_assert(ADJ_MREG >= 8 * ADJ_TMAX * (16 * ADJ_TMAX + 1), "the M(w) region holds the packed Z");
// the Z(w) blocks, the M(w) region, V, alpha, d and rz
__host__ __device__ __forceinline__ int adj_need(int)
{
    return 8 * (ADJ_TP * ADJ_VS + ADJ_TP) + 16 * (2 * ADJ_TP + 2 * ADJ_MREG);
}
__host__ __device__ __forceinline__ int adj_fixed() { return 16 * (CONT_THREADS / 64 + 8); }
// Larger rows form Y = Z V in their HBM scratch (row stride 32 ceil(2n/32),
// complex).

// Rows of at most 40 clicks (2n <= 80, at most ADJ_TMAX 16-wide tiles) form
// V^T Z V by column units: unit u of a row with T tiles covers column tile jt
// and row tiles rt0..rt1-1; it is held by one wavefront, which sums its share
// of R over the item's points in registers and writes it once, at the end of
// the item, into slot `slot` of the item's R scratch (ADJ_RSLOTS slots, summed
// in a fixed order by k_adj_reduce).
// Each column is split into as many parts as keep the eight wavefronts about
// equally loaded (a part costs (rt1 - rt0)(2 KS + 8 (jt + 1)) MFMAs); the
// units of each T are listed by decreasing cost, and with eight units wave w
// takes unit w (w < 4) or 11 - w, so that the two wavefronts of a SIMD hold a
// large and a small unit.
#define ADJ_RSLOTS GBS_RSLOTS
__device__ __forceinline__ int adj_col_units(int T)
{
    return T == 1 ? 1 : T == 2 ? 4 : 8;
}
__device__ __forceinline__ void adj_col_unit(int T, int u, int &jt, int &rt0, int &rt1, int &slot)
{
    // (jt, rt0, rt1, slot) packed 4 bits each
    constexpr unsigned short tab[5][8] = {
        {0x0010},
        {0x1010, 0x1121, 0x0010, 0x0121},
        {0x0131, 0x2010, 0x2121, 0x2232, 0x1010, 0x1121, 0x1232, 0x0010},
        {0x3020, 0x3241, 0x2020, 0x2241, 0x1020, 0x1241, 0x0020, 0x0241},
        {0x1050, 0x0050, 0x4251, 0x3251, 0x2251, 0x4020, 0x3020, 0x2020},
    };
    const unsigned v = tab[T - 1][u];
    jt = (v >> 12) & 15;
    rt0 = (v >> 8) & 15;
    rt1 = (v >> 4) & 15;
    slot = v & 15;
}

// 2x2 complex blocks of the fourth-order adjoint: general [[a, b], [c, d]] and
// symmetric [[a, b], [b, d]].
struct Blk {
    cplx a, b, c, d;
};
struct Sym {
    cplx a, b, d;
};
__device__ __forceinline__ Blk bmul(const Blk &x, const Blk &y)  // x y
{
    return Blk{cfma(x.a, y.a, cmul(x.b, y.c)), cfma(x.a, y.b, cmul(x.b, y.d)), cfma(x.c, y.a, cmul(x.d, y.c)),
               cfma(x.c, y.b, cmul(x.d, y.d))};
}
__device__ __forceinline__ Blk smul(const Sym &s, const Blk &y)  // s y
{
    return Blk{cfma(s.a, y.a, cmul(s.b, y.c)), cfma(s.a, y.b, cmul(s.b, y.d)), cfma(s.b, y.a, cmul(s.d, y.c)),
               cfma(s.b, y.b, cmul(s.d, y.d))};
}
__device__ __forceinline__ Blk bsmul(const Blk &x, const Sym &s)  // x s
{
    return Blk{cfma(x.a, s.a, cmul(x.b, s.b)), cfma(x.a, s.b, cmul(x.b, s.d)), cfma(x.c, s.a, cmul(x.d, s.b)),
               cfma(x.c, s.b, cmul(x.d, s.d))};
}
__device__ __forceinline__ Blk tmul(const Blk &x, const Blk &y)  // x^T y
{
    return Blk{cfma(x.a, y.a, cmul(x.c, y.c)), cfma(x.a, y.b, cmul(x.c, y.d)), cfma(x.b, y.a, cmul(x.d, y.c)),
               cfma(x.b, y.b, cmul(x.d, y.d))};
}
__device__ __forceinline__ Sym tmul_sym(const Blk &x, const Blk &y)  // x^T y, known symmetric
{
    return Sym{cfma(x.a, y.a, cmul(x.c, y.c)), cfma(x.a, y.b, cmul(x.c, y.d)), cfma(x.b, y.b, cmul(x.d, y.d))};
}
__device__ __forceinline__ Blk bmul_t(const Blk &x, const Blk &y)  // x y^T
{
    return Blk{cfma(x.a, y.a, cmul(x.b, y.b)), cfma(x.a, y.c, cmul(x.b, y.d)), cfma(x.c, y.a, cmul(x.d, y.b)),
               cfma(x.c, y.c, cmul(x.d, y.d))};
}
__device__ __forceinline__ Sym bmul_t_sym(const Blk &x, const Blk &y)  // x y^T, known symmetric
{
    return Sym{cfma(x.a, y.a, cmul(x.b, y.b)), cfma(x.a, y.c, cmul(x.b, y.d)), cfma(x.c, y.c, cmul(x.d, y.d))};
}
__device__ __forceinline__ Blk bsub(const Blk &x, const Blk &y)
{
    return Blk{csub(x.a, y.a), csub(x.b, y.b), csub(x.c, y.c), csub(x.d, y.d)};
}
__device__ __forceinline__ Sym ssub(const Sym &x, const Sym &y) { return Sym{csub(x.a, y.a), csub(x.b, y.b), csub(x.d, y.d)}; }
__device__ __forceinline__ Sym sadd(const Sym &x, const Sym &y) { return Sym{cadd(x.a, y.a), cadd(x.b, y.b), cadd(x.d, y.d)}; }
__device__ __forceinline__ Blk bneg(const Blk &x) { return Blk{cneg(x.a), cneg(x.b), cneg(x.c), cneg(x.d)}; }
__device__ __forceinline__ Blk bscale(const Blk &x, cplx k) { return Blk{cmul(x.a, k), cmul(x.b, k), cmul(x.c, k), cmul(x.d, k)}; }
__device__ __forceinline__ Sym sscale(const Sym &x, cplx k) { return Sym{cmul(x.a, k), cmul(x.b, k), cmul(x.d, k)}; }
// det(s)^{-1/2} on the principal branch (r) and s^{-1} = r^2 adj(s)
__device__ __forceinline__ Sym sinv(const Sym &s, cplx &r)
{
    r = crsqrt_p(cfnma(s.b, s.b, cmul(s.a, s.d)));
    const cplx r2 = cmul(r, r);
    return Sym{cmul(s.d, r2), cneg(cmul(s.b, r2)), cmul(s.a, r2)};
}

__device__ __forceinline__ void catomic(cplx *dst, cplx v)
{
    atomicAdd(&dst->re, v.re);
    atomicAdd(&dst->im, v.im);
}

// upper-triangle (column-major) packed index e -> (i, j), i <= j
__device__ __forceinline__ void upper_ij(int e, int &i, int &j)
{
    j = (int)floor(0.5 * (sqrt(8.0 * e + 1.0) - 1.0));
    while (j * (j + 1) / 2 > e) --j;
    while ((j + 1) * (j + 2) / 2 <= e) ++j;
    i = e - j * (j + 1) / 2;
}

template <int ORDER, bool BIG, bool DET>
__global__ __launch_bounds__(CONT_THREADS) void k_adj_contour(
    const int *__restrict__ offsets, const long long *__restrict__ voff,
    const double *__restrict__ alpha, const double *__restrict__ vt,
    const RowPlan *__restrict__ rows, const int *__restrict__ items, const int *__restrict__ q_end,
    int *__restrict__ q_head, const int *__restrict__ units, const int *__restrict__ unit_off,
    const int *__restrict__ unit4_off,
    const cplx *__restrict__ asw, const long long *__restrict__ roff, double *__restrict__ rscr,
    cplx *__restrict__ ascr, long long ascr_stride, const int *__restrict__ xq)
{
    extern __shared__ __attribute__((aligned(16))) double sh[];
    __shared__ int s_item;
    __shared__ cplx s_g[ORDER + 1];
    __shared__ double s_zmax[2 * CONT_THREADS / 64];
    __shared__ cplx s_wq[ADJ_QCHUNK];
    cplx *red = (cplx *)sh;                        // [waves]
    double *dyn = (double *)(red + CONT_THREADS / 64 + 8);
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int l16 = lane & 15, lq = lane >> 4;
    const int total = BIG ? 0 : *q_end;
    for (;;) {
        if (tid == 0) {
            if (BIG) {
                // larger rows: the queue of this workgroup's XCD first (workgroups
                // are dealt to the XCDs in turn), so that the rows in flight on
                // an XCD, whose V is read from its L2 at every point, are few;
                // the other XCDs' queues once it is empty (q_head: heads, q_end:
                // lengths then offsets, GBS_NXCD each)
                int it = -1;
                for (int d = 0; d < GBS_NXCD && it < 0; ++d) {
                    const int x = (blockIdx.x + d) % GBS_NXCD;
                    if (atomicAdd(&q_head[x], 0) >= q_end[x]) continue;
                    const int h = atomicAdd(&q_head[x], 1);
                    if (h < q_end[x]) it = xq[q_end[GBS_NXCD + x] + h];
                }
                s_item = it;
            } else {
                s_item = atomicAdd(q_head, 1);
            }
        }
        __syncthreads();
        const int item = s_item;
        __syncthreads();
        if (BIG ? item < 0 : item >= total) break;
        const int p = items[2 * item], ch = items[2 * item + 1];
        const int o = offsets[p], n = offsets[p + 1] - o, N = 2 * n;
        const RowPlan rp = rows[p];
        const int np = n * (n - 1) / 2;
        const long long vo = voff[p];
        // Vt[k*vs + i] = V[i][k].  Rows up to GBS_NSMALL clicks: V (zero-padded),
        // d, M(w) and Z(w) in LDS.  Larger rows: V read from HBM (L2), M(w) and
        // the Y = Z V panel in this workgroup's HBM scratch, Z(w) in LDS (at
        // order <= 2 only its diagonal blocks, plus a staged 32-row block of Z:
        // each pair block has a single writer and goes to the scratch)
        const int vs = BIG ? N : ADJ_VS;
        const double *Vt;
        double *al;
        cplx *dk, *rz, *Md0, *Zd0, *Zo0, *Yp, *Zs = nullptr;
        if (BIG) {
            Vt = vt + vo;
            al = dyn;
            dk = (cplx *)(al + N);
            rz = dk + N;
            Zd0 = rz + N;
            Md0 = ascr + blockIdx.x * ascr_stride;
            if (ORDER >= 3) {
                Zo0 = Zd0 + 3 * n;
                Yp = Md0 + 3 * n + 4 * np;
            } else {
                Zo0 = Md0 + 3 * n + 4 * np;
                Yp = Zo0 + 4 * np;
                Zs = Zd0 + 3 * n;
            }
        } else {
            // Z(w) first, then M(w), V, alpha, d, rz: every entry of Z then lies
            // within the 64 KB immediate offset of its LDS adds
            Zd0 = (cplx *)dyn;
            Zo0 = Zd0 + 3 * ADJ_DS;
            Md0 = Zd0 + ADJ_MREG;
            double *vl = (double *)(Md0 + ADJ_MREG);
            al = vl + ADJ_TP * ADJ_VS;
            dk = (cplx *)(al + ADJ_TP);
            rz = dk + ADJ_TP;
            Yp = nullptr;  // (no panel: Y stays in registers)
            for (int idx = tid; idx < ADJ_TP * ADJ_VS; idx += CONT_THREADS) {
                const int k = idx / ADJ_VS, i = idx - k * ADJ_VS;
                vl[idx] = k < N && i < N ? vt[vo + k * N + i] : 0.0;
            }
            for (int k = N + tid; k < ADJ_TP; k += CONT_THREADS) dk[k] = cmk(0.0, 0.0);
            Vt = vl;
        }
        const int dstr = BIG ? n : ADJ_DS, ostr = BIG ? np : ADJ_OS;
        cplx *Md1 = Md0 + dstr, *Md2 = Md1 + dstr;
        cplx *Mo0 = Md2 + dstr, *Mo1 = Mo0 + ostr, *Mo2 = Mo1 + ostr, *Mo3 = Mo2 + ostr;
        cplx *Zd1 = Zd0 + dstr, *Zd2 = Zd1 + dstr;
        cplx *Zo1 = Zo0 + ostr, *Zo2 = Zo1 + ostr, *Zo3 = Zo2 + ostr;
        // Z(w) accumulation.  Where the whole of Z sits in LDS (rows kept in
        // LDS, and the larger rows at order 3 and above) it is held as two
        // planes, the real parts and then the imaginary parts, zplane doubles
        // each, addressed by the complex index: each 64-bit LDS atomic of a
        // wavefront then steps by 8 bytes instead of 16, which halves its
        // bank passes.  (At order <= 2 the larger rows keep the pair blocks in
        // HBM and Z stays interleaved.)
        constexpr bool ZPLANES = !BIG || ORDER >= 3;
        const int zplane = BIG ? 3 * n + 4 * np : ADJ_MREG;
        // Deterministic mode: the cluster terms go into Z as 64-bit integers,
        // llrint(term x scale) (sums that do not depend on the order of the
        // adds), converted back after the point.  The scales are powers of two
        // with room for every term of an entry below the largest term of its
        // kind; the diagonal blocks and the pair blocks take scales of their own
        // (an entry of a pair block collects far fewer terms).  Over an item's
        // points the scales are carried: a point adds at the scales the previous
        // point's terms set (with one power of two of room) while it tracks its
        // own largest terms, and is run again at exact scales, after Z(w) is
        // cleared, only if they overrun those scales or sit more than two powers
        // of two below; the item's first point takes a pass that only finds them.
        double zmax = 0.0, zsc = 1.0, zmaxo = 0.0, zsco = 1.0;
        bool zhave = false;
        int zcap = 0, zcapo = 0;  // the scales' exponent caps: terms below 2^cap
        // the pair blocks follow the diagonal ones wherever they are added into
        const int zoff = BIG ? 3 * n : 3 * ADJ_DS;
        // (entries are addressed by their complex index from Zd0, so that the
        // arrays' fixed strides become immediate offsets of the LDS adds)
        // (pr: a pair-block entry; every call site passes a constant.  A pass
        // that only finds the largest terms runs the same code at scale 0.)
        auto zadd = [&](int idx, cplx v, bool pr) {
            if constexpr (DET) {
                const double m = fmax(fabs(v.re), fabs(v.im));
                const double mm = m <= DBL_MAX ? m : INFINITY;  // (NaN or inf: non-finite)
                if (pr)
                    zmaxo = fmax(zmaxo, mm);
                else
                    zmax = fmax(zmax, mm);
                const double sc = pr ? zsco : zsc;
                unsigned long long *zr = (unsigned long long *)Zd0 + (ZPLANES ? idx : 2 * idx);
                atomicAdd(zr, (unsigned long long)llrint(v.re * sc));
                atomicAdd(zr + (ZPLANES ? zplane : 1), (unsigned long long)llrint(v.im * sc));
            } else if constexpr (ZPLANES) {
                double *zr = (double *)Zd0 + idx;
                atomicAdd(zr, v.re);
                atomicAdd(zr + zplane, v.im);
            } else {
                catomic(Zd0 + idx, v);
            }
        };
        // diagonal-block array k at mode x; pair-block array k at pair position q
        auto zd = [&](int k, int x, cplx v) { zadd(k * dstr + x, v, false); };
        auto zo = [&](int k, int q, cplx v) { zadd(zoff + k * ostr + q, v, true); };
        for (int i = tid; i < N; i += CONT_THREADS) al[i] = alpha[2 * o + i];
        const int Qn = rp.K / 2 + 1;
        constexpr int QCH = BIG ? GBS_ADJ_CHUNK_BIG : ADJ_QCHUNK;
        const int q0 = ch * QCH, q1 = min(q0 + QCH, Qn);
        const int T = (N + 15) >> 4, KS = (N + 3) >> 2;
        // rows up to 40 clicks: this wavefront's share of R (its column unit's
        // tiles), summed over the item's points in registers
        dbl4 racc[ADJ_TMAX];
#pragma unroll
        for (int it = 0; it < ADJ_TMAX; ++it) racc[it] = dbl4{0.0, 0.0, 0.0, 0.0};
        const long long ro = roff[item];
        if (BIG) {
            for (int e = tid; e < N * (N + 1) / 2; e += CONT_THREADS) rscr[ro + e] = 0.0;
        } else {
            // R slots are written once, at the end of the item, by the column
            // units; the column strips of a slot that no unit covers are zero
            const int nun = adj_col_units(T), nup = N * (N + 1) / 2;
            for (int s = 0; s < ADJ_RSLOTS; ++s)
                for (int jt = 0; jt < T; ++jt) {
                    bool cov = false;
                    for (int u = 0; u < nun; ++u) {
                        int ujt, r0, r1, us;
                        adj_col_unit(T, u, ujt, r0, r1, us);
                        cov = cov || (ujt == jt && us == s);
                    }
                    if (cov) continue;
                    const int j0 = 16 * jt, j1 = min(16 * jt + 16, N);
                    for (int e = j0 * (j0 + 1) / 2 + tid; e < j1 * (j1 + 1) / 2; e += CONT_THREADS)
                        rscr[ro + (long long)s * nup + e] = 0.0;
                }
        }
        // the item's contour points w_q = rho e^{2 pi i q / K}
        if (tid < q1 - q0) {
            s_wq[tid] = cscale(unit_root(q0 + tid, rp.K), rp.rho);
        }
        __syncthreads();
        // (every pass over a point ends with a barrier, so the next point's d_k
        // and Z(w) may be written at once)
        for (int q = q0; q < q1; ++q) {
            const cplx w = s_wq[q - q0];
            for (int k = tid; k < N; k += CONT_THREADS) {
                const double am1 = al[k] - 1.0;
                const cplx z = cmk(fma(w.re, am1, 1.0), w.im * am1);
                const cplx r = crsqrt_p(z);
                dk[k] = cmul(r, r);
                rz[k] = r;
            }
            if (BIG) {
                for (int i = tid; i < 3 * n; i += CONT_THREADS) Zd0[i] = cmk(0.0, 0.0);
                if (ORDER != 2)
                    for (int i = tid; i < 4 * np; i += CONT_THREADS) Zo0[i] = cmk(0.0, 0.0);
            } else {
                for (int i = tid; i < ADJ_MREG; i += CONT_THREADS) Zd0[i] = cmk(0.0, 0.0);
            }
            __syncthreads();
            if (wid == 0) {
                // G_0(w)/G_0(rho) = exp(log det A/2 - log G_0(rho)) prod_k z_k^{-1/2}
                cplx pr = cmk(1.0, 0.0);
                for (int k = lane; k < N; k += 64) pr = cmul(pr, rz[k]);
                pr = cmul(warp_cprod(pr), cmk(exp(0.5 * rp.logdet_a - rp.log_g_rho), 0.0));
                if (lane <= ORDER) s_g[lane] = cmul(asw[((long)p * (ORDER + 1) + lane) * GBS_QCAP + q], pr);
            }
            // M(w) = V diag(d) V^T on the matrix cores, upper tiles over the waves
            if (ORDER >= 2) {
                constexpr int BS = BIG ? 2 : 1;
                const int TB = (N + 16 * BS - 1) / (16 * BS), nblk = TB * (TB + 1) / 2;
                // (the tiles are dealt from the last wavefront down: wavefront 0
                // forms G_0(w) first)
                for (int u = CONT_THREADS / 64 - 1 - wid; u < nblk; u += CONT_THREADS / 64) {
                    int it, jt;
                    upper_tile(u, it, jt);
                    m_block_mfma<BS, cplx, true, !BIG, !BIG>(n, it, jt, Vt, vs, dk, Md0, lane);
                }
            } else {
                for (int a = tid; a < n; a += CONT_THREADS) {
                    cplx m00 = cmk(0, 0), m01 = cmk(0, 0), m11 = cmk(0, 0);
#pragma unroll 1
                    for (int k = 0; k < N; ++k) {
                        const double v0 = Vt[k * vs + a], v1 = Vt[k * vs + n + a];
                        const cplx d = dk[k];
                        const double p00 = v0 * v0, p01 = v0 * v1, p11 = v1 * v1;
                        m00.re = fma(p00, d.re, m00.re); m00.im = fma(p00, d.im, m00.im);
                        m01.re = fma(p01, d.re, m01.re); m01.im = fma(p01, d.im, m01.im);
                        m11.re = fma(p11, d.re, m11.re); m11.im = fma(p11, d.im, m11.im);
                    }
                    Md0[a] = m00; Md1[a] = m01; Md2[a] = m11;
                }
            }
            __syncthreads();
            // clusters: Z += c_T E_T M_TT^{-1} E_T^T, c_T = gamma_|T| det(M_TT)^{-1/2}
            cplx bsum = cmk(0.0, 0.0);
            bool zredo = false;
            for (int zp = DET && !zhave ? 0 : 1; zp < 2; ++zp) {
                if (DET) {
                    zmax = zmaxo = 0.0;  // (this pass's terms only)
                    if (zp == 0) zsc = zsco = 0.0;
                }
                bsum = cmk(0.0, 0.0);
                const cplx g1 = s_g[1 <= ORDER ? 1 : 0];
                for (int a = tid; a < n; a += CONT_THREADS) {
                    const cplx a00 = Md0[a], a01 = Md1[a], a11 = Md2[a];
                    const cplx r = crsqrt_p(cfnma(a01, a01, cmul(a00, a11)));
                    const cplx c = cmul(g1, r);
                    const cplx id = cmul(r, r);
                    bsum = cadd(bsum, c);
                    const cplx cid = cmul(c, id);
                    zd(0, a, cmul(cid, a11));
                    zd(1, a, cscale(cmul(cid, a01), -1.0));
                    zd(2, a, cmul(cid, a00));
                }
                if (ORDER >= 2) {
                    const cplx g2 = s_g[2 <= ORDER ? 2 : 0];
                    const cplx g3 = s_g[3 <= ORDER ? 3 : 0];
                    const int *un = units + unit_off[2 * n];
                    const int nu = unit_off[2 * n + 1];
                    int unext = tid < nu ? un[tid] : 0;
    #pragma unroll 1
                    for (int ui = tid; ui < nu; ui += CONT_THREADS) {
                        const unsigned u = (unsigned)unext;
                        if (ui + CONT_THREADS < nu) unext = un[ui + CONT_THREADS];
                        const int a = u & 255, b = (u >> 8) & 255, c0 = (u >> 16) & 255, c1 = u >> 24;
                        const int pi = pair_pos<true>(n, a, b);
                        const cplx a00 = Md0[a], a01 = Md1[a], a11 = Md2[a];
                        const cplx b00 = Mo0[pi], b01 = Mo1[pi], b10 = Mo2[pi], b11 = Mo3[pi];
                        const cplx deta = cfnma(a01, a01, cmul(a00, a11));
                        const cplx ra = crsqrt_p(deta);
                        const cplx ideta = cmul(ra, ra);
                        const cplx ia00 = cmul(a11, ideta), ia11 = cmul(a00, ideta);
                        const cplx ia01 = cscale(cmul(a01, ideta), -1.0);
                        const cplx G00 = cfma(ia00, b00, cmul(ia01, b10));
                        const cplx G01 = cfma(ia00, b01, cmul(ia01, b11));
                        const cplx G10 = cfma(ia01, b00, cmul(ia11, b10));
                        const cplx G11 = cfma(ia01, b01, cmul(ia11, b11));
                        const cplx sb00 = csub(Md0[b], cfma(b00, G00, cmul(b10, G10)));
                        const cplx sb01 = csub(Md1[b], cfma(b00, G01, cmul(b10, G11)));
                        const cplx sb11 = csub(Md2[b], cfma(b01, G01, cmul(b11, G11)));
                        const cplx rb = crsqrt_p(cfnma(sb01, sb01, cmul(sb00, sb11)));
                        const cplx rab = cmul(ra, rb);
                        const cplx idetb = cmul(rb, rb);
                        const cplx ib00 = cmul(sb11, idetb), ib11 = cmul(sb00, idetb);
                        const cplx ib01 = cscale(cmul(sb01, idetb), -1.0);
                        // P^{-1} = [[ia + G ib G^T, -G ib], [-ib G^T, ib]]: its a block
                        // pa, its (a, b) block nH = -G ib (rows x_a, p_a), and ib
                        const cplx H00 = cfma(ib00, G00, cmul(ib01, G01)), H01 = cfma(ib01, G00, cmul(ib11, G01));
                        const cplx H10 = cfma(ib00, G10, cmul(ib01, G11)), H11 = cfma(ib01, G10, cmul(ib11, G11));
                        const cplx pa00 = cadd(ia00, cfma(H00, G00, cmul(H01, G01)));
                        const cplx pa01 = cadd(ia01, cfma(H00, G10, cmul(H01, G11)));
                        const cplx pa11 = cadd(ia11, cfma(H10, G10, cmul(H11, G11)));
                        const cplx nH00 = cneg(H00), nH01 = cneg(H01), nH10 = cneg(H10), nH11 = cneg(H11);
                        // coefficient of P^{-1} (the pair itself, carried by its first unit,
                        // plus the unit's triples) and the pair block of
                        // sum_c c_T U Sc^{-1} U^T (4x4 symmetric, 10 entries)
                        cplx cp = c0 == b + 1 ? cmul(g2, rab) : cmk(0.0, 0.0);
                        bsum = cadd(bsum, cp);
                        cplx A00 = cmk(0, 0), A01 = cmk(0, 0), A02 = cmk(0, 0), A03 = cmk(0, 0),
                             A11 = cmk(0, 0), A12 = cmk(0, 0), A13 = cmk(0, 0), A22 = cmk(0, 0),
                             A23 = cmk(0, 0), A33 = cmk(0, 0);
                        if (ORDER >= 3) {
                            // (pair positions stepped along c: pos(x, c + 1) = pos(x, c) + n - (c - x))
                            int cur_ac = pair_pos<true>(n, a, c0), cur_bc = pair_pos<true>(n, b, c0);
    #pragma unroll 1
                            for (int c = c0; c < c1; cur_ac += n - (c - a), cur_bc += n - (c - b), ++c) {
                                const cplx *xa = Mo0 + cur_ac, *xb = Mo0 + cur_bc;
                                if constexpr (!BIG) {
                                    // (indices from the LDS base, kept opaque, so that each
                                    // position's address is formed once and the arrays'
                                    // fixed strides ride as immediate offsets)
                                    // (Mo0 = Zd0 + ADJ_MREG + 3 ADJ_DS in this layout: Z(w), then
                                    // the M(w) region with its three diagonal-block arrays first)
                                    int ia_ = ADJ_MREG + 3 * ADJ_DS + cur_ac, ib_ = ADJ_MREG + 3 * ADJ_DS + cur_bc;
                                    asm("" : "+v"(ia_), "+v"(ib_));
                                    xa = Zd0 + ia_;
                                    xb = Zd0 + ib_;
                                }
                                const cplx x00 = xa[0], x01 = xa[ostr], x10 = xa[2 * ostr], x11 = xa[3 * ostr];
                                const cplx yy00 = xb[0], yy01 = xb[ostr], yy10 = xb[2 * ostr], yy11 = xb[3 * ostr];
                                const cplx m00 = Md0[c], m01 = Md1[c], m11 = Md2[c];
                                // U = P^{-1} B for B = [Xa; Xb] (rows x_a, p_a, x_b, p_b;
                                // columns x_c, p_c): rows a (U) and rows b (W); then
                                // Sc = Mcc - B^T U
                                const cplx U00 = cfma(pa00, x00, cfma(pa01, x10, cfma(nH00, yy00, cmul(nH01, yy10))));
                                const cplx U01 = cfma(pa00, x01, cfma(pa01, x11, cfma(nH00, yy01, cmul(nH01, yy11))));
                                const cplx U10 = cfma(pa01, x00, cfma(pa11, x10, cfma(nH10, yy00, cmul(nH11, yy10))));
                                const cplx U11 = cfma(pa01, x01, cfma(pa11, x11, cfma(nH10, yy01, cmul(nH11, yy11))));
                                const cplx W00 = cfma(nH00, x00, cfma(nH10, x10, cfma(ib00, yy00, cmul(ib01, yy10))));
                                const cplx W01 = cfma(nH00, x01, cfma(nH10, x11, cfma(ib00, yy01, cmul(ib01, yy11))));
                                const cplx W10 = cfma(nH01, x00, cfma(nH11, x10, cfma(ib01, yy00, cmul(ib11, yy10))));
                                const cplx W11 = cfma(nH01, x01, cfma(nH11, x11, cfma(ib01, yy01, cmul(ib11, yy11))));
                                const cplx sc00 = cfnma(x00, U00, cfnma(x10, U10, cfnma(yy00, W00, cfnma(yy10, W10, m00))));
                                const cplx sc01 = cfnma(x00, U01, cfnma(x10, U11, cfnma(yy00, W01, cfnma(yy10, W11, m01))));
                                const cplx sc11 = cfnma(x01, U01, cfnma(x11, U11, cfnma(yy01, W01, cfnma(yy11, W11, m11))));
                                const cplx rc = crsqrt_p(cfnma(sc01, sc01, cmul(sc00, sc11)));
                                const cplx ct = cmul(g3, cmul(rab, rc));
                                bsum = cadd(bsum, ct);
                                // c_T Sc^{-1}
                                cplx is00, is01, is11;
                                {
                                    const cplx k = cmul(ct, cmul(rc, rc));
                                    is00 = cmul(sc11, k);
                                    is11 = cmul(sc00, k);
                                    is01 = cmul(cneg(sc01), k);
                                }
                                zd(0, c, is00);
                                zd(1, c, is01);
                                zd(2, c, is11);
                                // rows a: Q_a = -P_a = -U_a c_T Sc^{-1} (formed with the
                                // sign the Z blocks take, so that no negated copy has to
                                // be made for the LDS adds)
                                const cplx Q00 = cfnma(U00, is00, cmul(cneg(U01), is01));
                                const cplx Q01 = cfnma(U00, is01, cmul(cneg(U01), is11));
                                const cplx Q10 = cfnma(U10, is00, cmul(cneg(U11), is01));
                                const cplx Q11 = cfnma(U10, is01, cmul(cneg(U11), is11));
                                zo(0, cur_ac, Q00);
                                zo(1, cur_ac, Q01);
                                zo(2, cur_ac, Q10);
                                zo(3, cur_ac, Q11);
                                A00 = cfnma(Q00, U00, cfnma(Q01, U01, A00));
                                A01 = cfnma(Q00, U10, cfnma(Q01, U11, A01));
                                A11 = cfnma(Q10, U10, cfnma(Q11, U11, A11));
                                A02 = cfnma(Q00, W00, cfnma(Q01, W01, A02));
                                A03 = cfnma(Q00, W10, cfnma(Q01, W11, A03));
                                A12 = cfnma(Q10, W00, cfnma(Q11, W01, A12));
                                A13 = cfnma(Q10, W10, cfnma(Q11, W11, A13));
                                // rows b: Q_b = -P_b = -W c_T Sc^{-1}
                                const cplx Q20 = cfnma(W00, is00, cmul(cneg(W01), is01));
                                const cplx Q21 = cfnma(W00, is01, cmul(cneg(W01), is11));
                                const cplx Q30 = cfnma(W10, is00, cmul(cneg(W11), is01));
                                const cplx Q31 = cfnma(W10, is01, cmul(cneg(W11), is11));
                                zo(0, cur_bc, Q20);
                                zo(1, cur_bc, Q21);
                                zo(2, cur_bc, Q30);
                                zo(3, cur_bc, Q31);
                                A22 = cfnma(Q20, W00, cfnma(Q21, W01, A22));
                                A23 = cfnma(Q20, W10, cfnma(Q21, W11, A23));
                                A33 = cfnma(Q30, W10, cfnma(Q31, W11, A33));
                                cp = cadd(cp, ct);
                            }
                        }
                        zd(0, a, cfma(cp, pa00, A00));
                        zd(1, a, cfma(cp, pa01, A01));
                        zd(2, a, cfma(cp, pa11, A11));
                        if (BIG && ORDER <= 2) {
                            // one unit per pair: the pair block has a single writer
                            Zo0[pi] = cfnma(cp, H00, A02);
                            Zo1[pi] = cfnma(cp, H01, A03);
                            Zo2[pi] = cfnma(cp, H10, A12);
                            Zo3[pi] = cfnma(cp, H11, A13);
                        } else {
                            zo(0, pi, cfnma(cp, H00, A02));
                            zo(1, pi, cfnma(cp, H01, A03));
                            zo(2, pi, cfnma(cp, H10, A12));
                            zo(3, pi, cfnma(cp, H11, A13));
                        }
                        zd(0, b, cfma(cp, ib00, A22));
                        zd(1, b, cfma(cp, ib01, A23));
                        zd(2, b, cfma(cp, ib11, A33));
                    }
                }
                if constexpr (ORDER >= 4) {
                    // quadruples T = {a, b, c, d}: units (a, b, c; d0 .. d0+len-1).  With
                    // the triple {a, b, c} eliminated as in the forward (ia = Maa^{-1},
                    // G = ia Mab, ib = Sb^{-1}, Zc = ia Mac, Wc = ib (Mbc - G^T Mac),
                    // ic = Sc^{-1}), each d has y = M3^{-1} r_d, r_d = [Mad; Mbd; Mcd],
                    // by back-substitution through those factors:
                    //   y3 = v = ic u,  y2 = W - Wc v,  y1 = Z - G y2 - Zc v,
                    // and M_TT^{-1} = [[M3^{-1} + y Sd^{-1} y^T, -y Sd^{-1}], [., Sd^{-1}]].
                    // c_T M_TT^{-1} goes into Z; the M3^{-1} part, the same for every d of
                    // the unit, once per unit with the sum of the unit's c_T.
                    const cplx g4 = s_g[ORDER >= 4 ? 4 : 0];
                    auto Mdiag = [&](int x) { return Sym{Md0[x], Md1[x], Md2[x]}; };
                    auto Mpair = [&](int x, int y) {
                        const int q = pair_pos<true>(n, x, y);
                        return Blk{Mo0[q], Mo1[q], Mo2[q], Mo3[q]};
                    };
                    auto zdiag = [&](int x, const Sym &v) {
                        zd(0, x, v.a);
                        zd(1, x, v.b);
                        zd(2, x, v.d);
                    };
                    auto zpair = [&](int x, int y, const Blk &v) {
                        const int q = pair_pos<true>(n, x, y);
                        zo(0, q, v.a);
                        zo(1, q, v.b);
                        zo(2, q, v.c);
                        zo(3, q, v.d);
                    };
                    const int *un4 = units + unit4_off[2 * n];
                    const int nu4 = unit4_off[2 * n + 1];
    #pragma unroll 1
                    for (int ui = tid; ui < nu4; ui += CONT_THREADS) {
                        const unsigned u4 = (unsigned)un4[ui];
                        const int a = u4 & 63, b = (u4 >> 6) & 63, c = (u4 >> 12) & 63, d0 = (u4 >> 18) & 63,
                                  d1 = d0 + (int)(u4 >> 24);
                        cplx ra, rb, rc;
                        const Sym ia = sinv(Mdiag(a), ra);
                        const Blk Mab = Mpair(a, b);
                        const Blk G = smul(ia, Mab);
                        const Sym ib = sinv(ssub(Mdiag(b), tmul_sym(Mab, G)), rb);
                        const Blk Mac = Mpair(a, c);
                        const Blk Zc = smul(ia, Mac);
                        const Blk Yc = bsub(Mpair(b, c), tmul(G, Mac));
                        const Blk Wc = smul(ib, Yc);
                        const Sym ic = sinv(ssub(ssub(Mdiag(c), tmul_sym(Mac, Zc)), tmul_sym(Yc, Wc)), rc);
                        const cplx rabc = cmul(cmul(ra, rb), rc);
                        cplx csum = cmk(0.0, 0.0);
    #pragma unroll 1
                        for (int d = d0; d < d1; ++d) {
                            const Blk x = Mpair(a, d);
                            const Blk Y = bsub(Mpair(b, d), tmul(G, x));
                            const Blk W = smul(ib, Y);
                            const Blk Z = smul(ia, x);
                            const Sym q = ssub(ssub(Mdiag(d), tmul_sym(x, Z)), tmul_sym(Y, W));
                            const Blk u = bsub(bsub(Mpair(c, d), tmul(Zc, x)), tmul(Wc, Y));
                            const Blk v = smul(ic, u);
                            cplx rd;
                            const Sym isd0 = sinv(ssub(q, tmul_sym(u, v)), rd);
                            const cplx ct = cmul(g4, cmul(rabc, rd));
                            csum = cadd(csum, ct);
                            const Sym isd = sscale(isd0, ct);
                            const Blk y2 = bsub(W, bmul(Wc, v));
                            const Blk y1 = bsub(bsub(Z, bmul(G, y2)), bmul(Zc, v));
                            const Blk t1 = bsmul(y1, isd), t2 = bsmul(y2, isd), t3 = bsmul(v, isd);
                            zdiag(d, isd);
                            zpair(a, d, bneg(t1));
                            zpair(b, d, bneg(t2));
                            zpair(c, d, bneg(t3));
                            zdiag(a, bmul_t_sym(t1, y1));
                            zdiag(b, bmul_t_sym(t2, y2));
                            zdiag(c, bmul_t_sym(t3, v));
                            zpair(a, b, bmul_t(t1, y2));
                            zpair(a, c, bmul_t(t1, v));
                            zpair(b, c, bmul_t(t2, v));
                        }
                        bsum = cadd(bsum, csum);
                        // csum M3^{-1}: cc = ic, ac = -Ua ic, bc = -Wc ic,
                        // aa = ia + G ib G^T + Ua ic Ua^T, ab = -G ib + Ua ic Wc^T,
                        // bb = ib + Wc ic Wc^T, with Ua = Zc - G Wc
                        const Blk Ua = bsub(Zc, bmul(G, Wc));
                        const Blk Uic = bsmul(Ua, ic), Wic = bsmul(Wc, ic), Gib = bsmul(G, ib);
                        const cplx ncs = cneg(csum);
                        zdiag(c, sscale(ic, csum));
                        zpair(a, c, bscale(Uic, ncs));
                        zpair(b, c, bscale(Wic, ncs));
                        zdiag(a, sscale(sadd(sadd(ia, bmul_t_sym(Gib, G)), bmul_t_sym(Uic, Ua)), csum));
                        zpair(a, b, bscale(bsub(bmul_t(Uic, Wc), Gib), csum));
                        zdiag(b, sscale(sadd(ib, bmul_t_sym(Wic, Wc)), csum));
                    }
                }
                if constexpr (DET) {
                    // the block's largest terms; each scale leaves room for one
                    // term per cluster holding the entry's modes: a diagonal
                    // entry's mode is in sum_{t < j} C(n-1, t) clusters, a pair
                    // entry's two modes in sum_{t < j-1} C(n-2, t)
                    double zm = zmax, zo_ = zmaxo;
                    for (int off = 32; off > 0; off >>= 1) {
                        zm = fmax(zm, __shfl_xor(zm, off));
                        zo_ = fmax(zo_, __shfl_xor(zo_, off));
                    }
                    if (lane == 0) {
                        s_zmax[wid] = zm;
                        s_zmax[CONT_THREADS / 64 + wid] = zo_;
                    }
                    __syncthreads();
                    zm = zo_ = 0.0;
                    for (int i = 0; i < CONT_THREADS / 64; ++i) {
                        zm = fmax(zm, s_zmax[i]);
                        zo_ = fmax(zo_, s_zmax[CONT_THREADS / 64 + i]);
                    }
                    zmax = zm;
                    zmaxo = zo_;
                    const bool fin = zm <= DBL_MAX && zo_ <= DBL_MAX;
                    // (non-finite terms: every entry becomes NaN below, whatever Z holds)
                    if (!fin) break;
                    int ed = 0, eo = 0;
                    frexp(zm, &ed);
                    frexp(zo_, &eo);
                    const bool fits = zp == 1 && (zm == 0.0 || (ed <= zcap && ed >= zcap - 2)) &&
                                      (zo_ == 0.0 || (eo <= zcapo && eo >= zcapo - 2));
                    if (!fits && !zredo) {
                        double ncl = 1.0, bin = 1.0;
                        for (int t = 1; t < ORDER && t < n; ++t) {
                            bin = bin * (n - t) / t;
                            ncl += bin;
                        }
                        double nclo = 1.0;
                        bin = 1.0;
                        for (int t = 1; t < ORDER - 1 && t < n - 1; ++t) {
                            bin = bin * (n - 1 - t) / t;
                            nclo += bin;
                        }
                        // exact caps for this point (ncl terms below 2^e sum to less
                        // than 2^62 at the scale 2^(61 - floor(log2 ncl) - e))
                        zcap = zm > 0.0 ? ed : zcap;
                        zcapo = zo_ > 0.0 ? eo : zcapo;
                        zsc = ldexp(1.0, 61 - ilogb(ncl) - zcap);
                        zsco = ldexp(1.0, 61 - ilogb(nclo) - zcapo);
                        zhave = true;
                        if (zp == 1) {
                            // the adds made at the old scales are discarded
                            if (BIG) {
                                for (int i = tid; i < 3 * n; i += CONT_THREADS) Zd0[i] = cmk(0.0, 0.0);
                                if (ORDER != 2)
                                    for (int i = tid; i < 4 * np; i += CONT_THREADS) Zo0[i] = cmk(0.0, 0.0);
                            } else {
                                for (int i = tid; i < ADJ_MREG; i += CONT_THREADS) Zd0[i] = cmk(0.0, 0.0);
                            }
                            zredo = true;
                        }
                        __syncthreads();
                        zp = 0;  // (the next pass adds at the new scales)
                        continue;
                    }
                    break;
                }
            }
            if constexpr (DET) {
                __syncthreads();
                // back to doubles (the scale is a power of two); non-finite terms
                // make every entry NaN, as the floating-point sums would
                unsigned long long *zi = (unsigned long long *)Zd0;
                double *zf = (double *)Zd0;
                const int nz = ZPLANES ? 2 * zplane : 6 * n;
                const double inv = 1.0 / zsc, invo = 1.0 / zsco;
                const bool bad = !(zmax <= DBL_MAX) || !(zmaxo <= DBL_MAX);
                for (int i = tid; i < nz; i += CONT_THREADS) {
                    const bool pr = ZPLANES && (i < zplane ? i : i - zplane) >= zoff;
                    zf[i] = bad ? NAN : (double)(long long)zi[i] * (pr ? invo : inv);
                }
                // the next point's scales: one power of two above this point's terms
                if (!bad && zhave) {
                    int ed = 0, eo = 0;
                    frexp(zmax, &ed);
                    frexp(zmaxo, &eo);
                    if (zmax > 0.0 && ed + 1 != zcap) {
                        zsc = ldexp(zsc, zcap - ed - 1);
                        zcap = ed + 1;
                    }
                    if (zmaxo > 0.0 && eo + 1 != zcapo) {
                        zsco = ldexp(zsco, zcapo - eo - 1);
                        zcapo = eo + 1;
                    }
                }
            }
            bsum = warp_csum(bsum);
            if (lane == 0) red[wid] = bsum;
            __syncthreads();
            // R += Re[(w/2) d_i d_j (V^T Z V)_ij] (+ diagonal beta terms) on the
            // matrix cores (below: the larger rows first, then the column units
            // of the rows kept in LDS)
            cplx beta = s_g[0];
            for (int i = 0; i < CONT_THREADS / 64; ++i) beta = cadd(beta, red[i]);
            const cplx hw = cscale(w, 0.5);
            // Z(r, s) for r, s in quadrature-major order (zero outside 2n x 2n)
            auto zget = [&](int r, int sidx) {
                const bool ok = r < N && sidx < N;
                const int a = r < n ? r : r - n, qa = r < n ? 0 : 1;
                const int b = sidx < n ? sidx : sidx - n, qb = sidx < n ? 0 : 1;
                const int lo = min(a, b), hi = max(a, b);
                const int kq = a < b ? 2 * qa + qb : 2 * qb + qa;
                const cplx *src = a == b ? Zd0 + (qa + qb) * dstr + a : Zo0 + kq * ostr + pair_pos<true>(n, lo, hi);
                cplx zl;
                if constexpr (ZPLANES) {
                    const double *zr = (const double *)Zd0 + (ok ? src - Zd0 : 0);
                    zl = cmk(zr[0], zr[zplane]);
                } else {
                    zl = *(ok ? src : Zd0);
                }
                return ok ? zl : cmk(0.0, 0.0);
            };
            if (BIG) {
                // Y = Z V for all 32 x 32 blocks (rb, cb), then X = V^T Y for the
                // upper blocks (ib <= jb), each phase dealt over all the
                // wavefronts; V comes from L2 (2x2 tiles share each operand
                // fetch), Y goes to this workgroup's HBM panel (row stride
                // 32 TB), and R is read-modified-written in the item's HBM slot
                // (each entry has one writer per point)
                const int TB = (T + 1) / 2, YS = 32 * TB;
                auto yblock = [&](int rb, int cb, auto zfn) {
                    dbl4 yre[2][2], yim[2][2];
#pragma unroll
                    for (int a = 0; a < 2; ++a)
#pragma unroll
                        for (int t = 0; t < 2; ++t) yre[a][t] = yim[a][t] = dbl4{0.0, 0.0, 0.0, 0.0};
                    const int r0 = (2 * rb) * 16 + l16, r1 = r0 + 16;
                    const int j0 = (2 * cb) * 16 + l16, j1 = j0 + 16;
#pragma unroll 2
                    for (int ks = 0; ks < KS; ++ks) {
                        const int sidx = ks * 4 + lq;
                        const cplx z0 = zfn(r0, sidx), z1 = zfn(r1, sidx);
                        const bool v0ok = j0 < N && sidx < N, v1ok = j1 < N && sidx < N;
                        const double v0l = Vt[v0ok ? j0 * vs + sidx : 0], v1l = Vt[v1ok ? j1 * vs + sidx : 0];
                        const double v0 = v0ok ? v0l : 0.0, v1 = v1ok ? v1l : 0.0;
                        yre[0][0] = mfma4(z0.re, v0, yre[0][0]);
                        yim[0][0] = mfma4(z0.im, v0, yim[0][0]);
                        yre[0][1] = mfma4(z0.re, v1, yre[0][1]);
                        yim[0][1] = mfma4(z0.im, v1, yim[0][1]);
                        yre[1][0] = mfma4(z1.re, v0, yre[1][0]);
                        yim[1][0] = mfma4(z1.im, v0, yim[1][0]);
                        yre[1][1] = mfma4(z1.re, v1, yre[1][1]);
                        yim[1][1] = mfma4(z1.im, v1, yim[1][1]);
                    }
#pragma unroll
                    for (int a = 0; a < 2; ++a)
#pragma unroll
                        for (int t = 0; t < 2; ++t)
#pragma unroll
                            for (int e = 0; e < 4; ++e) {
                                const int row = (2 * rb + a) * 16 + 4 * e + lq;
                                if (row < N) Yp[row * YS + (2 * cb + t) * 16 + l16] = cmk(yre[a][t][e], yim[a][t][e]);
                            }
                };
                if (ORDER >= 3) {
                    // Z is in LDS
                    for (int u = wid; u < TB * TB; u += CONT_THREADS / 64) yblock(u / TB, u % TB, zget);
                } else {
                    // the pair blocks of Z are in this workgroup's HBM scratch:
                    // each 32-row block of Z is gathered once into LDS (Zs, row
                    // stride 4 KS + 1, zero beyond 2n) and serves all its Y blocks
                    const int ZS = 4 * KS + 1;
                    for (int rb = 0; rb < TB; ++rb) {
                        for (int idx = tid; idx < 32 * 4 * KS; idx += CONT_THREADS) {
                            const int rr = idx / (4 * KS), sc = idx - rr * (4 * KS);
                            Zs[rr * ZS + sc] = zget(32 * rb + rr, sc);
                        }
                        __syncthreads();
                        for (int cb = wid; cb < TB; cb += CONT_THREADS / 64)
                            yblock(rb, cb, [&](int r, int sidx) { return Zs[(r - 32 * rb) * ZS + sidx]; });
                        __syncthreads();
                    }
                }
                __syncthreads();
                for (int u = wid; u < TB * (TB + 1) / 2; u += CONT_THREADS / 64) {
                    int ib, jb;
                    upper_tile(u, ib, jb);
                    dbl4 xre[2][2], xim[2][2];
#pragma unroll
                    for (int a = 0; a < 2; ++a)
#pragma unroll
                        for (int t = 0; t < 2; ++t) xre[a][t] = xim[a][t] = dbl4{0.0, 0.0, 0.0, 0.0};
                    const int i0 = (2 * ib) * 16 + l16, i1 = i0 + 16;
                    const int c0 = (2 * jb) * 16 + l16;
#pragma unroll 2
                    for (int ks = 0; ks < KS; ++ks) {
                        const int sidx = ks * 4 + lq;
                        const bool sok = sidx < N, a0ok = sok && i0 < N, a1ok = sok && i1 < N;
                        const double a0l = Vt[a0ok ? i0 * vs + sidx : 0], a1l = Vt[a1ok ? i1 * vs + sidx : 0];
                        const double a0 = a0ok ? a0l : 0.0, a1 = a1ok ? a1l : 0.0;
                        // (columns of Y beyond 2n hold zeros written above)
                        const cplx y0l = Yp[sok ? sidx * YS + c0 : 0];
                        const cplx y1l = Yp[sok ? sidx * YS + c0 + 16 : 0];
                        const cplx y0 = sok ? y0l : cmk(0.0, 0.0);
                        const cplx y1 = sok ? y1l : cmk(0.0, 0.0);
                        xre[0][0] = mfma4(a0, y0.re, xre[0][0]);
                        xim[0][0] = mfma4(a0, y0.im, xim[0][0]);
                        xre[0][1] = mfma4(a0, y1.re, xre[0][1]);
                        xim[0][1] = mfma4(a0, y1.im, xim[0][1]);
                        xre[1][0] = mfma4(a1, y0.re, xre[1][0]);
                        xim[1][0] = mfma4(a1, y0.im, xim[1][0]);
                        xre[1][1] = mfma4(a1, y1.re, xre[1][1]);
                        xim[1][1] = mfma4(a1, y1.im, xim[1][1]);
                    }
#pragma unroll
                    for (int a = 0; a < 2; ++a)
#pragma unroll
                        for (int t = 0; t < 2; ++t) {
                            const int jj = (2 * jb + t) * 16 + l16;
#pragma unroll
                            for (int e = 0; e < 4; ++e) {
                                const int ii = (2 * ib + a) * 16 + 4 * e + lq;
                                if (ii <= jj && jj < N) {
                                    const cplx f = cmul(hw, cmul(dk[ii], dk[jj]));
                                    double add = f.re * xre[a][t][e] - f.im * xim[a][t][e];
                                    if (ii == jj) {
                                        const double dr = 1.0 / (1.0 + rp.rho * (al[ii] - 1.0));
                                        const cplx tt = cmk(0.5 * rp.rho * dr - hw.re * dk[ii].re + hw.im * dk[ii].im,
                                                            -(hw.re * dk[ii].im + hw.im * dk[ii].re));
                                        add += beta.re * tt.re - beta.im * tt.im;
                                    }
                                    rscr[ro + (long long)jj * (jj + 1) / 2 + ii] += add;
                                }
                            }
                        }
                }
                __syncthreads();
            }
            if (!BIG) {
                // Z into the packed triangle Zp over the M(w) blocks (not read
                // again for this point): Zp[j (j + 1) / 2 + i] = Z(i, j), i <= j
                // (columns j and 16T-1-j together: 16T+1 entries, two per lane)
                cplx *Zp = Md0;
                for (int j = wid; j < 8 * T; j += CONT_THREADS / 64) {
                    const int TT = 16 * T;
                    cplx zv[2];
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        const int k = lane + 64 * c;
                        const int i = k <= j ? k : k - j - 1, col = k <= j ? j : TT - 1 - j;
                        zv[c] = k <= TT ? zget(i, col) : cmk(0.0, 0.0);
                    }
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        const int k = lane + 64 * c;
                        const int i = k <= j ? k : k - j - 1, col = k <= j ? j : TT - 1 - j;
                        if (k <= TT) Zp[col * (col + 1) / 2 + i] = zv[c];
                    }
                }
                __syncthreads();
                // Column unit (jt, rows rt0..rt1-1, slot): Y(rt, jt) = Z V for each
                // row tile rt of the part, then, with Y still in the accumulators
                // (the 16x16x4 accumulator layout is the B operand layout of the
                // next product), R(it, jt) += Re[f X(it, jt)] with X = V^T Y for
                // it <= jt (+ the diagonal beta terms in slot 0), summed in the
                // wavefront's registers over the item's points.  The units split
                // the columns so that the two wavefronts of each SIMD get about
                // the same number of MFMAs.
                const int nun = adj_col_units(T);
                for (int uw = wid; uw < nun; uw += CONT_THREADS / 64) {
                    const int u = nun == CONT_THREADS / 64 && uw >= 4 ? 11 - uw : uw;
                    int jt, rt0, rt1, slot;
                    adj_col_unit(T, u, jt, rt0, rt1, slot);
                    // (V and d_k are zero beyond 2n: no operand masks)
                    const int jj = jt * 16 + l16;
                    const bool jok = jj < N;
                    const cplx dkj = dk[jj];
                    const cplx *Zp = Md0;
                    for (int rt = rt0; rt < rt1; ++rt) {
                        const int r = rt * 16 + l16;
                        dbl4 yre = {0.0, 0.0, 0.0, 0.0}, yim = {0.0, 0.0, 0.0, 0.0};
                        // four k-steps per pass with the loads first (MFMAs keep
                        // the compiler from unrolling the loop); steps past KS
                        // read inside the padding (sidx < 16 T) and add zeros
                        for (int ks0 = 0; ks0 < KS; ks0 += 4) {
                            cplx z[4];
                            double v[4];
#pragma unroll
                            for (int u = 0; u < 4; ++u) {
                                const int sidx = min((ks0 + u) * 4 + lq, 16 * T - 1);
                                const int lo = min(r, sidx), hi = max(r, sidx);
                                z[u] = Zp[hi * (hi + 1) / 2 + lo];
                                v[u] = (ks0 + u) < KS ? Vt[jj * vs + sidx] : 0.0;
                            }
#pragma unroll
                            for (int u = 0; u < 4; ++u) {
                                yre = mfma4(z[u].re, v[u], yre);
                                yim = mfma4(z[u].im, v[u], yim);
                            }
                        }
                        // Re[hw dk_i dk_j X_ij] = sum_r Re[(hw dk_i V_ri) (dk_j Y_rj)]:
                        // the column factor scales Y in its accumulators, the row
                        // factor the A operand, and the real part goes straight into
                        // R.  Rows of Y beyond 2n are zero, so the A operand there
                        // only has to be finite.
                        dbl4 ure, uim;
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            ure[e] = dkj.re * yre[e] - dkj.im * yim[e];
                            uim[e] = dkj.im * yre[e] + dkj.re * yim[e];
                        }
#pragma unroll
                        for (int it = 0; it < ADJ_TMAX; ++it) {
                            if (it > jt) continue;
                            const int i = it * 16 + l16;
                            const cplx g = cmul(hw, dk[i]);
#pragma unroll
                            for (int e = 0; e < 4; ++e) {
                                // (rows of Y from 2n on are zero: their k-steps are skipped)
                                if (rt * 16 + 4 * e >= N) continue;
                                const int rr = rt * 16 + 4 * e + lq;
                                const double av = Vt[i * vs + rr];
                                racc[it] = mfma4(g.re * av, ure[e], racc[it]);
                                racc[it] = mfma4(-g.im * av, uim[e], racc[it]);
                            }
                        }
                    }
                    if (slot == 0 && jok) {
                        // diagonal beta terms, once per point
                        const double dr = 1.0 / (1.0 + rp.rho * (al[jj] - 1.0));
                        const cplx t = cmk(0.5 * rp.rho * dr - hw.re * dkj.re + hw.im * dkj.im,
                                           -(hw.re * dkj.im + hw.im * dkj.re));
                        const double add = beta.re * t.re - beta.im * t.im;
#pragma unroll
                        for (int it = 0; it < ADJ_TMAX; ++it)
#pragma unroll
                            for (int e = 0; e < 4; ++e)
                                if (it == jt && 4 * e + lq == l16) racc[it][e] += add;
                    }
                }
                __syncthreads();
            }
        }
        if (!BIG) {
            const int nun = adj_col_units(T);
            if (wid < nun) {
                const int u = nun == CONT_THREADS / 64 && wid >= 4 ? 11 - wid : wid;
                int jt, rt0, rt1, slot;
                adj_col_unit(T, u, jt, rt0, rt1, slot);
                double *Rs = rscr + ro + (long long)slot * (N * (N + 1) / 2);
                const int jj = jt * 16 + l16;
#pragma unroll
                for (int it = 0; it < ADJ_TMAX; ++it)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int ii = it * 16 + 4 * e + lq;
                        if (it <= jt && ii <= jj && jj < N) Rs[jj * (jj + 1) / 2 + ii] = racc[it][e];
                    }
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// k_v_transpose: for each larger row (perm[0..nbig)), its eigenvectors in the
// other orientation, W[i 2n + k] = V[i][k] (Vt holds V[i][k] at k 2n + i), into
// the row's work area of the eigen-decomposition (free after it), through
// 32 x 33 LDS tiles, followed by 16 zero rows
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_v_transpose(const int *__restrict__ offsets,
                                                     const int *__restrict__ perm,
                                                     const long long *__restrict__ voff,
                                                     const double *__restrict__ vt, double *__restrict__ wv)
{
    __shared__ double tile[32][33];
    const int p = perm[blockIdx.x];
    const int N = 2 * (offsets[p + 1] - offsets[p]);
    const double *src = vt + voff[p];
    double *dst = wv + 2 * voff[p];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const int nt = (N + 31) / 32;
    for (int t = 0; t < nt * nt; ++t) {
        const int bi = t / nt, bk = t % nt;
        // src rows k = 32 bk + ..., columns i = 32 bi + ...
        for (int r = ty; r < 32; r += 8) {
            const int k = 32 * bk + r, i = 32 * bi + tx;
            tile[r][tx] = k < N && i < N ? src[(long)k * N + i] : 0.0;
        }
        __syncthreads();
        for (int r = ty; r < 32; r += 8) {
            const int i = 32 * bi + r, k = 32 * bk + tx;
            if (i < N && k < N) dst[(long)i * N + k] = tile[tx][r];
        }
        __syncthreads();
    }
    // rows 2n .. 2n + 15 zero (read by the padded k-steps of Y = Z V; inside
    // the row's 2 (2n)^2 area for 2n >= 16)
    for (int e = threadIdx.x; e < 16 * N; e += blockDim.x) dst[(long)N * N + e] = 0.0;
}

// ---------------------------------------------------------------------------
// k_adj_pairs_big: the adjoint of rows above 40 clicks at order 2.  Per contour
// point, with V read from L2 and nothing of M(w) stored:
//  1. the 16 x 16 mode blocks (I, J), I <= J, of M(w) on the matrix cores, the
//     four quadrant products x_a x_b, x_a p_b, p_a x_b, p_a p_b of a block in
//     the same accumulator positions (the forward's scheme), after the mode
//     diagonals M_aa (formed first on the vector units, into LDS);
//  2. each lane's pairs (a, b) of a block straight from those registers:
//     c_T M_TT^{-1} split into its off-diagonal 2x2 block, written once into
//     this workgroup's scratch as the block's four 16 x 16 planes of Z(w)
//     (plane (q, q') holds Z(q_a, q'_b); tile-contiguous; a diagonal block
//     holds both orders of its pairs), and its two diagonal 2x2 blocks, added
//     with the singles' terms into Z's mode diagonals in LDS;
//  3. R += Re[(w/2) d_k d_l (V^T Z V)_kl] by row blocks of Z (the 16 rows of
//     one quadrature of one mode block, gathered into LDS, double-buffered so
//     that one barrier per block suffices): each wavefront owns whole columns
//     l of R (eigen index) and, per row block, forms its 16 x 16 tiles of
//     Y = Z V in the accumulators, whose layout is the B operand layout of
//     R's rank-16 update (A = (w/2) d_k V_rk), so Y never leaves the
//     registers.  V comes from L2 in the transposed copy k_v_transpose makes
//     (a wavefront's fetch of one k-step then reads four 128-byte runs), four
//     k-steps per pass with the loads first.  A wavefront's R tiles stay in
//     registers for the point and are then added into the item's R slot (one
//     writer per entry).
// Column l-tile lt goes to wavefront T-1-lt when lt >= T-8, else to lt+16-T
// (longest-first on their MFMA counts, 2 ceil(2n/4) + 8(lt+1)): at most two
// columns per wavefront; the first column's tile kt sits in racc[kt], the
// second's in racc[16 - kt] (2T - 17 < 16 keeps them apart for 2n <= 256).
// ---------------------------------------------------------------------------
#define ADJ_PB_RMAX 17
static_assert(GBS_MAX_N_APPROX <= 128, "2n <= 256: at most 16 column tiles");
static_assert(4 * GBS_MAX_N_APPROX <= CONT_THREADS, "four threads per mode for M's mode diagonals");
// (the k-steps of Y = Z V padded to a multiple of four: 16 ceil(2n/16) + 1)
__host__ __device__ __forceinline__ int adj_pb_zs(int n) { return 16 * ((2 * n + 15) / 16) + 1; }
// alpha (2n doubles), d and rz (2n each), M's and Z's mode diagonals (3n
// each) and two 16-row blocks of Z (row stride adj_pb_zs(n)), complex
__host__ __device__ __forceinline__ int adj_pb_lds(int n)
{
    return 8 * 2 * n + 16 * (2 * 2 * n + 6 * n + 32 * adj_pb_zs(n));
}

__global__ __launch_bounds__(CONT_THREADS) void k_adj_pairs_big(
    const int *__restrict__ offsets, const long long *__restrict__ voff,
    const double *__restrict__ alpha, const double *__restrict__ vt,
    const double *__restrict__ wv, const RowPlan *__restrict__ rows, const int *__restrict__ items,
    const int *__restrict__ q_end, int *__restrict__ q_head, const cplx *__restrict__ asw,
    const long long *__restrict__ roff, double *__restrict__ rscr, cplx *__restrict__ ascr,
    long long ascr_stride, const int *__restrict__ xq)
{
    constexpr int NW = CONT_THREADS / 64;
    extern __shared__ __attribute__((aligned(16))) double sh[];
    __shared__ int s_item;
    __shared__ cplx s_g[3];
    __shared__ cplx s_wq[ADJ_QCHUNK];
    cplx *red = (cplx *)sh;  // [waves]
    double *dyn = (double *)(red + NW + 8);
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int l16 = lane & 15, lq = lane >> 4;
    cplx *Zt = ascr + blockIdx.x * ascr_stride;
    for (;;) {
        if (tid == 0) {
            // this workgroup's XCD queue first, then the others (as k_adj_contour)
            int it = -1;
            for (int d = 0; d < GBS_NXCD && it < 0; ++d) {
                const int x = (blockIdx.x + d) % GBS_NXCD;
                if (atomicAdd(&q_head[x], 0) >= q_end[x]) continue;
                const int h = atomicAdd(&q_head[x], 1);
                if (h < q_end[x]) it = xq[q_end[GBS_NXCD + x] + h];
            }
            s_item = it;
        }
        __syncthreads();
        const int item = s_item;
        __syncthreads();
        if (item < 0) break;
        const int p = items[2 * item], ch = items[2 * item + 1];
        const int o = offsets[p], n = offsets[p + 1] - o, N = 2 * n;
        const RowPlan rp = rows[p];
        const double *Vt = vt + voff[p];       // Vt[k N + i] = V[i][k]
        const double *Wv = wv + 2 * voff[p];   // Wv[i N + k] = V[i][k]
        const int TM = (n + 15) >> 4, T = (N + 15) >> 4, KS = (N + 3) >> 2, ZS = adj_pb_zs(n);
        const int KS4 = 4 * T;  // k-steps of Y = Z V, padded (Zs and W zero past 2n)
        double *al = dyn;
        cplx *dk = (cplx *)(al + N);
        cplx *rz = dk + N;
        cplx *Md0 = rz + N, *Md1 = Md0 + n, *Md2 = Md1 + n;
        cplx *Zd0 = Md2 + n, *Zd1 = Zd0 + n, *Zd2 = Zd1 + n;  // Z(x_a, x_a), Z(x_a, p_a), Z(p_a, p_a)
        cplx *Zs0 = Zd0 + 3 * n, *Zs1 = Zs0 + 16 * ZS;
        // plane (q, q') = 2 q + q' of mode block (I, J), I <= J
        auto plane = [&](int I, int J, int pl) { return Zt + ((J * (J + 1) / 2 + I) * 4 + pl) * 256; };
        const long long ro = roff[item];
        for (int e = tid; e < N * (N + 1) / 2; e += CONT_THREADS) rscr[ro + e] = 0.0;
        for (int i = tid; i < N; i += CONT_THREADS) al[i] = alpha[2 * o + i];
        // columns 2n .. 16 T - 1 of the row blocks stay zero (never gathered)
        const int padc = 16 * T - N;
        for (int idx = tid; idx < 32 * padc; idx += CONT_THREADS) {
            const int r = idx / padc, c = N + idx % padc;
            (r < 16 ? Zs0 : Zs1)[(r & 15) * ZS + c] = cmk(0.0, 0.0);
        }
        const int Qn = rp.K / 2 + 1;
        const int q0 = ch * GBS_ADJ_CHUNK_BIG, q1 = min(q0 + GBS_ADJ_CHUNK_BIG, Qn);
        if (tid < q1 - q0) s_wq[tid] = cscale(unit_root(q0 + tid, rp.K), rp.rho);
        // this wavefront's columns of R (none when negative): column c1's tile kt
        // in racc[kt], column c2's in racc[16 - kt]
        const int c1 = T - 1 - wid, c2 = wid + T - 16;

        // the four quadrant products of mode block (I, J): lane holds the pairs
        // (16 I + 4 e + lq, 16 J + l16), e = 0..3
        auto quad = [&](int I, int J, dbl4 (&qq)[4][2]) {
#pragma unroll
            for (int h = 0; h < 4; ++h) qq[h][0] = qq[h][1] = dbl4{0.0, 0.0, 0.0, 0.0};
            const int ia = 16 * I + l16, jb = 16 * J + l16;
#pragma unroll 2
            for (int ks = 0; ks < KS; ++ks) {
                const int k = ks * 4 + lq;
                const bool kok = k < N, aok = kok && ia < n, bok = kok && jb < n;
                const cplx dl = dk[kok ? k : 0];
                const double axl = Vt[aok ? k * N + ia : 0], apl = Vt[aok ? k * N + n + ia : 0];
                const double bxl = Vt[bok ? k * N + jb : 0], bpl = Vt[bok ? k * N + n + jb : 0];
                const double ax = aok ? axl : 0.0, ap = aok ? apl : 0.0;
                const double bx = bok ? bxl : 0.0, bp = bok ? bpl : 0.0;
                const double axr = ax * dl.re, axi = ax * dl.im, apr = ap * dl.re, api = ap * dl.im;
                qq[0][0] = mfma4(axr, bx, qq[0][0]);
                qq[0][1] = mfma4(axi, bx, qq[0][1]);
                qq[1][0] = mfma4(axr, bp, qq[1][0]);
                qq[1][1] = mfma4(axi, bp, qq[1][1]);
                qq[2][0] = mfma4(apr, bx, qq[2][0]);
                qq[2][1] = mfma4(api, bx, qq[2][1]);
                qq[3][0] = mfma4(apr, bp, qq[3][0]);
                qq[3][1] = mfma4(api, bp, qq[3][1]);
            }
        };
        // the pairs of block (I, J) from its quadrant products: P = M_TT, T = {a, b},
        // eliminated through M_aa (ia) and the Schur complement of b (ib);
        // c_T P^{-1} = c_T [[ia + G ib G^T, -G ib], [-ib G^T, ib]], G = ia M_ab
        // per mode block u: the pairs' contributions to Z's mode-diagonal 2x2
        // blocks, summed in a fixed order (over the block's 16 partners by a
        // butterfly of lane shuffles), 16 modes x 3 entries for the rows a of
        // block I (side 0) and for the rows b of block J (side 1)
        cplx *Zq = Zt + TM * (TM + 1) / 2 * 1024;
        auto pairs = [&](int u, int I, int J, const dbl4 (&qq)[4][2], cplx g2, cplx &bs) {
            const int b = 16 * J + l16;
            cplx *t0 = plane(I, J, 0);
            cplx sb0 = cmk(0.0, 0.0), sb1 = sb0, sb2 = sb0;  // this lane's b, over e
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int ra_ = 4 * e + lq, a = 16 * I + ra_;
                // (lanes without a pair compute on safe indices; their terms are
                // replaced by zeros, so that every lane takes part in the sums)
                const bool ok = a < b && b < n;
                const int as = ok ? a : 0, bq = ok ? b : 0;
                const cplx b00 = cmk(qq[0][0][e], qq[0][1][e]), b01 = cmk(qq[1][0][e], qq[1][1][e]);
                const cplx b10 = cmk(qq[2][0][e], qq[2][1][e]), b11 = cmk(qq[3][0][e], qq[3][1][e]);
                const cplx a00 = Md0[as], a01 = Md1[as], a11 = Md2[as];
                const cplx ra = crsqrt_p(cfnma(a01, a01, cmul(a00, a11)));
                const cplx ideta = cmul(ra, ra);
                const cplx ia00 = cmul(a11, ideta), ia11 = cmul(a00, ideta);
                const cplx ia01 = cneg(cmul(a01, ideta));
                const cplx G00 = cfma(ia00, b00, cmul(ia01, b10));
                const cplx G01 = cfma(ia00, b01, cmul(ia01, b11));
                const cplx G10 = cfma(ia01, b00, cmul(ia11, b10));
                const cplx G11 = cfma(ia01, b01, cmul(ia11, b11));
                const cplx sb00 = csub(Md0[bq], cfma(b00, G00, cmul(b10, G10)));
                const cplx sb01 = csub(Md1[bq], cfma(b00, G01, cmul(b10, G11)));
                const cplx sb11 = csub(Md2[bq], cfma(b01, G01, cmul(b11, G11)));
                const cplx rb = crsqrt_p(cfnma(sb01, sb01, cmul(sb00, sb11)));
                const cplx cp = cmul(g2, cmul(ra, rb));
                const cplx zero = cmk(0.0, 0.0);
                bs = cadd(bs, ok ? cp : zero);
                const cplx idetb = cmul(rb, rb);
                const cplx ib00 = cmul(sb11, idetb), ib11 = cmul(sb00, idetb);
                const cplx ib01 = cneg(cmul(sb01, idetb));
                // (G ib) rows: (H00, H01), (H10, H11)
                const cplx H00 = cfma(ib00, G00, cmul(ib01, G01)), H01 = cfma(ib01, G00, cmul(ib11, G01));
                const cplx H10 = cfma(ib00, G10, cmul(ib01, G11)), H11 = cfma(ib01, G10, cmul(ib11, G11));
                const cplx pa00 = cadd(ia00, cfma(H00, G00, cmul(H01, G01)));
                const cplx pa01 = cadd(ia01, cfma(H00, G10, cmul(H01, G11)));
                const cplx pa11 = cadd(ia11, cfma(H10, G10, cmul(H11, G11)));
                // row a: the 16 lanes of this lq hold a's partners b
                cplx d0 = ok ? cmul(cp, pa00) : zero, d1 = ok ? cmul(cp, pa01) : zero;
                cplx d2 = ok ? cmul(cp, pa11) : zero;
#pragma unroll
                for (int off = 1; off < 16; off <<= 1) {
                    d0 = cadd(d0, cmk(__shfl_xor(d0.re, off), __shfl_xor(d0.im, off)));
                    d1 = cadd(d1, cmk(__shfl_xor(d1.re, off), __shfl_xor(d1.im, off)));
                    d2 = cadd(d2, cmk(__shfl_xor(d2.re, off), __shfl_xor(d2.im, off)));
                }
                if (l16 == 0) {
                    cplx *q = Zq + (u * 2) * 48 + ra_ * 3;
                    q[0] = d0;
                    q[1] = d1;
                    q[2] = d2;
                }
                if (ok) {
                    sb0 = cadd(sb0, cmul(cp, ib00));
                    sb1 = cadd(sb1, cmul(cp, ib01));
                    sb2 = cadd(sb2, cmul(cp, ib11));
                    const cplx ncp = cneg(cp);
                    const cplx zxx = cmul(ncp, H00), zxp = cmul(ncp, H01), zpx = cmul(ncp, H10),
                               zpp = cmul(ncp, H11);
                    const int at = ra_ * 16 + l16;
                    t0[at] = zxx;
                    t0[256 + at] = zxp;
                    t0[512 + at] = zpx;
                    t0[768 + at] = zpp;
                    if (I == J) {
                        // Z(q_b, q'_a) = Z(q'_a, q_b)
                        const int bt = l16 * 16 + ra_;
                        t0[bt] = zxx;
                        t0[256 + bt] = zpx;
                        t0[512 + bt] = zxp;
                        t0[768 + bt] = zpp;
                    }
                }
            }
            // row b: the four lq of this l16
#pragma unroll
            for (int off = 16; off < 64; off <<= 1) {
                sb0 = cadd(sb0, cmk(__shfl_xor(sb0.re, off), __shfl_xor(sb0.im, off)));
                sb1 = cadd(sb1, cmk(__shfl_xor(sb1.re, off), __shfl_xor(sb1.im, off)));
                sb2 = cadd(sb2, cmk(__shfl_xor(sb2.re, off), __shfl_xor(sb2.im, off)));
            }
            if (lq == 0) {
                cplx *q = Zq + (u * 2 + 1) * 48 + l16 * 3;
                q[0] = sb0;
                q[1] = sb1;
                q[2] = sb2;
            }
        };
        // rows 16 I .. 16 I + 15 of quadrature qr (row block rbi = qr TM + I) of
        // Z(w) into Zs (row stride ZS, columns in quadrature-major order); rows
        // past n are zero
        auto gather_z = [&](int rbi, cplx *Zs) {
            const int qr = rbi >= TM ? 1 : 0, I = rbi - qr * TM;
            for (int idx = tid; idx < 2 * TM * 256; idx += CONT_THREADS) {
                const int cb = idx >> 8, wv = idx & 255;
                const int qc = cb >= TM ? 1 : 0, J = cb - qc * TM;
                // (below the diagonal the stored block is (J, I): walk it in its
                // own row order)
                const int r = J < I ? wv & 15 : wv >> 4, c = J < I ? wv >> 4 : wv & 15;
                const int a = 16 * I + r, b = 16 * J + c;
                if (b >= n) continue;
                cplx v = cmk(0.0, 0.0);
                if (a < n) {
                    if (J < I)
                        v = plane(J, I, 2 * qc + qr)[c * 16 + r];
                    else if (J == I && r == c)
                        v = Zd0[(qr + qc) * n + a];
                    else
                        v = plane(I, J, 2 * qr + qc)[r * 16 + c];
                }
                Zs[r * ZS + qc * n + b] = v;
            }
        };
        __syncthreads();
        for (int q = q0; q < q1; ++q) {
            const cplx w = s_wq[q - q0];
            for (int k = tid; k < N; k += CONT_THREADS) {
                const double am1 = al[k] - 1.0;
                const cplx z = cmk(fma(w.re, am1, 1.0), w.im * am1);
                const cplx r = crsqrt_p(z);
                dk[k] = cmul(r, r);
                rz[k] = r;
            }
            for (int i = tid; i < 3 * n; i += CONT_THREADS) Zd0[i] = cmk(0.0, 0.0);
            __syncthreads();
            if (wid == 0) {
                // G_0(w)/G_0(rho) = exp(log det A/2 - log G_0(rho)) prod_k z_k^{-1/2}
                cplx pr = cmk(1.0, 0.0);
                for (int k = lane; k < N; k += 64) pr = cmul(pr, rz[k]);
                pr = cmul(warp_cprod(pr), cmk(exp(0.5 * rp.logdet_a - rp.log_g_rho), 0.0));
                if (lane <= 2) s_g[lane] = cmul(asw[((long)p * 3 + lane) * GBS_QCAP + q], pr);
            }
            // M's mode-diagonal 2x2 blocks, sum_k V_ak V_bk d_k on the vector
            // units, four partial sums per mode (threads 4a .. 4a + 3)
            {
                const int a = tid >> 2, part = tid & 3;
                cplx m00 = cmk(0.0, 0.0), m01 = m00, m11 = m00;
                if (a < n) {
                    for (int k = part; k < N; k += 4) {
                        const double vx = Vt[k * N + a], vp = Vt[k * N + n + a];
                        const cplx d = dk[k];
                        const double xx = vx * vx, xp = vx * vp, pp = vp * vp;
                        m00.re = fma(xx, d.re, m00.re); m00.im = fma(xx, d.im, m00.im);
                        m01.re = fma(xp, d.re, m01.re); m01.im = fma(xp, d.im, m01.im);
                        m11.re = fma(pp, d.re, m11.re); m11.im = fma(pp, d.im, m11.im);
                    }
                }
#pragma unroll
                for (int off = 1; off < 4; off <<= 1) {
                    m00.re += __shfl_xor(m00.re, off); m00.im += __shfl_xor(m00.im, off);
                    m01.re += __shfl_xor(m01.re, off); m01.im += __shfl_xor(m01.im, off);
                    m11.re += __shfl_xor(m11.re, off); m11.im += __shfl_xor(m11.im, off);
                }
                if (a < n && part == 0) {
                    Md0[a] = m00;
                    Md1[a] = m01;
                    Md2[a] = m11;
                }
            }
            __syncthreads();
            // singles: Z_aa += c_a M_aa^{-1}, c_a = gamma_1 det(M_aa)^{-1/2}
            cplx bsum = cmk(0.0, 0.0);
            const cplx g1 = s_g[1], g2 = s_g[2];
            for (int a = tid; a < n; a += CONT_THREADS) {
                const cplx a00 = Md0[a], a01 = Md1[a], a11 = Md2[a];
                const cplx r = crsqrt_p(cfnma(a01, a01, cmul(a00, a11)));
                const cplx c = cmul(g1, r);
                bsum = cadd(bsum, c);
                const cplx cid = cmul(c, cmul(r, r));
                Zd0[a] = cmul(cid, a11);
                Zd1[a] = cneg(cmul(cid, a01));
                Zd2[a] = cmul(cid, a00);
            }
            // every mode block (I, J), I <= J: quadrant products, then its pairs
            for (int u = wid; u < TM * (TM + 1) / 2; u += NW) {
                int I, J;
                upper_tile(u, I, J);
                dbl4 qq[4][2];
                quad(I, J, qq);
                pairs(u, I, J, qq, g2, bsum);
            }
            bsum = warp_csum(bsum);
            if (lane == 0) red[wid] = bsum;
            __syncthreads();
            cplx beta = s_g[0];
            for (int i = 0; i < NW; ++i) beta = cadd(beta, red[i]);
            const cplx hw = cscale(w, 0.5);
            // Z's mode diagonals: the singles' terms plus the pairs' partial sums
            // of every mode block holding the mode, in a fixed order (so the sum
            // does not depend on the order the wavefronts ran in)
            for (int a = tid; a < n; a += CONT_THREADS) {
                const int Ia = a >> 4, la = a & 15;
                cplx z0 = Zd0[a], z1 = Zd1[a], z2 = Zd2[a];
                for (int J = Ia; J < TM; ++J) {
                    const cplx *q = Zq + ((J * (J + 1) / 2 + Ia) * 2) * 48 + la * 3;
                    z0 = cadd(z0, q[0]);
                    z1 = cadd(z1, q[1]);
                    z2 = cadd(z2, q[2]);
                }
                for (int I = 0; I <= Ia; ++I) {
                    const cplx *q = Zq + ((Ia * (Ia + 1) / 2 + I) * 2 + 1) * 48 + la * 3;
                    z0 = cadd(z0, q[0]);
                    z1 = cadd(z1, q[1]);
                    z2 = cadd(z2, q[2]);
                }
                Zd0[a] = z0;
                Zd1[a] = z1;
                Zd2[a] = z2;
            }
            __syncthreads();
            dbl4 racc[ADJ_PB_RMAX];
#pragma unroll
            for (int t = 0; t < ADJ_PB_RMAX; ++t) racc[t] = dbl4{0.0, 0.0, 0.0, 0.0};
            const int l1 = 16 * c1 + l16, l2 = 16 * c2 + l16;
            const bool l1ok = c1 >= 0 && l1 < N, l2ok = c2 >= 0 && l2 < N;
            const cplx dl1 = l1ok ? dk[l1] : cmk(0.0, 0.0), dl2 = l2ok ? dk[l2] : cmk(0.0, 0.0);
            gather_z(0, Zs0);
            __syncthreads();
            for (int rbi = 0; rbi < 2 * TM; ++rbi) {
                const cplx *Zs = (rbi & 1) ? Zs1 : Zs0;
                if (rbi + 1 < 2 * TM) gather_z(rbi + 1, (rbi & 1) ? Zs0 : Zs1);
                const int qr = rbi >= TM ? 1 : 0, I = rbi - qr * TM;
                const int rbase = qr * n + 16 * I, nrow = min(16, n - 16 * I);
                if (c1 >= 0) {
                    // Y(rows of the block, column tiles c1 and c2) = Z V over the
                    // padded k-steps (Zs and W are zero past 2n; W's columns
                    // past 2n hold finite values, met by d_l = 0 below)
                    dbl4 y1r = {0.0, 0.0, 0.0, 0.0}, y1i = y1r, y2r = y1r, y2i = y1r;
                    const double *w1 = Wv + lq * N + 16 * c1 + l16;
                    const cplx *zrow = Zs + l16 * ZS + lq;
                    if (c2 >= 0) {
                        const double *w2 = Wv + lq * N + 16 * c2 + l16;
                        for (int ks0 = 0; ks0 < KS4; ks0 += 4) {
                            cplx z[4];
                            double v1[4], v2[4];
#pragma unroll
                            for (int u = 0; u < 4; ++u) {
                                z[u] = zrow[4 * (ks0 + u)];
                                v1[u] = w1[(long)4 * (ks0 + u) * N];
                                v2[u] = w2[(long)4 * (ks0 + u) * N];
                            }
#pragma unroll
                            for (int u = 0; u < 4; ++u) {
                                y1r = mfma4(z[u].re, v1[u], y1r);
                                y1i = mfma4(z[u].im, v1[u], y1i);
                                y2r = mfma4(z[u].re, v2[u], y2r);
                                y2i = mfma4(z[u].im, v2[u], y2i);
                            }
                        }
                    } else {
                        // one column: even and odd k-steps in separate
                        // accumulators (four independent chains), summed after
                        for (int ks0 = 0; ks0 < KS4; ks0 += 4) {
                            cplx z[4];
                            double v1[4];
#pragma unroll
                            for (int u = 0; u < 4; ++u) {
                                z[u] = zrow[4 * (ks0 + u)];
                                v1[u] = w1[(long)4 * (ks0 + u) * N];
                            }
#pragma unroll
                            for (int u = 0; u < 4; u += 2) {
                                y1r = mfma4(z[u].re, v1[u], y1r);
                                y1i = mfma4(z[u].im, v1[u], y1i);
                                y2r = mfma4(z[u + 1].re, v1[u + 1], y2r);
                                y2i = mfma4(z[u + 1].im, v1[u + 1], y2i);
                            }
                        }
                        y1r += y2r;
                        y1i += y2i;
                        y2r = y2i = dbl4{0.0, 0.0, 0.0, 0.0};
                    }
                    // column factor d_l into Y: B = d_l Y_rl
                    dbl4 b1r, b1i, b2r, b2i;
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        b1r[e] = dl1.re * y1r[e] - dl1.im * y1i[e];
                        b1i[e] = dl1.im * y1r[e] + dl1.re * y1i[e];
                        b2r[e] = dl2.re * y2r[e] - dl2.im * y2i[e];
                        b2i[e] = dl2.im * y2r[e] + dl2.re * y2i[e];
                    }
                    // R(kt, l) += Re[(g_k V_rk) B_rl], g_k = (w/2) d_k, for the
                    // tiles kt <= l, two row tiles kt, kt + 1 at a time so that
                    // up to four accumulators interleave.  V's block rows come
                    // from the transposed copy unmasked: rows past the block's
                    // end meet zero rows of Y, columns past 2n a zero g_k.
                    const double *wa = Wv + (long)(rbase + lq) * N + l16;
#pragma unroll
                    for (int kt = 0; kt < 16; kt += 2) {
                        if (kt > c1) continue;
                        double ar0[4], ai0[4], ar1[4], ai1[4];
                        {
                            const int k0 = 16 * kt + l16, k1 = k0 + 16;
                            const cplx g0 = k0 < N ? cmul(hw, dk[k0]) : cmk(0.0, 0.0);
                            const cplx g1 = k1 < N ? cmul(hw, dk[k1]) : cmk(0.0, 0.0);
#pragma unroll
                            for (int e = 0; e < 4; ++e) {
                                const double v0 = wa[(long)4 * e * N + 16 * kt];
                                const double v1 = wa[(long)4 * e * N + 16 * kt + 16];
                                ar0[e] = g0.re * v0;
                                ai0[e] = -g0.im * v0;
                                ar1[e] = g1.re * v1;
                                ai1[e] = -g1.im * v1;
                            }
                        }
                        auto upd = [&](auto U1, auto V0, auto V1) {
#pragma unroll
                            for (int e = 0; e < 4; ++e) {
                                racc[kt] = mfma4(ar0[e], b1r[e], racc[kt]);
                                if constexpr (decltype(U1)::value) racc[kt + 1] = mfma4(ar1[e], b1r[e], racc[kt + 1]);
                                if constexpr (decltype(V0)::value) racc[16 - kt] = mfma4(ar0[e], b2r[e], racc[16 - kt]);
                                if constexpr (decltype(V1)::value) racc[15 - kt] = mfma4(ar1[e], b2r[e], racc[15 - kt]);
                                racc[kt] = mfma4(ai0[e], b1i[e], racc[kt]);
                                if constexpr (decltype(U1)::value) racc[kt + 1] = mfma4(ai1[e], b1i[e], racc[kt + 1]);
                                if constexpr (decltype(V0)::value) racc[16 - kt] = mfma4(ai0[e], b2i[e], racc[16 - kt]);
                                if constexpr (decltype(V1)::value) racc[15 - kt] = mfma4(ai1[e], b2i[e], racc[15 - kt]);
                            }
                        };
                        using T_ = std::true_type;
                        using F_ = std::false_type;
                        // (kt <= c2 implies kt + 1 <= c1, as c2 < c1)
                        if (kt + 1 > c1)
                            upd(F_{}, F_{}, F_{});
                        else if (kt > c2)
                            upd(T_{}, F_{}, F_{});
                        else if (kt + 1 > c2)
                            upd(T_{}, T_{}, F_{});
                        else
                            upd(T_{}, T_{}, T_{});
                    }
                }
                __syncthreads();
            }
            // this wavefront's R tiles (+ the diagonal beta terms) into the item's slot
#pragma unroll 1
            for (int s = 0; s < 2; ++s) {
                const int lt = s == 0 ? c1 : c2;
                if (lt < 0) continue;
                const int jj = 16 * lt + l16;
#pragma unroll
                for (int t = 0; t < ADJ_PB_RMAX; ++t) {
                    const int kt = s == 0 ? t : 16 - t;
                    if (kt < 0 || kt > lt) continue;
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int ii = 16 * kt + 4 * e + lq;
                        if (ii > jj || jj >= N) continue;
                        double add = racc[t][e];
                        if (ii == jj) {
                            const double dr = 1.0 / (1.0 + rp.rho * (al[ii] - 1.0));
                            const cplx tt = cmk(0.5 * rp.rho * dr - hw.re * dk[ii].re + hw.im * dk[ii].im,
                                                -(hw.re * dk[ii].im + hw.im * dk[ii].re));
                            add += beta.re * tt.re - beta.im * tt.im;
                        }
                        rscr[ro + (long long)jj * (jj + 1) / 2 + ii] += add;
                    }
                }
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// k_adj_items: backward work items (row, chunk of ADJ_QCHUNK points) and the
// offsets of their R scratch
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_adj_items(int P, int nbig, const int *__restrict__ offsets,
                                                    const int *__restrict__ perm,
                                                    const RowPlan *__restrict__ rows,
                                                    int *__restrict__ items, long long *__restrict__ roff,
                                                    int *__restrict__ row_item0, int *__restrict__ counter,
                                                    int *__restrict__ xq)
{
    __shared__ int part[1024];
    __shared__ long long lpart[1024];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int per = (P + nt - 1) / nt;
    const int b = tid * per, e = min(P, b + per);
    auto nch = [&](int i) {
        const int p = perm[i];
        const int n = offsets[p + 1] - offsets[p];
        const RowPlan &rp = rows[p];
        if (n == 0 || rp.status != 0 || rp.K <= 0) return 0;
        const int qc = n > GBS_NSMALL ? GBS_ADJ_CHUNK_BIG : ADJ_QCHUNK;
        return (rp.K / 2 + 1 + qc - 1) / qc;
    };
    auto rsz = [&](int i) {
        const int p = perm[i];
        const int n = offsets[p + 1] - offsets[p];
        const long long N = 2 * n;
        return (n > GBS_NSMALL ? 1 : ADJ_RSLOTS) * (N * (N + 1) / 2);
    };
    __shared__ int s_big;
    if (tid == 0) s_big = 0;
    int s = 0, sb = 0;
    long long ls = 0;
    for (int i = b; i < e; ++i) {
        s += nch(i);
        if (i < nbig) sb += nch(i);
        ls += nch(i) * rsz(i);
    }
    part[tid] = s;
    lpart[tid] = ls;
    __syncthreads();
    if (sb) atomicAdd(&s_big, sb);
    if (tid == 0) {
        int acc = 0;
        long long lacc = 0;
        for (int t = 0; t < nt; ++t) {
            int v = part[t];
            long long lv = lpart[t];
            part[t] = acc;
            lpart[t] = lacc;
            acc += v;
            lacc += lv;
        }
        counter[2] = acc;
    }
    __syncthreads();
    if (tid == 0) {
        // items of perm[0..nbig) (the large rows) first: their own queue [6] / [7]
        counter[3] = s_big;
        counter[6] = s_big;
        counter[7] = 0;
    }
    int off = part[tid];
    long long loff = lpart[tid];
    for (int i = b; i < e; ++i) {
        const int c = nch(i), p = perm[i];
        const long long sz = rsz(i);
        row_item0[p] = c > 0 ? off : -1;
        for (int k = 0; k < c; ++k) {
            items[2 * (off + k)] = p;
            items[2 * (off + k) + 1] = k;
            roff[off + k] = loff + k * sz;
        }
        off += c;
        loff += c * sz;
    }
    // the larger rows' items by XCD queue: row i (in plan order) to queue
    // i % GBS_NXCD, its chunks together, rows in plan order (largest first)
    __shared__ int xcnt[GBS_NXCD];
    __syncthreads();
    if (tid < GBS_NXCD) {
        int c = 0;
        for (int i = tid; i < nbig; i += GBS_NXCD) c += nch(i);
        xcnt[tid] = c;
    }
    __syncthreads();
    if (tid < GBS_NXCD) {
        int o = 0;
        for (int x = 0; x < tid; ++x) o += xcnt[x];
        counter[8 + tid] = 0;
        counter[8 + GBS_NXCD + tid] = xcnt[tid];
        counter[8 + 2 * GBS_NXCD + tid] = o;
        for (int i = tid; i < nbig; i += GBS_NXCD) {
            const int c = nch(i), i0 = row_item0[perm[i]];
            for (int k = 0; k < c; ++k) xq[o++] = i0 + k;
        }
    }
}

// ---------------------------------------------------------------------------
// Psi accumulation.  mode 0: floating-point atomics (the order of the adds,
// and so the last bits, vary from run to run).  Deterministic gradients run
// the reduction twice: mode 1 only records the largest |term| (its bit
// pattern, which orders non-negative doubles; NaN above every number), mode 2
// adds the terms as 64-bit integers at the power-of-two scale k_det_scale
// derived from it; k_det_to_double converts Psi back.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void psi_add(double *dst, double s, int mode, unsigned long long *det)
{
    if (mode == 0) {
        atomicAdd(dst, s);
    } else if (mode == 1) {
        atomicMax(det, (unsigned long long)__double_as_longlong(fabs(s)));
    } else {
        atomicAdd((unsigned long long *)dst, (unsigned long long)llrint(s * __longlong_as_double((long long)det[1])));
    }
}

// det[1] = the scale for at most nterm terms per entry (0 when a term was
// not finite)
__global__ void k_det_scale(unsigned long long *det, int nterm)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double m = __longlong_as_double((long long)det[0]);
    double sc = 1.0;
    if (!(m <= DBL_MAX)) {
        sc = 0.0;
    } else if (m > 0.0) {
        int e = 0;
        frexp(m, &e);
        sc = ldexp(1.0, 61 - ilogb((double)nterm) - e);  // (the sum stays below 2^62)
    }
    det[1] = (unsigned long long)__double_as_longlong(sc);
}

__global__ void k_det_to_double(long n, double *x, const unsigned long long *det)
{
    const double sc = __longlong_as_double((long long)det[1]);
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const long long v = *(const long long *)&x[i];
        x[i] = sc > 0.0 ? (double)v / sc : NAN;
    }
}

// ---------------------------------------------------------------------------
// k_adj_reduce: per row, R = sum of the items' R (fixed order) plus the
// contour-independent diagonal term of log G_0(rho) and log P_vac(Cbar)
// (their A^{-1} parts cancel, leaving -w_p rho/2 M(rho)), then A_bar = V R V^T,
// added into Psi at the row's mode pairs: Psi[u][v] = sum over rows holding
// both modes of A_bar at their positions (global fp64 atomics; Psi cleared
// before the launch).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_adj_reduce(int M, const int *__restrict__ offsets,
                                                    const int *__restrict__ modes,
                                                    const long long *__restrict__ voff,
                                                    const double *__restrict__ alpha,
                                                    const double *__restrict__ vt,
                                                    const RowPlan *__restrict__ rows,
                                                    const double *__restrict__ dl,
                                                    const int *__restrict__ status,
                                                    const int *__restrict__ row_item0,
                                                    const long long *__restrict__ roff,
                                                    const double *__restrict__ rscr,
                                                    double *__restrict__ psi, int mode,
                                                    unsigned long long *__restrict__ det)
{
    extern __shared__ __attribute__((aligned(16))) double sh[];
    const int p = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
    const int o = offsets[p], n = offsets[p + 1] - o, N = 2 * n;
    const RowPlan rp = rows[p];
    const long long vo = voff[p];
    if (n == 0 || n > GBS_NSMALL) return;
    const int it0 = row_item0[p];
    if (it0 < 0 || rp.status != 0 || (status[p] & GBS_PS_FAILED) || !isfinite(dl[p]) || dl[p] == 0.0) return;
    const int nit = (rp.K / 2 + 1 + ADJ_QCHUNK - 1) / ADJ_QCHUNK;
    double *V = sh;            // V[i][k] row-major
    double *R = V + N * N;     // full symmetric
    double *T = R + N * N;
    int *g = (int *)(T + N * N);   // global index of the row's local index
    for (int idx = tid; idx < N * N; idx += nt) {
        const int k = idx / N, i = idx - k * N;
        V[i * N + k] = vt[vo + idx];
    }
    for (int i = tid; i < N; i += nt) g[i] = modes[o + (i < n ? i : i - n)] + (i < n ? 0 : M);
    const int nup = N * (N + 1) / 2;
    for (int e = tid; e < nup; e += nt) {
        int i, j;
        upper_ij(e, i, j);
        double s = 0.0;
        for (int it = 0; it < nit; ++it)
            for (int sl = 0; sl < ADJ_RSLOTS; ++sl) s += rscr[roff[it0 + it] + (long long)sl * nup + e];
        if (i == j) {
            const double dr = 1.0 / (1.0 + rp.rho * (alpha[2 * o + i] - 1.0));
            s += -0.5 * dl[p] * rp.rho * dr;
        }
        R[i * N + j] = s;
        R[j * N + i] = s;
    }
    __syncthreads();
    // T = R V^T, A_bar = V T
    for (int idx = tid; idx < N * N; idx += nt) {
        const int k = idx / N, j = idx - k * N;
        double s = 0.0;
        for (int l = 0; l < N; ++l) s = fma(R[k * N + l], V[j * N + l], s);
        T[k * N + j] = s;
    }
    __syncthreads();
    const long D = 2L * M;
    for (int idx = tid; idx < N * N; idx += nt) {
        const int i = idx / N, j = idx - i * N;
        double s = 0.0;
        for (int k = 0; k < N; ++k) s = fma(V[i * N + k], T[k * N + j], s);
        psi_add(psi + g[i] * D + g[j], s, mode, det);
    }
}

// k_adj_reduce for the larger rows (perm[0..nbig)): R and T = R V^T in HBM
// scratch (2 N^2 per row), A_bar = V T added into Psi.
__global__ __launch_bounds__(256) void k_adj_reduce_big(int M, const int *__restrict__ offsets,
                                                        const int *__restrict__ modes,
                                                        const int *__restrict__ perm,
                                                        const long long *__restrict__ voff,
                                                        const double *__restrict__ alpha,
                                                        const double *__restrict__ vt,
                                                        const RowPlan *__restrict__ rows,
                                                        const double *__restrict__ dl,
                                                        const int *__restrict__ status,
                                                        const int *__restrict__ row_item0,
                                                        const long long *__restrict__ roff,
                                                        const double *__restrict__ rscr,
                                                        double *__restrict__ wbig,
                                                        double *__restrict__ psi, int mode,
                                                        unsigned long long *__restrict__ det)
{
    __shared__ int g[2 * GBS_MAX_N_APPROX];
    const int p = perm[blockIdx.x], tid = threadIdx.x, nt = blockDim.x;
    const int o = offsets[p], n = offsets[p + 1] - o, N = 2 * n;
    const RowPlan rp = rows[p];
    const int it0 = row_item0[p];
    if (n == 0 || it0 < 0 || rp.status != 0 || (status[p] & GBS_PS_FAILED) || !isfinite(dl[p]) ||
        dl[p] == 0.0)
        return;
    const int nit = (rp.K / 2 + 1 + GBS_ADJ_CHUNK_BIG - 1) / GBS_ADJ_CHUNK_BIG;
    const long long vo = voff[p];
    const double *Vt = vt + vo;          // Vt[k*N + i] = V[i][k]
    double *R = wbig + 2 * vo, *T = R + (long)N * N;
    for (int i = tid; i < N; i += nt) g[i] = modes[o + (i < n ? i : i - n)] + (i < n ? 0 : M);
    const int nup = N * (N + 1) / 2;
    for (int e = tid; e < nup; e += nt) {
        int i, j;
        upper_ij(e, i, j);
        double s = 0.0;
        for (int it = 0; it < nit; ++it) s += rscr[roff[it0 + it] + e];
        if (i == j) {
            const double dr = 1.0 / (1.0 + rp.rho * (alpha[2 * o + i] - 1.0));
            s += -0.5 * dl[p] * rp.rho * dr;
        }
        R[(long)i * N + j] = s;
        R[(long)j * N + i] = s;
    }
    __syncthreads();
    for (int idx = tid; idx < N * N; idx += nt) {
        const int k = idx / N, j = idx - k * N;
        double s = 0.0;
        for (int l = 0; l < N; ++l) s = fma(R[(long)k * N + l], Vt[(long)l * N + j], s);
        T[idx] = s;
    }
    __syncthreads();
    const long D = 2L * M;
    for (int idx = tid; idx < N * N; idx += nt) {
        const int i = idx / N, j = idx - i * N;
        double s = 0.0;
        for (int k = 0; k < N; ++k) s = fma(Vt[(long)k * N + i], T[(long)k * N + j], s);
        psi_add(psi + g[i] * D + g[j], s, mode, det);
    }
}

// Model adjoint, one workgroup: Q_bar = -(W/2) Q^{-1} - Q^{-1} Psi Q^{-1} with W the
// sum of w_p over rows with a result; sigma_bar = Q_bar; then through
// sigma = D sigma0 D + (I - D^2)/2 and sigma0 = O diag(e^{-2r}, e^{2r}) O^T / 2.
__global__ __launch_bounds__(1024) void k_adj_model(int M, int P, const double *__restrict__ qi,
                                                    const double *__restrict__ params,
                                                    const double *__restrict__ dl,
                                                    const int *__restrict__ status,
                                                    double *__restrict__ psi, double *__restrict__ tmp,
                                                    double *__restrict__ grad)
{
    __shared__ double red[1024];
    const int D = 2 * M, tid = threadIdx.x, nt = blockDim.x;
    const double *ure = params, *uim = params + (long)M * M;
    const double *r = params + 2L * M * M, *eta = r + M;
    double ws = 0.0;
    for (int p = tid; p < P; p += nt)
        if ((status[p] & GBS_PS_FAILED) == 0 && isfinite(dl[p])) ws += dl[p];
    ws = block_sum(ws, red);
    // tmp = Psi Q^{-1}
    for (int idx = tid; idx < D * D; idx += nt) {
        const int i = idx / D, j = idx - i * D;
        double s = 0.0;
        for (int k = 0; k < D; ++k) s = fma(psi[(long)i * D + k], qi[(long)k * D + j], s);
        tmp[idx] = s;
    }
    __syncthreads();
    // psi <- sigma_bar = -(W/2) Q^{-1} - Q^{-1} tmp
    for (int idx = tid; idx < D * D; idx += nt) {
        const int i = idx / D, j = idx - i * D;
        double s = 0.0;
        for (int k = 0; k < D; ++k) s = fma(qi[(long)i * D + k], tmp[(long)k * D + j], s);
        psi[idx] = -0.5 * ws * qi[idx] - s;
    }
    __syncthreads();
    auto O = [&](int i, int k) {
        if (i < M) return k < M ? ure[i * M + k] : -uim[i * M + k - M];
        return k < M ? uim[(i - M) * M + k] : ure[(i - M) * M + k - M];
    };
    auto sq = [&](int i) { return sqrt(eta[i % M]); };
    // tmp = sigma0_bar O with sigma0_bar = D sigma_bar D
    for (int idx = tid; idx < D * D; idx += nt) {
        const int i = idx / D, k = idx - i * D;
        double s = 0.0;
        for (int j = 0; j < D; ++j) s = fma(psi[(long)i * D + j] * sq(j), O(j, k), s);
        tmp[idx] = sq(i) * s;
    }
    __syncthreads();
    // r_bar_j = -e^{-2 r_j} (O^T sigma0_bar O)_{jj} + e^{2 r_j} (O^T sigma0_bar O)_{M+j,M+j}
    for (int j = tid; j < M; j += nt) {
        double bx = 0.0, bp = 0.0;
        for (int i = 0; i < D; ++i) {
            bx = fma(O(i, j), tmp[(long)i * D + j], bx);
            bp = fma(O(i, M + j), tmp[(long)i * D + M + j], bp);
        }
        grad[j] = -exp(-2.0 * r[j]) * bx + exp(2.0 * r[j]) * bp;
    }
    __syncthreads();
    // eta_bar_m = (1/eta_m) sum_{i in quads(m)} sum_j sigma0_bar_ij sigma0_ij
    //             - (sigma_bar_{m,m} + sigma_bar_{M+m,M+m}) / 2,
    // with sum_j sigma0_bar_ij sigma0_ij = sum_k O_ik (lambda_k / 2) (sigma0_bar O)_ik,
    // lambda = (e^{-2r}, e^{2r})
    for (int m = tid; m < M; m += nt) {
        double s = 0.0;
        for (int qd = 0; qd < 2; ++qd) {
            const int i = m + qd * M;
            for (int k = 0; k < M; ++k) {
                s = fma(O(i, k) * (0.5 * exp(-2.0 * r[k])), tmp[(long)i * D + k], s);
                s = fma(O(i, M + k) * (0.5 * exp(2.0 * r[k])), tmp[(long)i * D + M + k], s);
            }
        }
        grad[M + m] = s / eta[m] - 0.5 * (psi[(long)m * D + m] + psi[(long)(M + m) * D + M + m]);
    }
}

__global__ void k_zero(long n, double *x)
{
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        x[i] = 0.0;
}

}  // namespace
long long adj_pair_scratch(int n);
namespace {

template <int ORDER>
int backward_order(gbs_ctx *ctx, gbs_plan *pl, const double *dl, const int32_t *status,
                   double *grad_r, double *grad_eta)
{
    hipStream_t st = ctx->stream;
    DevModel &m = ctx->model;
    const int P = pl->P, nmax = pl->max_n, M = m.M;
    size_t lds_f = sizeof(cplx) * (GBS_KMAX + GBS_KMAX / 2);
    if (int rc = func_lds_limit(ctx, (const void *)k_adj_fit<ORDER>, (int)lds_f)) return rc;
    int ts = timer_begin(ctx, TG_ADJ_FIT);
    hipLaunchKernelGGL(k_adj_fit<ORDER>, dim3(P), dim3(FIT_THREADS), lds_f, st, pl->d_offsets,
                       pl->d_rows, pl->d_sw, dl, status, pl->d_asw);
    timer_end(ctx, ts);
    ts = timer_begin(ctx, TG_ADJ_CLUSTER);
    hipLaunchKernelGGL(k_adj_items, dim3(1), dim3(1024), 0, st, P, pl->nbig, pl->d_offsets, pl->d_perm,
                       pl->d_rows, pl->d_aitems, pl->d_roff, pl->d_ritem0, pl->d_counter, pl->d_axq);
    if constexpr (ORDER == 2) {
        if (pl->nbig > 0) {
            // larger rows at order 2: M(w) never stored, the pair blocks of Z(w) in
            // this workgroup's scratch, 16-row blocks of Z(w) in LDS
            const void *fn = (const void *)k_adj_pairs_big;
            int lds_static = 0;
            if (int rc = func_static_lds(ctx, fn, &lds_static)) return rc;
            const int lds_b = adj_fixed() + adj_pb_lds(nmax);
            if (lds_b + lds_static > ctx->lds_per_block)
                return set_err(ctx, GBS_E_INVAL, "rows too large for the gradient kernel's LDS");
            if (adj_pair_scratch(nmax) > pl->ascr_stride)
                return set_err(ctx, GBS_E_INVAL, "gradient scratch smaller than the rows need");
            int occ = 1;
            if (int rc = func_lds_limit(ctx, fn, lds_b)) return rc;
            if (int rc = func_occupancy(ctx, fn, CONT_THREADS, lds_b, &occ)) return rc;
            int grid = std::min(occ * ctx->num_cu, pl->ascr_blocks);
            hipLaunchKernelGGL(k_v_transpose, dim3(pl->nbig), dim3(256), 0, st, pl->d_offsets, pl->d_perm,
                               pl->d_voff, pl->d_v, pl->d_wbig);
            hipLaunchKernelGGL(k_adj_pairs_big, dim3(grid), dim3(CONT_THREADS), lds_b, st, pl->d_offsets,
                               pl->d_voff, pl->d_alpha, pl->d_v, pl->d_wbig, pl->d_rows, pl->d_aitems,
                               pl->d_counter + 8 + GBS_NXCD, pl->d_counter + 8, pl->d_asw, pl->d_roff,
                               pl->d_rscr, pl->d_ascr, pl->ascr_stride, pl->d_axq);
        }
    } else if (pl->nbig > 0) {
        // larger rows: V and M(w) in HBM, Z(w) (all of it at order 3, its diagonal
        // blocks and a 32-row block of it otherwise) in LDS
        const bool det = ctx->deterministic;
        const void *fn = det ? (const void *)k_adj_contour<ORDER, true, true>
                             : (const void *)k_adj_contour<ORDER, true, false>;
        int lds_static = 0;
        if (int rc = func_static_lds(ctx, fn, &lds_static)) return rc;
        const int nb = nmax, npb = nb * (nb - 1) / 2;
        const int lds_b = adj_fixed() + 8 * 2 * nb + 16 * 2 * 2 * nb + 16 * 3 * nb +
                          (ORDER >= 3 ? 16 * 4 * npb : 16 * 32 * (4 * ((2 * nb + 3) / 4) + 1));
        if (lds_b + lds_static > ctx->lds_per_block)
            return set_err(ctx, GBS_E_INVAL, "rows too large for the gradient kernel's LDS");
        int occ = 1;
        if (int rc = func_lds_limit(ctx, fn, lds_b)) return rc;
        if (int rc = func_occupancy(ctx, fn, CONT_THREADS, lds_b, &occ)) return rc;
        int grid = std::min(occ * ctx->num_cu, pl->ascr_blocks);
        hipLaunchKernelGGL((det ? k_adj_contour<ORDER, true, true> : k_adj_contour<ORDER, true, false>),
                           dim3(grid), dim3(CONT_THREADS), lds_b, st,
                           pl->d_offsets, pl->d_voff, pl->d_alpha, pl->d_v, pl->d_rows, pl->d_aitems,
                           pl->d_counter + 8 + GBS_NXCD, pl->d_counter + 8,
                           pl->d_cluster_items, pl->d_cluster_off + 2 * (pl->max_n + 1),
                           pl->order >= 4 ? pl->d_cluster_off + 4 * (pl->max_n + 1) : nullptr, pl->d_asw,
                           pl->d_roff, pl->d_rscr, pl->d_ascr, pl->ascr_stride, pl->d_axq);
    }
    const int ns = pl->max_n_small;
    if (pl->nbig < P) {
        const bool det = ctx->deterministic;
        const void *fn = det ? (const void *)k_adj_contour<ORDER, false, true>
                             : (const void *)k_adj_contour<ORDER, false, false>;
        int lds_static = 0;
        if (int rc = func_static_lds(ctx, fn, &lds_static)) return rc;
        int lds_a = 0;
        for (int k = 1; k <= ns; ++k) lds_a = std::max(lds_a, adj_need(k));
        lds_a += adj_fixed();
        if (lds_a + lds_static > ctx->lds_per_block)
            return set_err(ctx, GBS_E_INVAL, "rows too large for the gradient kernel's LDS");
        int occ = 1;
        if (int rc = func_lds_limit(ctx, fn, lds_a)) return rc;
        if (int rc = func_occupancy(ctx, fn, CONT_THREADS, lds_a, &occ)) return rc;
        hipLaunchKernelGGL((det ? k_adj_contour<ORDER, false, true> : k_adj_contour<ORDER, false, false>),
                           dim3(occ * ctx->num_cu), dim3(CONT_THREADS),
                           lds_a, st, pl->d_offsets, pl->d_voff, pl->d_alpha, pl->d_v, pl->d_rows,
                           pl->d_aitems, pl->d_counter + 2, pl->d_counter + 3,
                           pl->d_cluster_items, pl->d_cluster_off + 2 * (pl->max_n + 1),
                           pl->order >= 4 ? pl->d_cluster_off + 4 * (pl->max_n + 1) : nullptr, pl->d_asw,
                           pl->d_roff, pl->d_rscr, (cplx *)nullptr, 0LL, (const int *)nullptr);
    }
    timer_end(ctx, ts);
    ts = timer_begin(ctx, TG_ADJ_ROWS);
    const int D = 2 * M;
    hipLaunchKernelGGL(k_zero, dim3((D * D + 255) / 256), dim3(256), 0, st, (long)D * D, pl->d_qibar);
    // deterministic gradients: the reduction twice (largest term, then the
    // terms as integers at the scale it fixes), Psi then back to doubles
    const bool det = ctx->deterministic;
    if (det) hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, st, 2L, (double *)pl->d_det);
    for (int mode = det ? 1 : 0; mode <= (det ? 2 : 0); ++mode) {
        if (mode == 2) hipLaunchKernelGGL(k_det_scale, dim3(1), dim3(64), 0, st, pl->d_det, P);
        if (pl->nbig < P) {
            const int N = 2 * ns;
            size_t lds_r = sizeof(double) * 3 * (size_t)N * N + sizeof(int) * N;
            if (int rc = func_lds_limit(ctx, (const void *)k_adj_reduce, (int)lds_r)) return rc;
            hipLaunchKernelGGL(k_adj_reduce, dim3(P), dim3(256), lds_r, st, M, pl->d_offsets, pl->d_modes,
                               pl->d_voff, pl->d_alpha, pl->d_v, pl->d_rows, dl, status, pl->d_ritem0,
                               pl->d_roff, pl->d_rscr, pl->d_qibar, mode, pl->d_det);
        }
        if (pl->nbig > 0)
            hipLaunchKernelGGL(k_adj_reduce_big, dim3(pl->nbig), dim3(256), 0, st, M, pl->d_offsets,
                               pl->d_modes, pl->d_perm, pl->d_voff, pl->d_alpha, pl->d_v, pl->d_rows, dl,
                               status, pl->d_ritem0, pl->d_roff, pl->d_rscr, pl->d_wbig, pl->d_qibar, mode,
                               pl->d_det);
    }
    if (det)
        hipLaunchKernelGGL(k_det_to_double, dim3((D * D + 255) / 256), dim3(256), 0, st, (long)D * D,
                           pl->d_qibar, pl->d_det);
    timer_end(ctx, ts);
    ts = timer_begin(ctx, TG_ADJ_MODEL);
    hipLaunchKernelGGL(k_adj_model, dim3(1), dim3(1024), 0, st, M, P, m.qi_hi, m.params, dl,
                       status, pl->d_qibar, pl->d_qitmp, pl->d_grad);
    timer_end(ctx, ts);
    HIP_TRY(ctx, hipMemcpyAsync(grad_r, pl->d_grad, M * sizeof(double), hipMemcpyDeviceToDevice, st));
    HIP_TRY(ctx, hipMemcpyAsync(grad_eta, pl->d_grad + M, M * sizeof(double), hipMemcpyDeviceToDevice, st));
    HIP_TRY(ctx, hipGetLastError());
    return 0;
}

}  // namespace

int adj_workspace(gbs_ctx *ctx, gbs_plan *pl);

// complex entries of k_adj_pairs_big's per-workgroup scratch for rows of up to
// n clicks: the four 16 x 16 planes of each upper 16 x 16 mode block of Z(w),
// then each block's partial sums of Z's mode diagonals (2 x 16 x 3)
long long adj_pair_scratch(int n)
{
    const long long tm = (n + 15) / 16;
    return tm * (tm + 1) / 2 * (4 * 256 + 96);
}

int approx_backward(gbs_ctx *ctx, gbs_plan *pl, const double *dl_dev, const int32_t *status_dev,
                    double *grad_r_dev, double *grad_eta_dev)
{
    int rc = adj_workspace(ctx, pl);
    if (rc) return rc;
    if (pl->P == 0) {
        hipLaunchKernelGGL(k_zero, dim3(1), dim3(256), 0, ctx->stream, (long)ctx->model.M, grad_r_dev);
        hipLaunchKernelGGL(k_zero, dim3(1), dim3(256), 0, ctx->stream, (long)ctx->model.M, grad_eta_dev);
        HIP_TRY(ctx, hipGetLastError());
        return 0;
    }
    switch (pl->order) {
    case 1: return backward_order<1>(ctx, pl, dl_dev, status_dev, grad_r_dev, grad_eta_dev);
    case 2: return backward_order<2>(ctx, pl, dl_dev, status_dev, grad_r_dev, grad_eta_dev);
    case 3: return backward_order<3>(ctx, pl, dl_dev, status_dev, grad_r_dev, grad_eta_dev);
    case 4: return backward_order<4>(ctx, pl, dl_dev, status_dev, grad_r_dev, grad_eta_dev);
    default: return set_err(ctx, GBS_E_INVAL, "order must be 1, 2, 3 or 4");
    }
}
