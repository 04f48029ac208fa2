// A plain kernel for the same order-j estimate, kept for speed-up comparisons
// and as an independent check of the tuned contour kernel: one workgroup per
// row, the row's contour points one after another, M(w) = V diag(d) V^T by
// plain dot products into a packed symmetric array, and every cluster
// determinant det(M_TT) by its own unpivoted LDL^T (no reuse between clusters,
// no work queue, no matrix cores).  det(M_TT)^{-1/2} is the product of the
// principal inverse square roots of the pivots: every pivot of a complex
// symmetric matrix whose Hermitian part is positive definite has a positive
// real part, so this is the branch continuous from w = 0.  The eigen-
// decomposition, the sector transform and the fits are the tuned path's.
#include "contour_common.h"

#define PLAIN_THREADS 256

namespace {

// packed upper-triangle index of (i, j)
__device__ __forceinline__ int pidx(int i, int j)
{
    return i <= j ? j * (j + 1) / 2 + i : i * (i + 1) / 2 + j;
}

// cluster number c (singles, then pairs a < b, then triples a < b < c, then
// quadruples, each in colexicographic order) -> its modes; returns the size
__device__ __forceinline__ int cluster_modes(int c, int n, int *m)
{
    if (c < n) {
        m[0] = c;
        return 1;
    }
    c -= n;
    const int np = n * (n - 1) / 2;
    if (c < np) {
        int b = 1;
        while ((b + 1) * b / 2 <= c) ++b;
        m[0] = c - b * (b - 1) / 2;
        m[1] = b;
        return 2;
    }
    c -= np;
    const int nt3 = n * (n - 1) * (n - 2) / 6;
    int t = 4;
    if (c >= nt3) {
        c -= nt3;
        int y = 3;
        while ((y + 1) * y * (y - 1) * (y - 2) / 24 <= c) ++y;
        c -= y * (y - 1) * (y - 2) * (y - 3) / 24;
        m[3] = y;
    } else {
        t = 3;
    }
    int z = 2;
    while ((z + 1) * z * (z - 1) / 6 <= c) ++z;
    c -= z * (z - 1) * (z - 2) / 6;
    int b = 1;
    while ((b + 1) * b / 2 <= c) ++b;
    m[0] = c - b * (b - 1) / 2;
    m[1] = b;
    m[2] = z;
    return t;
}

template <int ORDER>
__global__ __launch_bounds__(PLAIN_THREADS) void k_plain(const int *__restrict__ offsets,
                                                         const long long *__restrict__ voff,
                                                         const double *__restrict__ alpha,
                                                         const double *__restrict__ vt,
                                                         const RowPlan *__restrict__ rows,
                                                         cplx *__restrict__ sw)
{
    extern __shared__ __attribute__((aligned(16))) double sh[];
    __shared__ cplx red[PLAIN_THREADS / 64][ORDER + 1];
    __shared__ cplx s_w, s_g;
    const int p = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int o = offsets[p], n = offsets[p + 1] - o, N = 2 * n;
    const RowPlan rp = rows[p];
    if (n == 0 || rp.status != 0 || rp.K <= 0) return;
    double *Vt = sh;                      // N x N, eigenvector k contiguous
    cplx *d = (cplx *)(Vt + N * N);       // N
    cplx *rz = d + N;                     // N
    cplx *Mp = rz + N;                    // N(N+1)/2, packed upper triangle
    const long long vo = voff[p];
    for (int i = tid; i < N * N; i += PLAIN_THREADS) Vt[i] = vt[vo + i];
    int nc = n;
    if (ORDER >= 2) nc += n * (n - 1) / 2;
    if (ORDER >= 3) nc += n * (n - 1) * (n - 2) / 6;
    if (ORDER >= 4) nc += n * (n - 1) * (n - 2) * (n - 3) / 24;
    const int Q = rp.K / 2 + 1;
    __syncthreads();
    for (int q = 0; q < Q; ++q) {
        if (tid == 0) {
            s_w = cscale(unit_root(q, rp.K), rp.rho);
        }
        __syncthreads();
        const cplx w = s_w;
        for (int k = tid; k < N; k += PLAIN_THREADS) {
            const double am1 = alpha[2 * o + k] - 1.0;
            const cplx r = crsqrt_p(cmk(fma(w.re, am1, 1.0), w.im * am1));
            rz[k] = r;
            d[k] = cmul(r, r);
        }
        __syncthreads();
        if (tid == 0) {
            cplx g = cmk(exp(0.5 * rp.logdet_a - rp.log_g_rho), 0.0);
            for (int k = 0; k < N; ++k) g = cmul(g, rz[k]);
            s_g = g;
        }
        for (int e = tid; e < N * (N + 1) / 2; e += PLAIN_THREADS) {
            int j = 0;
            while ((j + 1) * (j + 2) / 2 <= e) ++j;
            const int i = e - j * (j + 1) / 2;
            cplx s = cmk(0.0, 0.0);
            for (int k = 0; k < N; ++k) {
                const double v = Vt[k * N + i] * Vt[k * N + j];
                s.re = fma(v, d[k].re, s.re);
                s.im = fma(v, d[k].im, s.im);
            }
            Mp[e] = s;
        }
        __syncthreads();
        cplx acc[ORDER + 1];
        for (int t = 0; t <= ORDER; ++t) acc[t] = cmk(0.0, 0.0);
        for (int c = tid; c < nc; c += PLAIN_THREADS) {
            int m[4];
            const int t = cluster_modes(c, n, m);
            const int S = 2 * t;
            int idx[2 * ORDER];
            for (int u = 0; u < t; ++u) {
                idx[u] = m[u];
                idx[t + u] = n + m[u];
            }
            cplx L[2 * ORDER][2 * ORDER], dv[2 * ORDER];
            cplx r = cmk(1.0, 0.0);
            for (int k = 0; k < S; ++k) {
                cplx dk = Mp[pidx(idx[k], idx[k])];
                for (int l = 0; l < k; ++l) dk = csub(dk, cmul(cmul(L[k][l], L[k][l]), dv[l]));
                dv[k] = dk;
                const cplx id = crecip(dk);
                for (int i = k + 1; i < S; ++i) {
                    cplx s = Mp[pidx(idx[i], idx[k])];
                    for (int l = 0; l < k; ++l) s = csub(s, cmul(cmul(L[i][l], L[k][l]), dv[l]));
                    L[i][k] = cmul(s, id);
                }
                r = cmul(r, crsqrt_p(dk));
            }
            acc[t] = cadd(acc[t], r);
        }
        for (int t = 1; t <= ORDER; ++t) {
            const cplx v = warp_csum(acc[t]);
            if (lane == 0) red[wid][t] = v;
        }
        __syncthreads();
        if (tid <= ORDER) {
            cplx s = cmk(tid == 0 ? 1.0 : 0.0, 0.0);
            if (tid > 0)
                for (int wv = 0; wv < PLAIN_THREADS / 64; ++wv) s = cadd(s, red[wv][tid]);
            sw[((long)p * (ORDER + 1) + tid) * GBS_QCAP + q] = cmul(s_g, s);
        }
        __syncthreads();
    }
}

template <int ORDER>
int plain_order(gbs_ctx *ctx, gbs_plan *pl)
{
    const int N = 2 * pl->max_n;
    const int lds = sizeof(double) * N * N + sizeof(cplx) * (2 * N + N * (N + 1) / 2);
    if (int rc = func_lds_limit(ctx, (const void *)k_plain<ORDER>, lds)) return rc;
    hipLaunchKernelGGL(k_plain<ORDER>, dim3(pl->P), dim3(PLAIN_THREADS), lds, ctx->stream,
                       pl->d_offsets, pl->d_voff, pl->d_alpha, pl->d_v, pl->d_rows, pl->d_sw);
    return 0;
}

}  // namespace

int plain_contour(gbs_ctx *ctx, gbs_plan *pl)
{
    if (pl->max_n > GBS_NSMALL)
        return set_err(ctx, GBS_E_INVAL, "the plain kernel takes rows of at most 40 clicks");
    switch (pl->order) {
    case 1: return plain_order<1>(ctx, pl);
    case 2: return plain_order<2>(ctx, pl);
    case 3: return plain_order<3>(ctx, pl);
    case 4: return plain_order<4>(ctx, pl);
    default: return set_err(ctx, GBS_E_INVAL, "order must be 1, 2, 3 or 4");
    }
}
