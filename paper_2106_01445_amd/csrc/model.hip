// Model build on the device, in double-double (Methods, Model; loss added).
//
//   sigma = D O diag(e^{-2r}, e^{2r}) O^T D / 2 + (I - D^2)/2,   Q = sigma + I/2
//   O = [[Re U, -Im U], [Im U, Re U]],  D = diag(sqrt eta, sqrt eta)
//
// Q is factored Q = L L^T (one workgroup, right-looking), inverted column by
// column from L (one workgroup per column) and log det Q, det(Q)^{-1/2} kept.
// Everything stays in HBM as hi/lo fp64 planes, row-major (2M)^2, xxpp order.
#include "internal.h"

namespace {

__device__ __forceinline__ dd ld_dd(const double *hi, const double *lo, long i)
{
    return dd{hi[i], lo[i]};
}
__device__ __forceinline__ void st_dd(double *hi, double *lo, long i, dd v)
{
    hi[i] = v.hi;
    lo[i] = v.lo;
}

// e^{-2 r_k}, e^{2 r_k} (dd) and sqrt(eta_k) (dd).  Layout of expd:
// [0,2M) hi of d, [2M,4M) lo of d, [4M,5M) hi of s, [5M,6M) lo of s.
__global__ void k_model_scalars(int M, const double *__restrict__ r,
                                const double *__restrict__ eta, double *__restrict__ expd)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= M) return;
    dd em = dd_exp(dd_make(-2.0 * r[k]));
    dd ep = dd_exp(dd_make(2.0 * r[k]));
    dd s = eta[k] > 0.0 ? dd_sqrt(dd_make(eta[k])) : dd_make(0.0);
    int D = 2 * M;
    expd[k] = em.hi;
    expd[D + k] = em.lo;
    expd[M + k] = ep.hi;
    expd[D + M + k] = ep.lo;
    expd[2 * D + k] = s.hi;
    expd[2 * D + M + k] = s.lo;
}

__device__ __forceinline__ double o_entry(int M, const double *ure, const double *uim, int i,
                                          int k)
{
    if (i < M) return k < M ? ure[i * M + k] : -uim[i * M + k - M];
    return k < M ? uim[(i - M) * M + k] : ure[(i - M) * M + k - M];
}

// One thread per entry (i, j) of Q.
__global__ void k_build_q(int M, const double *__restrict__ ure, const double *__restrict__ uim,
                          const double *__restrict__ eta, const double *__restrict__ expd,
                          const double *__restrict__ sigma, double *__restrict__ q_hi,
                          double *__restrict__ q_lo)
{
    int D = 2 * M;
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    int i = blockIdx.y;
    if (j >= D || i >= D) return;
    dd q;
    if (sigma) {
        q = dd_make(sigma[(long)i * D + j]);
        if (i == j) q = dd_add_d(q, 0.5);
    } else {
        dd acc = dd_make(0.0);
        for (int k = 0; k < D; ++k) {
            double a = o_entry(M, ure, uim, i, k);
            double b = o_entry(M, ure, uim, j, k);
            if (a == 0.0 || b == 0.0) continue;
            dd t = dd_mul(two_prod(a, b), dd{expd[k], expd[D + k]});
            acc = dd_add(acc, t);
        }
        acc = dd_mul_d(acc, 0.5);
        dd si = dd{expd[2 * D + (i % M)], expd[2 * D + M + (i % M)]};
        dd sj = dd{expd[2 * D + (j % M)], expd[2 * D + M + (j % M)]};
        q = dd_mul(dd_mul(acc, si), sj);
        // diagonal: (1 - eta)/2 from the loss channel plus 1/2 = 1 - eta/2
        if (i == j) q = dd_add(q, two_sum(1.0, -0.5 * eta[i % M]));
    }
    st_dd(q_hi, q_lo, (long)i * D + j, q);
}

// In-place right-looking Cholesky in one workgroup.  scal: [0] log det Q,
// [1],[2] det(Q)^{-1/2} (dd), [3] 1 if not positive definite,
// [8 .. 8+2D) 1/L_jj as dd (hi then lo planes).
__global__ void k_chol(int D, double *__restrict__ l_hi, double *__restrict__ l_lo,
                       double *__restrict__ scal)
{
    __shared__ double s_inv_hi, s_inv_lo;
    __shared__ int s_bad;
    const int tid = threadIdx.x, nt = blockDim.x;
    double logdet = 0.0;
    dd rdet = dd_make(1.0);
    if (tid == 0) s_bad = 0;
    __syncthreads();
    for (int j = 0; j < D; ++j) {
        if (tid == 0) {
            dd piv = ld_dd(l_hi, l_lo, (long)j * D + j);
            if (!(piv.hi > 0.0)) {
                s_bad = 1;
            } else {
                dd l = dd_sqrt(piv);
                dd inv = dd_recip(l);
                st_dd(l_hi, l_lo, (long)j * D + j, l);
                s_inv_hi = inv.hi;
                s_inv_lo = inv.lo;
                scal[8 + j] = inv.hi;
                scal[8 + D + j] = inv.lo;
                logdet += 2.0 * (log(l.hi) + l.lo / l.hi);
                rdet = dd_mul(rdet, inv);
            }
        }
        __syncthreads();
        if (s_bad) break;
        dd inv = dd{s_inv_hi, s_inv_lo};
        for (int i = j + 1 + tid; i < D; i += nt) {
            long ij = (long)i * D + j;
            st_dd(l_hi, l_lo, ij, dd_mul(ld_dd(l_hi, l_lo, ij), inv));
        }
        __syncthreads();
        int m = D - j - 1;
        for (int idx = tid; idx < m * m; idx += nt) {
            int ii = idx / m, kk = idx - ii * m;
            if (kk > ii) continue;
            int i = j + 1 + ii, k = j + 1 + kk;
            dd lij = ld_dd(l_hi, l_lo, (long)i * D + j);
            dd lkj = ld_dd(l_hi, l_lo, (long)k * D + j);
            long ik = (long)i * D + k;
            st_dd(l_hi, l_lo, ik, dd_sub(ld_dd(l_hi, l_lo, ik), dd_mul(lij, lkj)));
        }
        __syncthreads();
    }
    if (tid == 0) {
        scal[0] = logdet;
        scal[1] = rdet.hi;
        scal[2] = rdet.lo;
        scal[3] = s_bad ? 1.0 : 0.0;
    }
}

// Column j of Q^{-1} = L^{-T} L^{-1} e_j, one 64-lane workgroup per column.
__global__ void k_chol_inv(int D, const double *__restrict__ l_hi, const double *__restrict__ l_lo,
                           const double *__restrict__ scal, double *__restrict__ qi_hi,
                           double *__restrict__ qi_lo)
{
    extern __shared__ double sh[];
    double *b_hi = sh, *b_lo = sh + D;
    const int j = blockIdx.x, lane = threadIdx.x, nt = blockDim.x;
    if (scal[3] != 0.0) return;
    for (int i = lane; i < D; i += nt) {
        b_hi[i] = (i == j) ? 1.0 : 0.0;
        b_lo[i] = 0.0;
    }
    __syncthreads();
    // forward: L y = e_j  (y_i = 0 for i < j)
    for (int k = j; k < D; ++k) {
        dd yk = dd_mul(dd{b_hi[k], b_lo[k]}, dd{scal[8 + k], scal[8 + D + k]});
        __syncthreads();
        for (int i = k + 1 + lane; i < D; i += nt) {
            dd v = dd_sub(dd{b_hi[i], b_lo[i]}, dd_mul(ld_dd(l_hi, l_lo, (long)i * D + k), yk));
            b_hi[i] = v.hi;
            b_lo[i] = v.lo;
        }
        if (lane == 0) {
            b_hi[k] = yk.hi;
            b_lo[k] = yk.lo;
        }
        __syncthreads();
    }
    // backward: L^T x = y
    for (int k = D - 1; k >= 0; --k) {
        dd xk = dd_mul(dd{b_hi[k], b_lo[k]}, dd{scal[8 + k], scal[8 + D + k]});
        __syncthreads();
        for (int i = lane; i < k; i += nt) {
            dd v = dd_sub(dd{b_hi[i], b_lo[i]}, dd_mul(ld_dd(l_hi, l_lo, (long)k * D + i), xk));
            b_hi[i] = v.hi;
            b_lo[i] = v.lo;
        }
        if (lane == 0) {
            b_hi[k] = xk.hi;
            b_lo[k] = xk.lo;
        }
        __syncthreads();
    }
    for (int i = lane; i < D; i += nt) {
        qi_hi[(long)i * D + j] = b_hi[i];
        qi_lo[(long)i * D + j] = b_lo[i];
    }
}

}  // namespace

static void free_model(DevModel &m)
{
    double **ptrs[] = {&m.q_hi, &m.q_lo, &m.qi_hi, &m.qi_lo, &m.chol_hi, &m.chol_lo,
                       &m.params, &m.scal, &m.expd};
    for (double **p : ptrs) {
        if (*p) (void)hipFree(*p);
        *p = nullptr;
    }
}

// Allocate model buffers for M modes (reallocating when M changes).
int model_alloc(gbs_ctx *ctx, int M)
{
    DevModel &m = ctx->model;
    if (m.M == M && m.q_hi) return 0;
    free_model(m);
    m.M = M;
    m.have = false;
    size_t D = 2 * (size_t)M, DD = D * D * sizeof(double);
    double **mats[] = {&m.q_hi, &m.q_lo, &m.qi_hi, &m.qi_lo, &m.chol_hi, &m.chol_lo};
    for (double **p : mats)
        if (hipMalloc((void **)p, DD) != hipSuccess) {
            free_model(m);
            m.M = 0;
            return set_err(ctx, -3, "model: device allocation failed");
        }
    if (hipMalloc((void **)&m.params, (2 * (size_t)M * M + 2 * M) * sizeof(double)) != hipSuccess ||
        hipMalloc((void **)&m.scal, (8 + 2 * D) * sizeof(double)) != hipSuccess ||
        hipMalloc((void **)&m.expd, 6 * (size_t)M * sizeof(double)) != hipSuccess) {
        free_model(m);
        m.M = 0;
        return set_err(ctx, -3, "model: device allocation failed");
    }
    return 0;
}

void model_release(gbs_ctx *ctx) { free_model(ctx->model); ctx->model.M = 0; }

// Build Q, its factor and inverse.  Parameters must already be in
// ctx->model.params (U_re, U_im, r, eta) unless sigma_dev is given.
int model_build_dev(gbs_ctx *ctx, const double *sigma_dev, bool sync)
{
    DevModel &m = ctx->model;
    int M = m.M, D = 2 * M;
    hipStream_t st = ctx->stream;
    const double *ure = m.params, *uim = m.params + (size_t)M * M;
    const double *r = m.params + 2 * (size_t)M * M, *eta = r + M;
    const int tslot = timer_begin(ctx, TG_MODEL);
    if (!sigma_dev) {
        hipLaunchKernelGGL(k_model_scalars, dim3((M + 63) / 64), dim3(64), 0, st, M, r, eta,
                           m.expd);
    }
    hipLaunchKernelGGL(k_build_q, dim3((D + 127) / 128, D), dim3(128), 0, st, M, ure, uim, eta,
                       m.expd, sigma_dev, m.q_hi, m.q_lo);
    HIP_TRY(ctx, hipMemcpyAsync(m.chol_hi, m.q_hi, (size_t)D * D * sizeof(double),
                                hipMemcpyDeviceToDevice, st));
    HIP_TRY(ctx, hipMemcpyAsync(m.chol_lo, m.q_lo, (size_t)D * D * sizeof(double),
                                hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(k_chol, dim3(1), dim3(1024), 0, st, D, m.chol_hi, m.chol_lo, m.scal);
    hipLaunchKernelGGL(k_chol_inv, dim3(D), dim3(64), 2 * D * sizeof(double), st, D, m.chol_hi,
                       m.chol_lo, m.scal, m.qi_hi, m.qi_lo);
    timer_end(ctx, tslot);
    HIP_TRY(ctx, hipGetLastError());
    if (!sync) {
        m.have = true;  // a non-PD Q is flagged on the device and reported per row
        return 0;
    }
    double flag = 0.0;
    HIP_TRY(ctx, hipMemcpyAsync(&flag, m.scal + 3, sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(ctx, hipStreamSynchronize(st));
    if (flag != 0.0) {
        m.have = false;
        return set_err(ctx, -2, "covariance + I/2 is not positive definite");
    }
    m.have = true;
    return 0;
}
