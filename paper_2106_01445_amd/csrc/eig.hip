// Per-row set-up of the order-j estimate: A = (Q^{-1})_CC = V diag(alpha) V^T
// with the working matrices in HBM (L2-resident), one workgroup per row.
//
//   1. Householder reduction of A to tridiagonal form (symmetric rank-2
//      updates of the trailing block, Golub & Van Loan, Matrix Computations,
//      section 8.3.1);
//   2. the orthogonal factor accumulated explicitly, last reflector first;
//   3. implicit QL iterations with Wilkinson shifts on the tridiagonal matrix
//      (ibid., section 8.3.3, in its QL form): one thread chases the bulge of a
//      sweep and records its plane rotations, then every thread applies them to
//      its own row of the factor;
//   4. the contour plan of the row from its spectrum.
// The factor is kept column-major, which is the layout the contour kernels
// read (eigenvector k contiguous).
#include "contour_common.h"

#define EIG_THREADS 256

namespace {

__global__ __launch_bounds__(EIG_THREADS) void k_eig(
    int M, const double *__restrict__ qi, const double *__restrict__ scal,
    const int *__restrict__ offsets, const int *__restrict__ modes, const int *__restrict__ perm,
    const long long *__restrict__ voff, double *__restrict__ wbuf, double *__restrict__ alpha_out,
    double *__restrict__ vt_out, RowPlan *__restrict__ rows, int frozen)
{
    __shared__ double red[EIG_THREADS];
    __shared__ double v[EIG_THREADS], w[EIG_THREADS];
    __shared__ double dg[EIG_THREADS], ed[EIG_THREADS], tau[EIG_THREADS];
    __shared__ double rc[EIG_THREADS], rs[EIG_THREADS];
    __shared__ int s_m, s_lo, s_fail;
    const int p = perm[blockIdx.x];
    const int o = offsets[p], n = offsets[p + 1] - o, N = 2 * n;
    const int tid = threadIdx.x, nt = blockDim.x;
    const double logdetQ = scal[0];
    const long long vo = voff[p];
    double *W = wbuf + 2 * vo;  // A, row-major, reduced in place (2 N^2 per row reserved)
    double *Qf = vt_out + vo;   // orthogonal factor, column-major: Qf[c * N + r]
    const int D = 2 * M;
    for (int idx = tid; idx < N * N; idx += nt) {
        const int i = idx / N, j = idx - i * N;
        const int ri = i < n ? modes[o + i] : modes[o + i - n] + M;
        const int rj = j < n ? modes[o + j] : modes[o + j - n] + M;
        W[idx] = qi[(long)ri * D + rj];
    }
    __syncthreads();
    // 1. reduction: step k annihilates W[k][k+2..], reflector v (length m = N-k-1)
    //    stored in row k right of the diagonal, tau[k]; diagonal dg, coupling ed
    for (int k = 0; k + 2 < N; ++k) {
        const int m = N - k - 1;
        double *Wk = W + (long)k * N + k + 1;
        double sg = 0.0;
        for (int i = tid; i < m; i += nt) {
            const double x = Wk[i];
            v[i] = x;
            if (i > 0) sg += x * x;
        }
        sg = block_sum(sg, red);
        if (tid == 0) {
            const double x0 = v[0];
            dg[k] = W[(long)k * N + k];
            if (sg == 0.0) {
                tau[k] = 0.0;
                ed[k] = x0;
            } else {
                const double al = -copysign(sqrt(x0 * x0 + sg), x0);
                const double v0 = x0 - al;
                v[0] = v0;
                tau[k] = 2.0 / (v0 * v0 + sg);
                ed[k] = al;
            }
        }
        __syncthreads();
        const double tk = tau[k];
        for (int i = tid; i < m; i += nt) Wk[i] = v[i];
        if (tk != 0.0) {
            // p = tau W2 v (W2 symmetric: column sums), then w = p - (tau/2)(p.v) v
            double *W2 = W + (long)(k + 1) * N + k + 1;
            double pv = 0.0;
            for (int j = tid; j < m; j += nt) {
                double s = 0.0;
                for (int i = 0; i < m; ++i) s = fma(W2[(long)i * N + j], v[i], s);
                w[j] = tk * s;
                pv += w[j] * v[j];
            }
            pv = block_sum(pv, red);
            const double kk = 0.5 * tk * pv;
            for (int j = tid; j < m; j += nt) w[j] -= kk * v[j];
            __syncthreads();
            for (int idx = tid; idx < m * m; idx += nt) {
                const int i = idx / m, j = idx - i * m;
                W2[(long)i * N + j] -= v[i] * w[j] + w[i] * v[j];
            }
        }
        __syncthreads();
    }
    if (tid == 0) {
        if (N >= 2) {
            dg[N - 2] = W[(long)(N - 2) * N + N - 2];
            ed[N - 2] = W[(long)(N - 2) * N + N - 1];
        }
        if (N >= 1) {  // (an empty row has nothing to reduce)
            dg[N - 1] = W[(long)(N - 1) * N + N - 1];
            ed[N - 1] = 0.0;
        }
        s_fail = 0;
    }
    // 2. factor: Qf = H_0 H_1 ... H_{N-3}, applied to the identity last first
    for (int idx = tid; idx < N * N; idx += nt) {
        const int c = idx / N, r = idx - c * N;
        Qf[idx] = r == c ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int k = N - 3; k >= 0; --k) {
        const double tk = tau[k];
        if (tk == 0.0) continue;
        const int m = N - k - 1;
        const double *vk = W + (long)k * N + k + 1;
        for (int i = tid; i < m; i += nt) v[i] = vk[i];
        __syncthreads();
        // u_j = tau sum_i v_i Qf[k+1+i][k+1+j]; Qf[k+1+i][k+1+j] -= v_i u_j
        for (int j = tid; j < m; j += nt) {
            const double *col = Qf + (long)(k + 1 + j) * N + k + 1;
            double s = 0.0;
            for (int i = 0; i < m; ++i) s = fma(col[i], v[i], s);
            w[j] = tk * s;
        }
        __syncthreads();
        for (int idx = tid; idx < m * m; idx += nt) {
            const int j = idx / m, i = idx - j * m;
            Qf[(long)(k + 1 + j) * N + k + 1 + i] -= v[i] * w[j];
        }
        __syncthreads();
    }
    // 3. implicit QL on (dg, ed); ed[i] couples i and i+1
    const double eps = 2.220446049250313e-16;
    for (int l = 0; l < N; ++l) {
        for (int iter = 0;; ++iter) {
            if (tid == 0) {
                int m = l;
                for (; m < N - 1; ++m)
                    if (fabs(ed[m]) <= eps * (fabs(dg[m]) + fabs(dg[m + 1]))) break;
                int lo = m;  // rotations recorded for i in [lo, m-1]
                if (m != l && iter < 60) {
                    // (|g| < 1e16 and every other quantity of the sweep is O(1),
                    // since ed[l] is above eps |dg|: plain square roots suffice)
                    double g = (dg[l + 1] - dg[l]) / (2.0 * ed[l]);
                    double r = sqrt(fma(g, g, 1.0));
                    g = dg[m] - dg[l] + ed[l] / (g + copysign(r, g));
                    double s = 1.0, c = 1.0, pp = 0.0;
                    bool early = false;
                    for (int i = m - 1; i >= l; --i) {
                        const double f = s * ed[i], b = c * ed[i];
                        r = sqrt(fma(f, f, g * g));
                        ed[i + 1] = r;
                        if (r == 0.0) {
                            dg[i + 1] -= pp;
                            ed[m] = 0.0;
                            early = true;
                            break;
                        }
                        s = f / r;
                        c = g / r;
                        g = dg[i + 1] - pp;
                        r = (dg[i] - g) * s + 2.0 * c * b;
                        pp = s * r;
                        dg[i + 1] = g + pp;
                        g = c * r - b;
                        rc[i] = c;
                        rs[i] = s;
                        lo = i;
                    }
                    if (!early) {
                        dg[l] -= pp;
                        ed[l] = g;
                        ed[m] = 0.0;
                    }
                } else if (m != l) {
                    s_fail = 1;
                    m = l;
                }
                s_m = m;
                s_lo = lo;
            }
            __syncthreads();
            const int m = s_m, lo = s_lo;
            if (m == l) break;
            // rows of the factor: Qf[r][i], Qf[r][i+1] rotated for i = m-1 down to lo
            for (int r = tid; r < N; r += nt) {
                double up = Qf[(long)m * N + r];
                for (int i = m - 1; i >= lo; --i) {
                    const double lo_v = Qf[(long)i * N + r];
                    const double c = rc[i], s = rs[i];
                    Qf[(long)(i + 1) * N + r] = s * lo_v + c * up;
                    up = c * lo_v - s * up;
                }
                Qf[(long)lo * N + r] = up;
            }
            __syncthreads();
        }
    }
    // 4. spectrum and plan
    double lsum = 0.0, amin = 1e300, dev = 0.0;
    for (int i = tid; i < N; i += nt) {
        const double a = dg[i];
        alpha_out[2 * o + i] = a;
        lsum += log(a);
        amin = fmin(amin, a);
        dev = fmax(dev, fabs(a - 1.0));
    }
    const double logdetA = block_sum(lsum, red);
    amin = -block_max(-amin, red);
    dev = block_max(dev, red);
    if (tid == 0) {
        RowPlan rp = rows[p];
        row_plan(rp, n, dg, 1, logdetQ, logdetA, amin, dev, scal[3] != 0.0 || s_fail != 0, frozen & 1,
                 (frozen & 2) != 0);
        rows[p] = rp;
    }
}

}  // namespace

int eig_rows(gbs_ctx *ctx, gbs_plan *pl)
{
    if (pl->P == 0) return 0;
    hipLaunchKernelGGL(k_eig, dim3(pl->P), dim3(EIG_THREADS), 0, ctx->stream, ctx->model.M,
                       ctx->model.qi_hi, ctx->model.scal, pl->d_offsets, pl->d_modes, pl->d_perm,
                       pl->d_voff, pl->d_wbig, pl->d_alpha, pl->d_v, pl->d_rows,
                       (pl->frozen ? 1 : 0) | (pl->whole ? 2 : 0));
    HIP_TRY(ctx, hipGetLastError());
    return 0;
}
