// Per-row set-up of the order-j estimate: A = (Q^{-1})_CC = V diag(alpha) V^T
// with the working matrices in HBM (L2-resident), one workgroup per row.
//
//   1. Householder reduction of A to tridiagonal form (symmetric rank-2
//      updates of the trailing block, Golub & Van Loan, Matrix Computations,
//      section 8.3.1);
//   2. the orthogonal factor accumulated explicitly, last reflector first;
//   3. implicit symmetric QR steps with Wilkinson shifts on the tridiagonal
//      matrix (ibid., section 8.3): one thread chases the bulge of a step with
//      plane rotations and records them, then every thread applies them to its
//      own row of the factor;
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
    // 3. implicit symmetric QR steps with Wilkinson shifts on (dg, ed); ed[i]
    //    couples i and i+1.  The active block [lo, hi] is the lowest unreduced
    //    one.  One thread chases the bulge of a step down the block with plane
    //    rotations G_k on (k, k+1), choosing G_0 from the shifted first column
    //    and every later one to annihilate the bulge below the subdiagonal,
    //    and records (c_k, s_k); every thread then applies the rotations in
    //    order to its own row of the factor (Qf <- Qf G_k).
    const double eps = 2.220446049250313e-16;
    if (tid == 0) {
        s_fail = 0;
        s_m = N - 1;
    }
    __syncthreads();
    // (ed[i] is negligible when |ed[i]| <= eps (|dg[i]| + |dg[i+1]|))
    auto small = [&](int i) { return fabs(ed[i]) <= eps * (fabs(dg[i]) + fabs(dg[i + 1])); };
    for (int guard = 0; guard < 60 * N + 60; ++guard) {
        if (tid < 64) {
            // wavefront 0 finds the active block: hi = the highest index at or
            // below s_m whose coupling to the row above is not negligible (the
            // negligible ones set to zero), lo = the lowest index joined to hi
            // by non-negligible couplings; 64 candidates per ballot
            const int top = s_m;
            int hi = 0;
            for (int base = top; base > 0; base -= 64) {
                const int idx = base - tid;
                const bool stop = idx > 0 && !small(idx - 1);
                const unsigned long long bal = __ballot(stop);
                if (bal != 0ull) {
                    hi = base - __ffsll((long long)bal) + 1;
                    break;
                }
            }
            for (int idx = hi + 1 + tid; idx <= top; idx += 64) ed[idx - 1] = 0.0;
            int lo = -1;
            if (hi > 0) {
                for (int base = hi - 1;; base -= 64) {
                    const int idx = base - tid;
                    const bool stop = idx >= 0 && (idx == 0 || small(idx - 1));
                    const unsigned long long bal = __ballot(stop);
                    if (bal != 0ull) {
                        lo = base - __ffsll((long long)bal) + 1;
                        break;
                    }
                }
            }
            if (tid == 0) {
                if (hi > 0) {
                    if (lo > 0) ed[lo - 1] = 0.0;
                    // Wilkinson shift: the eigenvalue of the trailing 2 x 2 block
                    // closer to its last diagonal entry
                    const double e = ed[hi - 1];
                    const double dd = 0.5 * (dg[hi - 1] - dg[hi]);
                    const double den = dd + copysign(sqrt(fma(dd, dd, e * e)), dd);
                    const double mu = den != 0.0 ? dg[hi] - e * e / den : dg[hi];
                    // the chase: a = dg[k] and b = ed[k] as rotated by the previous
                    // step are carried in registers, d = dg[k + 1] and en = ed[k + 1]
                    // are still the block's own values
                    double a = dg[lo], b = ed[lo];
                    double x = a - mu, z = b, bulge = 0.0;
                    for (int k = lo; k < hi; ++k) {
                        const double d = dg[k + 1];
                        const double en = k + 1 < hi ? ed[k + 1] : 0.0;
                        const double r = sqrt(fma(x, x, z * z));
                        double c = 1.0, sn = 0.0;
                        if (r != 0.0) {
                            c = x / r;
                            sn = z / r;
                        }
                        if (k > lo) ed[k - 1] = r;  // the bulge is gone
                        const double cs = c * sn, c2 = c * c, s2 = sn * sn;
                        dg[k] = c2 * a + 2.0 * cs * b + s2 * d;
                        const double dn = s2 * a - 2.0 * cs * b + c2 * d;
                        const double ek = cs * (d - a) + (c2 - s2) * b;
                        ed[k] = ek;
                        if (k + 1 < hi) {
                            bulge = sn * en;
                            b = c * en;
                        }
                        rc[k] = c;
                        rs[k] = sn;
                        x = ek;
                        z = bulge;
                        a = dn;
                    }
                    dg[hi] = a;
                }
                s_m = hi;
                s_lo = lo;
                if (hi > 0 && guard == 60 * N + 59) s_fail = 1;
            }
        }
        __syncthreads();
        const int hi = s_m, lo = s_lo;
        if (hi == 0) break;
        // the factor's rows: columns k and k+1 rotated for k = lo .. hi-1
        for (int r = tid; r < N; r += nt) {
            double qk = Qf[(long)lo * N + r];
            for (int k = lo; k < hi; ++k) {
                const double qn = Qf[(long)(k + 1) * N + r];
                const double c = rc[k], sn = rs[k];
                Qf[(long)k * N + r] = c * qk + sn * qn;
                qk = c * qn - sn * qk;
            }
            Qf[(long)hi * N + r] = qk;
        }
        __syncthreads();
    }
    if (tid == 0 && s_m > 0) s_fail = 1;
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
