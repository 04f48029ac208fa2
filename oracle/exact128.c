/*
 * Exact click probabilities in binary128 (oracle, test infrastructure only).
 *
 * The signed sum over the 2^n subsets of the clicked set (Methods, Probability
 * of any sample; the click projector of Methods, Model) cancels by up to ~1e11
 * at 20 modes, so an fp64 evaluation loses up to 5 digits.  This file runs the
 * whole chain -- covariance from (U, r, eta), conditioning on the unclicked
 * modes, and every subset determinant -- in __float128 so that its result is
 * the exact probability of the fp64 inputs to ~1e-20 relative.
 *
 *   sigma = D O diag(e^{-2r}, e^{2r}) O^T D / 2 + (I - D^2)/2,  Q = sigma + I/2
 *   P_vac(Cbar) = det(Q_Cbar)^{-1/2}
 *   W = Q_CC - Q_{C,Cbar} Q_Cbar^{-1} Q_{Cbar,C}
 *   p(C) = P_vac(Cbar) * sum_{T subset C} (-1)^{|T|} det(W_T)^{-1/2}
 *
 * Every determinant is the squared product of a fresh Cholesky factor's
 * diagonal (no reuse between subsets: slow and plain on purpose).
 * Build: gcc -O2 -shared -fPIC exact128.c -lquadmath
 */
#include <quadmath.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

typedef __float128 R;

/* In-place lower Cholesky of the symmetric n x n row-major matrix a.
 * Returns prod_i 1/L_ii = det(a)^{-1/2}, or -1 if a is not positive definite. */
static R chol_rsqrt_det(R *a, int n)
{
    R inv = 1.0Q;
    for (int j = 0; j < n; ++j) {
        R d = a[j * n + j];
        for (int k = 0; k < j; ++k) d -= a[j * n + k] * a[j * n + k];
        if (!(d > 0)) return -1.0Q;
        R l = sqrtq(d);
        a[j * n + j] = l;
        inv /= l;
        for (int i = j + 1; i < n; ++i) {
            R s = a[i * n + j];
            for (int k = 0; k < j; ++k) s -= a[i * n + k] * a[j * n + k];
            a[i * n + j] = s / l;
        }
    }
    return inv;
}

static void build_q(int M, const double *Ure, const double *Uim, const double *r,
                    const double *eta, const double *sigma, R *Q)
{
    int D = 2 * M;
    if (sigma) {
        for (int i = 0; i < D * D; ++i) Q[i] = (R)sigma[i];
    } else {
        R *O = (R *)malloc(sizeof(R) * D * D);
        R *d = (R *)malloc(sizeof(R) * D);
        R *s = (R *)malloc(sizeof(R) * D);
        for (int i = 0; i < M; ++i)
            for (int j = 0; j < M; ++j) {
                O[i * D + j] = (R)Ure[i * M + j];
                O[i * D + M + j] = -(R)Uim[i * M + j];
                O[(M + i) * D + j] = (R)Uim[i * M + j];
                O[(M + i) * D + M + j] = (R)Ure[i * M + j];
            }
        for (int j = 0; j < M; ++j) {
            d[j] = expq(-2.0Q * (R)r[j]);
            d[M + j] = expq(2.0Q * (R)r[j]);
            s[j] = s[M + j] = sqrtq((R)eta[j]);
        }
        for (int i = 0; i < D; ++i)
            for (int j = 0; j < D; ++j) {
                R acc = 0;
                for (int k = 0; k < D; ++k) acc += O[i * D + k] * d[k] * O[j * D + k];
                Q[i * D + j] = s[i] * s[j] * acc / 2.0Q;
            }
        for (int i = 0; i < D; ++i) Q[i * D + i] += (1.0Q - s[i] * s[i]) / 2.0Q;
        free(O); free(d); free(s);
    }
    for (int i = 0; i < D; ++i) Q[i * D + i] += 0.5Q;
}

/* sigma (or the model) -> Q in binary128, split into hi + lo doubles. */
int oracle128_q_matrix(int M, const double *Ure, const double *Uim, const double *r,
                       const double *eta, const double *sigma, double *q_hi, double *q_lo)
{
    int D = 2 * M;
    R *Q = (R *)malloc(sizeof(R) * D * D);
    build_q(M, Ure, Uim, r, eta, sigma, Q);
    for (int i = 0; i < D * D; ++i) {
        q_hi[i] = (double)Q[i];
        q_lo[i] = (double)(Q[i] - (R)q_hi[i]);
    }
    free(Q);
    return 0;
}

/* Exact p for each CSR row.  p is returned as p_hi + p_lo; logp = log p;
 * kappa = sum |terms| / |sum| (cancellation factor of the signed sum).
 * Returns 0, or -(row+1) if some block is not positive definite. */
int oracle128_exact(int M, const double *Ure, const double *Uim, const double *r,
                    const double *eta, const double *sigma, int P, const int *offsets,
                    const int *modes, double *p_hi, double *p_lo, double *logp,
                    double *kappa)
{
    int D = 2 * M;
    R *Q = (R *)malloc(sizeof(R) * D * D);
    build_q(M, Ure, Uim, r, eta, sigma, Q);
    R *Qb = (R *)malloc(sizeof(R) * D * D);
    R *Y = (R *)malloc(sizeof(R) * D * D);
    R *W = (R *)malloc(sizeof(R) * D * D);
    R *Wt = (R *)malloc(sizeof(R) * D * D);
    int *isc = (int *)malloc(sizeof(int) * M);
    int *cb = (int *)malloc(sizeof(int) * D);
    int *cc = (int *)malloc(sizeof(int) * D);
    int rc = 0;
    for (int p = 0; p < P && rc == 0; ++p) {
        int n = offsets[p + 1] - offsets[p];
        const int *C = modes + offsets[p];
        memset(isc, 0, sizeof(int) * M);
        for (int a = 0; a < n; ++a) isc[C[a]] = 1;
        int nb = 0;
        for (int m = 0; m < M; ++m)
            if (!isc[m]) cb[nb++] = m;
        for (int a = 0; a < nb; ++a) cb[nb + a] = cb[a] + M;
        for (int a = 0; a < n; ++a) { cc[a] = C[a]; cc[n + a] = C[a] + M; }
        int B = 2 * nb, Cn = 2 * n;
        /* Cholesky of Q_Cbar -> P_vac(Cbar) */
        for (int i = 0; i < B; ++i)
            for (int j = 0; j < B; ++j) Qb[i * B + j] = Q[cb[i] * D + cb[j]];
        R pv = (B > 0) ? chol_rsqrt_det(Qb, B) : 1.0Q;
        if (pv < 0) { rc = -(p + 1); break; }
        /* Y = L^{-1} Q_{Cbar,C}; W = Q_CC - Y^T Y */
        for (int i = 0; i < B; ++i)
            for (int c = 0; c < Cn; ++c) {
                R s = Q[cb[i] * D + cc[c]];
                for (int k = 0; k < i; ++k) s -= Qb[i * B + k] * Y[k * Cn + c];
                Y[i * Cn + c] = s / Qb[i * B + i];
            }
        for (int a = 0; a < Cn; ++a)
            for (int c = 0; c < Cn; ++c) {
                R s = Q[cc[a] * D + cc[c]];
                for (int k = 0; k < B; ++k) s -= Y[k * Cn + a] * Y[k * Cn + c];
                W[a * Cn + c] = s;
            }
        /* signed subset sum */
        R total = 0, absum = 0;
        int idx[512];
        for (long mask = 0; mask < (1L << n); ++mask) {
            int t = 0;
            for (int a = 0; a < n; ++a)
                if (mask >> a & 1) idx[t++] = a;
            for (int a = 0; a < t; ++a) idx[t + a] = idx[a] + n;
            int T2 = 2 * t;
            R term = 1.0Q;
            if (t > 0) {
                for (int i = 0; i < T2; ++i)
                    for (int j = 0; j < T2; ++j) Wt[i * T2 + j] = W[idx[i] * Cn + idx[j]];
                term = chol_rsqrt_det(Wt, T2);
                if (term < 0) { rc = -(p + 1); break; }
            }
            total += (t & 1) ? -term : term;
            absum += term;
        }
        R prob = pv * total;
        p_hi[p] = (double)prob;
        p_lo[p] = (double)(prob - (R)p_hi[p]);
        logp[p] = (prob > 0) ? (double)logq(prob) : -INFINITY;
        kappa[p] = (total != 0) ? (double)(absum / fabsq(total)) : INFINITY;
    }
    free(Q); free(Qb); free(Y); free(W); free(Wt); free(isc); free(cb); free(cc);
    return rc;
}
