/*
 * Photon-number sector weights of one cluster in binary128 (oracle, test
 * infrastructure only).
 *
 * Methods, Partition function and Moments calculation: the sector weight of
 * kappa photons in the sub-ensemble with the cluster T forced empty is the
 * kappa-th power-series coefficient of its generating function
 *
 *   G_T(w) = det(W)^{-1/2} prod_mu (1 - w lambda_mu)^{-1/2},  lambda = 1 - 1/mu,
 *
 * where W is the Q-covariance of the sub-ensemble (2n x 2n, xxpp order) and mu
 * runs over the eigenvalues of the Schur complement S = W_ZZ - W_ZT W_TT^{-1}
 * W_TZ of the cluster's rows (Z = the clicked modes outside T).  With
 * l_k = sum_mu lambda_mu^k / (2k) the coefficients f of exp(sum_k l_k w^k)
 * follow from f_0 = 1, k f_k = sum_{i=1..k} i l_i f_{k-i}.
 *
 * Everything here is __float128 (about 33 digits): the Schur complement, a
 * cyclic Jacobi eigen-solver for S (Golub & Van Loan, Matrix Computations,
 * section 8.5, written for this file), det(W) by Cholesky, the power sums and
 * the series.  The fp64 W is taken as exact, so the result measures the
 * rounding of the fp64 series in oracle/sectors.py on the same input.
 * Build: gcc -O2 -shared -fPIC sectors128.c -lquadmath
 */
#include <quadmath.h>
#include <stdlib.h>
#include <string.h>

typedef __float128 R;

/* log det of the symmetric positive definite n x n matrix a (destroyed), by
 * Cholesky; returns 0 and sets *ok = 0 if a is not positive definite. */
static R chol_logdet(R *a, int n, int *ok)
{
    R ld = 0;
    *ok = 1;
    for (int j = 0; j < n; ++j) {
        R d = a[j * n + j];
        for (int k = 0; k < j; ++k) d -= a[j * n + k] * a[j * n + k];
        if (!(d > 0)) {
            *ok = 0;
            return 0;
        }
        R l = sqrtq(d);
        a[j * n + j] = l;
        ld += 2 * logq(l);
        for (int i = j + 1; i < n; ++i) {
            R s = a[i * n + j];
            for (int k = 0; k < j; ++k) s -= a[i * n + k] * a[j * n + k];
            a[i * n + j] = s / l;
        }
    }
    return ld;
}

/* Eigenvalues of the symmetric n x n matrix a (destroyed) by cyclic Jacobi
 * sweeps: each rotation in the (p, q) plane zeroes a_pq; sweeps repeat until
 * the off-diagonal mass is below 1e-66 of the diagonal's.  ev[n] out. */
static void jacobi_eigenvalues(R *a, int n, R *ev)
{
    for (int sweep = 0; sweep < 100; ++sweep) {
        R off = 0, dia = 0;
        for (int i = 0; i < n; ++i) {
            dia += a[i * n + i] * a[i * n + i];
            for (int j = i + 1; j < n; ++j) off += a[i * n + j] * a[i * n + j];
        }
        if (off <= 1e-66Q * dia) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                const R apq = a[p * n + q];
                if (apq == 0) continue;
                /* angle with tan(2 theta) = 2 a_pq / (a_qq - a_pp); t = tan theta,
                   the root of smaller magnitude */
                const R th = (a[q * n + q] - a[p * n + p]) / (2 * apq);
                R t = 1 / (fabsq(th) + sqrtq(th * th + 1));
                if (th < 0) t = -t;
                const R c = 1 / sqrtq(t * t + 1), s = t * c;
                for (int k = 0; k < n; ++k) {
                    /* rows p and q, then columns p and q (symmetric storage kept whole) */
                    const R akp = a[k * n + p], akq = a[k * n + q];
                    a[k * n + p] = c * akp - s * akq;
                    a[k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {
                    const R apk = a[p * n + k], aqk = a[q * n + k];
                    a[p * n + k] = c * apk - s * aqk;
                    a[q * n + k] = s * apk + c * aqk;
                }
            }
    }
    for (int i = 0; i < n; ++i) ev[i] = a[i * n + i];
}

/* Solve the small symmetric positive definite system a x = b for m right-hand
 * sides (a: t2 x t2, b: t2 x m, both row-major; a destroyed, b overwritten). */
static int spd_solve(R *a, int t2, R *b, int m)
{
    int ok;
    R tmp = chol_logdet(a, t2, &ok);
    (void)tmp;
    if (!ok) return 0;
    for (int c = 0; c < m; ++c) {
        for (int i = 0; i < t2; ++i) {
            R s = b[i * m + c];
            for (int k = 0; k < i; ++k) s -= a[i * t2 + k] * b[k * m + c];
            b[i * m + c] = s / a[i * t2 + i];
        }
        for (int i = t2 - 1; i >= 0; --i) {
            R s = b[i * m + c];
            for (int k = i + 1; k < t2; ++k) s -= a[k * t2 + i] * b[k * m + c];
            b[i * m + c] = s / a[i * t2 + i];
        }
    }
    return 1;
}

/*
 * g_T[kappa], kappa = 0..L-1, for the cluster T (t positions in 0..n-1 of the
 * clicked set) of the sub-ensemble with Q-covariance W (2n x 2n fp64,
 * row-major, xxpp).  Output as hi + lo doubles.  Returns 0 on success, -1 if
 * W or W_TT is not positive definite.
 */
int oracle128_sector_weights(int n, const double *W, int t, const int *T, int L, double *out_hi,
                             double *out_lo)
{
    const int N = 2 * n, t2 = 2 * t, z2 = N - t2;
    int *it = (int *)malloc(sizeof(int) * (t2 + 1)), *iz = (int *)malloc(sizeof(int) * (z2 + 1));
    char *in_t = (char *)calloc(n, 1);
    for (int i = 0; i < t; ++i) in_t[T[i]] = 1;
    for (int i = 0; i < t; ++i) {
        it[i] = T[i];
        it[t + i] = T[i] + n;
    }
    int k = 0;
    for (int a = 0; a < n; ++a)
        if (!in_t[a]) iz[k++] = a;
    for (int a = 0; a < n; ++a)
        if (!in_t[a]) iz[k++] = a + n;
    R *w = (R *)malloc(sizeof(R) * N * N);
    for (int i = 0; i < N * N; ++i) w[i] = (R)W[i];
    int ok = 1;
    R ldw = chol_logdet(w, N, &ok);
    for (int i = 0; i < N * N; ++i) w[i] = (R)W[i];
    R *S = (R *)malloc(sizeof(R) * (z2 * z2 + 1));
    for (int i = 0; i < z2; ++i)
        for (int j = 0; j < z2; ++j) S[i * z2 + j] = w[iz[i] * N + iz[j]];
    if (ok && t > 0) {
        /* S -= W_ZT W_TT^{-1} W_TZ */
        R *att = (R *)malloc(sizeof(R) * t2 * t2), *x = (R *)malloc(sizeof(R) * t2 * (z2 + 1));
        for (int i = 0; i < t2; ++i)
            for (int j = 0; j < t2; ++j) att[i * t2 + j] = w[it[i] * N + it[j]];
        for (int i = 0; i < t2; ++i)
            for (int j = 0; j < z2; ++j) x[i * z2 + j] = w[it[i] * N + iz[j]];
        ok = spd_solve(att, t2, x, z2);
        if (ok)
            for (int i = 0; i < z2; ++i)
                for (int j = 0; j < z2; ++j) {
                    R s = 0;
                    for (int q = 0; q < t2; ++q) s += w[iz[i] * N + it[q]] * x[q * z2 + j];
                    S[i * z2 + j] -= s;
                }
        free(att);
        free(x);
    }
    if (!ok) {
        free(it); free(iz); free(in_t); free(w); free(S);
        return -1;
    }
    R *mu = (R *)malloc(sizeof(R) * (z2 + 1));
    jacobi_eigenvalues(S, z2, mu);
    /* l_k = sum lambda^k / (2k), then the exponential series */
    R *l = (R *)calloc(L + 1, sizeof(R)), *f = (R *)calloc(L + 1, sizeof(R));
    R *pw = (R *)malloc(sizeof(R) * (z2 + 1));
    for (int i = 0; i < z2; ++i) pw[i] = 1 - 1 / mu[i];
    for (int kk = 1; kk < L; ++kk) {
        R s = 0;
        for (int i = 0; i < z2; ++i) s += pw[i];
        l[kk] = s / (2 * kk);
        for (int i = 0; i < z2; ++i) pw[i] *= 1 - 1 / mu[i];
    }
    f[0] = 1;
    for (int kk = 1; kk < L; ++kk) {
        R s = 0;
        for (int i = 1; i <= kk; ++i) s += i * l[i] * f[kk - i];
        f[kk] = s / kk;
    }
    const R pref = expq(-ldw / 2);
    for (int kk = 0; kk < L; ++kk) {
        const R g = pref * f[kk];
        out_hi[kk] = (double)g;
        out_lo[kk] = (double)(g - (R)out_hi[kk]);
    }
    free(it); free(iz); free(in_t); free(w); free(S); free(mu); free(l); free(f); free(pw);
    return 0;
}
