/*
 * Plain CPU oracle for the Gaussian-process profile likelihood.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant with
 * the GPU path.
 *
 * Written straight from the definitions of Franey, Ranjan & Chipman,
 * "A Short Note on Gaussian Process Modeling for Large Datasets using
 * Graphics Processing Units" (arXiv 1203.1269):
 *   - model y(x_i) = mu + z(x_i)                          (Sec. 2, eq. 1)
 *   - power-exponential correlation, product form       (Sec. 2, eq. 2)
 *   - Matern correlation (smoothness 3/2 and 5/2), the alternative that
 *     Sec. 2 names, in the same product-over-dimensions form
 *   - closed-form mu_hat and sigma_hat^2                  (Sec. 2, eq. 3)
 *   - profile likelihood -2 log L                         (Sec. 2, eq. 4)
 *   - determinant and solves through a Cholesky factor   (Sec. 2, text after
 *     eq. 4; Sec. 3, "CPU implementation")
 *
 * The arithmetic type REAL is chosen at compile time: the file is compiled
 * once with REAL = double (symbols *_f64) and once with REAL = long double
 * (symbols *_f80, x87 80-bit, unit roundoff 2^-64).  <tgmath.h> dispatches
 * exp/pow/log/sqrt/fabs to the matching precision.  The long-double build
 * exists only to measure how sensitive each FP64 result is to rounding.
 *
 * Readings of the paper used here (the paper is silent or ambiguous):
 *   - nugget: R_delta = R + delta*I, so R_ii = 1 + delta.
 *   - the reported "nll" is log|R_delta| + n*ln(sigma_hat^2); the literal
 *     eq. 4 value is that plus n*ln(n) and is returned as nll_paper.
 *   - 0^p = 0; natural logarithms.
 *   - Cholesky failure: info = 1-based index of the first pivot that is not
 *     strictly positive (or is NaN); all outputs NaN.
 *   - Q == 0 exactly: sigma2 = 0, nll = -inf, info = -1.
 *   - invalid theta (negative or non-finite): info = -3, outputs NaN.
 */
#include <tgmath.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef REAL
#define REAL double
#endif
#ifndef SFX
#define SFX(name) name##_f64
#endif

/* Output record per theta: logdet, mu, sigma2, nll, nll_paper, Q, aa, ab. */
#define ORC_NOUT 8

/* Correlation families (fam):
 *   0  power exponential, eq. 2: exp(-theta_k |x_ik - x_jk|^p)
 *   1  Matern, smoothness 3/2:  (1 + sqrt(3) h) exp(-sqrt(3) h)
 *   2  Matern, smoothness 5/2:  (1 + sqrt(5) h + 5 h^2 / 3) exp(-sqrt(5) h)
 * with h = theta_k |x_ik - x_jk| for the Matern families (the half-integer
 * closed forms of 2^(1-nu) / Gamma(nu) (sqrt(2 nu) h)^nu K_nu(sqrt(2 nu) h));
 * every family is a product of such factors over the d dimensions. */
static REAL corr_factor(int fam, REAL diff, REAL th, REAL p)
{
    if (fam == 0) {
        REAL pw = (diff == 0) ? (REAL)0 : pow(diff, p);
        return exp(-th * pw);
    }
    REAL h = th * diff;
    if (fam == 1) {
        REAL c = sqrt((REAL)3);
        return (1 + c * h) * exp(-c * h);
    }
    REAL c = sqrt((REAL)5);
    return (1 + c * h + c * c * h * h / 3) * exp(-c * h);
}

/* -d ln(factor) / d theta_k:
 *   fam 0: |x_ik - x_jk|^p
 *   fam 1: diff * 3 h / (1 + sqrt(3) h)
 *   fam 2: diff * 5 h (1 + sqrt(5) h) / (3 (1 + sqrt(5) h + 5 h^2 / 3)) */
static REAL corr_dlog(int fam, REAL diff, REAL th, REAL p)
{
    if (fam == 0) return (diff == 0) ? (REAL)0 : pow(diff, p);
    REAL h = th * diff;
    if (fam == 1) {
        REAL c = sqrt((REAL)3);
        return diff * c * c * h / (1 + c * h);
    }
    REAL c = sqrt((REAL)5);
    return diff * c * c * h * (1 + c * h) / (3 * (1 + c * h + c * c * h * h / 3));
}

static int family_ok(int fam, double p)
{
    if (fam == 0) return p > 0 && p <= 2;
    return fam == 1 || fam == 2;
}

/* eq. 2 (or a Matern family) written literally as a product over dimensions
 * of per-dimension factors, plus the nugget on the diagonal.  Full
 * symmetric n x n, row-major. */
static void build_corr(int n, int d, const double *X, const REAL *theta,
                       REAL p, int fam, REAL delta, REAL *R)
{
    for (int i = 0; i < n; ++i) {
        R[(size_t)i * n + i] = (REAL)1 + delta;
        for (int j = 0; j < i; ++j) {
            REAL prod = 1;
            for (int k = 0; k < d; ++k) {
                REAL diff = fabs((REAL)X[(size_t)i * d + k] - (REAL)X[(size_t)j * d + k]);
                prod *= corr_factor(fam, diff, theta[k], p);
            }
            R[(size_t)i * n + j] = prod;
            R[(size_t)j * n + i] = prod;
        }
    }
}

/* Unblocked Cholesky, column by column (Cholesky-Crout / dot-product form):
 *   L_jj = sqrt(A_jj - sum_{m<j} L_jm^2)
 *   L_ij = (A_ij - sum_{m<j} L_im L_jm) / L_jj,  i > j
 * In place on the lower triangle of a row-major matrix; the strict upper
 * triangle is set to zero.  Returns 0 or the 1-based failing pivot. */
static int cholesky(int n, REAL *A)
{
    for (int j = 0; j < n; ++j) {
        REAL *rj = A + (size_t)j * n;
        REAL s = rj[j];
        for (int m = 0; m < j; ++m) s -= rj[m] * rj[m];
        if (!(s > 0)) return j + 1;
        REAL ljj = sqrt(s);
        rj[j] = ljj;
        for (int i = j + 1; i < n; ++i) {
            REAL *ri = A + (size_t)i * n;
            REAL t = ri[j];
            for (int m = 0; m < j; ++m) t -= ri[m] * rj[m];
            ri[j] = t / ljj;
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) A[(size_t)i * n + j] = 0;
    return 0;
}

/* Forward substitution L z = v (L lower, row-major). */
static void forward_solve(int n, const REAL *L, const REAL *v, REAL *z)
{
    for (int i = 0; i < n; ++i) {
        const REAL *ri = L + (size_t)i * n;
        REAL t = v[i];
        for (int m = 0; m < i; ++m) t -= ri[m] * z[m];
        z[i] = t / ri[i];
    }
}

/* Back substitution L^T w = z. */
static void back_solve(int n, const REAL *L, const REAL *z, REAL *w)
{
    for (int i = n - 1; i >= 0; --i) {
        REAL t = z[i];
        for (int m = i + 1; m < n; ++m) t -= L[(size_t)m * n + i] * w[m];
        w[i] = t / L[(size_t)i * n + i];
    }
}

static int theta_ok(int d, const double *theta)
{
    for (int k = 0; k < d; ++k)
        if (!(theta[k] >= 0) || !isfinite(theta[k])) return 0;
    return 1;
}

static void fill_nan(double *out)
{
    for (int q = 0; q < ORC_NOUT; ++q) out[q] = NAN;
}

/* One profile-likelihood evaluation for one theta.  `work` holds n*n + 4n
 * REALs.  Steps follow Sec. 2: build R (eq. 2), factor it, log|R| from the
 * factor, a = L^-1 1 and b = L^-1 y, then eq. 3 and eq. 4. */
static int eval_one(int n, int d, const double *X, const double *y,
                    const double *theta_in, REAL p, int fam, REAL delta,
                    double *out, REAL *work, REAL *mu_out, REAL *sigma2_out)
{
    if (!theta_ok(d, theta_in)) { fill_nan(out); return -3; }
    REAL theta[64];
    for (int k = 0; k < d; ++k) theta[k] = (REAL)theta_in[k];
    REAL *A = work;
    REAL *ones = work + (size_t)n * n;
    REAL *yv = ones + n;
    REAL *a = yv + n;
    REAL *b = a + n;

    build_corr(n, d, X, theta, p, fam, delta, A);
    int info = cholesky(n, A);
    if (info != 0) { fill_nan(out); return info; }

    REAL logdet = 0;
    for (int j = 0; j < n; ++j) logdet += log(A[(size_t)j * n + j]);
    logdet *= 2;

    for (int i = 0; i < n; ++i) { ones[i] = 1; yv[i] = (REAL)y[i]; }
    forward_solve(n, A, ones, a);
    forward_solve(n, A, yv, b);

    /* eq. 3: mu = (1'R^-1 1)^-1 1'R^-1 y = (a.b)/(a.a) */
    REAL aa = 0, ab = 0;
    for (int i = 0; i < n; ++i) { aa += a[i] * a[i]; ab += a[i] * b[i]; }
    REAL mu = ab / aa;
    /* Q = (y - 1 mu)' R^-1 (y - 1 mu) = |b - mu a|^2, evaluated in two passes */
    REAL Q = 0;
    for (int i = 0; i < n; ++i) { REAL r = b[i] - mu * a[i]; Q += r * r; }
    REAL sigma2 = Q / (REAL)n;
    if (mu_out) *mu_out = mu;
    if (sigma2_out) *sigma2_out = sigma2;

    out[0] = (double)logdet;
    out[1] = (double)mu;
    out[2] = (double)sigma2;
    out[5] = (double)Q;
    out[6] = (double)aa;
    out[7] = (double)ab;
    if (Q == 0) {
        out[3] = -INFINITY;
        out[4] = -INFINITY;
        return -1;
    }
    /* eq. 4 */
    REAL nll = logdet + (REAL)n * log(sigma2);
    out[3] = (double)nll;
    out[4] = (double)(logdet + (REAL)n * log(Q));
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Exported entry points (plain C ABI for ctypes).                          */

/* R_delta for one theta, full symmetric, row-major, written as double. */
int SFX(orc_corr)(int n, int d, const double *X, const double *theta,
                  double p, int fam, double delta, double *R_out)
{
    if (n < 1 || d < 1 || d > 64 || !family_ok(fam, p)) return -100;
    REAL th[64];
    for (int k = 0; k < d; ++k) th[k] = (REAL)theta[k];
    REAL *R = (REAL *)malloc(sizeof(REAL) * (size_t)n * n);
    if (!R) return -101;
    build_corr(n, d, X, th, (REAL)p, fam, (REAL)delta, R);
    for (size_t q = 0; q < (size_t)n * n; ++q) R_out[q] = (double)R[q];
    free(R);
    return 0;
}

/* Cholesky of a caller matrix (row-major n x n, double in, double out). */
int SFX(orc_cholesky)(int n, const double *A_in, double *L_out)
{
    REAL *A = (REAL *)malloc(sizeof(REAL) * (size_t)n * n);
    if (!A) return -101;
    for (size_t q = 0; q < (size_t)n * n; ++q) A[q] = (REAL)A_in[q];
    int info = cholesky(n, A);
    for (size_t q = 0; q < (size_t)n * n; ++q) L_out[q] = (double)A[q];
    free(A);
    return info;
}

/* Full evaluation for B thetas (row-major B x d).  out: B x ORC_NOUT,
 * info: B.  nthreads <= 0 uses the OpenMP default. Returns -100 on invalid
 * sizes/scalars, else 0. */
int SFX(orc_nll_batch)(int n, int d, const double *X, const double *y,
                       int B, const double *theta, double p, int fam, double delta,
                       double *out, int32_t *info, int nthreads)
{
    if (n < 1 || d < 1 || d > 64 || B < 0) return -100;
    if (!family_ok(fam, p) || !(delta >= 0) || !isfinite(delta)) return -100;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#else
    nthreads = 1;
#endif
    int status = 0;
#pragma omp parallel num_threads(nthreads)
    {
        REAL *work = (REAL *)malloc(sizeof(REAL) * ((size_t)n * n + 4 * (size_t)n));
        if (!work) {
#pragma omp atomic write
            status = -101;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (int t = 0; t < B; ++t)
                info[t] = eval_one(n, d, X, y, theta + (size_t)t * d, (REAL)p, fam,
                                   (REAL)delta, out + (size_t)t * ORC_NOUT, work, NULL, NULL);
            free(work);
        }
    }
    return status;
}

/* Gradient of nll = log|R| + n ln(sigma2) with respect to theta.
 * d nll / d theta_k = tr(R^-1 dR_k) - n * alpha' dR_k alpha / Q, with
 * alpha = R^-1 (y - 1 mu), dR_k,ij = -R_ij G_k,ij (i != j) with
 * G_k,ij = -d ln(factor_k) / d theta_k (|x_ik - x_jk|^p for eq. 2).
 * The mu derivative drops out because 1' alpha = 0 at mu = mu_hat.
 * R^-1 is formed column by column from the Cholesky factor (n forward and
 * back solves).  grad: B x d.  Also fills `out` like orc_nll_batch. */
int SFX(orc_grad_batch)(int n, int d, const double *X, const double *y,
                        int B, const double *theta, double p, int fam, double delta,
                        double *out, int32_t *info, double *grad, int nthreads)
{
    if (n < 1 || d < 1 || d > 64 || B < 0) return -100;
    if (!family_ok(fam, p) || !(delta >= 0) || !isfinite(delta)) return -100;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#else
    nthreads = 1;
#endif
    int status = 0;
#pragma omp parallel num_threads(nthreads)
    {
        size_t nn = (size_t)n * n;
        REAL *work = (REAL *)malloc(sizeof(REAL) * (3 * nn + 8 * (size_t)n));
        if (!work) {
#pragma omp atomic write
            status = -101;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (int t = 0; t < B; ++t) {
                const double *th_in = theta + (size_t)t * d;
                double *o = out + (size_t)t * ORC_NOUT;
                double *g = grad + (size_t)t * d;
                REAL *L = work;              /* factor */
                REAL *R = work + nn;         /* R_delta */
                REAL *Ri = work + 2 * nn;    /* R_delta^-1 */
                REAL *v = work + 3 * nn;
                REAL *z = v + n, *w = z + n, *alpha = w + n;
                REAL mu = 0;
                int inf = eval_one(n, d, X, y, th_in, (REAL)p, fam, (REAL)delta, o, work, &mu, NULL);
                info[t] = inf;
                if (inf != 0) {
                    for (int k = 0; k < d; ++k) g[k] = NAN;
                    continue;
                }
                REAL th[64];
                for (int k = 0; k < d; ++k) th[k] = (REAL)th_in[k];
                build_corr(n, d, X, th, (REAL)p, fam, (REAL)delta, R);
                memcpy(L, R, sizeof(REAL) * nn);
                cholesky(n, L);
                for (int c = 0; c < n; ++c) {
                    for (int i = 0; i < n; ++i) v[i] = (i == c);
                    forward_solve(n, L, v, z);
                    back_solve(n, L, z, w);
                    for (int i = 0; i < n; ++i) Ri[(size_t)i * n + c] = w[i];
                }
                for (int i = 0; i < n; ++i) v[i] = (REAL)y[i] - mu;
                forward_solve(n, L, v, z);
                back_solve(n, L, z, alpha);
                REAL Q = 0;
                for (int i = 0; i < n; ++i) Q += v[i] * alpha[i];
                for (int k = 0; k < d; ++k) {
                    REAL gk = 0;
                    for (int i = 0; i < n; ++i)
                        for (int j = 0; j < n; ++j) {
                            if (i == j) continue;
                            REAL diff = fabs((REAL)X[(size_t)i * d + k] - (REAL)X[(size_t)j * d + k]);
                            REAL G = corr_dlog(fam, diff, th[k], (REAL)p);
                            gk += R[(size_t)i * n + j] * G *
                                  ((REAL)n / Q * alpha[i] * alpha[j] - Ri[(size_t)i * n + j]);
                        }
                    g[k] = (double)gk;
                }
            }
            free(work);
        }
    }
    return status;
}

/* Predictions at N test points with the fitted model (Sec. 3: predictions
 * use one R, one factorisation and back-solves per test point; Sec. 4: the
 * SSPE over a test set).  The paper does not print the predictor; this is
 * the best linear unbiased predictor of the model of Sec. 2 and its mean
 * squared error, written from their definitions with R_delta applied
 * through forward and back solves:
 *   r_i(x)  = prod_k factor_k(|x_k - x_ik|)              (eq. 2, no nugget)
 *   mean(x) = mu + r(x)' R^-1 (y - 1 mu)
 *   mse(x)  = sigma2 (1 - r' R^-1 r + (1 - 1' R^-1 r)^2 / (1' R^-1 1))
 * with mu, sigma2 of eq. 3.  Xs: N x d row-major.  fit: ORC_NOUT values as
 * orc_nll_batch.  Returns info as orc_nll_batch (outputs NaN unless 0). */
int SFX(orc_predict)(int n, int d, const double *X, const double *y, const double *theta_in,
                     double p_in, int fam, double delta_in, int N, const double *Xs,
                     double *fit, double *mean, double *mse)
{
    if (n < 1 || d < 1 || d > 64 || N < 0) return -100;
    if (!family_ok(fam, p_in) || !(delta_in >= 0) || !isfinite(delta_in)) return -100;
    const REAL p = (REAL)p_in, delta = (REAL)delta_in;
    size_t nn = (size_t)n * n;
    REAL *work = (REAL *)malloc(sizeof(REAL) * (2 * nn + 8 * (size_t)n));
    if (!work) return -101;
    REAL mu = 0, sigma2 = 0;
    int info = eval_one(n, d, X, y, theta_in, p, fam, delta, fit, work, &mu, &sigma2);
    if (info != 0 && info != -1) {
        for (int j = 0; j < N; ++j) mean[j] = mse[j] = NAN;
        free(work);
        return info;
    }
    REAL th[64];
    for (int k = 0; k < d; ++k) th[k] = (REAL)theta_in[k];
    REAL *L = work + nn;
    REAL *v = work + 2 * nn, *z = v + n, *alpha = z + n, *u = alpha + n, *r = u + n;
    REAL *one_inv = r + n;
    build_corr(n, d, X, th, p, fam, delta, L);
    cholesky(n, L);
    /* alpha = R^-1 (y - 1 mu), R^-1 1 */
    for (int i = 0; i < n; ++i) v[i] = (REAL)y[i] - mu;
    forward_solve(n, L, v, z);
    back_solve(n, L, z, alpha);
    for (int i = 0; i < n; ++i) v[i] = 1;
    forward_solve(n, L, v, z);
    back_solve(n, L, z, one_inv);
    REAL oRo = 0;
    for (int i = 0; i < n; ++i) oRo += one_inv[i];
    for (int j = 0; j < N; ++j) {
        for (int i = 0; i < n; ++i) {
            REAL prod = 1;
            for (int k = 0; k < d; ++k) {
                REAL diff = fabs((REAL)Xs[(size_t)j * d + k] - (REAL)X[(size_t)i * d + k]);
                prod *= corr_factor(fam, diff, th[k], p);
            }
            r[i] = prod;
        }
        /* u = R^-1 r by a forward and a back solve */
        forward_solve(n, L, r, z);
        back_solve(n, L, z, u);
        REAL m = mu, rRr = 0, oRr = 0;
        for (int i = 0; i < n; ++i) {
            m += r[i] * alpha[i];
            rRr += r[i] * u[i];
            oRr += u[i];
        }
        mean[j] = (double)m;
        mse[j] = (double)(sigma2 * (1 - rRr + (1 - oRr) * (1 - oRr) / oRo));
    }
    free(work);
    return info;
}

int SFX(orc_nout)(void) { return ORC_NOUT; }
