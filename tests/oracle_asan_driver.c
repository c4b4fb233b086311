/* Drives every entry point of the C oracle (FP64 and 80-bit builds) on small
 * inputs, for a build with AddressSanitizer and UndefinedBehaviorSanitizer:
 * random design, several thetas (one invalid, one that makes R singular),
 * both correlation families, predictions and gradients.  Prints OK when
 * every call returned and the finite results are finite. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#define DECL(sfx)                                                                              \
    int orc_corr_##sfx(int, int, const double *, const double *, double, int, double, double *); \
    int orc_cholesky_##sfx(int, const double *, double *);                                     \
    int orc_nll_batch_##sfx(int, int, const double *, const double *, int, const double *,     \
                            double, int, double, double *, int32_t *, int);                   \
    int orc_grad_batch_##sfx(int, int, const double *, const double *, int, const double *,    \
                             double, int, double, double *, int32_t *, double *, int);        \
    int orc_predict_##sfx(int, int, const double *, const double *, const double *, double,    \
                          int, double, int, const double *, double *, double *, double *);    \
    int orc_nout_##sfx(void);
DECL(f64)
DECL(f80)

static double urand(unsigned *s) { *s = *s * 1664525u + 1013904223u; return (*s >> 8) / 16777216.0; }

#define RUN(sfx)                                                                                \
    do {                                                                                        \
        const int nout = orc_nout_##sfx();                                                      \
        double *out = malloc(sizeof(double) * nout * B), *grad = malloc(sizeof(double) * d * B); \
        int32_t info[8];                                                                        \
        double *R = malloc(sizeof(double) * n * n), *L = malloc(sizeof(double) * n * n);       \
        for (int fam = 0; fam < 3; ++fam) {                                                     \
            const double p = fam == 0 ? 1.95 : 0.0;                                             \
            if (orc_nll_batch_##sfx(n, d, X, y, B, th, p, fam, 1e-6, out, info, 2) != 0) bad++; \
            if (orc_grad_batch_##sfx(n, d, X, y, B, th, p, fam, 1e-6, out, info, grad, 2) != 0) \
                bad++;                                                                          \
            for (int t = 0; t < B; ++t)                                                         \
                if (info[t] == 0 && !isfinite(out[(size_t)t * nout + 3])) bad++;                \
            if (orc_corr_##sfx(n, d, X, th, p, fam, 1e-6, R) != 0) bad++;                       \
            if (orc_cholesky_##sfx(n, R, L) != 0) bad++;                                        \
            double fit[16], mean[5], mse[5];                                                    \
            if (orc_predict_##sfx(n, d, X, y, th, p, fam, 1e-6, 5, Xs, fit, mean, mse) != 0)    \
                bad++;                                                                          \
        }                                                                                       \
        free(out); free(grad); free(R); free(L);                                                \
    } while (0)

int main(void)
{
    enum { n = 37, d = 3, B = 5 };
    unsigned s = 7;
    double X[n * d], y[n], Xs[5 * d], th[B * d];
    for (int i = 0; i < n * d; ++i) X[i] = urand(&s);
    for (int i = 0; i < n; ++i) y[i] = sin(6.0 * X[i * d]) + 0.01 * urand(&s);
    for (int i = 0; i < 5 * d; ++i) Xs[i] = urand(&s);
    for (int i = 0; i < B * d; ++i) th[i] = 0.5 + 5.0 * urand(&s);
    th[1 * d + 1] = -1.0;                                   /* invalid theta */
    for (int k = 0; k < d; ++k) th[3 * d + k] = 0.0;        /* R = all ones + nugget */
    int bad = 0;
    RUN(f64);
    RUN(f80);
    printf(bad ? "BAD %d\n" : "OK\n", bad);
    return bad != 0;
}
