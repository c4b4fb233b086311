// Predictions with the fitted model at N test points (the paper obtains them
// with one R, one Cholesky factorisation and back-solves per test point,
// Sec. 3, and scores them by the SSPE over a test set, Sec. 4).
//
// The right-hand sides [1 y] and the cross-correlations r(x*_j) are stored as
// extra rows below the padded matrix and are factored with it: the TRSM and
// trailing updates treat them as rows below the diagonal, which leaves
// a = L^-1 1, b = L^-1 y and w_j = L^-1 r(x*_j) in those rows.  Then
//   mu = a.b / a.a,  Q = |b - mu a|^2,  sigma2 = Q / n               (eq. 3)
//   mean_j = mu + w_j.(b - mu a)                = mu + r' R^-1 (y - 1 mu)
//   mse_j  = sigma2 (1 - w_j.w_j + (1 - a.w_j)^2 / a.a)
// (r' R^-1 r = w.w, 1' R^-1 r = a.w, 1' R^-1 1 = a.a).
#include <math.h>

#include "kernels.hpp"

namespace gpk {
namespace {

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// one thread per (extra row, column), looping over the thetas: the
// theta-independent per-dimension terms of a (test point, design point) pair
// are computed once and reused for every theta, as in the correlation build
template <int PMODE, int DM>
__global__ __launch_bounds__(256)
void pred_rows_kernel(double *__restrict__ A0, int lda, size_t bstride, int np,
                      const double *__restrict__ X, int n, int d, double p,
                      const double *__restrict__ y, const double *__restrict__ theta,
                      const double *__restrict__ Xs, int N, int extra, int batch)
{
    const size_t total = (size_t)extra * np;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int r = (int)(e % extra);   // row below the matrix
        const int c = (int)(e / extra);   // column = design point
        double *dst = A0 + np + (size_t)r + (size_t)c * lda;
        if (c < n && r >= TB && r - TB < N) {
            const double *xs = Xs + (size_t)(r - TB) * d;
            const double *xc = X + (size_t)c * d;
            double D[DM];
#pragma unroll
            for (int k = 0; k < DM; ++k)
                D[k] = (k < d) ? corr_term<PMODE>(fabs(xs[k] - xc[k]), p) : 0.0;
            for (int b = 0; b < batch; ++b) {
                double t[DM];
#pragma unroll
                for (int k = 0; k < DM; ++k) t[k] = (k < d) ? theta[(size_t)b * d + k] : 0.0;
                dst[(size_t)b * bstride] = corr_value<PMODE, DM>(t, D);
            }
        } else {
            double v = 0.0;
            if (c < n && r == 0) v = 1.0;
            else if (c < n && r == 1) v = y[c];
            for (int b = 0; b < batch; ++b) dst[(size_t)b * bstride] = v;
        }
    }
}

// one 256-thread workgroup per theta: the fit from rows a and b
__global__ __launch_bounds__(256)
void pred_fit_kernel(const double *__restrict__ A0, int lda, size_t bstride, int np, int n,
                     const double *__restrict__ lpart, int nparts,
                     const int32_t *__restrict__ info, gp_result *__restrict__ fit)
{
    const int b = blockIdx.x;
    __shared__ double red[4][3];
    const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
    const double *ab_rows = A0 + (size_t)b * bstride + np;
    double aa = 0.0, ab = 0.0;
    for (int i = tid; i < n; i += 256) {
        const double a = ab_rows[(size_t)i * lda], bb = ab_rows[(size_t)i * lda + 1];
        aa = fma(a, a, aa);
        ab = fma(a, bb, ab);
    }
    aa = wave_sum(aa);
    ab = wave_sum(ab);
    if (lane == 0) { red[wave][0] = aa; red[wave][1] = ab; }
    __syncthreads();
    aa = red[0][0] + red[1][0] + red[2][0] + red[3][0];
    ab = red[0][1] + red[1][1] + red[2][1] + red[3][1];
    const double mu = ab / aa;
    __syncthreads();
    double Q = 0.0;
    for (int i = tid; i < n; i += 256) {
        const double e = fma(-mu, ab_rows[(size_t)i * lda], ab_rows[(size_t)i * lda + 1]);
        Q = fma(e, e, Q);
    }
    Q = wave_sum(Q);
    double ld = 0.0;
    for (int q = tid; q < nparts; q += 256) ld += lpart[(size_t)b * nparts + q];
    ld = wave_sum(ld);
    if (lane == 0) { red[wave][0] = Q; red[wave][2] = ld; }
    __syncthreads();
    if (tid == 0) {
        Q = red[0][0] + red[1][0] + red[2][0] + red[3][0];
        ld = red[0][2] + red[1][2] + red[2][2] + red[3][2];
        gp_result res;
        res.ir_iters = 0;
        const int inf = info[b];
        if (inf != 0) {
            res.logdet = res.mu = res.sigma2 = res.nll = NAN;
            res.info = inf;
        } else if (Q == 0.0) {
            res.logdet = ld;
            res.mu = mu;
            res.sigma2 = 0.0;
            res.nll = -INFINITY;
            res.info = -1;
        } else {
            const double s2 = Q / (double)n;
            res.logdet = ld;
            res.mu = mu;
            res.sigma2 = s2;
            res.nll = ld + (double)n * log(s2);
            res.info = 0;
        }
        fit[b] = res;
    }
}

// grid (ceil(N / 64), theta); lane l of every wave <-> test point 64 x + l,
// the PP_WAVES waves split the design points and meet in LDS
constexpr int PP_WAVES = 16;

__global__ __launch_bounds__(64 * PP_WAVES)
void pred_point_kernel(const double *__restrict__ A0, int lda, size_t bstride, int np, int n,
                       int N, const gp_result *__restrict__ fit, double *__restrict__ mean,
                       double *__restrict__ mse)
{
    const int b = blockIdx.y;
    __shared__ double part[PP_WAVES][3][64];
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int j = blockIdx.x * 64 + lane;
    const double *rows = A0 + (size_t)b * bstride + np;
    const gp_result f = fit[b];
    const double mu = f.mu;
    double s1 = 0.0, s2 = 0.0, s3 = 0.0;
    if (j < N) {
        const double *wj = rows + TB + j;
        for (int i = wave; i < n; i += PP_WAVES) {
            const double a = rows[(size_t)i * lda], bb = rows[(size_t)i * lda + 1];
            const double w = wj[(size_t)i * lda];
            s1 = fma(w, fma(-mu, a, bb), s1);
            s2 = fma(w, w, s2);
            s3 = fma(a, w, s3);
        }
    }
    part[wave][0][lane] = s1;
    part[wave][1][lane] = s2;
    part[wave][2][lane] = s3;
    // a.a = 1' R^-1 1, shared by all test points of this theta
    double aa = 0.0;
    for (int i = threadIdx.x; i < n; i += 64 * PP_WAVES) {
        const double a = rows[(size_t)i * lda];
        aa = fma(a, a, aa);
    }
    aa = wave_sum(aa);
    __shared__ double aaw[PP_WAVES];
    if (lane == 0) aaw[wave] = aa;
    __syncthreads();
    if (wave == 0 && j < N) {
        aa = 0.0;
        for (int w = 0; w < PP_WAVES; ++w) aa += aaw[w];
        s1 = s2 = s3 = 0.0;
#pragma unroll
        for (int w = 0; w < PP_WAVES; ++w) {
            s1 += part[w][0][lane];
            s2 += part[w][1][lane];
            s3 += part[w][2][lane];
        }
        const size_t o = (size_t)b * N + j;
        if (f.info != 0 && f.info != -1) {
            mean[o] = mse[o] = NAN;
        } else {
            mean[o] = mu + s1;
            const double t = 1.0 - s3;
            mse[o] = f.sigma2 * (1.0 - s2 + t * t / aa);
        }
    }
}

template <int DM>
void launch_pred_rows_dm(unsigned grid, double *A, int lda, size_t bstride, int np,
                         const double *X, int n, int d, double p, const double *y,
                         const double *theta, const double *Xs, int N, int extra, int batch,
                         hipStream_t s)
{
#define GPK_PRED_LAUNCH(PM)                                                                   \
    pred_rows_kernel<PM, DM><<<grid, 256, 0, s>>>(A, lda, bstride, np, X, n, d, p, y, theta, \
                                                  Xs, N, extra, batch)
    GPK_DISPATCH_PMODE(p, GPK_PRED_LAUNCH);
#undef GPK_PRED_LAUNCH
}

}  // namespace

void launch_pred_rows(double *A, int lda, size_t bstride, int np, const double *X, int n, int d,
                      double p, const double *y, const double *theta, const double *Xs, int N,
                      int extra, int batch, hipStream_t s)
{
    ProfScope ps(K_PRED_ROWS, 3.0 * d * (double)N * n * batch, 8.0 * extra * (double)np * batch,
                 s);
    const size_t total = (size_t)extra * np;
    const unsigned grid = (unsigned)min((total + 255) / 256, (size_t)16384);
    if (d <= 8)
        launch_pred_rows_dm<8>(grid, A, lda, bstride, np, X, n, d, p, y, theta, Xs, N, extra,
                               batch, s);
    else
        launch_pred_rows_dm<GP_DMAX>(grid, A, lda, bstride, np, X, n, d, p, y, theta, Xs, N,
                                     extra, batch, s);
}

void launch_pred_reduce(const double *A, int lda, size_t bstride, int np, int n,
                        const double *lpart, int nparts, const int32_t *info, int N, int batch,
                        gp_result *fit, double *mean, double *mse, hipStream_t s)
{
    ProfScope ps(K_PRED_REDUCE, 6.0 * (double)n * (N + 1) * batch,
                 8.0 * (double)n * (N + 2) * batch, s);
    pred_fit_kernel<<<batch, 256, 0, s>>>(A, lda, bstride, np, n, lpart, nparts, info, fit);
    if (N > 0) {
        dim3 grid((N + 63) / 64, batch);
        pred_point_kernel<<<grid, 64 * PP_WAVES, 0, s>>>(A, lda, bstride, np, n, N, fit, mean,
                                                         mse);
    }
}

}  // namespace gpk
