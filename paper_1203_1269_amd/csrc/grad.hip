// Adjoint gradient of nll = log|R| + n ln(sigma2) with respect to theta.
//
// With r = y - 1 mu and alpha = R^-1 r (mu at its optimum, so 1' alpha = 0
// and the mu derivative drops out):
//   d nll / d theta_k = tr(R^-1 dR_k) - n alpha' dR_k alpha / Q,
//   dR_k,ij = -R_ij G_k,ij (i != j), G_k,ij = -d ln R_ij / d theta_k
//   (|x_ik - x_jk|^p for eq. 2; corr_dlog for the Matern families),
// i.e. g_k = sum_{i != j} R_ij G_k,ij ((n/Q) alpha_i alpha_j - (R^-1)_ij).
// Gradient methods are what the paper names as the alternative to the
// genetic algorithm for maximising the likelihood (Sec. 2).
//
// R^-1 comes from the factorisation of the bordered matrix
//     [ R  I ]        [ L      0 ] [ L'  L^-1 ]
//     [ I  0 ]   =    [ L^-T   * ] [ 0   *    ]
// carried through its first n_pad columns only: the TRSM steps produce
// L^-T in the bottom-left block and the trailing updates leave
// 0 - L^-T L^-1 = -R^-1 in the bottom-right block.  Row i of the border is
// zero left of column i, so each step only touches border rows it can reach
// (the row limits in factor_bordered), which keeps the cost at the n^3 of a
// Cholesky factorisation plus inversion, all on the same MFMA kernels.
#include <math.h>

#include "kernels.hpp"

namespace gpk {

namespace {

constexpr int GR_THREADS = 256;

// Border of the augmented matrix: identity in the bottom-left block, zero in
// the bottom-right block (only its lower triangle is ever read).
__global__ void border_init_kernel(double *__restrict__ A0, int lda, size_t bstride, int np)
{
    const int b = blockIdx.y;
    double *A = A0 + (size_t)b * bstride;
    const size_t per = (size_t)np * np;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < 2 * per;
         e += (size_t)gridDim.x * blockDim.x) {
        const size_t q = e % per;
        const int r = (int)(q % np), c = (int)(q / np);
        if (e < per)
            A[(size_t)(np + r) + (size_t)c * lda] = (r == c) ? 1.0 : 0.0;          // bottom-left
        else
            A[(size_t)(np + r) + (size_t)(np + c) * lda] = 0.0;                     // bottom-right
    }
}

// alpha = R^-1 (y - 1 mu) = -M (y - 1 mu), M = bottom-right block (lower
// triangle stored).  One workgroup per (64-row block I, theta); wave w takes
// the column blocks J = w, w+4, ...; tiles above the diagonal are read as the
// transpose of the stored tile through a per-wave LDS buffer.
__global__ __launch_bounds__(GR_THREADS)
void alpha_kernel(const double *__restrict__ A0, int lda, size_t bstride, int np, int n,
                  const double *__restrict__ y, const gp_result *__restrict__ res,
                  double *__restrict__ alpha)
{
    __shared__ double tr[4][TB][TB + 1];
    __shared__ double rv[4][TB];
    __shared__ double part[4][TB];
    const int I = blockIdx.x, b = blockIdx.y;
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const double *A = A0 + (size_t)b * bstride;
    const double mu = res[b].mu;
    const int T = np / TB;
    const int i = I * TB + lane;
    double acc = 0.0;
    for (int J = wave; J < T; J += 4) {
        const int j = J * TB + lane;
        rv[wave][lane] = (j < n) ? y[j] - mu : 0.0;
        if (J <= I) {
            // stored tile (I, J): lane = row i, loop over the columns
            const double *p = A + (size_t)(np + i) + (size_t)(np + J * TB) * lda;
            __builtin_amdgcn_wave_barrier();
#pragma unroll 8
            for (int jj = 0; jj < TB; ++jj) acc = fma(p[(size_t)jj * lda], rv[wave][jj], acc);
        } else {
            // tile (J, I) stored; transpose through LDS
            const double *p = A + (size_t)(np + J * TB) + (size_t)(np + I * TB) * lda;
#pragma unroll 8
            for (int ii = 0; ii < TB; ++ii) tr[wave][ii][lane] = p[(size_t)lane + (size_t)ii * lda];
            __builtin_amdgcn_wave_barrier();
#pragma unroll 8
            for (int jj = 0; jj < TB; ++jj) acc = fma(tr[wave][lane][jj], rv[wave][jj], acc);
        }
        __builtin_amdgcn_wave_barrier();
    }
    part[wave][lane] = acc;
    __syncthreads();
    if (wave == 0) {
        const double s = part[0][lane] + part[1][lane] + part[2][lane] + part[3][lane];
        alpha[(size_t)b * np + i] = (i < n) ? -s : 0.0;
    }
}

// Per (lower 64 x 64 tile, theta): sum over the tile's pairs i > j of
// w_ij G_k,ij with w_ij = R_ij ((n/Q) alpha_i alpha_j + M_ij), M = -R^-1.
// R_ij and G_k,ij are regenerated from X; M_ij is read from the factor.
template <int DM, int PMODE>
__global__ __launch_bounds__(GR_THREADS)
void adjoint_tile_kernel(const double *__restrict__ A0, int lda, size_t bstride, int np, int n,
                         int d, double p, const double *__restrict__ X,
                         const double *__restrict__ theta, const double *__restrict__ alpha,
                         const gp_result *__restrict__ res, double *__restrict__ part)
{
    __shared__ double xi[DM][TB], xj[DM][TB], ai[TB], aj[TB], th[DM];
    __shared__ double red[GR_THREADS / 64][DM];
    const int t = blockIdx.x, b = blockIdx.y;
    int I = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while ((I + 1) * (I + 2) / 2 <= t) ++I;
    while (I * (I + 1) / 2 > t) --I;
    const int J = t - I * (I + 1) / 2;
    const int tid = threadIdx.x;
    for (int e = tid; e < DM * TB; e += GR_THREADS) {
        const int k = e / TB, q = e % TB;
        const int gi = I * TB + q, gj = J * TB + q;
        xi[k][q] = (k < d && gi < n) ? X[(size_t)gi * d + k] : 0.0;
        xj[k][q] = (k < d && gj < n) ? X[(size_t)gj * d + k] : 0.0;
    }
    if (tid < TB) {
        ai[tid] = alpha[(size_t)b * np + I * TB + tid];
        aj[tid] = alpha[(size_t)b * np + J * TB + tid];
    }
    if (tid < DM) th[tid] = (tid < d) ? theta[(size_t)b * d + tid] : 0.0;
    __syncthreads();

    const double nq = (double)n / (res[b].sigma2 * (double)n);   // n / Q
    const double *A = A0 + (size_t)b * bstride;
    const int i = tid % TB, gi = I * TB + i;
    double acc[DM];
#pragma unroll
    for (int k = 0; k < DM; ++k) acc[k] = 0.0;
    for (int m = 0; m < TB / (GR_THREADS / TB); ++m) {
        const int j = tid / TB + m * (GR_THREADS / TB);
        const int gj = J * TB + j;
        if (gi >= n || gj >= n || gi <= gj) continue;
        double D[DM];
#pragma unroll
        for (int k = 0; k < DM; ++k)
            D[k] = (k < d) ? corr_term<PMODE>(fabs(xi[k][i] - xj[k][j]), p) : 0.0;
        const double Rij = corr_value<PMODE, DM>(th, D);
        const double Mij = A[(size_t)(np + gi) + (size_t)(np + gj) * lda];
        const double wgt = Rij * fma(nq * ai[i], aj[j], Mij);
#pragma unroll
        for (int k = 0; k < DM; ++k) acc[k] = fma(wgt, corr_dlog<PMODE>(th[k], D[k]), acc[k]);
    }
    const int wave = tid / 64, lane = tid % 64;
#pragma unroll
    for (int k = 0; k < DM; ++k) {
        double v = acc[k];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) red[wave][k] = v;
    }
    __syncthreads();
    if (tid < d) {
        double v = 0.0;
        for (int w = 0; w < GR_THREADS / 64; ++w) v += red[w][tid];
        part[((size_t)b * gridDim.x + t) * d + tid] = v;
    }
}

// grad[b][k] = 2 sum over tiles (pairs i > j stand for both orders), in a
// fixed order; NaN when the evaluation failed.
__global__ void grad_reduce_kernel(const double *__restrict__ part, int ntiles, int d,
                                   const gp_result *__restrict__ res, double *__restrict__ grad)
{
    const int b = blockIdx.x;
    for (int k = threadIdx.x; k < d; k += blockDim.x) {
        double v = 0.0;
        for (int t = 0; t < ntiles; ++t) v += part[((size_t)b * ntiles + t) * d + k];
        grad[(size_t)b * d + k] = (res[b].info == 0) ? 2.0 * v : NAN;
    }
}

template <int DM>
void launch_adjoint_dm(const double *A, int lda, size_t bstride, int np, int n, int d, double p,
                       const double *X, const double *theta, const double *alpha,
                       const gp_result *res, double *part, int batch, hipStream_t s)
{
    const int T = np / TB;
    dim3 grid(T * (T + 1) / 2, batch);
#define GPK_ADJ_LAUNCH(PM)                                                                  \
    adjoint_tile_kernel<DM, PM><<<grid, GR_THREADS, 0, s>>>(A, lda, bstride, np, n, d, p, X, \
                                                            theta, alpha, res, part)
    GPK_DISPATCH_PMODE(p, GPK_ADJ_LAUNCH);
#undef GPK_ADJ_LAUNCH
}

}  // namespace

void launch_border_init(double *A, int lda, size_t bstride, int np, int batch, hipStream_t s)
{
    ProfScope ps(K_BORDER, 0.0, 16.0 * np * np * batch, s);
    const size_t total = (size_t)2 * np * np;
    const int blocks = (int)min((size_t)4096, (total + 255) / 256);
    border_init_kernel<<<dim3(blocks, batch), 256, 0, s>>>(A, lda, bstride, np);
}

void launch_alpha(const double *A, int lda, size_t bstride, int np, int n, const double *y,
                  const gp_result *res, double *alpha, int batch, hipStream_t s)
{
    ProfScope ps(K_ALPHA, 2.0 * np * np * batch, 8.0 * np * np * batch, s);
    alpha_kernel<<<dim3(np / TB, batch), GR_THREADS, 0, s>>>(A, lda, bstride, np, n, y, res, alpha);
}

void launch_adjoint(const double *A, int lda, size_t bstride, int np, int n, int d, double p,
                    const double *X, const double *theta, const double *alpha,
                    const gp_result *res, double *part, double *grad, int batch, hipStream_t s)
{
    const int T = np / TB;
    const int ntiles = T * (T + 1) / 2;
    {
        const double pairs = 0.5 * (double)np * np;
        ProfScope ps(K_ADJOINT, (4.0 * d + 6.0) * pairs * batch, 8.0 * pairs * batch, s);
        if (d <= 4)
            launch_adjoint_dm<4>(A, lda, bstride, np, n, d, p, X, theta, alpha, res, part, batch, s);
        else if (d <= 8)
            launch_adjoint_dm<8>(A, lda, bstride, np, n, d, p, X, theta, alpha, res, part, batch, s);
        else if (d <= 16)
            launch_adjoint_dm<16>(A, lda, bstride, np, n, d, p, X, theta, alpha, res, part, batch, s);
        else
            launch_adjoint_dm<GP_DMAX>(A, lda, bstride, np, n, d, p, X, theta, alpha, res, part,
                                       batch, s);
    }
    grad_reduce_kernel<<<batch, 64, 0, s>>>(part, ntiles, d, res, grad);
}

}  // namespace gpk
