// Correlation build R_delta (paper Sec. 2, eq. 2, plus the nugget on the
// diagonal) and per-theta initialisation.
//
// One workgroup owns one 64 x 64 tile on or below the diagonal and a chunk of
// thetas.  The two 64-point slabs of X are staged in LDS (dimension-major so
// that consecutive lanes read consecutive points); the power terms
// |x_ik - x_jk|^p do not depend on theta, so each lane computes them once per
// entry and reuses them for every theta in the chunk.  The product of
// exponentials in eq. 2 is evaluated as one exponential of the sum (the
// Matern families: one exponential of the sum times the product of the
// per-dimension polynomials).  The kernel is bound by the HBM writes of R
// (8 bytes per entry per theta); for p outside {1, 2} the FP64 pow() per
// (entry, dimension) is amortised over the theta chunk.
#include <math.h>

#include "kernels.hpp"

namespace gpk {

namespace {

constexpr int CB_THREADS = 256;
#ifndef CB_CHUNK_N
#define CB_CHUNK_N 128
#endif
constexpr int CB_CHUNK = CB_CHUNK_N;   // most thetas per workgroup

__global__ void init_kernel(const double *__restrict__ theta, int d, int batch,
                            int32_t *__restrict__ info, const uint8_t *__restrict__ mask)
{
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch || (mask && !mask[b])) return;
    int ok = 1;
    for (int k = 0; k < d; ++k) {
        double t = theta[(size_t)b * d + k];
        if (!(t >= 0.0) || !isfinite(t)) ok = 0;
    }
    info[b] = ok ? 0 : -3;
}

__device__ __forceinline__ void tile_of(int t, int &ti, int &tj)
{
    // lower tiles enumerated row by row: t = ti (ti + 1) / 2 + tj, tj <= ti
    int r = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while ((r + 1) * (r + 2) / 2 <= t) ++r;
    while (r * (r + 1) / 2 > t) --r;
    ti = r;
    tj = t - r * (r + 1) / 2;
}

template <int DM, int PMODE>  // PMODE: see corr_term / corr_value
__global__ __launch_bounds__(CB_THREADS)
void corr_build_kernel(const double *__restrict__ X, int n, int d, double p, double delta,
                       const double *__restrict__ theta, int batch, int chunk,
                       double *__restrict__ R, int lda, size_t bstride,
                       const uint8_t *__restrict__ mask)
{
    __shared__ double xi[DM][TB];
    __shared__ double xj[DM][TB];
    __shared__ double th[CB_CHUNK][DM];

    int ti, tj;
    tile_of(blockIdx.x, ti, tj);
    const int tid = threadIdx.x;
    const int b0 = blockIdx.y * chunk;
    const int nb = min(chunk, batch - b0);   // chunk <= CB_CHUNK
    if (mask) {   // a chunk with no selected theta has nothing to write
        int any = 0;
        for (int c = 0; c < nb; ++c) any |= mask[b0 + c];
        if (!any) return;   // uniform over the workgroup
    }

    for (int e = tid; e < DM * TB; e += CB_THREADS) {
        int k = e / TB, q = e % TB;
        int gi = ti * TB + q, gj = tj * TB + q;
        xi[k][q] = (k < d && gi < n) ? X[(size_t)gi * d + k] : 0.0;
        xj[k][q] = (k < d && gj < n) ? X[(size_t)gj * d + k] : 0.0;
    }
    for (int e = tid; e < CB_CHUNK * DM; e += CB_THREADS) {
        int c = e / DM, k = e % DM;
        th[c][k] = (c < nb && k < d) ? theta[(size_t)(b0 + c) * d + k] : 0.0;
    }
    __syncthreads();

    const int i = tid % TB;              // row within the tile
    const int gi = ti * TB + i;
    double *Rb = R + (size_t)b0 * bstride;

    for (int m = 0; m < TB / (CB_THREADS / TB); ++m) {
        const int j = tid / TB + m * (CB_THREADS / TB);
        const int gj = tj * TB + j;
        const size_t off = (size_t)gi + (size_t)gj * lda;
        if (gi >= n || gj >= n || gi == gj) {
            double v = (gi == gj) ? ((gi < n) ? 1.0 + delta : 1.0) : 0.0;
            for (int c = 0; c < nb; ++c)
                if (!mask || mask[b0 + c]) Rb[off + (size_t)c * bstride] = v;
            continue;
        }
        double D[DM];
#pragma unroll
        for (int k = 0; k < DM; ++k)
            D[k] = (k < d) ? corr_term<PMODE>(fabs(xi[k][i] - xj[k][j]), p) : 0.0;
        for (int c = 0; c < nb; ++c) {
            if (mask && !mask[b0 + c]) continue;
            Rb[off + (size_t)c * bstride] = corr_value<PMODE, DM>(th[c], D);
        }
    }
}

__global__ void pad_identity_kernel(double *__restrict__ A, int lda, size_t bstride, int n,
                                    int np)
{
    // rows/cols in [n, np): grid.x covers np * (np - n) entries of the lower part
    const int b = blockIdx.y;
    const int w = np - n;
    const size_t total = (size_t)np * w;
    double *Ab = A + (size_t)b * bstride;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        int r = (int)(e % np);       // any row
        int c = n + (int)(e / np);   // padded column
        // column c (padded) and row c (padded): identity pattern
        Ab[(size_t)r + (size_t)c * lda] = (r == c) ? 1.0 : 0.0;
        Ab[(size_t)c + (size_t)r * lda] = (r == c) ? 1.0 : 0.0;
    }
}

template <int DM>
void launch_corr_dm(const double *X, int n, int d, double p, double delta, const double *theta,
                    int batch, double *R, int lda, size_t bstride, int np, hipStream_t s,
                    const uint8_t *mask)
{
    const int T = np / TB;
    // thetas per workgroup: CB_CHUNK where there are tiles enough to fill the
    // GPU, fewer for small matrices (more workgroups, power terms recomputed)
    const long tiles = (long)T * (T + 1) / 2;
    int chunk = CB_CHUNK;
    while (chunk > 8 && tiles * ((batch + chunk - 1) / chunk) < 1024) chunk /= 2;
    dim3 grid((unsigned)tiles, (batch + chunk - 1) / chunk);
#define GPK_CORR_LAUNCH(PM)                                                                  \
    corr_build_kernel<DM, PM><<<grid, CB_THREADS, 0, s>>>(X, n, d, p, delta, theta, batch,    \
                                                          chunk, R, lda, bstride, mask)
    GPK_DISPATCH_PMODE(p, GPK_CORR_LAUNCH);
#undef GPK_CORR_LAUNCH
}

}  // namespace

void launch_init(const double *theta, int d, int batch, int32_t *info, hipStream_t s,
                 const uint8_t *mask)
{
    ProfScope ps(K_INIT, 0.0, 12.0 * batch * d, s);
    init_kernel<<<(batch + 255) / 256, 256, 0, s>>>(theta, d, batch, info, mask);
}

void launch_corr_build(const double *X, int n, int d, double p, double delta,
                       const double *theta, int batch, double *R, int lda, size_t bstride,
                       int np, hipStream_t s, const uint8_t *mask)
{
    const double lower = 0.5 * (double)np * (np + 1);
    ProfScope ps(K_CORR_BUILD, 2.0 * d * lower * batch, 8.0 * lower * batch, s);
    if (d <= 4)
        launch_corr_dm<4>(X, n, d, p, delta, theta, batch, R, lda, bstride, np, s, mask);
    else if (d <= 8)
        launch_corr_dm<8>(X, n, d, p, delta, theta, batch, R, lda, bstride, np, s, mask);
    else if (d <= 16)
        launch_corr_dm<16>(X, n, d, p, delta, theta, batch, R, lda, bstride, np, s, mask);
    else
        launch_corr_dm<GP_DMAX>(X, n, d, p, delta, theta, batch, R, lda, bstride, np, s, mask);
}

void launch_pad_identity(double *A, int lda, size_t bstride, int n, int np, int batch,
                         hipStream_t s)
{
    if (np <= n) return;
    ProfScope ps(K_PAD, 0.0, 16.0 * np * (np - n) * batch, s);
    size_t total = (size_t)np * (np - n);
    int blocks = (int)min((size_t)1024, (total + 255) / 256);
    pad_identity_kernel<<<dim3(blocks, batch), 256, 0, s>>>(A, lda, bstride, n, np);
}

}  // namespace gpk
