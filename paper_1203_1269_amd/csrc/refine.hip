// Iterative refinement of the two solves R x = [1 y] for the mixed-precision
// mode.  The factor L comes from a factorisation whose trailing updates ran
// in FP32, so x = L^-T L^-1 v is only FP32-accurate; each sweep computes the
// residual s = v - R x in FP64 with R regenerated from X (no FP64 copy of R
// is kept) and adds the correction L^-T L^-1 s.  Then
//   mu = 1'x_1 / 1'x_1 ... = (1'R^-1 y) / (1'R^-1 1)    (eq. 3),
//   Q  = (y - 1 mu)' (x_y - mu x_1) = (y - 1 mu)' R^-1 (y - 1 mu),
// and nll = log|R| + n ln(Q/n) with log|R| from the factor's diagonal
// (refinement cannot change it; its error is that of the factorisation).
#include <math.h>

#include "kernels.hpp"

namespace gpk {

namespace {

constexpr int RS_THREADS = 1024;
constexpr int RS_WAVES = RS_THREADS / 64;

__device__ __forceinline__ double wsum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// x = L^-T L^-1 v for the two right-hand sides v = rhs[b][0..np), rhs[b][np..2np)
// (in place in x: x[b][0..2np)).  One workgroup per matrix, z and x kept in LDS.
__global__ __launch_bounds__(RS_THREADS)
void solve2_kernel(const double *__restrict__ A0, int lda, size_t bstride, int np,
                   const double *rhs, double *x)   // rhs and x may be the same buffer
{
    extern __shared__ double zs[];   // z0[np], z1[np]
    __shared__ double part[RS_WAVES][2][64];
    double *z0 = zs, *z1 = zs + np;
    const int b = blockIdx.x;
    const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
    const double *A = A0 + (size_t)b * bstride;
    const double *v = rhs + (size_t)b * 2 * np;
    const int T = np / TB;

    // forward: L z = v, 64-row blocks top-down
    for (int ib = 0; ib < T; ++ib) {
        const int r = ib * TB + lane;
        double s0 = 0.0, s1 = 0.0;
        for (int c = wave; c < ib * TB; c += RS_WAVES) {
            const double l = A[(size_t)r + (size_t)c * lda];
            s0 = fma(l, z0[c], s0);
            s1 = fma(l, z1[c], s1);
        }
        part[wave][0][lane] = s0;
        part[wave][1][lane] = s1;
        __syncthreads();
        if (wave == 0) {
            double t0 = v[r], t1 = v[np + r];
            for (int w = 0; w < RS_WAVES; ++w) { t0 -= part[w][0][lane]; t1 -= part[w][1][lane]; }
            double Lrow[TB];
            const double *pd = A + r + (size_t)ib * TB * lda;
#pragma unroll
            for (int j = 0; j < TB; ++j) Lrow[j] = pd[(size_t)j * lda];
#pragma unroll
            for (int j = 0; j < TB; ++j) {
                const double q0 = __shfl(t0 / Lrow[j], j, 64);
                const double q1 = __shfl(t1 / Lrow[j], j, 64);
                if (lane == j) { t0 = q0; t1 = q1; }
                else if (lane > j) { t0 = fma(-Lrow[j], q0, t0); t1 = fma(-Lrow[j], q1, t1); }
            }
            z0[r] = t0;
            z1[r] = t1;
        }
        __syncthreads();
    }
    // backward: L' x = z, 64-row blocks bottom-up; x overwrites z in LDS.
    // Column i of L below the block is contiguous: wave w takes the columns
    // i = w, w + 16, ... of the block and reduces over the rows below.
    for (int ib = T - 1; ib >= 0; --ib) {
        const int below = (ib + 1) * TB;
        for (int ci = wave; ci < TB; ci += RS_WAVES) {
            const int i = ib * TB + ci;
            double s0 = 0.0, s1 = 0.0;
            for (int m = below + lane; m < np; m += 64) {
                const double l = A[(size_t)m + (size_t)i * lda];
                s0 = fma(l, z0[m], s0);
                s1 = fma(l, z1[m], s1);
            }
            s0 = wsum(s0);
            s1 = wsum(s1);
            if (lane == 0) { part[0][0][ci] = s0; part[0][1][ci] = s1; }
        }
        __syncthreads();
        if (wave == 0) {
            const int i = ib * TB + lane;
            double t0 = z0[i] - part[0][0][lane];
            double t1 = z1[i] - part[0][1][lane];
            // lane i holds column i of the diagonal block: Lcol[j] = L(j, i)
            double Lcol[TB];
            const double *pc = A + (size_t)ib * TB + (size_t)i * lda;
#pragma unroll
            for (int j = 0; j < TB; ++j) Lcol[j] = pc[j];
#pragma unroll
            for (int j = TB - 1; j >= 0; --j) {
                // lane j finishes x_j = t_j / L_jj; lanes i < j subtract L(j, i) x_j
                const double q0 = __shfl(t0 / Lcol[j], j, 64);
                const double q1 = __shfl(t1 / Lcol[j], j, 64);
                if (lane == j) { t0 = q0; t1 = q1; }
                else if (lane < j) { t0 = fma(-Lcol[j], q0, t0); t1 = fma(-Lcol[j], q1, t1); }
            }
            z0[i] = t0;
            z1[i] = t1;
        }
        __syncthreads();
    }
    double *xo = x + (size_t)b * 2 * np;
    for (int r = tid; r < np; r += RS_THREADS) { xo[r] = z0[r]; xo[np + r] = z1[r]; }
}

constexpr int RF_THREADS = 256;
constexpr int RF_CHUNK = 16;   // thetas sharing the power terms

// s[b] = v[b] - R(theta_b) x[b] for both right-hand sides, R regenerated in
// FP64 from X.  Workgroup = (64-row block I, chunk of RF_CHUNK thetas); it
// sweeps all column blocks J.  Thread = (row i, column phase jq).  Rows and
// columns >= n are padding (identity in R).
template <int DM, int PMODE>
__global__ __launch_bounds__(RF_THREADS)
void residual_kernel(const double *__restrict__ X, int n, int d, double p, double delta,
                     const double *__restrict__ theta, int batch, int np,
                     const double *__restrict__ v, const double *__restrict__ x,
                     double *__restrict__ s)
{
    __shared__ double xi[DM][TB], xj[DM][TB];
    __shared__ double th[RF_CHUNK][DM];
    __shared__ double xv[RF_CHUNK][2][TB];
    __shared__ double red[RF_THREADS / 64][RF_CHUNK][2][TB];
    const int I = blockIdx.x;
    const int b0 = blockIdx.y * RF_CHUNK;
    const int nb = min(RF_CHUNK, batch - b0);
    const int tid = threadIdx.x, i = tid % TB, jq = tid / TB;
    const int gi = I * TB + i;
    for (int e = tid; e < DM * TB; e += RF_THREADS) {
        const int k = e / TB, q = e % TB, g = I * TB + q;
        xi[k][q] = (k < d && g < n) ? X[(size_t)g * d + k] : 0.0;
    }
    for (int e = tid; e < RF_CHUNK * DM; e += RF_THREADS) {
        const int c = e / DM, k = e % DM;
        th[c][k] = (c < nb && k < d) ? theta[(size_t)(b0 + c) * d + k] : 0.0;
    }
    double acc[RF_CHUNK][2];
#pragma unroll
    for (int c = 0; c < RF_CHUNK; ++c) acc[c][0] = acc[c][1] = 0.0;

    const int T = np / TB;
    for (int J = 0; J < T; ++J) {
        __syncthreads();
        for (int e = tid; e < DM * TB; e += RF_THREADS) {
            const int k = e / TB, q = e % TB, g = J * TB + q;
            xj[k][q] = (k < d && g < n) ? X[(size_t)g * d + k] : 0.0;
        }
        for (int e = tid; e < RF_CHUNK * 2 * TB; e += RF_THREADS) {
            const int c = e / (2 * TB), h = (e / TB) % 2, q = e % TB;
            xv[c][h][q] = (c < nb) ? x[(size_t)(b0 + c) * 2 * np + (size_t)h * np + J * TB + q] : 0.0;
        }
        __syncthreads();
        for (int j = jq; j < TB; j += RF_THREADS / TB) {
            const int gj = J * TB + j;
            if (gi >= n || gj >= n || gi == gj) {
                const double rv = (gi == gj) ? ((gi < n) ? 1.0 + delta : 1.0) : 0.0;
                if (rv != 0.0) {
#pragma unroll
                    for (int c = 0; c < RF_CHUNK; ++c) {
                        acc[c][0] = fma(rv, xv[c][0][j], acc[c][0]);
                        acc[c][1] = fma(rv, xv[c][1][j], acc[c][1]);
                    }
                }
                continue;
            }
            double D[DM];
#pragma unroll
            for (int k = 0; k < DM; ++k)
                D[k] = (k < d) ? corr_term<PMODE>(fabs(xi[k][i] - xj[k][j]), p) : 0.0;
#pragma unroll
            for (int c = 0; c < RF_CHUNK; ++c) {
                const double rij = corr_value<PMODE, DM>(th[c], D);
                acc[c][0] = fma(rij, xv[c][0][j], acc[c][0]);
                acc[c][1] = fma(rij, xv[c][1][j], acc[c][1]);
            }
        }
    }
    // reduce the column phases, then s = v - R x
#pragma unroll
    for (int c = 0; c < RF_CHUNK; ++c) { red[jq][c][0][i] = acc[c][0]; red[jq][c][1][i] = acc[c][1]; }
    __syncthreads();
    for (int e = tid; e < RF_CHUNK * 2 * TB; e += RF_THREADS) {
        const int c = e / (2 * TB), h = (e / TB) % 2, q = e % TB;
        if (c >= nb) continue;
        double rx = 0.0;
        for (int w = 0; w < RF_THREADS / 64; ++w) rx += red[w][c][h][q];
        const size_t o = (size_t)(b0 + c) * 2 * np + (size_t)h * np + I * TB + q;
        s[o] = v[o] - rx;
    }
}

// rhs[b] = [1 y] (zero beyond n); x[b] = 0.
__global__ void rhs_init_kernel(const double *__restrict__ y, int n, int np, int batch,
                                double *__restrict__ rhs)
{
    const size_t total = (size_t)batch * 2 * np;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int q = (int)(e % np);
        const int h = (int)((e / np) % 2);
        rhs[e] = (q < n) ? (h == 0 ? 1.0 : y[q]) : 0.0;
    }
}

// x += dx; per-theta max |residual| / max |rhs| into rnorm (for convergence).
__global__ void axpy_kernel(double *__restrict__ x, const double *__restrict__ dx, size_t total)
{
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x)
        x[e] += dx[e];
}

// Final assembly after refinement: mu, Q, sigma2, nll, log|R| (partials).
__global__ __launch_bounds__(RS_THREADS)
void refine_reduce_kernel(const double *__restrict__ x, const double *__restrict__ y, int n, int np,
                          const double *__restrict__ lpart, int nparts,
                          const int32_t *__restrict__ info, const double *__restrict__ s,
                          int sweeps, gp_result *__restrict__ out)
{
    __shared__ double red[RS_WAVES][4];
    const int b = blockIdx.x, tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
    const double *x1 = x + (size_t)b * 2 * np, *xy = x1 + np;
    const double *s1 = s + (size_t)b * 2 * np, *sy = s1 + np;
    // rs = max |s|, rv = max |v| + n max |x| (|R|_inf <= n (1 + delta) bounds the
    // normwise backward error eta = |s|_inf / (|R|_inf |x|_inf + |v|_inf) from below)
    double a = 0.0, c = 0.0, rs = 0.0, rv = 0.0;
    for (int r = tid; r < n; r += RS_THREADS) {
        a += x1[r];
        c += xy[r];
        rs = fmax(rs, fmax(fabs(s1[r]), fabs(sy[r])));
        rv = fmax(rv, fmax(1.0, fabs(y[r])) + (double)n * fmax(fabs(x1[r]), fabs(xy[r])));
    }
    a = wsum(a);
    c = wsum(c);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        rs = fmax(rs, __shfl_xor(rs, off, 64));
        rv = fmax(rv, __shfl_xor(rv, off, 64));
    }
    if (lane == 0) { red[wave][0] = a; red[wave][1] = c; red[wave][2] = rs; red[wave][3] = rv; }
    __syncthreads();
    double aa = 0.0, ab = 0.0, rmax = 0.0, vmax = 0.0;
    for (int w = 0; w < RS_WAVES; ++w) {
        aa += red[w][0]; ab += red[w][1];
        rmax = fmax(rmax, red[w][2]); vmax = fmax(vmax, red[w][3]);
    }
    const double mu = ab / aa;
    __syncthreads();
    double Q = 0.0;
    for (int r = tid; r < n; r += RS_THREADS) Q = fma(y[r] - mu, fma(-mu, x1[r], xy[r]), Q);
    Q = wsum(Q);
    double ld = 0.0;
    for (int q = tid; q < nparts; q += RS_THREADS) ld += lpart[(size_t)b * nparts + q];
    ld = wsum(ld);
    if (lane == 0) { red[wave][0] = Q; red[wave][1] = ld; }
    __syncthreads();
    if (tid == 0) {
        Q = 0.0; ld = 0.0;
        for (int w = 0; w < RS_WAVES; ++w) { Q += red[w][0]; ld += red[w][1]; }
        gp_result res;
        res.ir_iters = sweeps;
        const int inf = info[b];
        // converged when the normwise backward error of the refined solution
        // is at the FP64 level
        const bool conv = rmax <= 1e-13 * vmax;
        if (inf != 0) {
            res.logdet = res.mu = res.sigma2 = res.nll = NAN;
            res.info = inf;
        } else if (!(Q > 0.0)) {
            res.logdet = ld; res.mu = mu; res.sigma2 = 0.0; res.nll = -INFINITY;
            res.info = (Q == 0.0) ? -1 : -2;
        } else {
            const double s2 = Q / (double)n;
            res.logdet = ld; res.mu = mu; res.sigma2 = s2;
            res.nll = ld + (double)n * log(s2);
            res.info = conv ? 0 : -2;
        }
        out[b] = res;
    }
}

template <int DM>
void launch_residual_dm(const double *X, int n, int d, double p, double delta, const double *theta,
                        int batch, int np, const double *v, const double *x, double *s,
                        hipStream_t st)
{
    dim3 grid(np / TB, (batch + RF_CHUNK - 1) / RF_CHUNK);
#define GPK_RES_LAUNCH(PM)                                                                  \
    residual_kernel<DM, PM><<<grid, RF_THREADS, 0, st>>>(X, n, d, p, delta, theta, batch, np, \
                                                         v, x, s)
    GPK_DISPATCH_PMODE(p, GPK_RES_LAUNCH);
#undef GPK_RES_LAUNCH
}

void launch_residual(const double *X, int n, int d, double p, double delta, const double *theta,
                     int batch, int np, const double *v, const double *x, double *s, hipStream_t st)
{
    ProfScope ps(K_RESIDUAL, (double)np * np * batch * (4.0 + 2.0 * d), 32.0 * np * batch, st);
    if (d <= 4) launch_residual_dm<4>(X, n, d, p, delta, theta, batch, np, v, x, s, st);
    else if (d <= 8) launch_residual_dm<8>(X, n, d, p, delta, theta, batch, np, v, x, s, st);
    else if (d <= 16) launch_residual_dm<16>(X, n, d, p, delta, theta, batch, np, v, x, s, st);
    else launch_residual_dm<GP_DMAX>(X, n, d, p, delta, theta, batch, np, v, x, s, st);
}

void launch_solve2(const double *A, int lda, size_t bstride, int np, const double *rhs, double *x,
                   int batch, hipStream_t st)
{
    allow_dynamic_lds((const void *)solve2_kernel, (int)(2 * GP_NMAX * sizeof(double)));
    const double lower = 0.5 * (double)np * (np + 1);
    ProfScope ps(K_SOLVE2, 8.0 * lower * batch, 16.0 * lower * batch, st);
    solve2_kernel<<<batch, RS_THREADS, (size_t)2 * np * sizeof(double), st>>>(A, lda, bstride, np,
                                                                              rhs, x);
}

__global__ void fallback_mask_kernel(const gp_result *__restrict__ out, int batch,
                                     uint8_t *__restrict__ mask)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    const int inf = out[b].info;
    mask[b] = (inf > 0 || inf == -2) ? 1 : 0;
}

}  // namespace

void launch_fallback_mask(const gp_result *out, int batch, uint8_t *mask, hipStream_t s)
{
    fallback_mask_kernel<<<(batch + 255) / 256, 256, 0, s>>>(out, batch, mask);
}

void refine_solves(const double *A, int lda, size_t bstride, int np, const gp_dataset *ds,
                   const double *theta, int batch, const double *lpart, const int32_t *info,
                   double *rhs, double *x, double *s, int sweeps, gp_result *out, hipStream_t st)
{
    const size_t total = (size_t)batch * 2 * np;
    const int blocks = (int)min((size_t)4096, (total + 255) / 256);
    rhs_init_kernel<<<blocks, 256, 0, st>>>(ds->y, ds->n, np, batch, rhs);
    launch_solve2(A, lda, bstride, np, rhs, x, batch, st);
    for (int it = 0; it < sweeps; ++it) {
        launch_residual(ds->X, ds->n, ds->d, family_p(ds), ds->delta, theta, batch, np, rhs, x, s, st);
        launch_solve2(A, lda, bstride, np, s, s, batch, st);   // correction in place
        axpy_kernel<<<blocks, 256, 0, st>>>(x, s, total);
    }
    // residual of the refined solution, for the convergence flag
    launch_residual(ds->X, ds->n, ds->d, family_p(ds), ds->delta, theta, batch, np, rhs, x, s, st);
    refine_reduce_kernel<<<batch, RS_THREADS, 0, st>>>(x, ds->y, ds->n, np, lpart, np / TB, info, s,
                                                       sweeps, out);
}

}  // namespace gpk
