// Forward solves L [a b] = [1 y] and the reductions of eq. 3-4 (paper Sec. 2):
//   mu = (a.b)/(a.a),  Q = |b - mu a|^2 (two-pass),  sigma2 = Q/n,
//   nll = log|R| + n ln(sigma2),  log|R| = sum of the per-tile partials.
// One workgroup per matrix.  The solve is blocked by 64 columns and
// right-looking: wave 0 finishes the 64 x 64 triangular block with
// lane-to-lane broadcasts, then all 16 waves subtract that block column times
// its solution from the rows below (both right-hand sides; consecutive
// threads take consecutive rows, so every column segment of L is read as one
// contiguous run).  The solution
// vectors live in LDS (2 n_pad doubles), so n_pad <= 8192.
// The kernel streams the n^2/2 lower entries of L once: HBM bound.
// A launch may cover only the column blocks [ib0, ib1) (a solve segment that
// runs as soon as those columns of L are final): it then starts from, or
// leaves, the partial solution in z (2 n_pad doubles per matrix), and only
// the segment that ends at the last block does the reductions.
// In a ragged batch each matrix has its own order, n and y (RagMat): the
// launch covers the blocks of the largest, and a matrix's last block is
// where its own segment ends and its reductions are done.
#include <math.h>

#include <mutex>
#include <set>
#include <utility>

#include "kernels.hpp"

namespace gpk {

namespace {

constexpr int SV_THREADS = 1024;
constexpr int SV_WAVES = SV_THREADS / 64;

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__global__ __launch_bounds__(SV_THREADS)
void solve_reduce_kernel(const double *__restrict__ A0, int lda, size_t bstride, int np, int n,
                         const double *__restrict__ y, const double *__restrict__ lpart,
                         int nparts, const int32_t *__restrict__ info,
                         gp_result *__restrict__ out, const uint8_t *__restrict__ mask,
                         int ir_tag, double *__restrict__ zg, int ib0, int ib1,
                         const RagMat *__restrict__ rag)
{
    if (mask && !mask[blockIdx.x]) return;
    extern __shared__ double zs[];          // z0[np], z1[np]
    __shared__ double red[SV_WAVES][3];
    const int b = blockIdx.x;
    // the partial solution in zg keeps the launch's stride (2 np per matrix)
    double *zb = zg ? zg + (size_t)b * 2 * np : nullptr;
    size_t boff = (size_t)b * bstride;
    int nlp = nparts;   // log-det partials of this matrix
    if (rag) {   // uniform over the workgroup
        const RagMat m = rag[b];
        if (ib0 * TB >= m.live) return;   // this matrix was finished before
        np = m.live;
        lda = m.lda;
        boff = m.off;
        n = m.n;
        y = m.y;
        nlp = m.live / TB;
        ib1 = min(ib1, np / TB);
    }
    double *z0 = zs, *z1 = zs + np;

    const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
    const double *A = A0 + boff;
    const int T = np / TB;

    if (ib0 == 0) {
        // right-hand sides [1 y] (0 in the padded rows)
        for (int r = tid; r < np; r += SV_THREADS) {
            z0[r] = (r < n) ? 1.0 : 0.0;
            z1[r] = (r < n) ? y[r] : 0.0;
        }
    } else {
        for (int r = tid; r < np; r += SV_THREADS) {
            z0[r] = zb[r];
            z1[r] = zb[np + r];
        }
    }
    __syncthreads();
    for (int ib = ib0; ib < ib1; ++ib) {
        const int c0 = ib * TB;
        // wave 0: triangular solve of the 64 x 64 diagonal block (lane = row)
        if (wave == 0) {
            const int r = c0 + lane;
            double t0 = z0[r], t1 = z1[r];
            double Lrow[TB];
            const double *pd = A + r + (size_t)c0 * lda;
#pragma unroll
            for (int j = 0; j < TB; ++j) Lrow[j] = pd[(size_t)j * lda];
#pragma unroll
            for (int j = 0; j < TB; ++j) {
                // lane j holds the finished right-hand sides of row j
                const double q0 = __shfl(t0 / Lrow[j], j, 64);
                const double q1 = __shfl(t1 / Lrow[j], j, 64);
                if (lane == j) { t0 = q0; t1 = q1; }
                else if (lane > j) { t0 = fma(-Lrow[j], q0, t0); t1 = fma(-Lrow[j], q1, t1); }
            }
            z0[r] = t0;
            z1[r] = t1;
        }
        __syncthreads();
        // all waves: rows below the block lose L(rows, block) z(block); each
        // column segment of L is read as one contiguous run
        const int rows = np - c0 - TB;
        if (rows > 0) {
            for (int r = c0 + TB + tid; r < np; r += SV_THREADS) {
                const double *pr = A + r + (size_t)c0 * lda;
                double s0 = 0.0, s1 = 0.0;
#pragma unroll 16
                for (int j = 0; j < TB; ++j) {
                    const double v = pr[(size_t)j * lda];
                    s0 = fma(v, z0[c0 + j], s0);
                    s1 = fma(v, z1[c0 + j], s1);
                }
                z0[r] -= s0;
                z1[r] -= s1;
            }
        }
        __syncthreads();
    }
    if (ib1 < T) {   // not the last segment: keep the partial solution
        for (int r = tid; r < np; r += SV_THREADS) {
            zb[r] = z0[r];
            zb[np + r] = z1[r];
        }
        return;
    }

    // aa = a.a, ab = a.b over the n real rows
    double aa = 0.0, ab = 0.0;
    for (int r = tid; r < n; r += SV_THREADS) { aa = fma(z0[r], z0[r], aa); ab = fma(z0[r], z1[r], ab); }
    aa = wave_sum(aa);
    ab = wave_sum(ab);
    if (lane == 0) { red[wave][0] = aa; red[wave][1] = ab; }
    __syncthreads();
    aa = 0.0; ab = 0.0;
    for (int w = 0; w < SV_WAVES; ++w) { aa += red[w][0]; ab += red[w][1]; }
    const double mu = ab / aa;
    __syncthreads();
    double Q = 0.0;
    for (int r = tid; r < n; r += SV_THREADS) {
        const double e = fma(-mu, z0[r], z1[r]);
        Q = fma(e, e, Q);
    }
    Q = wave_sum(Q);
    double ld = 0.0;
    for (int q = tid; q < nlp; q += SV_THREADS) ld += lpart[(size_t)b * nparts + q];
    ld = wave_sum(ld);
    if (lane == 0) { red[wave][0] = Q; red[wave][2] = ld; }
    __syncthreads();
    if (tid == 0) {
        Q = 0.0; ld = 0.0;
        for (int w = 0; w < SV_WAVES; ++w) { Q += red[w][0]; ld += red[w][2]; }
        gp_result res;
        res.ir_iters = ir_tag;
        int inf = info[b];
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
        out[rag ? rag[b].dst : b] = res;
    }
}

}  // namespace

void launch_solve_reduce(const double *A, int lda, size_t bstride, int np, int n, const double *y,
                         const double *lpart, int nparts, const int32_t *info, int batch,
                         gp_result *out, hipStream_t s, const uint8_t *mask, int ir_tag)
{
    const size_t shm = (size_t)2 * np * sizeof(double);
    allow_dynamic_lds((const void *)solve_reduce_kernel, (int)(2 * GP_NMAX * sizeof(double)));
    const double lower = 0.5 * (double)np * (np + 1);
    ProfScope ps(K_SOLVE_REDUCE, 4.0 * lower * batch, (8.0 * lower + 16.0 * n) * batch, s);
    solve_reduce_kernel<<<batch, SV_THREADS, shm, s>>>(A, lda, bstride, np, n, y, lpart, nparts,
                                                       info, out, mask, ir_tag, nullptr, 0,
                                                       np / TB, nullptr);
}

void launch_solve_segment(const double *A, int lda, size_t bstride, int np, int n,
                          const double *y, const double *lpart, int nparts,
                          const int32_t *info, int batch, gp_result *out, double *z, int ib0,
                          int ib1, hipStream_t s, const RagMat *rag)
{
    if (ib1 <= ib0) return;
    const size_t shm = (size_t)2 * np * sizeof(double);
    allow_dynamic_lds((const void *)solve_reduce_kernel, (int)(2 * GP_NMAX * sizeof(double)));
    // entries of L read: the lower part of columns [64 ib0, 64 ib1)
    const double c0 = 64.0 * ib0, c1 = 64.0 * ib1;
    const double entries = (c1 - c0) * np - 0.5 * (c1 * c1 - c0 * c0) + 0.5 * (c1 - c0);
    ProfScope ps(K_SOLVE_REDUCE, 4.0 * entries * batch, (8.0 * entries + 32.0 * np) * batch, s);
    solve_reduce_kernel<<<batch, SV_THREADS, shm, s>>>(A, lda, bstride, np, n, y, lpart, nparts,
                                                       info, out, nullptr, 0, z, ib0, ib1,
                                                       rag);
}

void allow_dynamic_lds(const void *fn, int bytes)
{
    static std::mutex mu;
    static std::set<std::pair<int, const void *>> done;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return;
    std::lock_guard<std::mutex> lock(mu);
    if (done.insert(std::make_pair(dev, fn)).second)
        (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

}  // namespace gpk
