// Batched multi-start L-BFGS on -2logL with its state on the device.
//
// The paper fits the GP with a genetic algorithm and names multi-start
// gradient methods as the alternative, each needing many likelihood
// evaluations (Sec. 2).  Here S minimisations run together: every
// value+gradient evaluation of the starts still in play is one batched
// gp_nll_grad call, and the L-BFGS bookkeeping (two-loop recursion over a
// ring buffer of m curvature pairs, the trial points of a backtracking
// Armijo line search, acceptance, history update) runs in small kernels on
// the same stream.  The host loop only reads, once per line-search trial,
// how many starts are still searching (the batch size of the next
// evaluation).
//
// Parametrisation phi = log(theta) (theta stays positive; trial points are
// clipped to [log theta_lo, log theta_hi]); d(nll)/d(phi_k) = theta_k
// d(nll)/d(theta_k).  A start stops when max_k |d nll / d phi_k| <= gtol, when
// its line search fails max_ls times in a row, or after `iters` iterations.
#include <math.h>
#include <string.h>

#include "kernels.hpp"

namespace gpk {
namespace {

constexpr int LB_SMAX = 1024;   // starts per call (one workgroup packs them)
constexpr int LB_MMAX = 32;     // curvature pairs kept

struct LbState {
    double *phi, *f, *g;        // current iterate, S x d / S / S x d
    double *nphi, *nf, *ng;     // accepted trial
    double *dir, *slope, *step, *trial;
    double *hs, *hy;            // S x m x d ring buffers
    int32_t *pending, *active, *hcount, *hhead, *its, *idx;
    int32_t *ctrl;              // [0] trial count, [1] active count
    double *theta_c, *grad_c;   // compact evaluation batch: S x d each
    gp_result *out_c;
    char *gws;                  // gp_nll_grad workspace
    size_t gws_bytes;
    size_t total;
};

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

bool lb_layout(int n, int d, int S, int m, LbState &L, char *base)
{
    if (S < 1 || S > LB_SMAX || m < 1 || m > LB_MMAX || d < 1 || d > GP_DMAX) return false;
    const size_t gb = gp_grad_workspace_bytes(n, d, S);
    if (gb == 0) return false;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base ? base + off : nullptr;
        off = al(off + bytes);
        return p;
    };
    const size_t sd = sizeof(double) * (size_t)S * d, s1 = sizeof(double) * (size_t)S;
    const size_t si = sizeof(int32_t) * (size_t)S;
    L.phi = (double *)take(sd);
    L.f = (double *)take(s1);
    L.g = (double *)take(sd);
    L.nphi = (double *)take(sd);
    L.nf = (double *)take(s1);
    L.ng = (double *)take(sd);
    L.dir = (double *)take(sd);
    L.slope = (double *)take(s1);
    L.step = (double *)take(s1);
    L.trial = (double *)take(sd);
    L.hs = (double *)take(sd * m);
    L.hy = (double *)take(sd * m);
    L.pending = (int32_t *)take(si);
    L.active = (int32_t *)take(si);
    L.hcount = (int32_t *)take(si);
    L.hhead = (int32_t *)take(si);
    L.its = (int32_t *)take(si);
    L.idx = (int32_t *)take(si);
    L.ctrl = (int32_t *)take(4 * sizeof(int32_t));
    L.theta_c = (double *)take(sd);
    L.grad_c = (double *)take(sd);
    L.out_c = (gp_result *)take(sizeof(gp_result) * (size_t)S);
    L.gws = take(gb);
    L.gws_bytes = gb;
    L.total = off;
    return true;
}

__device__ __forceinline__ bool result_bad(const gp_result &r)
{
    return r.info != 0 || !isfinite(r.nll);
}

// phi = log(theta0); the first evaluation batch is every start
__global__ void lb_start_kernel(const double *__restrict__ theta0, int S, int d, LbState L)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    for (int k = 0; k < d; ++k) {
        const double t = theta0[(size_t)s * d + k];
        L.phi[(size_t)s * d + k] = log(t);
        L.theta_c[(size_t)s * d + k] = t;
    }
    L.idx[s] = s;
    L.hcount[s] = 0;
    L.hhead[s] = 0;
    L.its[s] = 0;
}

// values and gradients of the first evaluation; active starts
__global__ void lb_first_kernel(int S, int d, double gtol, LbState L, double *__restrict__ trace)
{
    const int s = threadIdx.x;
    __shared__ int cnt;
    if (s == 0) cnt = 0;
    __syncthreads();
    if (s < S) {
        const gp_result r = L.out_c[s];
        const bool bad = result_bad(r);
        const double fs = bad ? INFINITY : r.nll;
        double gmax = 0.0;
        for (int k = 0; k < d; ++k) {
            const double gk = L.grad_c[(size_t)s * d + k] * exp(L.phi[(size_t)s * d + k]);
            L.g[(size_t)s * d + k] = gk;
            gmax = fmax(gmax, fabs(gk));
        }
        L.f[s] = fs;
        const int act = isfinite(fs) && gmax > gtol;
        L.active[s] = act;
        if (trace) trace[s] = fs;
        if (act) atomicAdd(&cnt, 1);
    }
    __syncthreads();
    if (s == 0) L.ctrl[1] = cnt;
}

// search direction by the two-loop recursion (newest pair first), the
// initial step, the Armijo slope; every active start starts searching
__global__ void lb_direction_kernel(int S, int d, int m, LbState L)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    L.pending[s] = 0;
    if (!L.active[s]) return;
    double q[GP_DMAX], alpha[LB_MMAX];
    const double *gs = L.g + (size_t)s * d;
    for (int k = 0; k < d; ++k) q[k] = gs[k];
    const int hc = L.hcount[s], hh = L.hhead[s];
    const double *HS = L.hs + (size_t)s * m * d, *HY = L.hy + (size_t)s * m * d;
    for (int t = 0; t < hc; ++t) {   // newest first
        const int slot = (hh - 1 - t + 2 * m) % m;
        const double *sv = HS + (size_t)slot * d, *yv = HY + (size_t)slot * d;
        double ys = 0.0, sq = 0.0;
        for (int k = 0; k < d; ++k) { ys += yv[k] * sv[k]; sq += sv[k] * q[k]; }
        const double a = (1.0 / ys) * sq;
        alpha[t] = a;
        for (int k = 0; k < d; ++k) q[k] -= a * yv[k];
    }
    if (hc > 0) {   // scale by s.y / y.y of the newest pair
        const int slot = (hh - 1 + m) % m;
        const double *sv = HS + (size_t)slot * d, *yv = HY + (size_t)slot * d;
        double sy = 0.0, yy = 0.0;
        for (int k = 0; k < d; ++k) { sy += sv[k] * yv[k]; yy += yv[k] * yv[k]; }
        const double sc = sy / yy;
        for (int k = 0; k < d; ++k) q[k] *= sc;
    }
    for (int t = hc - 1; t >= 0; --t) {   // oldest first
        const int slot = (hh - 1 - t + 2 * m) % m;
        const double *sv = HS + (size_t)slot * d, *yv = HY + (size_t)slot * d;
        double ys = 0.0, yq = 0.0;
        for (int k = 0; k < d; ++k) { ys += yv[k] * sv[k]; yq += yv[k] * q[k]; }
        const double bq = (1.0 / ys) * yq;
        for (int k = 0; k < d; ++k) q[k] += (alpha[t] - bq) * sv[k];
    }
    double pg = 0.0;
    for (int k = 0; k < d; ++k) pg += -q[k] * gs[k];
    int h = hc;
    if (pg >= 0.0) {   // not a descent direction: restart from steepest descent
        h = 0;
        L.hcount[s] = 0;
        for (int k = 0; k < d; ++k) q[k] = gs[k];
    }
    double pmax = 0.0, slope = 0.0;
    for (int k = 0; k < d; ++k) {
        const double p = -q[k];
        L.dir[(size_t)s * d + k] = p;
        pmax = fmax(pmax, fabs(p));
        slope += gs[k] * p;
        L.nphi[(size_t)s * d + k] = L.phi[(size_t)s * d + k];
        L.ng[(size_t)s * d + k] = gs[k];
    }
    L.nf[s] = L.f[s];
    L.slope[s] = slope;
    // unit step once curvature pairs exist; before that at most 1 in log(theta)
    L.step[s] = h == 0 ? fmin(1.0, 1.0 / fmax(pmax, 1e-300)) : 1.0;
    L.pending[s] = 1;
}

// trial points of the searching starts, packed in start order (one block)
__global__ void lb_pack_kernel(int S, int d, double lo, double hi, LbState L)
{
    __shared__ int pos[LB_SMAX];
    const int s = threadIdx.x;
    const int pend = s < S ? L.pending[s] : 0;
    pos[s] = pend;
    __syncthreads();
    for (int off = 1; off < LB_SMAX; off <<= 1) {   // inclusive scan
        const int v = s >= off ? pos[s - off] : 0;
        __syncthreads();
        pos[s] += v;
        __syncthreads();
    }
    if (pend) {
        const int k = pos[s] - 1;
        L.idx[k] = s;
        for (int c = 0; c < d; ++c) {
            const double t = fmin(hi, fmax(lo, L.phi[(size_t)s * d + c] +
                                                   L.step[s] * L.dir[(size_t)s * d + c]));
            L.trial[(size_t)s * d + c] = t;
            L.theta_c[(size_t)k * d + c] = exp(t);
        }
    }
    if (s == LB_SMAX - 1) L.ctrl[0] = pos[s];
}

// Armijo test of the evaluated trials; accepted ones stop searching,
// rejected ones halve their step
__global__ void lb_accept_kernel(int K, int d, double c1, LbState L)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    const int s = L.idx[k];
    const gp_result r = L.out_c[k];
    const double ft = result_bad(r) ? INFINITY : r.nll;
    if (ft <= L.f[s] + c1 * L.step[s] * L.slope[s]) {
        for (int c = 0; c < d; ++c) {
            const double t = L.trial[(size_t)s * d + c];
            L.nphi[(size_t)s * d + c] = t;
            L.ng[(size_t)s * d + c] = L.grad_c[(size_t)k * d + c] * exp(t);
        }
        L.nf[s] = ft;
        L.pending[s] = 0;
    } else {
        L.step[s] *= 0.5;
    }
}

// end of an iteration: curvature pair (if s.y is safely positive), move,
// convergence test; trace row of this iteration
__global__ void lb_update_kernel(int S, int d, int m, double gtol, LbState L,
                                 double *__restrict__ trace_row)
{
    const int s = threadIdx.x;
    __shared__ int cnt;
    if (s == 0) cnt = 0;
    __syncthreads();
    if (s < S) {
        if (L.active[s]) {
            const bool moved = !L.pending[s];
            if (moved) {
                double sy = 0.0, ss = 0.0, yy = 0.0;
                for (int c = 0; c < d; ++c) {
                    const double sv = L.nphi[(size_t)s * d + c] - L.phi[(size_t)s * d + c];
                    const double yv = L.ng[(size_t)s * d + c] - L.g[(size_t)s * d + c];
                    sy += sv * yv; ss += sv * sv; yy += yv * yv;
                }
                if (sy > 1e-12 * sqrt(ss * yy)) {
                    const int slot = L.hhead[s];
                    for (int c = 0; c < d; ++c) {
                        L.hs[((size_t)s * m + slot) * d + c] =
                            L.nphi[(size_t)s * d + c] - L.phi[(size_t)s * d + c];
                        L.hy[((size_t)s * m + slot) * d + c] =
                            L.ng[(size_t)s * d + c] - L.g[(size_t)s * d + c];
                    }
                    L.hhead[s] = (slot + 1) % m;
                    L.hcount[s] = min(L.hcount[s] + 1, m);
                }
                double gmax = 0.0;
                for (int c = 0; c < d; ++c) {
                    L.phi[(size_t)s * d + c] = L.nphi[(size_t)s * d + c];
                    L.g[(size_t)s * d + c] = L.ng[(size_t)s * d + c];
                    gmax = fmax(gmax, fabs(L.g[(size_t)s * d + c]));
                }
                L.f[s] = L.nf[s];
                L.its[s] += 1;
                L.active[s] = gmax > gtol;
            } else {
                L.active[s] = 0;   // the line search failed
            }
        }
        if (trace_row) trace_row[s] = L.f[s];
        if (L.active[s]) atomicAdd(&cnt, 1);
    }
    __syncthreads();
    if (s == 0) L.ctrl[1] = cnt;
}

__global__ void lb_finish_kernel(int S, int d, LbState L, double *__restrict__ theta,
                                 double *__restrict__ nll, double *__restrict__ gnorm,
                                 int32_t *__restrict__ iters)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    double gmax = 0.0;
    for (int c = 0; c < d; ++c) {
        theta[(size_t)s * d + c] = exp(L.phi[(size_t)s * d + c]);
        gmax = fmax(gmax, fabs(L.g[(size_t)s * d + c]));
    }
    nll[s] = L.f[s];
    gnorm[s] = gmax;
    iters[s] = L.its[s];
}

}  // namespace
}  // namespace gpk

using namespace gpk;

extern "C" {

size_t gp_lbfgs_workspace_bytes(int32_t n, int32_t d, int32_t starts, int32_t m)
{
    LbState L;
    return lb_layout(n, d, starts, m, L, nullptr) ? L.total : 0;
}

gp_status gp_lbfgs(const gp_dataset *ds, int32_t starts, double *theta,
                   const gp_lbfgs_config *cfg, void *ws, size_t ws_bytes, double *nll,
                   double *gnorm, int32_t *iters, double *trace, gp_lbfgs_summary *summary,
                   hipStream_t stream)
{
    if (!ds || !dataset_valid(ds) || !theta || !cfg || !ws || !nll || !gnorm || !iters ||
        !summary)
        return GP_EINVAL;
    if (((uintptr_t)ws & 255) != 0) return GP_EINVAL;
    if (cfg->iters < 0 || cfg->max_ls < 1 || cfg->reserved != 0 || !(cfg->c1 > 0.0 && cfg->c1 < 1.0) ||
        !(cfg->gtol >= 0.0) || !(cfg->theta_lo > 0.0) || !(cfg->theta_hi > cfg->theta_lo) ||
        !isfinite(cfg->theta_hi))
        return GP_EINVAL;
    const int S = starts, d = ds->d, m = cfg->m;
    LbState L;
    if (!lb_layout(ds->n, d, S, m, L, nullptr)) return GP_EINVAL;
    if (ws_bytes < L.total) return GP_EWORKSPACE;
    lb_layout(ds->n, d, S, m, L, (char *)ws);
    const double lo = log(cfg->theta_lo), hi = log(cfg->theta_hi);
    const int tb = 256, nb = (S + tb - 1) / tb;
    summary->iterations = 0;
    summary->evaluations = 0;

    auto eval = [&](int K) {
        return gp_nll_grad(ds, K, L.theta_c, GP_FP64, L.gws, L.gws_bytes, L.out_c, L.grad_c,
                           stream);
    };
    auto read_ctrl = [&](int32_t *h) {
        return hipMemcpyAsync(h, L.ctrl, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, stream) ==
                       hipSuccess &&
                   hipStreamSynchronize(stream) == hipSuccess
                   ? GP_OK
                   : GP_ELAUNCH;
    };

    lb_start_kernel<<<nb, tb, 0, stream>>>(theta, S, d, L);
    gp_status rc = eval(S);
    if (rc != GP_OK) return rc;
    summary->evaluations = 1;
    lb_first_kernel<<<1, LB_SMAX, 0, stream>>>(S, d, cfg->gtol, L, trace);
    int32_t ctrl[2] = {0, 0};
    for (int it = 0; it < cfg->iters; ++it) {
        if ((rc = read_ctrl(ctrl)) != GP_OK) return rc;
        if (ctrl[1] == 0) break;
        lb_direction_kernel<<<nb, tb, 0, stream>>>(S, d, m, L);
        for (int t = 0; t < cfg->max_ls; ++t) {
            lb_pack_kernel<<<1, LB_SMAX, 0, stream>>>(S, d, lo, hi, L);
            if ((rc = read_ctrl(ctrl)) != GP_OK) return rc;
            const int K = ctrl[0];
            if (K == 0) break;
            if ((rc = eval(K)) != GP_OK) return rc;
            summary->evaluations += 1;
            lb_accept_kernel<<<(K + tb - 1) / tb, tb, 0, stream>>>(K, d, cfg->c1, L);
        }
        lb_update_kernel<<<1, LB_SMAX, 0, stream>>>(S, d, m, cfg->gtol, L,
                                                    trace ? trace + (size_t)(it + 1) * S : nullptr);
        summary->iterations = it + 1;
    }
    lb_finish_kernel<<<nb, tb, 0, stream>>>(S, d, L, theta, nll, gnorm, iters);
    return hipGetLastError() == hipSuccess ? GP_OK : GP_ELAUNCH;
}

}  // extern "C"
