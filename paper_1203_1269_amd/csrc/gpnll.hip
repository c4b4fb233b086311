// C ABI of libgpnll.so: argument checks, workspace carving and the launch
// sequence of the likelihood hot path.  Declarations and contracts are in
// include/gpnll.h.
#include <math.h>
#include <string.h>

#include "kernels.hpp"

using namespace gpk;

namespace {

constexpr size_t ALIGN = 256;

inline size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

constexpr int IR_SWEEPS = 2;   // refinement sweeps of the mixed mode

struct Layout {
    int np;
    size_t mat;      // offset of the matrices
    size_t bstride;  // doubles per matrix
    size_t lpart;    // offset of the log-det partials
    size_t info;     // offset of info
    size_t lk;       // diagonal-factor copies for TRSM, batch * 64 * 64 doubles
    size_t z;        // forward-solve state between solve segments, batch * 2 np doubles
    size_t rhs, x, s; // refinement vectors (mixed mode), batch * 2 np doubles each
    size_t mask;     // per-theta FP64 fallback mask (mixed modes), batch bytes
    size_t crt_res, crt_ex; // INT8 residues and row exponents (GP_MIXED)
    size_t total;
};

bool layout_for(int n, int batch, Layout &L, int prec = GP_FP64)
{
    if (n < 2 || n > GP_NMAX || batch < 1 || batch > GP_BATCH_MAX) return false;
    L.np = pad64(n);
    L.bstride = (size_t)L.np * L.np;
    size_t off = 0;
    L.mat = off;
    off = align_up(off + L.bstride * sizeof(double) * batch);
    L.lpart = off;
    off = align_up(off + sizeof(double) * (size_t)(L.np / TB) * batch);
    L.info = off;
    off = align_up(off + sizeof(int32_t) * (size_t)batch);
    L.lk = off;
    off = align_up(off + sizeof(double) * TB * TB * (size_t)batch);
    L.z = off;
    off = align_up(off + sizeof(double) * 2 * (size_t)L.np * batch);
    L.rhs = L.x = L.s = L.mask = L.crt_res = L.crt_ex = off;
    if (prec == GP_MIXED) {
        L.mask = off;
        off += align_up((size_t)batch);
        L.crt_ex = off;
        off += align_up(sizeof(int32_t) * (size_t)L.np * batch);
        L.crt_res = off;
        off += align_up(crt_residue_bytes(L.np, GP_MIXED_RANK, batch));
    }
    if (prec == GP_MIXED_FAST) {
        const size_t vec = align_up(sizeof(double) * 2 * (size_t)L.np * batch);
        L.rhs = off;
        L.x = off + vec;
        L.s = off + 2 * vec;
        L.mask = off + 3 * vec;
        off += 3 * vec + align_up((size_t)batch);
    }
    L.total = off;
    return true;
}

// Predictions: the matrix carries 64 + 64 ceil(N / 64) extra rows below it
// ([1 y] and the test points' cross-correlations).
struct PredLayout {
    int np, extra, lda;
    size_t mat, bstride, lpart, info, lk, total;
};

bool pred_layout_for(int n, int batch, int N, PredLayout &P)
{
    if (n < 2 || n > GP_NMAX || batch < 1 || batch > GP_BATCH_MAX || N < 0 || N > (1 << 20))
        return false;
    P.np = pad64(n);
    P.extra = TB + pad64(N);
    P.lda = P.np + P.extra;
    P.bstride = (size_t)P.lda * P.np;
    size_t off = 0;
    P.mat = off;
    off = align_up(off + P.bstride * sizeof(double) * batch);
    P.lpart = off;
    off = align_up(off + sizeof(double) * (size_t)(P.np / TB) * batch);
    P.info = off;
    off = align_up(off + sizeof(int32_t) * (size_t)batch);
    P.lk = off;
    off = align_up(off + sizeof(double) * TB * TB * (size_t)batch);
    P.total = off;
    return true;
}

bool dataset_ok(const gp_dataset *ds)
{
    if (!ds || !ds->X || !ds->y) return false;
    if (ds->n < 2 || ds->n > GP_NMAX || ds->d < 1 || ds->d > GP_DMAX) return false;
    if (!family_ok(ds)) return false;
    if (!(ds->delta >= 0.0) || !isfinite(ds->delta)) return false;
    return true;
}

bool prec_ok(int32_t prec)
{
    return prec == GP_FP64 || prec == GP_MIXED || prec == GP_MIXED_FAST;
}

bool aligned16(const void *p) { return ((uintptr_t)p & 15) == 0; }
bool aligned256(const void *p) { return ((uintptr_t)p & 255) == 0; }

gp_status launched()
{
    return hipGetLastError() == hipSuccess ? GP_OK : GP_ELAUNCH;
}

}  // namespace

extern "C" {

size_t gp_workspace_bytes(int32_t n, int32_t d, int32_t batch, int32_t prec)
{
    Layout L;
    if (d < 1 || d > GP_DMAX || !prec_ok(prec)) return 0;
    if (!layout_for(n, batch, L, prec)) return 0;
    return L.total;
}

}  // extern "C"

namespace gpk {

bool dataset_valid(const gp_dataset *ds) { return dataset_ok(ds); }

gp_status nll_batch_impl(const gp_dataset *ds, int32_t batch, const double *theta, int32_t prec,
                         void *ws, size_t ws_bytes, gp_result *out, hipStream_t stream,
                         bool lookahead)
{
    if (!dataset_ok(ds) || batch < 1 || batch > GP_BATCH_MAX || !theta || !out || !ws ||
        !prec_ok(prec))
        return GP_EINVAL;
    if (!aligned256(ws)) return GP_EINVAL;
    Layout L;
    if (!layout_for(ds->n, batch, L, prec)) return GP_EINVAL;
    if (ws_bytes < L.total) return GP_EWORKSPACE;

    char *base = (char *)ws;
    double *A = (double *)(base + L.mat);
    double *lpart = (double *)(base + L.lpart);
    int32_t *info = (int32_t *)(base + L.info);
    const int np = L.np;

    launch_init(theta, ds->d, batch, info, stream);
    launch_corr_build(ds->X, ds->n, ds->d, family_p(ds), ds->delta, theta, batch, A, np,
                      L.bstride, np, stream);
    double *lk = (double *)(base + L.lk);
    // FP64 and GP_MIXED: the forward solves follow the factorisation panel by
    // panel (solve segments on their own stream), ending with eq. 3-4
    SolvePlan plan{ds->y, ds->n, (double *)(base + L.z), out};
    factor_batch(A, np, L.bstride, np, batch, info, lpart, lk, stream, prec, false, nullptr,
                 (int8_t *)(base + L.crt_res), (int32_t *)(base + L.crt_ex), lookahead, 0,
                 prec == GP_MIXED_FAST ? nullptr : &plan);
    if (prec == GP_FP64) return launched();
    if (prec == GP_MIXED_FAST)
        refine_solves(A, np, L.bstride, np, ds, theta, batch, lpart, info,
                      (double *)(base + L.rhs), (double *)(base + L.x), (double *)(base + L.s),
                      IR_SWEEPS, out, stream);
    // thetas whose mixed result failed (pivot, or refinement in GP_MIXED_FAST)
    // are redone on the FP64 path; their results carry ir_iters = -1
    uint8_t *mask = (uint8_t *)(base + L.mask);
    launch_fallback_mask(out, batch, mask, stream);
    launch_init(theta, ds->d, batch, info, stream, mask);
    launch_corr_build(ds->X, ds->n, ds->d, family_p(ds), ds->delta, theta, batch, A, np,
                      L.bstride, np, stream, mask);
    factor_batch(A, np, L.bstride, np, batch, info, lpart, lk, stream, GP_FP64, false, mask,
                 nullptr, nullptr, lookahead);
    launch_solve_reduce(A, np, L.bstride, np, ds->n, ds->y, lpart, np / TB, info, batch, out,
                        stream, mask, -1);
    return launched();
}

}  // namespace gpk

extern "C" {

gp_status gp_nll_batch(const gp_dataset *ds, int32_t batch, const double *theta, int32_t prec,
                       void *ws, size_t ws_bytes, gp_result *out, hipStream_t stream)
{
    return nll_batch_impl(ds, batch, theta, prec, ws, ws_bytes, out, stream, true);
}

gp_status gp_nll(const gp_dataset *ds, const double *theta, int32_t prec, void *ws,
                 size_t ws_bytes, gp_result *out, hipStream_t stream)
{
    return gp_nll_batch(ds, 1, theta, prec, ws, ws_bytes, out, stream);
}

gp_status gp_corr_build(const gp_dataset *ds, int32_t batch, const double *theta, double *R,
                        int32_t ldr, int32_t *info, hipStream_t stream)
{
    if (!dataset_ok(ds) || batch < 1 || batch > GP_BATCH_MAX || !theta || !R || !info)
        return GP_EINVAL;
    const int np = pad64(ds->n);
    if (ldr < np) return GP_EINVAL;
    launch_init(theta, ds->d, batch, info, stream);
    launch_corr_build(ds->X, ds->n, ds->d, family_p(ds), ds->delta, theta, batch, R, ldr,
                      (size_t)ldr * ldr, np, stream);
    return launched();
}

size_t gp_cholesky_ws_bytes(int32_t n, int32_t batch)
{
    if (n < 1 || n > GP_NMAX || batch < 1 || batch > GP_BATCH_MAX) return 0;
    return align_up(sizeof(double) * (size_t)(pad64(n) / TB) * batch) +
           align_up(sizeof(double) * TB * TB * (size_t)batch);
}

gp_status gp_cholesky_batch(int32_t n, int32_t batch, double *A, int32_t lda, int32_t *info,
                            double *logdet, void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (n < 1 || n > GP_NMAX || batch < 1 || batch > GP_BATCH_MAX || !A || !info || !logdet ||
        !ws)
        return GP_EINVAL;
    const int np = pad64(n);
    if (lda < np || !aligned16(A) || (lda % 2) != 0) return GP_EINVAL;
    if (ws_bytes < gp_cholesky_ws_bytes(n, batch)) return GP_EWORKSPACE;
    double *lpart = (double *)ws;
    double *lk = (double *)((char *)ws + align_up(sizeof(double) * (size_t)(np / TB) * batch));
    const size_t bstride = (size_t)lda * lda;
    launch_pad_identity(A, lda, bstride, n, np, batch, stream);
    factor_batch(A, lda, bstride, np, batch, info, lpart, lk, stream, GP_FP64);
    launch_logdet_sum(lpart, np / TB, batch, logdet, stream);
    return launched();
}

struct GradLayout {
    int np, ntiles;
    size_t lda, bstride, mat, lpart, info, lk, z, alpha, part, total;
};

static bool grad_layout_for(int n, int d, int batch, GradLayout &L)
{
    if (n < 2 || n > GP_NMAX || batch < 1 || batch > GP_BATCH_MAX || d < 1 || d > GP_DMAX)
        return false;
    L.np = pad64(n);
    const int T = L.np / TB;
    L.ntiles = T * (T + 1) / 2;
    L.lda = (size_t)2 * L.np;
    L.bstride = L.lda * L.lda;
    size_t off = 0;
    L.mat = off;
    off = align_up(off + L.bstride * sizeof(double) * batch);
    L.lpart = off;
    off = align_up(off + sizeof(double) * (size_t)T * batch);
    L.info = off;
    off = align_up(off + sizeof(int32_t) * (size_t)batch);
    L.lk = off;
    off = align_up(off + sizeof(double) * TB * TB * (size_t)batch);
    L.z = off;
    off = align_up(off + sizeof(double) * 2 * (size_t)L.np * batch);
    L.alpha = off;
    off = align_up(off + sizeof(double) * (size_t)L.np * batch);
    L.part = off;
    off = align_up(off + sizeof(double) * (size_t)L.ntiles * d * batch);
    L.total = off;
    return true;
}

size_t gp_predict_workspace_bytes(int32_t n, int32_t d, int32_t batch, int32_t N)
{
    PredLayout P;
    if (d < 1 || d > GP_DMAX || !pred_layout_for(n, batch, N, P)) return 0;
    return P.total;
}

gp_status gp_predict(const gp_dataset *ds, int32_t batch, const double *theta,
                     const double *Xstar, int32_t N, int32_t prec, void *ws, size_t ws_bytes,
                     gp_result *fit, double *mean, double *mse, hipStream_t stream)
{
    if (!dataset_ok(ds) || batch < 1 || batch > GP_BATCH_MAX || !theta || !fit || !ws ||
        prec != GP_FP64 || N < 0)
        return GP_EINVAL;
    if (N > 0 && (!Xstar || !mean || !mse)) return GP_EINVAL;
    if (!aligned256(ws)) return GP_EINVAL;
    PredLayout P;
    if (!pred_layout_for(ds->n, batch, N, P)) return GP_EINVAL;
    if (ws_bytes < P.total) return GP_EWORKSPACE;
    char *base = (char *)ws;
    double *A = (double *)(base + P.mat);
    double *lpart = (double *)(base + P.lpart);
    int32_t *info = (int32_t *)(base + P.info);
    const int np = P.np;
    launch_init(theta, ds->d, batch, info, stream);
    launch_corr_build(ds->X, ds->n, ds->d, family_p(ds), ds->delta, theta, batch, A, P.lda,
                      P.bstride, np, stream);
    launch_pred_rows(A, P.lda, P.bstride, np, ds->X, ds->n, ds->d, family_p(ds), ds->y, theta,
                     Xstar, N, P.extra, batch, stream);
    factor_batch(A, P.lda, P.bstride, np, batch, info, lpart, (double *)(base + P.lk), stream,
                 GP_FP64, false, nullptr, nullptr, nullptr, true, P.extra);
    launch_pred_reduce(A, P.lda, P.bstride, np, ds->n, lpart, np / TB, info, N, batch, fit, mean,
                       mse, stream);
    return launched();
}

size_t gp_grad_workspace_bytes(int32_t n, int32_t d, int32_t batch)
{
    GradLayout L;
    if (!grad_layout_for(n, d, batch, L)) return 0;
    return L.total;
}

gp_status gp_nll_grad(const gp_dataset *ds, int32_t batch, const double *theta, int32_t prec,
                      void *ws, size_t ws_bytes, gp_result *out, double *grad, hipStream_t stream)
{
    if (!dataset_ok(ds) || batch < 1 || batch > GP_BATCH_MAX || !theta || !out || !grad || !ws ||
        prec != GP_FP64)
        return GP_EINVAL;
    if (!aligned16(ws)) return GP_EINVAL;
    GradLayout L;
    if (!grad_layout_for(ds->n, ds->d, batch, L)) return GP_EINVAL;
    if (ws_bytes < L.total) return GP_EWORKSPACE;

    char *base = (char *)ws;
    double *A = (double *)(base + L.mat);
    double *lpart = (double *)(base + L.lpart);
    int32_t *info = (int32_t *)(base + L.info);
    double *alpha = (double *)(base + L.alpha);
    double *part = (double *)(base + L.part);
    const int np = L.np;
    const int lda = (int)L.lda;

    launch_init(theta, ds->d, batch, info, stream);
    launch_corr_build(ds->X, ds->n, ds->d, family_p(ds), ds->delta, theta, batch, A, lda,
                      L.bstride, np, stream);
    launch_border_init(A, lda, L.bstride, np, batch, stream);
    // the forward solves and eq. 3-4 follow the factorisation panel by panel
    // (solve segments on their own stream, reading only the top n_pad rows)
    SolvePlan plan{ds->y, ds->n, (double *)(base + L.z), out};
    factor_batch(A, lda, L.bstride, np, batch, info, lpart, (double *)(base + L.lk), stream,
                 GP_FP64, true, nullptr, nullptr, nullptr, true, 0, &plan);
    launch_alpha(A, lda, L.bstride, np, ds->n, ds->y, out, alpha, batch, stream);
    launch_adjoint(A, lda, L.bstride, np, ds->n, ds->d, family_p(ds), ds->X, theta, alpha, out,
                   part, grad, batch, stream);
    return launched();
}

}  // extern "C"
