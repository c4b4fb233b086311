// Internal launchers of the gfx950 kernels.  Every launcher enqueues on
// `stream` and returns immediately; the caller checks hipGetLastError().
//
// Matrix storage: batch of column-major FP64 matrices, leading dimension
// `lda`, batch stride `bstride` doubles, factorised extent `np` (a multiple
// of 64, np <= lda).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "gpnll.h"
#include "profile.hpp"

namespace gpk {

constexpr int TB = 64;          // base tile / inner panel width
#ifndef OUTER_NB
#define OUTER_NB 512   // outer panel width (K of the trailing update), FP64 paths
#endif

inline int pad64(int n) { return (n + TB - 1) / TB * TB; }

// Correlation families inside the library: launchers take the family where
// they take the power exponent p.  p in (0, 2] is the power exponential of
// eq. 2; P_MATERN32 / P_MATERN52 select the Matern families.  Kernels are
// specialised on PMODE: 0 power exponential with general p, 1 p == 1,
// 2 p == 2, 3 Matern 3/2, 4 Matern 5/2.
constexpr double P_MATERN32 = -1.5;
constexpr double P_MATERN52 = -2.5;

// Family and exponent of a dataset: a known family, p in (0, 2] for the
// power exponential, reserved field zero.
inline bool family_ok(const gp_dataset *ds)
{
    if (ds->reserved != 0) return false;
    if (ds->corr == GP_CORR_POWEXP) return ds->p > 0.0 && ds->p <= 2.0;
    return ds->corr == GP_CORR_MATERN32 || ds->corr == GP_CORR_MATERN52;
}

inline double family_p(const gp_dataset *ds)
{
    return ds->corr == GP_CORR_MATERN32 ? P_MATERN32
         : ds->corr == GP_CORR_MATERN52 ? P_MATERN52 : ds->p;
}

// Theta-independent per-dimension term: |d|^p (power exponential), |d|
// (Matern).
template <int PMODE>
__device__ __forceinline__ double corr_term(double diff, double p)
{
    if (PMODE == 2) return diff * diff;
    if (PMODE == 0) return (diff == 0.0) ? 0.0 : pow(diff, p);
    return diff;
}

// Correlation from the per-dimension terms D[0..DM) (zero beyond d) and theta
// th[0..DM).  Power exponential: exp(-sum th_k D_k).  Matern: with
// h_k = th_k D_k and c = sqrt(3) or sqrt(5), prod_k poly(h_k) exp(-c sum h_k),
// poly = 1 + c h (3/2) or 1 + c h + c^2 h^2 / 3 (5/2).  Where exp(-c sum h_k)
// would underflow (c sum h_k > 700) the product is taken as
// exp(ln(poly) - c sum h_k); with c sum h_k < 2e4 every factor is below 1.4e8,
// so poly stays finite for d <= 32, and beyond 2e4 the value is 0 (ln(poly)
// is then below 700).
template <int PMODE, int DM>
__device__ __forceinline__ double corr_value(const double *th, const double *D)
{
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < DM; ++k) s = fma(th[k], D[k], s);
    if (PMODE <= 2) return exp(-s);
    constexpr double c = PMODE == 3 ? 1.7320508075688772 : 2.23606797749979;
    const double e = c * s;
    if (!(e < 2.0e4)) return 0.0;
    double poly = 1.0;
#pragma unroll
    for (int k = 0; k < DM; ++k) {
        const double h = th[k] * D[k];
        poly *= (PMODE == 3) ? fma(c, h, 1.0) : fma(h, fma(c * c / 3.0, h, c), 1.0);
    }
    return (e <= 700.0) ? poly * exp(-e) : exp(log(poly) - e);
}

// G_k = -d ln(correlation) / d theta_k from the per-dimension term D_k:
// D_k (power exponential); D_k c^2 h / (1 + c h) (Matern 3/2);
// D_k c^2 h (1 + c h) / (3 (1 + c h + c^2 h^2 / 3)) (Matern 5/2).
template <int PMODE>
__device__ __forceinline__ double corr_dlog(double th, double D)
{
    if (PMODE <= 2) return D;
    constexpr double c = PMODE == 3 ? 1.7320508075688772 : 2.23606797749979;
    const double h = th * D;
    if (PMODE == 3) return D * (c * c) * h / fma(c, h, 1.0);
    return D * (c * c) * h * fma(c, h, 1.0) / (3.0 * fma(h, fma(c * c / 3.0, h, c), 1.0));
}

// Host dispatch of a kernel template on the family / exponent p.
#define GPK_DISPATCH_PMODE(p, LAUNCH)                \
    do {                                             \
        if ((p) == P_MATERN32) { LAUNCH(3); }        \
        else if ((p) == P_MATERN52) { LAUNCH(4); }   \
        else if ((p) == 2.0) { LAUNCH(2); }          \
        else if ((p) == 1.0) { LAUNCH(1); }          \
        else { LAUNCH(0); }                          \
    } while (0)

// Raise the dynamic-LDS limit of kernel `fn` to `bytes` on the current
// device, once per (device, kernel) for the life of the process.
void allow_dynamic_lds(const void *fn, int bytes);

// Optional per-theta mask (mask[b] == 0: the launch leaves theta b alone;
// nullptr: all thetas) used to rerun a subset of a batch on the FP64 path.

// Ragged batches (matrices of different orders in one launch, FP64 path):
// matrix b starts at A0 + off with leading dimension lda and order `live`
// (its padded size, a multiple of 64); launches sized for the largest order
// leave everything of matrix b at or beyond `live` alone.  n and y are the
// dataset's, for the solves.  With rag == nullptr every matrix is at
// A0 + b bstride with the launch's lda and order.
struct RagMat {
    size_t off;
    int32_t lda, live;
    int32_t n, dst;     // dst: index of the matrix's result in `out`
    const double *y;
};
// rag[0 .. count) = src (count <= RAG_CHUNK), a kernel-argument copy so the
// descriptors need no host buffer that outlives the call
constexpr int RAG_CHUNK = 32;
void launch_rag_fill(RagMat *rag, const RagMat *src, int count, hipStream_t s);

// theta validity and info initialisation.
void launch_init(const double *theta, int d, int batch, int32_t *info, hipStream_t s,
                 const uint8_t *mask = nullptr);

// Correlation build: R_delta tiles on and below the diagonal, identity padding.
void launch_corr_build(const double *X, int n, int d, double p, double delta,
                       const double *theta, int batch, double *R, int lda,
                       size_t bstride, int np, hipStream_t s, const uint8_t *mask = nullptr);

// Identity padding of rows/columns n..np-1 (lower part) of caller matrices.
void launch_pad_identity(double *A, int lda, size_t bstride, int n, int np, int batch,
                         hipStream_t s);

// Factorisation steps.
// lk: batch * 64 * 64 doubles, the current diagonal factor copy for TRSM.
// Block column c0 of an outer panel starting at kc0 (K = c0 - kc0 columns
// of the panel before it): potrf_diag updates and factors the diagonal tile,
// panel_trsm updates the rows below (up to np) and solves them against it.
void launch_potrf_diag(double *A, int lda, size_t bstride, int c0, int kc0, int K, int batch,
                       int32_t *info, double *lpart, int nparts, double *lk, hipStream_t s,
                       const uint8_t *mask = nullptr, const RagMat *rag = nullptr);
void launch_panel_trsm(double *A, int lda, size_t bstride, int np, int c0, int kc0, int K,
                       int batch, const double *lk, hipStream_t s, const uint8_t *mask = nullptr,
                       const RagMat *rag = nullptr);
// C(r, c) -= sum_{k in [kc0, kc0+K)} A(r, k) A(c, k) for c in [cs, ce) and
// r in [c's 128-tile row .. np), i.e. the lower part of the column range.
// prec selects the arithmetic of the trailing updates (GP_FP64 or
// GP_MIXED_FAST); updates of a single 64-column block are always FP64.
void launch_syrk_update(double *A, int lda, size_t bstride, int np, int cs, int ce,
                        int kc0, int K, int batch, hipStream_t s, int prec,
                        const uint8_t *mask = nullptr, const RagMat *rag = nullptr,
                        const int32_t *hlive = nullptr);

// Forward solves L [a b] = [1 y] and eq. 3-4 run along with the
// factorisation: the solve of the columns of each finished outer panel (a
// solve segment) goes to a stream of its own while later panels are
// factored; z (batch x 2 np doubles) carries the partial solution from one
// segment to the next, and the last segment writes `out`.
struct SolvePlan {
    const double *y;
    int n;
    double *z;
    gp_result *out;
    const RagMat *rag = nullptr;   // ragged batch: n and y per matrix
};

// The whole blocked factorisation plus log-det partials.  With
// `bordered`, A has order 2 np and holds [[R, I], [I, 0]]; only the first np
// columns are factored, which leaves L^-T bottom-left and -R^-1 bottom-right.
// With a solve plan the forward solves and eq. 3-4 are done as well.
// Synchronizes and destroys the side streams the factorisation created for
// caller stream `caller` on the current device (if any), before the caller
// destroys that stream.
void release_side_streams(hipStream_t caller);

void factor_batch(double *A, int lda, size_t bstride, int np, int batch, int32_t *info,
                  double *lpart, double *lk, hipStream_t s, int prec, bool bordered = false,
                  const uint8_t *mask = nullptr, int8_t *crt_res = nullptr,
                  int32_t *crt_ex = nullptr, bool lookahead = true, int extra = 0,
                  const SolvePlan *plan = nullptr, const RagMat *rag = nullptr,
                  const int32_t *hlive = nullptr);

// Predictions: rows np .. np + extra - 1 below the n_pad x n_pad matrix ride
// through the factorisation as rows below the diagonal (factor_batch with
// `extra`), so each is turned into its forward solve L^-1 v:
//   row np:       1 (c < n), 0 otherwise        -> a = L^-1 1
//   row np + 1:   y_c                            -> b = L^-1 y
//   rows np + 2 .. np + 63: zero
//   row np + 64 + j: r_c(x*_j) = correlation of x*_j and x_c (c < n; no nugget)
//                                                -> w_j = L^-1 r(x*_j)
// (leading dimension np + extra, extra = 64 + 64 ceil(N / 64)).
void launch_pred_rows(double *A, int lda, size_t bstride, int np, const double *X, int n, int d,
                      double p, const double *y, const double *theta, const double *Xs, int N,
                      int extra, int batch, hipStream_t s);
// fit (as gp_result) from rows a, b; then per test point
//   mean = mu + w.(b - mu a),  mse = sigma2 (1 - w.w + (1 - a.w)^2 / a.a)
void launch_pred_reduce(const double *A, int lda, size_t bstride, int np, int n,
                        const double *lpart, int nparts, const int32_t *info, int N, int batch,
                        gp_result *fit, double *mean, double *mse, hipStream_t s);

// Host-side check of a dataset descriptor (pointers, sizes, family, delta).
bool dataset_valid(const gp_dataset *ds);

// gp_nll_batch with the lookahead of the factorisation switchable (the
// request server runs several calls side by side and turns it off).
gp_status nll_batch_impl(const gp_dataset *ds, int32_t batch, const double *theta, int32_t prec,
                         void *ws, size_t ws_bytes, gp_result *out, hipStream_t stream,
                         bool lookahead);

// Ragged FP64 batch over several datasets (multi.hip): counts[k] thetas of
// dataset k, packed per dataset in order; one launch sequence for all.
size_t ragged_workspace_bytes(const gp_dataset *ds, int32_t nds, const int32_t *counts);
gp_status nll_ragged_impl(const gp_dataset *ds, int32_t nds, const int32_t *counts,
                          const double *theta, void *ws, size_t ws_bytes, gp_result *out,
                          hipStream_t stream, bool lookahead);

// GP_MIXED trailing update by modular arithmetic on INT8 MFMA (crt.hip):
// per row of the panel block P (rows pe .. np-1, K columns from kc0) an
// exponent and the residues of its fixed-point integers modulo CRT_NMOD
// moduli, then C -= P P^T over the columns [cs, ce) (multiples of 64 from
// pe) reconstructed from the per-modulus INT8 products.  K is 256, 512, 768
// or 1024.
constexpr int CRT_NMOD = 16;
struct CrtConst {
    int b;                    // fraction bits of the per-row fixed point
    int pad_;
    double Mscaled;           // (m_1 ... m_N) 2^-2b
    float mf[CRT_NMOD];       // moduli and reciprocals (FP32: reduction of the products)
    float inv[CRT_NMOD];
    double md[CRT_NMOD];      // moduli and reciprocals (FP64: residues of the split)
    double invd[CRT_NMOD];
    double t29[CRT_NMOD];     // 2^29 mod m_l
    double f1[CRT_NMOD];      // y_l / m_l = f1 + f2, f1 a multiple of 2^-40
    double f2[CRT_NMOD];
};
bool crt_setup(int K, CrtConst &c);
// constants for rank K (computed once per K), nullptr if K is not handled
const CrtConst *crt_constants(int K);
// residue bytes for `batch` matrices of order np at rank K (rows padded to 128)
size_t crt_residue_bytes(int np, int K, int batch);
void launch_crt_split(const double *A, int lda, size_t bstride, int np, int pe, int kc0, int K,
                      int batch, const CrtConst &cc, int8_t *sl, int32_t *ex, hipStream_t s,
                      const uint8_t *mask = nullptr);
void launch_syrk_update_crt(double *A, int lda, size_t bstride, int np, int pe, int cs, int ce,
                            int K, int batch, const CrtConst &cc, const int8_t *sl,
                            const int32_t *ex, hipStream_t s, const uint8_t *mask = nullptr);

// Iterative refinement of R x = [1 y] with FP64 residuals (R regenerated
// from X) and corrections through the factor A; then mu, sigma2, nll.
// rhs, x, s: batch * 2 np doubles each.
void refine_solves(const double *A, int lda, size_t bstride, int np, const gp_dataset *ds,
                   const double *theta, int batch, const double *lpart, const int32_t *info,
                   double *rhs, double *x, double *s, int sweeps, gp_result *out, hipStream_t st);

// Gradient pieces (grad.hip).
void launch_border_init(double *A, int lda, size_t bstride, int np, int batch, hipStream_t s);
void launch_alpha(const double *A, int lda, size_t bstride, int np, int n, const double *y,
                  const gp_result *res, double *alpha, int batch, hipStream_t s);
void launch_adjoint(const double *A, int lda, size_t bstride, int np, int n, int d, double p,
                    const double *X, const double *theta, const double *alpha,
                    const gp_result *res, double *part, double *grad, int batch, hipStream_t s);

// Log-determinant alone: logdet[b] = sum of the nparts partials.
void launch_logdet_sum(const double *lpart, int nparts, int batch, double *logdet,
                       hipStream_t s);

// Forward solves with [1 y], mu, sigma2, nll; writes gp_result.
// ir_tag goes to gp_result.ir_iters of the thetas written.
void launch_solve_reduce(const double *A, int lda, size_t bstride, int np, int n,
                         const double *y, const double *lpart, int nparts,
                         const int32_t *info, int batch, gp_result *out, hipStream_t s,
                         const uint8_t *mask = nullptr, int ir_tag = 0);
// Columns [64 ib0, 64 ib1) of the forward solve (right-hand sides from
// [1 y] when `first`, else from z); the last segment also does the
// reductions of eq. 3-4 and writes out, the others store the state to z.
void launch_solve_segment(const double *A, int lda, size_t bstride, int np, int n,
                          const double *y, const double *lpart, int nparts,
                          const int32_t *info, int batch, gp_result *out, double *z, int ib0,
                          int ib1, hipStream_t s, const RagMat *rag = nullptr);

// mask[b] = 1 for thetas whose mixed-precision result must be recomputed in
// FP64 (failed pivot or refinement above the FP64 backward-error level).
void launch_fallback_mask(const gp_result *out, int batch, uint8_t *mask, hipStream_t s);

}  // namespace gpk
