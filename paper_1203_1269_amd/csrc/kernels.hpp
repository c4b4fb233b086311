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
constexpr int OUTER_NB = 256;   // outer panel width (K of the trailing update)

inline int pad64(int n) { return (n + TB - 1) / TB * TB; }

// theta validity, info and log-det partial initialisation.
void launch_init(const double *theta, int d, int batch, int32_t *info, hipStream_t s);

// a1: R_delta tiles on and below the diagonal, identity padding.
void launch_corr_build(const double *X, int n, int d, double p, double delta,
                       const double *theta, int batch, double *R, int lda,
                       size_t bstride, int np, hipStream_t s);

// Identity padding of rows/columns n..np-1 (lower part) of caller matrices.
void launch_pad_identity(double *A, int lda, size_t bstride, int n, int np, int batch,
                         hipStream_t s);

// a2: factorisation steps.
void launch_potrf_diag(double *A, int lda, size_t bstride, int c0, int batch,
                       int32_t *info, double *lpart, int nparts, hipStream_t s);
void launch_trsm_panel(double *A, int lda, size_t bstride, int np, int c0, int batch,
                       hipStream_t s);
// C(r, c) -= sum_{k in [kc0, kc0+K)} A(r, k) A(c, k) for c in [cs, ce) and
// r in [c's 128-tile row .. np), i.e. the lower part of the column range.
void launch_syrk_update(double *A, int lda, size_t bstride, int np, int cs, int ce,
                        int kc0, int K, int batch, hipStream_t s);

// The whole blocked factorisation (a2) plus log-det partials (a3).
void factor_batch(double *A, int lda, size_t bstride, int np, int batch, int32_t *info,
                  double *lpart, hipStream_t s);

// a3 alone: logdet[b] = sum of the nparts partials.
void launch_logdet_sum(const double *lpart, int nparts, int batch, double *logdet,
                       hipStream_t s);

// a4 + a6: forward solves with [1 y], mu, sigma2, nll; writes gp_result.
void launch_solve_reduce(const double *A, int lda, size_t bstride, int np, int n,
                         const double *y, const double *lpart, int nparts,
                         const int32_t *info, int batch, gp_result *out, hipStream_t s);

}  // namespace gpk
