/*
 * gpnll.h -- C ABI of the MI355X (gfx950) Gaussian-process profile-likelihood
 * library (libgpnll.so).
 *
 * The library evaluates, for many correlation parameters theta, the profile
 * negative log-likelihood of the model y(x_i) = mu + z(x_i) (Franey, Ranjan &
 * Chipman, arXiv 1203.1269, Sec. 2, eq. 1) with the power-exponential
 * correlation (eq. 2) plus a nugget delta on the diagonal:
 *
 *     R_ij   = exp(-sum_k theta_k |x_ik - x_jk|^p)   (i != j),  R_ii = 1 + delta
 *     mu     = (1' R^-1 1)^-1 1' R^-1 y                            (eq. 3)
 *     sigma2 = (y - 1 mu)' R^-1 (y - 1 mu) / n                     (eq. 3)
 *     nll    = log|R| + n ln(sigma2)                               (eq. 4)
 *
 * eq. 4 as printed carries n ln[(y-1mu)'R^-1(y-1mu)], i.e. nll + n ln n; that
 * value is nll + n*log(n) and is not returned separately.
 *
 * Conventions shared by every entry point:
 *   - Every pointer argument is a DEVICE pointer owned by the caller unless
 *     marked "host".  The library never allocates, frees or keeps device
 *     memory; all scratch space is the caller's workspace `ws`.
 *   - Calls are asynchronous and stream-ordered on `stream`; the returned
 *     status reports argument and launch errors only and never waits.
 *   - Numerical status is per theta, written on the device in
 *     gp_result.info (one bad theta never fails the batch):
 *        0   success
 *        k>0 the k-th pivot (1-based) of the Cholesky factorisation was not
 *            strictly positive or was NaN; all outputs NaN
 *        -1  (y - 1 mu)' R^-1 (y - 1 mu) == 0 exactly: sigma2 = 0, nll = -inf
 *        -3  theta has a negative or non-finite entry; all outputs NaN
 *   - Matrices are column-major.  Internally the order is padded to
 *     n_pad = 64 * ceil(n / 64) with an identity block, which changes neither
 *     the determinant nor the solves.
 *   - Limits: 2 <= n <= GP_NMAX, 1 <= d <= GP_DMAX, 0 < p <= 2, delta >= 0.
 */
#ifndef GPNLL_H
#define GPNLL_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GP_NMAX 8192
#define GP_DMAX 32

typedef enum {
    GP_OK = 0,
    GP_EINVAL = -1,      /* invalid argument (sizes, scalars, null pointers) */
    GP_EWORKSPACE = -2,  /* workspace smaller than gp_workspace_bytes()      */
    GP_ELAUNCH = -3      /* a kernel launch failed (hipGetLastError)         */
} gp_status;

typedef enum {
    GP_FP64 = 0          /* every step in FP64 (FP64 MFMA for the trailing updates) */
} gp_prec;

/* One result per theta (40 bytes). */
typedef struct {
    double logdet;   /* log|R_delta| = 2 sum_j ln L_jj (Sec. 2, via the Cholesky factor) */
    double mu;       /* eq. 3 */
    double sigma2;   /* eq. 3 */
    double nll;      /* log|R_delta| + n ln(sigma2)  (eq. 4 up to the constant n ln n) */
    int32_t info;    /* see the conventions above */
    int32_t ir_iters;/* refinement sweeps taken (0 on the FP64 path) */
} gp_result;

/* A resident dataset.  X: device, n x d, row-major (x_i is row i).
 * y: device, n.  p, delta: host scalars of eq. 2 and the nugget. */
typedef struct {
    const double *X;
    const double *y;
    int32_t n;
    int32_t d;
    double p;
    double delta;
} gp_dataset;

/* Bytes of workspace that gp_nll_batch needs for `batch` thetas on a dataset
 * of n points in d dimensions at precision `prec`.  Returns 0 for invalid
 * arguments.  The workspace holds one padded n_pad x n_pad FP64 matrix per
 * theta plus O(n) vectors per theta. */
size_t gp_workspace_bytes(int32_t n, int32_t d, int32_t batch, int32_t prec);

/* Profile likelihood for `batch` thetas (theta: device, batch x d,
 * row-major) on one dataset (ds: host struct).  out: device, batch results.
 * Steps, all on the GPU: correlation build (eq. 2 + nugget), blocked
 * right-looking Cholesky, log-determinant, forward solves with [1 y] and the
 * reductions of eq. 3-4 (Sec. 2, the three expensive components (i)-(iii)).
 * ws: device workspace of at least gp_workspace_bytes(n, d, batch, prec)
 * bytes, 256-byte aligned. */
gp_status gp_nll_batch(const gp_dataset *ds, int32_t batch, const double *theta,
                       int32_t prec, void *ws, size_t ws_bytes, gp_result *out,
                       hipStream_t stream);

/* gp_nll_batch with batch = 1. */
gp_status gp_nll(const gp_dataset *ds, const double *theta, int32_t prec,
                 void *ws, size_t ws_bytes, gp_result *out, hipStream_t stream);

/* Step a1 alone: write R_delta (eq. 2 plus nugget) for `batch` thetas.
 * R: device, batch matrices of order n_pad = 64*ceil(n/64), column-major with
 * leading dimension ldr (>= n_pad) and batch stride ldr*ldr doubles.  Written:
 * every 64 x 64 tile on or below the diagonal (diagonal tiles in full); the
 * padding rows/columns hold the identity.  Tiles above the diagonal are not
 * touched.  info: device, batch int32, set to 0 or -3 (invalid theta). */
gp_status gp_corr_build(const gp_dataset *ds, int32_t batch, const double *theta,
                        double *R, int32_t ldr, int32_t *info, hipStream_t stream);

/* Step a2/a3 alone: in-place blocked Cholesky R = L L' of `batch` symmetric
 * matrices of order n (lower triangle referenced), column-major, leading
 * dimension lda >= 64*ceil(n/64), batch stride lda*lda doubles.  Rows and
 * columns n..n_pad-1 are overwritten with the identity.  On return the lower
 * triangle holds L and the strict upper triangle of each 64 x 64 diagonal
 * tile is zero.  info: device, batch int32; must be zero on entry (entries
 * that are nonzero on entry are left unchanged and mark that matrix as
 * already failed).  logdet: device, batch doubles, 2 sum_j ln L_jj.
 * ws: device workspace of at least gp_cholesky_ws_bytes(n, batch). */
size_t gp_cholesky_ws_bytes(int32_t n, int32_t batch);
gp_status gp_cholesky_batch(int32_t n, int32_t batch, double *A, int32_t lda,
                            int32_t *info, double *logdet, void *ws, size_t ws_bytes,
                            hipStream_t stream);

/* Per-launch timing for measurement.  gp_profile_begin(max_launches) makes
 * every later kernel launch of this library record two hipEvents on its own
 * stream, tagged with that launch's algorithmic FP64 FLOPs and HBM bytes
 * (counted on the padded order n_pad).  gp_profile_end waits for the recorded
 * events, sums time, FLOPs and bytes per kernel kind into `stats` (host
 * array of max_stats entries) and returns the number of kinds written, or a
 * negative gp_status (GP_EWORKSPACE if more than max_launches launches were
 * made).  Host-side event objects only; no device memory.  One host thread
 * at a time. */
typedef struct {
    char name[32];
    int32_t launches;
    int32_t pad_;
    double ms;      /* summed event time of the launches */
    double flops;   /* summed algorithmic FLOPs */
    double bytes;   /* summed algorithmic HBM bytes */
} gp_kernel_stat;

gp_status gp_profile_begin(int32_t max_launches);
int32_t gp_profile_end(gp_kernel_stat *stats, int32_t max_stats);

#ifdef __cplusplus
}
#endif
#endif /* GPNLL_H */
