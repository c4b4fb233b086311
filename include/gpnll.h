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
 *     (or a Matern family, gp_corr below)
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
 *     status reports argument and launch errors only and never waits.  The
 *     factorisation overlaps its trailing updates with the next panel on a
 *     second stream, and runs the forward solve of each finished panel on a
 *     third: the library creates these two streams (default priority) and
 *     four events per (device, caller stream) on first use and keeps them
 *     until the process ends (for at most 64 caller streams; calls on
 *     further streams factor without the lookahead, with the same results);
 *     their work is joined back into `stream` before the call's last
 *     kernel, so the call still behaves as ordered on `stream`.  Calls that share a stream must not be issued from several
 *     host threads at the same time.
 *   - Numerical status is per theta, written on the device in
 *     gp_result.info (one bad theta never fails the batch):
 *        0   success
 *        k>0 the k-th pivot (1-based) of the Cholesky factorisation was not
 *            strictly positive or was NaN; all outputs NaN
 *        -1  (y - 1 mu)' R^-1 (y - 1 mu) == 0 exactly: sigma2 = 0, nll = -inf
 *        -3  theta has a negative or non-finite entry; all outputs NaN
 *        -4  (request server only) the micro-batch could not be launched
 *   - Matrices are column-major.  Internally the order is padded to
 *     n_pad = 64 * ceil(n / 64) with an identity block, which changes neither
 *     the determinant nor the solves.
 *   - Limits: 2 <= n <= GP_NMAX, 1 <= d <= GP_DMAX, 0 < p <= 2 (power
 *     exponential family), delta >= 0,
 *     1 <= batch <= GP_BATCH_MAX (larger batches are rejected with GP_EINVAL;
 *     split them over several calls).
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
#define GP_BATCH_MAX 65535
#define GP_MIXED_MODULI 16  /* INT8 moduli of the GP_MIXED trailing update */
#define GP_MIXED_RANK 768   /* rank of the GP_MIXED trailing updates (outer panel width) */

typedef enum {
    GP_OK = 0,
    GP_EINVAL = -1,      /* invalid argument (sizes, scalars, null pointers) */
    GP_EWORKSPACE = -2,  /* workspace smaller than gp_workspace_bytes()      */
    GP_ELAUNCH = -3      /* a kernel launch failed (hipGetLastError)         */
} gp_status;

typedef enum {
    GP_FP64 = 0,         /* every step in FP64 (FP64 MFMA for the trailing updates) */
    GP_MIXED = 1,        /* matched accuracy: the rank-768 trailing updates
                            C -= P P^T run on INT8 MFMA by modular
                            arithmetic: each row of P is rounded to a
                            fixed-point integer (per-row power-of-two scale,
                            56 fraction bits at rank 768), the integer
                            product is formed exactly modulo
                            GP_MIXED_MODULI pairwise coprime moduli <= 256
                            (one INT8 product with exact INT32 accumulation
                            per modulus) and recovered by the Chinese
                            remainder theorem in FP64; every other step in
                            FP64.  The update is as accurate as the FP64 one
                            (error below K 2^-56 of the row scales):
                            -2logL and log|R| agree with the FP64 path well
                            within 1e-8 relative.  A theta whose
                            factorisation loses positive definiteness is
                            recomputed on the FP64 path within the same
                            call (gp_result.ir_iters = -1). */
    GP_MIXED_FAST = 2    /* rank-512 trailing updates on FP32 MFMA with FP32
                            accumulation; correlation build, diagonal
                            factorisation, TRSM and log-det in FP64; the solves
                            R x = [1 y] are refined with FP64 residuals (R
                            regenerated from X) for 2 sweeps before mu and
                            sigma2 are formed.  log|R| keeps the error of the
                            factorisation; errors against the FP64 result are
                            reported, not bounded (they grow with the
                            conditioning of R).  A theta whose mixed
                            factorisation loses positive definiteness or
                            whose refinement stays above the FP64 backward
                            error is recomputed on the FP64 path within the
                            same call (gp_result.ir_iters = -1). */
} gp_prec;

/* One result per theta (40 bytes). */
typedef struct {
    double logdet;   /* log|R_delta| = 2 sum_j ln L_jj (Sec. 2, via the Cholesky factor) */
    double mu;       /* eq. 3 */
    double sigma2;   /* eq. 3 */
    double nll;      /* log|R_delta| + n ln(sigma2)  (eq. 4 up to the constant n ln n) */
    int32_t info;    /* see the conventions above */
    int32_t ir_iters;/* refinement sweeps (0 on the FP64 and GP_MIXED paths;
                        -1 when a mixed theta was recomputed in FP64) */
} gp_result;

/* Correlation families (gp_dataset.corr).  Each is a product over the d
 * dimensions of one factor per dimension:
 *   GP_CORR_POWEXP    exp(-theta_k |x_ik - x_jk|^p), 0 < p <= 2     (eq. 2)
 *   GP_CORR_MATERN32  (1 + sqrt(3) h) exp(-sqrt(3) h)
 *   GP_CORR_MATERN52  (1 + sqrt(5) h + 5 h^2 / 3) exp(-sqrt(5) h)
 * with h = theta_k |x_ik - x_jk|: the Matern correlations of smoothness 3/2
 * and 5/2, the alternative Sec. 2 names as numerically more stable; p is not
 * used by them. */
typedef enum {
    GP_CORR_POWEXP = 0,
    GP_CORR_MATERN32 = 1,
    GP_CORR_MATERN52 = 2
} gp_corr;

/* A resident dataset.  X: device, n x d, row-major (x_i is row i).
 * y: device, n.  p, delta: host scalars of eq. 2 and the nugget.  corr: a
 * gp_corr value (GP_CORR_POWEXP for eq. 2); 48 bytes. */
typedef struct {
    const double *X;
    const double *y;
    int32_t n;
    int32_t d;
    double p;
    double delta;
    int32_t corr;
    int32_t reserved;   /* must be 0 */
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

/* The correlation build alone: write R_delta (eq. 2 plus nugget) for `batch` thetas.
 * R: device, batch matrices of order n_pad = 64*ceil(n/64), column-major with
 * leading dimension ldr (>= n_pad) and batch stride ldr*ldr doubles.  Written:
 * every 64 x 64 tile on or below the diagonal (diagonal tiles in full); the
 * padding rows/columns hold the identity.  Tiles above the diagonal are not
 * touched.  info: device, batch int32, set to 0 or -3 (invalid theta). */
gp_status gp_corr_build(const gp_dataset *ds, int32_t batch, const double *theta,
                        double *R, int32_t ldr, int32_t *info, hipStream_t stream);

/* The factorisation and log-determinant alone (Sec. 2: the determinant and the solves of eq. 3-4 come
 * from a factorisation of R; Sec. 3: the factorisation is the dominant cost
 * of an evaluation): in-place blocked Cholesky R = L L' of `batch` symmetric
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

/* Value and adjoint gradient of nll with respect to theta for `batch`
 * thetas (FP64 only; prec must be GP_FP64):
 *   d nll/d theta_k = tr(R^-1 dR/dtheta_k) - n r'R^-1 (dR/dtheta_k) R^-1 r / (r'R^-1 r),
 *   r = y - 1 mu, dR_ij/dtheta_k = -R_ij |x_ik - x_jk|^p for i != j (eq. 2;
 *   for the Matern families the derivative of their per-dimension factor).
 * (Sec. 2: gradient-based optimisers need this next to the likelihood.)
 * R^-1 is obtained by carrying the blocked factorisation through the first
 * n_pad columns of [[R, I], [I, 0]] (order 2 n_pad), which leaves -R^-1 in
 * the bottom-right block.  out: device, batch results as gp_nll_batch;
 * grad: device, batch x d row-major, NaN where info != 0.  ws: at least
 * gp_grad_workspace_bytes(n, d, batch) bytes (four n_pad^2 doubles per
 * theta), 16-byte aligned. */
size_t gp_grad_workspace_bytes(int32_t n, int32_t d, int32_t batch);
gp_status gp_nll_grad(const gp_dataset *ds, int32_t batch, const double *theta,
                      int32_t prec, void *ws, size_t ws_bytes, gp_result *out,
                      double *grad, hipStream_t stream);

/* Batched multi-start L-BFGS on -2logL (the paper fits with a genetic
 * algorithm and names multi-start gradient methods as the alternative, each
 * needing many likelihood evaluations, Sec. 2).  `starts` independent
 * minimisations over phi = log(theta): two-loop recursion over the last m
 * curvature pairs, backtracking line search (halving, Armijo constant c1,
 * at most max_ls trials per iteration; the first step of a start without
 * curvature pairs is at most 1 in phi; trial points clipped to
 * [log theta_lo, log theta_hi]); a pair is kept when s.y > 1e-12 |s| |y|; a
 * direction that is not a descent direction restarts that start from the
 * steepest descent.  A start stops when max_k |d(-2logL)/d phi_k| <= gtol,
 * when its line search fails, or after `iters` iterations.  Every
 * value+gradient evaluation is one gp_nll_grad call over the starts still
 * searching (FP64); the search state lives in the workspace and is updated
 * by kernels on `stream`.
 * theta: device, starts x d; in: the starts, out: the final iterates.
 * nll, gnorm (max_k |d(-2logL)/d log theta_k|): device, starts doubles;
 * iters: device, starts int32 (accepted steps).  trace: device,
 * (iters + 1) x starts doubles or NULL: row t holds every start's -2logL
 * after iteration t (rows past summary->iterations are not written).
 * summary: host, filled on return.  ws: at least
 * gp_lbfgs_workspace_bytes(n, d, starts, m) bytes, 256-byte aligned.
 * 1 <= starts <= 1024, 1 <= m <= 32.  Blocking: the call synchronises
 * `stream` once per line-search trial (it reads how many starts are still
 * searching) and returns when the fit is done.  GP_EINVAL for invalid
 * arguments before anything is launched. */
typedef struct {
    int32_t iters;       /* outer iterations */
    int32_t m;           /* curvature pairs kept */
    int32_t max_ls;      /* line-search trials per iteration */
    int32_t reserved;    /* must be 0 */
    double c1;           /* Armijo constant, (0, 1) */
    double gtol;         /* stop when max |d(-2logL)/d log theta_k| <= gtol */
    double theta_lo, theta_hi;   /* 0 < theta_lo < theta_hi */
} gp_lbfgs_config;
typedef struct {
    int32_t iterations;  /* outer iterations run */
    int32_t evaluations; /* gp_nll_grad calls */
} gp_lbfgs_summary;
size_t gp_lbfgs_workspace_bytes(int32_t n, int32_t d, int32_t starts, int32_t m);
gp_status gp_lbfgs(const gp_dataset *ds, int32_t starts, double *theta,
                   const gp_lbfgs_config *cfg, void *ws, size_t ws_bytes, double *nll,
                   double *gnorm, int32_t *iters, double *trace, gp_lbfgs_summary *summary,
                   hipStream_t stream);

/* Predictions at N test points with the model fitted at each of `batch`
 * thetas (the paper obtains them with one R, one Cholesky factorisation and
 * back-solves per test point, Sec. 3, and scores them by the sum of squared
 * prediction errors over a test set, Sec. 4).  The paper does not print the
 * predictor; this is the best linear unbiased one of the model of Sec. 2 and
 * its mean squared error:
 *     mean(x) = mu + r(x)' R^-1 (y - 1 mu)
 *     mse(x)  = sigma2 (1 - r' R^-1 r + (1 - 1' R^-1 r)^2 / (1' R^-1 1))
 * with r_i(x) the correlation of x and x_i (the dataset's family, no nugget) and mu,
 * sigma2 of eq. 3.  FP64 throughout (prec must be GP_FP64).
 * Xstar: device, N x d row-major test points (may be NULL when N == 0).
 * fit: device, batch results as gp_nll_batch.  mean, mse: device, batch x N
 * (NaN where the fit's info is > 0 or -3).  ws: at least
 * gp_predict_workspace_bytes(n, d, batch, N) bytes ((n_pad + 64 +
 * 64 ceil(N/64)) x n_pad doubles per theta plus O(n)), 256-byte aligned. */
size_t gp_predict_workspace_bytes(int32_t n, int32_t d, int32_t batch, int32_t N);
gp_status gp_predict(const gp_dataset *ds, int32_t batch, const double *theta,
                     const double *Xstar, int32_t N, int32_t prec, void *ws, size_t ws_bytes,
                     gp_result *fit, double *mean, double *mse, hipStream_t stream);

/* Uneven-n batching in one call: counts[k] thetas for dataset ds[k]
 * (k < nds; any n, d and correlation family per dataset), the thetas of
 * dataset k stored as a counts[k] x d_k row-major block, blocks concatenated
 * in dataset order in `theta` (device); results in the same order in `out`
 * (device, sum of counts).  The paper evaluated one theta at a time and
 * names concurrent evaluations as the parallelism it could not use (Sec. 3).
 *   GP_FP64: one ragged batch.  Each theta's matrix has its own order
 *     (n_pad of its dataset); the correlation build runs per dataset, then
 *     one launch sequence factors and solves all matrices together (each
 *     launch covers the matrices that still have columns at that step), so
 *     the panel steps of every theta advance in the same kernels.  The sum
 *     of counts is at most GP_BATCH_MAX.
 *   GP_MIXED, GP_MIXED_FAST: each dataset's thetas run as one gp_nll_batch
 *     (without the factorisation lookahead), the per-dataset batches side by
 *     side on a pool of eight library-owned streams (default priority,
 *     created on first use per device and caller stream and kept for the
 *     life of the process; for at most 32 caller streams, further ones run
 *     the batches one after another on `stream`) that fork from and join
 *     back into `stream`.
 * Either way each result is bitwise the one gp_nll_batch gives for that
 * dataset and theta.  ds, counts: host arrays; counts[k] = 0 skips dataset k
 * (its descriptor is then not read).  ws: at least
 * gp_multi_workspace_bytes(ds, nds, counts, prec) bytes, 256-byte aligned
 * (FP64: the matrices at their own orders plus per-theta vectors at the
 * largest; mixed: one gp_nll_batch workspace per dataset with work).
 * Returns GP_EINVAL for an invalid descriptor or count before anything is
 * launched. */
size_t gp_multi_workspace_bytes(const gp_dataset *ds, int32_t nds, const int32_t *counts,
                                int32_t prec);
gp_status gp_nll_multi(const gp_dataset *ds, int32_t nds, const int32_t *counts,
                       const double *theta, int32_t prec, void *ws, size_t ws_bytes,
                       gp_result *out, hipStream_t stream);

/* ------------------------------------------------------------------------ */
/* Continuous-batching request server (host API over gp_nll_batch).
 * The paper evaluates one theta at a time and notes that evaluating the
 * likelihood for many parameter values concurrently is the natural
 * parallelism it could not use (Sec. 3); the server does that across
 * requests that arrive over time, for several resident datasets of uneven n.
 *
 * gp_server_create: datasets (host array of descriptors whose X, y stay
 *   resident on the device), an arena of caller-owned device memory (256-byte
 *   aligned) from which every micro-batch's footprint is carved (admission by
 *   HBM footprint), max_batch thetas per micro-batch, nstreams concurrent
 *   micro-batches (streams of default priority), prec (GP_FP64, GP_MIXED or
 *   GP_MIXED_FAST).  Creates streams, events and pinned host staging.
 * gp_server_submit: queues host requests (copied).  GP_EWORKSPACE if a
 *   request could never fit the arena.
 * gp_server_poll: non-blocking; retires finished micro-batches into `out`
 *   (at most max_out completions; a batch is reported whole or not at all,
 *   so max_out is 0 (admit only) or at least max_batch, else GP_EINVAL)
 *   and launches queued work while a stream and arena space are free: the
 *   oldest request picks the dataset, up to max_batch queued requests of it
 *   (arrival order) form the batch, shrunk until it fits; with `ragged`, up
 *   to max_batch queued requests (arrival order) of at most 8 datasets, the
 *   oldest request's and those closest to it in order n (several requests
 *   of one dataset share the correlation build's power terms), form the
 *   batch (shrunk from the newest until it fits) and run as one ragged FP64
 *   batch.  Returns the number
 *   of completions written or a negative gp_status.  A result of a batch whose
 *   launch failed has info = -4.
 * gp_server_outstanding: requests queued or on the GPU.
 * gp_server_destroy: waits for the streams, frees host resources and the
 *   streams the factorisation made beside the server's streams.
 * One host thread drives a server. */
typedef struct gp_server gp_server;
typedef struct {
    int64_t id;
    int32_t dataset;
    int32_t pad_;
    double theta[GP_DMAX];   /* first d entries used */
} gp_request;
typedef struct {
    int64_t id;
    int32_t dataset;
    int32_t batch;           /* size of the micro-batch it ran in */
    gp_result result;
} gp_completion;
typedef struct {
    int32_t max_batch;
    int32_t nstreams;
    int32_t prec;
    int32_t graphs;          /* 1: launch each micro-batch as a captured HIP
                                graph (kept per stream and updated in place
                                for the same dataset and batch size); 0: direct
                                kernel launches */
    int32_t ragged;          /* 1 (GP_FP64, graphs 0): a micro-batch holds
                                requests of up to 8 datasets, run as one
                                ragged batch (the FP64 path of gp_nll_multi);
                                0: one dataset per micro-batch */
} gp_server_config;

gp_status gp_server_create(const gp_dataset *datasets, int32_t ndatasets, void *arena,
                           size_t arena_bytes, const gp_server_config *cfg, gp_server **out);
gp_status gp_server_submit(gp_server *server, const gp_request *reqs, int32_t count);
int32_t gp_server_poll(gp_server *server, gp_completion *out, int32_t max_out);
int64_t gp_server_outstanding(const gp_server *server);
size_t gp_server_arena_used(const gp_server *server);
gp_status gp_server_destroy(gp_server *server);

/* gp_nll_batch for callers that cannot allocate device memory (code under
 * HIP stream capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same computation and results as gp_nll_batch, with the workspace taken
 * from a fixed array of GP_NOALLOC_BYTES in the library's device memory
 * (one copy per GPU, held from the library's load on that GPU until the
 * process ends) instead of a caller buffer, and without the factorisation
 * lookahead (no library streams are created).  The call allocates nothing.
 * Returns GP_EWORKSPACE when gp_workspace_bytes(n, d, batch, prec) exceeds
 * GP_NOALLOC_BYTES (e.g. n = 1024 fits 8 FP64 thetas), GP_EINVAL for
 * invalid arguments, GP_ELAUNCH if the array's device address cannot be
 * obtained.  Every call on a GPU uses that GPU's one array: calls that
 * overlap on one GPU (other streams or host threads) race, and each call
 * overwrites the array's previous contents. */
#define GP_NOALLOC_BYTES (64u << 20)
gp_status gp_nll_batch_noalloc(const gp_dataset *ds, int32_t batch, const double *theta,
                               int32_t prec, gp_result *out, hipStream_t stream);

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
