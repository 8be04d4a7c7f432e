/*
 * tsne355 — exact t-SNE hot path on AMD Instinct MI355X (gfx950).
 *
 * C ABI of libtsne355.so. The library computes the perplexity-calibrated
 * input affinities P and runs the exact KL-gradient iteration of t-SNE as
 * described in "bigMap: Big Data Mapping with parallelized t-SNE" (Garriga
 * and Bartumeus, arXiv 1812.09869), section "ptSNE: parallelized t-SNE",
 * Eqs. 1-6, 9 and 10. Output maps are 2-D.
 *
 * Conventions (all entry points):
 *   - Array arguments are DEVICE pointers unless stated otherwise: dense,
 *     row-major, FP32 unless stated otherwise. X is n x d, maps are n x 2.
 *   - Every call is asynchronous on `stream` (a hipStream_t; NULL means the
 *     default stream). Nothing is allocated: the caller owns all memory,
 *     including the workspace `ws`, a device buffer of at least
 *     tsne_workspace_bytes() bytes, 256-byte aligned.
 *   - Arguments are validated on the host before any launch; a bad argument
 *     returns an error code at once and launches nothing. Conditions found
 *     on the device (non-finite values, a row whose bisection did not
 *     converge, a workspace that does not hold affinities for this n) set a
 *     flag word inside the workspace, returned by tsne_sync_status().
 *   - Return values are tsne_status codes; tsne_last_error() gives a message
 *     for the last failing call of the calling thread.
 *   - Calls that share a workspace must be ordered on one stream.
 *   - State kept by the library between calls, per device, created on first
 *     use and held until the process ends: one non-blocking side stream and
 *     two events on which the all-zero tiles of a force or cost pass run
 *     beside the rest of the pass (forked from `stream` and joined back into
 *     it, so a caller sees plain stream order; passes on one device are
 *     serialised by a mutex while they are enqueued); four side streams and
 *     their events for the per-thread affinities of tsne_pt_epoch; the
 *     scratch array of tsne_mlp_forward_noalloc. All streams have the
 *     default priority. Beyond that, only the thread-local error message.
 */
#ifndef TSNE355_H
#define TSNE355_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define TSNE_API __attribute__((visibility("default")))
#else
#define TSNE_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TSNE_OK = 0,
  TSNE_E_ARG = 1,        /* null pointer, n < 2, d < 1, bad mode, bad range */
  TSNE_E_PERPLEXITY = 2, /* perplexity not in (1, n - 1): Eq. 2 caps it at n - 1 */
  TSNE_E_WORKSPACE = 3,  /* workspace too small or misaligned */
  TSNE_E_DEVICE = 4,     /* a HIP runtime call failed */
  TSNE_E_NONFINITE = 5,  /* device: non-finite input, Z, gradient or map */
  TSNE_E_NOCONV = 6,     /* device: a row's bisection hit max_bisect */
  TSNE_E_STATE = 7       /* device: workspace holds no affinities for this n */
} tsne_status;

/* Precision of the squared-distance contraction d = |x|^2 + |y|^2 - 2 x.y
 * (Eq. 1's ||x_i - x_j||^2 in GEMM form) that feeds the affinities. All modes
 * run on MFMA; the bisection and every reduction stay FP64/FP32 as documented
 * below.
 *
 * FP32, BF16 and FP16 keep the cancellation of the GEMM form: where |x|^2 is
 * much larger than d, one rounding of the large terms moves d by
 * u |x|^2 (u the unit roundoff), and p_ij by beta_i times that.
 *
 * The x3 modes remove it. Every centred coordinate is cut on one grid for the
 * whole input into three integer slices (x = sigma (h1 + 2^-b h2 + 2^-2b h3)
 * plus a remainder below sigma 2^(-2b-1), with b <= 10 for FP16 and <= 8 for
 * BF16 and 2b + log2(K) <= 24 for K = d rounded up to 32). One MFMA product
 * per operand pair gives the leading slice sum, an integer below 2^24 that
 * the FP32 accumulation adds exactly; seven more give the rest, 2^-b lower.
 * The norms are FP32 (hi, lo) pairs, and n_i + n_j - 2 x.y is formed with an
 * error-free sum of the hi parts (TwoSum) and an exact leading difference
 * (Sterbenz), so d carries about one FP32 rounding of d itself. */
typedef enum {
  TSNE_DIST_FP64 = 0,   /* FP64 MFMA on the centred input (default) */
  TSNE_DIST_FP32 = 1,   /* FP32 MFMA */
  TSNE_DIST_BF16 = 2,   /* BF16 operands, FP32 accumulate */
  TSNE_DIST_BF16X3 = 3, /* three BF16 slices, eight products, compensated combine */
  TSNE_DIST_FP16 = 4,   /* FP16 operands, FP32 accumulate */
  TSNE_DIST_FP16X3 = 5  /* three FP16 slices, eight products, compensated combine */
} tsne_dist_mode;

/* Options of the affinity stage. A NULL pointer selects the defaults
 * {TSNE_DIST_FP64, 200, 1e-6, 1}.
 *
 * reorder != 0: after P is formed, the points are renumbered internally so
 * that points close in the input space are contiguous (a bisection tree
 * that splits every segment of the order along its leading principal
 * direction, with leaves of one 256-row tile), and P is rebuilt in that
 * order. Tiles of P that then hold only zeros (flushed sub-normal values
 * included) are skipped by the attractive part of every force pass and cost
 * evaluation. Results are those of the same computation in another
 * summation order; inputs and outputs of every call stay in the caller's
 * order. Skipped when d > 2048 or n <= 256. */
typedef struct {
  int32_t dist_mode;  /* tsne_dist_mode */
  int32_t max_bisect; /* bisection passes per row, >= 1 */
  double tol_h;       /* stop when |H_i - ln(perplexity)| <= tol_h (nats), > 0 */
  int32_t reorder;    /* 1: group points by affinity components (default); 0: keep order */
  int32_t implicit_p; /* 0: store P (default); 1: store only what rebuilds it, and recompute
                         P in every pass (tsne_*_implicit, any distance mode) */
} tsne_aff_opts;

/* Learning-rate rules of an update. */
typedef enum {
  /* the given learning_rate, scaled per coordinate by adaptive gains (the
   * conventional t-SNE schedule of Eq. 10 and the paragraph after it) */
  TSNE_LR_GAINS = 0,
  /* the paper's own rule (Eq. 11, section "Internal parametric
   * configuration"): eta = ln(n - 1) (Y_max - Y_min) / 2, where
   * Y_max - Y_min is the larger of the two coordinate ranges of the map the
   * gradient is taken at; no gains (g is neither read nor written and may be
   * NULL), learning_rate and min_gain are ignored */
  TSNE_LR_RANGE = 1
} tsne_lr_rule;

/* Parameters of one update (Eq. 10 and the paragraph after it). */
typedef struct {
  float exaggeration;  /* alpha: multiplies p_ij in the gradient (early exaggeration) */
  float momentum;      /* mu */
  float learning_rate; /* eta (TSNE_LR_GAINS) */
  float min_gain;      /* floor of the adaptive gains (TSNE_LR_GAINS) */
  int32_t recentre;    /* nonzero: subtract the mean of the map after the update */
  int32_t lr_rule;     /* tsne_lr_rule; anything else is TSNE_E_ARG */
} tsne_step_params;

/* Bytes of workspace for n points in d dimensions with the given distance
 * mode; 0 if the arguments are out of range. Host-only, no device work.
 * (The distance mode is the only option the size depends on, so it is
 * passed alone rather than as a tsne_aff_opts; an implicit-P workspace has
 * its own size function below.) */
TSNE_API size_t tsne_workspace_bytes(int64_t n, int32_t d, int32_t dist_mode);

/*
 * Input affinities (Eqs. 1-3). x: n x d FP32 (device). For every row i the
 * precision beta_i of the Gaussian kernel is found by bisection so that the
 * entropy of p_{.|i} equals ln(perplexity) (Eq. 2, in nats); then
 * p_ij = (p_{j|i} + p_{i|j}) / (2n) is stored in the workspace (FP32, upper
 * triangle, tile-packed; entries below the normal FP32 range are stored as
 * 0). Self terms are zero. Errors: TSNE_E_ARG,
 * TSNE_E_PERPLEXITY, TSNE_E_WORKSPACE, TSNE_E_DEVICE; device flags may set
 * TSNE_E_NONFINITE (non-finite x) or TSNE_E_NOCONV.
 */
TSNE_API int tsne_affinities(const float *x, int64_t n, int32_t d, double perplexity,
                    const tsne_aff_opts *opts, void *ws, size_t ws_bytes, void *stream);

/*
 * Input affinities from given dissimilarities instead of points (any measure
 * of similarity may enter the method, section "ptSNE: parallelized t-SNE";
 * the paper's dwt1005 set gives shortest-path distances). dis: n x n FP32
 * (device, row-major), symmetric and non-negative; the diagonal is ignored.
 * The dissimilarity takes the place of ||x_i - x_j||, so Eq. 1 uses its
 * square; everything after that is tsne_affinities. The workspace is that of
 * tsne_workspace_bytes(n, 1, TSNE_DIST_FP64). opts->dist_mode and
 * opts->reorder are ignored (no coordinates: the caller's order is kept).
 * P takes the upper-triangle value dis[i][j], i < j, for both orders of a
 * pair. Errors as tsne_affinities; a negative or non-finite off-diagonal
 * entry sets TSNE_E_NONFINITE on the device.
 */
TSNE_API int tsne_affinities_dissim(const float *dis, int64_t n, double perplexity,
                                    const tsne_aff_opts *opts, void *ws, size_t ws_bytes,
                                    void *stream);

/*
 * One iteration of the exact gradient descent from state (y, u, g), each
 * n x 2 FP32 on the device, updated in place:
 *   grad_i = 4 sum_j (alpha p_ij - q_ij) w_ij (y_i - y_j),
 *            w_ij = 1 / (1 + |y_i - y_j|^2), q_ij = w_ij / Z      (Eqs. 4, 6)
 *   g <- (grad > 0) != (u > 0) ? g + 0.2 : 0.8 g;  g <- max(g, min_gain)
 *   u <- momentum u - learning_rate g grad;  y <- y + u           (Eq. 10)
 *   y <- y - mean(y) if recentre.
 * With lr_rule TSNE_LR_RANGE the gains step is skipped and
 *   u <- momentum u - eta grad,  eta = ln(n - 1) (Y_max - Y_min) / 2 (Eq. 11)
 * at the map y passed in.
 * grad_out (nullable, n x 2 FP32) receives the gradient; z_out (nullable,
 * device double) receives Z. Requires a workspace filled by
 * tsne_affinities for the same n. Z and all row sums are reduced in FP64 in
 * a fixed order: repeated calls give bitwise identical results.
 */
TSNE_API int tsne_step(void *ws, int64_t n, float *y, float *u, float *g, const tsne_step_params *prm,
              float *grad_out, double *z_out, void *stream);

/* The two halves of tsne_step, for callers that time or schedule them
 * separately. tsne_forces runs the pair pass over the stored tiles at map y
 * (Student-t kernel, Z, attractive and repulsive row sums; Eqs. 4 and 6) and
 * keeps the partial sums in the workspace; tsne_update reduces them, forms
 * the gradient with exaggeration prm->exaggeration and applies the update
 * of tsne_step to (y, u, g). tsne_update must follow tsne_forces for the same
 * y on the same stream. */
TSNE_API int tsne_forces(void *ws, int64_t n, const float *y, void *stream);
TSNE_API int tsne_update(void *ws, int64_t n, float *y, float *u, float *g,
                         const tsne_step_params *prm, float *grad_out, double *z_out,
                         void *stream);

/* Gradient of Eq. 6 (with exaggeration alpha) at map y, without an update.
 * grad_out: n x 2 FP32 (device, required); z_out nullable device double. */
TSNE_API int tsne_gradient(void *ws, int64_t n, const float *y, float alpha, float *grad_out,
                  double *z_out, void *stream);

/* KL cost of Eq. 5 and the pseudo-normalised cost of Eq. 9 at map y, with
 * the true P (no exaggeration). out: device double[2] = {KL, C_norm}. */
TSNE_API int tsne_cost(void *ws, int64_t n, const float *y, double *out, void *stream);

/* ------------------------------------------------------------------------
 * Implicit P. For n beyond what a stored P fits (the packed FP32 triangle
 * takes 2 n^2 bytes), tsne_affinities with implicit_p = 1 keeps only the row
 * statistics, the contraction operands in the internal order (the centred
 * input in FP64, or the FP32 / 16-bit operands of a reduced distance mode)
 * and a buffer of tiles. The affinity stage ends with one pass over every
 * tile that finds the all-zero tiles of P; every force pass and cost
 * evaluation then recomputes the nonzero tiles buffer by buffer (their
 * distances on MFMA in the workspace's distance mode, Eq. 1 with the stored
 * beta, m and S, Eq. 3) and consumes them at once, and gives the zero tiles
 * the repulsion-only body. P, gradients, costs and maps are bitwise those of
 * the stored path in the same mode; a pass does up to N^2 D / 2 more
 * multiply-adds of the mode's contraction (fewer by the zero tiles' share).
 * The stored-P entry points (tsne_step, tsne_forces, tsne_gradient,
 * tsne_cost, tsne_export_p_rows, the batched launch) reject such a workspace
 * on the device (TSNE_E_STATE), and these reject a stored-P workspace.
 * ---------------------------------------------------------------------- */

/* Bytes of an implicit-P workspace for n points in d dimensions with the
 * given distance mode (tsne_dist_mode; 0 if out of range). Host-only. */
TSNE_API size_t tsne_workspace_bytes_implicit(int64_t n, int32_t d, int32_t dist_mode);

/* tsne_step, tsne_gradient and tsne_cost on an implicit-P workspace. d and
 * dist_mode are those the affinities were computed with (the workspace keeps
 * the contraction operands of that mode; a workspace prepared for another n,
 * d or mode is refused on the device with TSNE_E_STATE, before any of its
 * buffers is touched; a mode outside tsne_dist_mode is TSNE_E_ARG). */
TSNE_API int tsne_step_implicit(void *ws, int64_t n, int32_t d, int32_t dist_mode, float *y,
                                float *u, float *g, const tsne_step_params *prm, float *grad_out,
                                double *z_out, void *stream);
TSNE_API int tsne_gradient_implicit(void *ws, int64_t n, int32_t d, int32_t dist_mode,
                                    const float *y, float alpha, float *grad_out, double *z_out,
                                    void *stream);
TSNE_API int tsne_cost_implicit(void *ws, int64_t n, int32_t d, int32_t dist_mode,
                                const float *y, double *out, void *stream);

/* Synchronises the stream and returns the first device-side condition
 * recorded in the workspace (TSNE_OK if none). Clears nothing. */
TSNE_API int tsne_sync_status(void *ws, void *stream);

/* Message for the last failing call on this thread ("" if none). */
TSNE_API const char *tsne_last_error(void);

/* Test hooks. Row statistics of the calibration: beta (double), row minimum
 * m of the squared distances (float), normaliser S = sum_j exp(-beta (d_ij -
 * m)) (double), entropy H in nats (double), bisection passes (int32,
 * negative if not converged). Any pointer may be NULL. */
TSNE_API int tsne_export_rowstats(void *ws, int64_t n, double *beta, float *m, double *S, double *H,
                         int32_t *evals, void *stream);

/* Test hook: out (device double[4]) = {sum_{i != j} p_ij, sum_{i != j} p_ij ln p_ij,
 * Z of the last force pass, perplexity}. */
TSNE_API int tsne_export_scalars(void *ws, int64_t n, double *out, void *stream);

/* Test hook: dense rows row0 .. row0 + nrows - 1 of P (nrows x n FP32). */
TSNE_API int tsne_export_p_rows(void *ws, int64_t n, int64_t row0, int64_t nrows, float *out,
                       void *stream);

/* Test hook: the internal order and the zero-tile flags (device buffers,
 * either may be NULL). perm (int32[n]): perm[r] is the caller's index of the
 * point at internal position r (the identity when reordering is off).
 * flags (uint8[nb (nb + 1) / 2], nb = ceil(n / 256)): one byte per tile of
 * the upper triangle of P in row-major tile order, 0 when every entry of the
 * tile is zero. */
TSNE_API int tsne_export_order(void *ws, int64_t n, int32_t *perm, uint8_t *flags, void *stream);

/* ------------------------------------------------------------------------
 * Batched iteration: many independent problems advanced together, one
 * launch per phase for all of them (the GPU counterpart of the paper's
 * independent partial t-SNEs, section "Parallelized implementation").
 * Each problem has its own workspace, filled by tsne_affinities, and its own
 * state (y, u, g: n x 2 FP32 device arrays). Every problem's result is
 * bitwise identical to calling tsne_step on it alone.
 * ---------------------------------------------------------------------- */
typedef struct {
  void *ws;    /* workspace holding the problem's affinities */
  int64_t n;   /* number of points */
  float *y, *u, *g;
} tsne_batch_problem;

/* Bytes of the batch workspace (device) for `count` problems; 0 if count < 1. */
TSNE_API size_t tsne_batch_workspace_bytes(int32_t count);

/* Writes the device table of the problems (host array) into batch_ws and
 * synchronises the stream. The same array must be passed to tsne_batch_step;
 * a mismatch is detected on the device and the step does nothing. */
TSNE_API int tsne_batch_plan(const tsne_batch_problem *problems, int32_t count, void *batch_ws,
                             size_t batch_ws_bytes, void *stream);

/* One iteration (as tsne_step) of every problem, with the same parameters. */
TSNE_API int tsne_batch_step(const tsne_batch_problem *problems, int32_t count,
                             const void *batch_ws, const tsne_step_params *prm, void *stream);

/* The cost of tsne_cost (Eqs. 5 and 9) of every problem at its current map
 * y, in one launch per phase. out: device double[2 count], {KL, C_norm} of
 * problem p at out[2p]. */
TSNE_API int tsne_batch_cost(const tsne_batch_problem *problems, int32_t count,
                             const void *batch_ws, double *out, void *stream);

/* ------------------------------------------------------------------------
 * Parallel scheme, ptSNE (section "Parallelized implementation"). The n
 * points are split into `threads` chunks, contiguous pieces of a per-epoch
 * order of the points (sizes differ by at most one, larger chunks first).
 * Partial t-SNE k runs on chunks k, k+1, ..., k+layers-1 (cyclic), so every
 * chunk is shared by `layers` successive partial problems and every point has
 * one 2-D position per layer. An epoch (subsection "epochs"):
 *   mix:     chunk (k + l) mod threads enters partial problem k at its points'
 *            layer-l positions; momentum state starts at zero;
 *   run:     affinities of the partial problem's own points (Eqs. 1-3), then
 *            `iters` iterations of Eqs. 10-11 (learning rate from the map's
 *            extent, external momentum, no exaggeration, no gains, no
 *            re-centring), all partial problems in one batched launch per
 *            phase;
 *   pool:    every partial result is written back to the layer it was read
 *            from, so each (point, layer) is read and written exactly once.
 * A round is floor(sqrt(n)) epochs; `iters` defaults to ceil(sqrt(z)) with
 * the thread size z = n layers / threads (subsections "thread-size" and
 * "rounds"). Monitors (section comparing t-SNE and ptSNE): the mean over the
 * partial problems of their pseudo-normalised cost (Eq. 9) and the mean over
 * the layers of the embedding size, the diagonal of the layer's box.
 * ---------------------------------------------------------------------- */
typedef struct {
  int32_t threads;    /* partial problems, 1 <= threads <= n */
  int32_t layers;     /* chunks per partial problem, 1 <= layers <= threads */
  double perplexity;  /* of every partial problem, in (1, smallest thread size - 1) */
  float momentum;     /* the external momentum of Eq. 10 */
  int32_t iters;      /* iterations per epoch; <= 0: ceil(sqrt(n layers / threads)) */
  int32_t dist_mode;  /* tsne_dist_mode of the partial affinities */
  int32_t reorder;    /* tsne_aff_opts.reorder of the partial affinities */
  int32_t reserved;   /* must be 0 */
} tsne_pt_opts;

/* Bytes of the ptSNE workspace (device, 256-byte aligned) for n points in d
 * dimensions; 0 if the options are invalid. Host-only. It holds the pooled
 * rows of all partial problems, their workspaces and the batch table. */
TSNE_API size_t tsne_pt_workspace_bytes(int64_t n, int32_t d, const tsne_pt_opts *opts);

/* Iterations per epoch for these options (opts->iters if positive). */
TSNE_API int32_t tsne_pt_iterations(int64_t n, const tsne_pt_opts *opts);

/* Prepares the workspace (thread table, batch plan); synchronises the stream.
 * Errors: TSNE_E_ARG, TSNE_E_PERPLEXITY, TSNE_E_WORKSPACE, TSNE_E_DEVICE. */
TSNE_API int tsne_pt_init(int64_t n, int32_t d, const tsne_pt_opts *opts, void *ws, size_t bytes,
                          void *stream);

/* One epoch. x: n x d FP32; order: int32[n], a permutation of 0..n-1 (the
 * master's mixing draw; entries outside [0, n) are recorded as TSNE_E_ARG for
 * tsne_pt_sync_status and the epoch's result is then undefined); maps:
 * layers x n x 2 FP32, read and updated in place; monitors: nullable device
 * double[2] = {mean partial C_norm, mean layer size} after the epoch. All
 * pointers are device pointers; asynchronous on `stream`. The workspace must
 * have been prepared by tsne_pt_init with the same n, d and options. */
TSNE_API int tsne_pt_epoch(const float *x, int64_t n, int32_t d, const tsne_pt_opts *opts,
                           const int32_t *order, float *maps, void *ws, size_t bytes,
                           double *monitors, void *stream);

/* Synchronises the stream; returns the first condition recorded by the
 * epochs (an order entry out of range) or by any partial problem's
 * workspace (tsne_sync_status), else TSNE_OK. */
TSNE_API int tsne_pt_sync_status(int64_t n, int32_t d, const tsne_pt_opts *opts, void *ws,
                                 size_t bytes, void *stream);

/* Test hook: the workspace of partial problem k (0 <= k < threads) inside the
 * ptSNE workspace, and its number of points. Host-only pointer arithmetic;
 * after an epoch the single-problem export hooks read that epoch's
 * affinities of the partial problem through it (rows in the order of the
 * thread's chunks k, k+1, ..., each in the epoch's order). */
TSNE_API int tsne_pt_partial(int64_t n, int32_t d, const tsne_pt_opts *opts, void *ws,
                             size_t bytes, int32_t k, void **ws_k, int64_t *n_k);

/* Message of the last failing tsne_pt_* call on this thread. */
TSNE_API const char *tsne_pt_last_error(void);

/* ------------------------------------------------------------------------
 * Perplexity-adaptive kernel density estimate of a 2-D map (paKDE, section
 * "Perplexity-adaptive Kernel Density Estimation"). Each map point j gets the
 * precision beta_j of the same perplexity search as the input affinities
 * (Eqs. 1-2 on the squared map distances |y_j - y_k|^2); the density is the
 * sample smoothing estimator with bivariate Gaussian kernels of bandwidth
 * h_j^2 = 2 sigma_j^2 = 1 / beta_j:
 *   f(c) = (S / n) sum_j (beta_j / pi) exp(-beta_j |c - y_j|^2),
 * at the centre c of every cell of a regular raster with cells of area S
 * (the probability mass of the cell; a raster covering the map sums to ~1).
 * ---------------------------------------------------------------------- */
typedef struct {
  float x0, y0;    /* corner of the raster: cell (v, u) spans [x0 + u cx, x0 + (u+1) cx] x ... */
  float cx, cy;    /* cell sizes (> 0); S = cx cy */
  int32_t gx, gy;  /* cells along x and y; the output is gy x gx, row v = y index */
} tsne_raster;

/* Bytes of the workspace of tsne_kde_bandwidths for n map points (0 if n < 3).
 * Host-only. It holds the row statistics and one 256 x n distance block. */
TSNE_API size_t tsne_kde_workspace_bytes(int64_t n);

/* beta (device double[n]) of every point of the map y (device n x 2 FP32),
 * for the given perplexity (1 < perplexity < n - 1). Device conditions (a row
 * that did not converge, non-finite input) are read with tsne_sync_status on
 * this workspace. */
TSNE_API int tsne_kde_bandwidths(const float *y, int64_t n, double perplexity, double *beta,
                                 void *ws, size_t ws_bytes, void *stream);

/* f(c) of every raster cell into out (device FP32, gy x gx, row-major), from
 * the map y (n x 2 FP32) and its precisions beta (n FP64), all on the device.
 * The sum over points is FP32 within chunks of 256 points and FP64 across
 * chunks. Errors: TSNE_E_ARG for null pointers or an invalid raster. */
TSNE_API int tsne_kde_raster(const float *y, int64_t n, const double *beta,
                             const tsne_raster *grid, float *out, void *stream);

/* ------------------------------------------------------------------------
 * Learned surrogate (not in the paper): an MLP d_in -> H -> H -> 2 with ReLU
 * that maps input points to their embedding, trained on (x, y) pairs that
 * the exact path produced. Exact t-SNE (tsne_step) stays the fallback: a
 * short refinement seeded from the network's output.
 *
 * Parameters are one packed FP32 device array: W1 [H][d_in], b1 [H],
 * W2 [H][H], b2 [H], W3 [2][H], b3 [2] (row-major, out x in). Inputs are
 * standardised as (x - mean) * invstd (mean, invstd: device float[d_in]).
 * The two wide layers run as BF16 MFMA contractions with FP32 accumulation
 * (operands rounded to nearest even), the output layer in FP32.
 * Limits: 1 <= d_in <= 64, H in {64, 128, 192, 256}.
 * ---------------------------------------------------------------------- */

/* Number of packed parameters (79,362 for d_in = 50, H = 256). */
TSNE_API int64_t tsne_mlp_param_count(int32_t d_in, int32_t hidden);

/* Workspace bytes for batches of up to `batch` rows; train != 0 adds the
 * buffers of the backward pass. 0 if the arguments are out of range. */
TSNE_API size_t tsne_mlp_workspace_bytes(int32_t d_in, int32_t hidden, int64_t batch,
                                         int32_t train);

/* out (n x 2 FP32) = network(x) for the n rows of x (n x d_in FP32). Rows are
 * processed in chunks of the batch size the workspace was sized for. */
TSNE_API int tsne_mlp_forward(const float *params, int32_t d_in, int32_t hidden,
                              const float *mean, const float *invstd, const float *x, int64_t n,
                              float *out, void *ws, size_t ws_bytes, void *stream);

/* tsne_mlp_forward for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same kernels and results, with the BF16 weight copies kept in a
 * device-resident scratch array of the library (512 KiB per device, held until
 * the process ends) instead of a caller workspace. No allocation happens in
 * the call. The scratch is shared by every call on a device and keeps the
 * last call's contents, so calls that overlap on one device (different
 * streams, threads) race. The stream must belong to the current device.
 * Errors: TSNE_E_ARG as tsne_mlp_forward; TSNE_E_WORKSPACE if the network's
 * scratch would exceed the array (no supported d_in, hidden does). */
TSNE_API int tsne_mlp_forward_noalloc(const float *params, int32_t d_in, int32_t hidden,
                                      const float *mean, const float *invstd, const float *x,
                                      int64_t n, float *out, void *stream);

/* Gradient of L = (1 / (2B)) sum_b |net(x_b) - y_b|^2 over a batch of B rows,
 * rows idx[0..B) of x and y (idx: device int32, or NULL for rows 0..B-1).
 * grad: packed FP32 like params (fully overwritten); loss: device double. */
TSNE_API int tsne_mlp_gradient(const float *params, int32_t d_in, int32_t hidden,
                               const float *mean, const float *invstd, const float *x,
                               const float *y, const int32_t *idx, int64_t batch, float *grad,
                               double *loss, void *ws, size_t ws_bytes, void *stream);

/* One Adam step t (1-based) on count packed FP32 parameters, in place on
 * params, m and v: m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
 * p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps). */
TSNE_API int tsne_mlp_adam(float *params, const float *grad, float *m, float *v, int64_t count,
                           float lr, float beta1, float beta2, float eps, int32_t t,
                           void *stream);

#ifdef __cplusplus
}
#endif

#endif /* TSNE355_H */
