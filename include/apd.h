/*
 * apd.h -- C ABI of libapd, the MI355X (gfx950) library that fits
 * anisotropic power diagrams (APDs) to prescribed cell volumes.
 *
 * Method: Buze, Feydy, Roper, Sedighiani, Bourne, "Anisotropic power
 * diagrams for polycrystal modelling: efficient generation of curved grains
 * via optimal transport", arXiv 2403.03571.
 *
 * Conventions shared by every call
 * --------------------------------
 * - Pointers documented "device" are HIP device pointers the caller owns
 *   (for example the data_ptr() of a torch tensor on the ctx's device);
 *   pointers documented "host" are ordinary host memory.  The library never
 *   frees caller memory.  It owns only the scratch inside an apd_ctx.
 * - Every call enqueues its GPU work on the ctx's stream and returns once
 *   its outputs are written, so outputs are ready on return.  Evaluations
 *   (apd_dual_objective_grad, the passes of the fits) wait for their last
 *   kernel to publish its results in pinned host memory rather than for
 *   the stream: that kernel's tail, which writes no output, may still be
 *   running on return, and later work on the same stream is ordered after
 *   it as usual.
 * - Pixels: the box [lo, hi] is cut into grid[0] x ... x grid[dim-1] equal
 *   boxes (Section 2.3, eq. (2.6)); pixel j has integer coordinates k with
 *   j = row-major index, the LAST axis fastest, and centre
 *   y_d = lo_d + (k_d + 1/2) (hi_d - lo_d) / grid_d.
 * - Labels are 0-based seed indices (the paper's H_j runs over 1..N).
 *   A pixel equidistant (equal cost) from several seeds goes to the lowest
 *   index.
 * - Every call returns an apd_status; on error, apd_last_error(ctx) holds a
 *   message until the next call on the same ctx.  No call aborts the
 *   process.
 */
#ifndef APD_H
#define APD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    APD_OK = 0,
    APD_ERR_INVALID_ARG = 1,   /* bad dim, n, grid, box, NULL pointer, bad option */
    APD_ERR_NOT_SPD = 2,       /* some A_i is not symmetric positive definite */
    APD_ERR_VOLUMES = 3,       /* some v_i <= 0 or sum v != domain measure (rel. 1e-12) */
    APD_ERR_NOT_CONVERGED = 4, /* budget spent; the best iterate is returned */
    APD_ERR_LINESEARCH = 5,    /* no descent step found even after a restart */
    APD_ERR_DEVICE = 6,        /* a HIP runtime call failed */
    APD_ERR_OOM = 7,           /* device scratch could not be allocated */
    APD_ERR_NONFINITE = 8      /* NaN or Inf in x, A or w */
} apd_status;

/* Arithmetic used to decide the assignment (Algorithm 1).  Every tier
 * returns the same labels as an exact double-precision evaluation of
 * C_ij = (y_j - x_i)^T A_i (y_j - x_i) - w_i: the faster tiers re-evaluate in
 * double every pixel whose top-two cost gap is within their rounding bound. */
typedef enum {
    APD_FP64 = 0, /* every pair in double precision */
    APD_FP32 = 1, /* single precision + certified double re-check */
    APD_BF16 = 2, /* bf16 matrix cores (split hi/lo operands, fp32
                     accumulation) + certified double re-check */
    APD_BF16_RECHECK = APD_BF16  /* the same tier, by its boundary name */
} apd_precision;

typedef struct apd_ctx apd_ctx;

/* Create a context on HIP device `device`, enqueuing on `hip_stream`
 * (a hipStream_t; NULL = the device's null stream).  *out receives the
 * context.  Errors: APD_ERR_DEVICE if the device cannot be selected. */
apd_status apd_create(apd_ctx **out, int device, void *hip_stream);

/* Release the context and its device scratch.  NULL is allowed. */
void apd_destroy(apd_ctx *ctx);

/* Message of the last failed call on ctx ("" if none).  Valid until the
 * next call on ctx. */
const char *apd_last_error(const apd_ctx *ctx);

/* Change the stream later calls enqueue on. */
apd_status apd_set_stream(apd_ctx *ctx, void *hip_stream);

/* One APD problem (Algorithm 2's inputs D, Omega, N, X, Lambda, J, V).
 * x, A, v, mass are DEVICE pointers, row-major:
 *   x [n][dim]          seed points (Section 2.1)
 *   A [n][dim][dim]     anisotropy matrices, symmetric positive definite
 *                       (Section 2.1); only the upper triangle is read
 *   v [n]               target volumes, v_i > 0, sum v = the domain measure
 *                       (|Omega|, or sum_j |P_j| with pixel weights)
 *                       (Section 2.1); may be NULL for apd_assign
 *   mass [J] or NULL    pixel weights q_j in [0, 255]: pixel j has measure
 *                       |P_j| = (q_j / 255) |P| in the objective, the
 *                       volumes and the centroids (the general-tessellation
 *                       form of Section 2.3 on the regular grid): a mask of
 *                       a non-rectangular domain (0 outside), with partial
 *                       weights on boundary pixels.  NULL: every pixel full.
 *                       Labels do not depend on it.  Limit:
 *                       255 J (2 max_d M_d)^2 < 2^64.                      */
typedef struct {
    int32_t dim;        /* 2 or 3 */
    int32_t power;      /* cost C_ij = |y_j - x_i|_{A_i}^power - w_i: 0 or 2 the
                           anisotropic power diagram (every tier); 1, 3 or 4
                           the other costs the paper's discussion (Section 4)
                           names, evaluated in APD_FP64 only (other tiers and
                           the batched and warm-start calls give INVALID_ARG);
                           the norm is computed from the squared norm q,
                           clamped at 0, as sqrt(q), q sqrt(q) or q q */
    int64_t n;          /* number of seeds N >= 1 */
    int32_t grid[3];    /* pixels per axis M_d >= 1 (entries >= dim ignored) */
    int32_t reserved1;
    double lo[3];       /* box Omega = [lo, hi] (Section 2.1), lo_d < hi_d */
    double hi[3];
    const double *x;
    const double *A;
    const double *v;
    const uint8_t *mass;
} apd_problem;

/* Algorithm 1 (pixel method): labels[j] = argmin_i C_ij for every pixel j,
 * with C_ij = |y_j - x_i|^2_{A_i} - w_i (eq. (2.1) at pixel centres).
 *   w        [n]  device, weights
 *   labels   [J]  device int32 output, J = prod(grid)
 *   rel_gap  [J]  device float output or NULL: a lower bound of pixel j's
 *                 relative top-two gap (C_(2) - C_(1)) / C_(2), the costs
 *                 taken in the gauge w - max_i w_i where all are >= 0 (the
 *                 set-valued argmin of Algorithm 1 has one element when it is
 *                 > 0).  Pixels the pass re-evaluated in double get the
 *                 exact gap of the double costs, rounded down (its
 *                 runner-up over the tile's candidate list, or, when lower,
 *                 the bound under which no seed outside the list costs);
 *                 the others a bound from the single-precision costs and
 *                 their rounding bounds (with candidate lists, where the
 *                 runner-up was left out of the pixel's list, from the
 *                 list's U: a weaker bound).  1 for a single seed, 0 when
 *                 the two smallest costs tie.
 * Errors: INVALID_ARG, NOT_SPD, NONFINITE, DEVICE, OOM. */
apd_status apd_assign(apd_ctx *ctx, const apd_problem *prob, const double *w,
                      int32_t *labels, float *rel_gap, apd_precision prec);

/* One evaluation of the discretised dual problem at w (Section 2.3):
 *   *g        host   g~(w) of eq. (2.7)
 *   grad [n]  device v_i - m_i |P|, eq. (2.8), m_i = pixels in cell i
 *             (with pixel weights: v_i - sum over the cell of |P_j|)
 *   counts[n] device int64 m_i (with pixel weights: sum of q_j over the
 *             cell, in units of |P|/255) (may be NULL)
 *   centroids [n][dim] device: discrete centroid of cell i (Algorithm 3),
 *             x_i for an empty cell (may be NULL)
 *   *maxrel   host   max_i |v_i - m_i |P|| / v_i, the quantity Algorithm 2's
 *             stopping rule tests (may be NULL)
 * prob->v is required.  Errors: as apd_assign, plus VOLUMES. */
apd_status apd_dual_objective_grad(apd_ctx *ctx, const apd_problem *prob, const double *w,
                                   double *g, double *grad, int64_t *counts,
                                   double *centroids, double *maxrel, apd_precision prec);

/* apd_dual_objective_grad for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same evaluation and outputs, with every scratch buffer of
 * the pass (scalars, block partials, moments, eigenvalue ranges, re-check
 * queue, candidate lists) in one static device array of 96 MiB that each
 * device holds from the library's load until the process ends.  The call
 * allocates nothing; ctx must exist (apd_create allocates its own small
 * buffers, among them the pinned copy of the scalars this call reads back).
 * It clears what must start at zero with a kernel and synchronises the
 * ctx's stream before returning.  Problems whose buffers do not fit --
 * about (100 n + 4 J) bytes plus, with candidate lists, 1 KiB per tile of
 * 1024 pixels and 2 KiB per super-tile: up to about 2 * 10^7 pixels at
 * n = 10^4 -- are rejected with APD_ERR_OOM and a message giving the size
 * needed.  Candidate lists keep at most 256 seeds per tile and 512 per
 * super-tile (longer lists fall back to every seed, as with the regular
 * call).  Every call on a device shares that device's array: calls that
 * overlap in time on one device (other threads, other streams) race and
 * must be serialised by the caller.
 * Errors: as apd_dual_objective_grad, plus OOM for problems too large. */
apd_status apd_dual_objective_grad_noalloc(apd_ctx *ctx, const apd_problem *prob, const double *w,
                                           double *g, double *grad, int64_t *counts,
                                           double *centroids, double *maxrel, apd_precision prec);

typedef struct {
    double eps;         /* relative volume tolerance (eq. (2.5)); 0.01 = 1 %    */
    int32_t max_iter;   /* accepted L-BFGS steps                                */
    int32_t max_evals;  /* objective evaluations (passes)                       */
    int32_t history;    /* stored curvature pairs (10)                          */
    int32_t warm;       /* 0: start from W_0 = 0 (Algorithm 2); 1: from w_inout */
    apd_precision prec; /* tier of every pass                                   */
    int32_t refine;     /* apd_fit_weights only: if the tolerance is not reached,
                           refine the grid and restart from the weights reached,
                           at most this many times (0: never; the last step of
                           Algorithm 2).  Every axis is scaled by
                           max(3/2, (|P| 2^D / (eps min v))^(1/D)), rounded up,
                           which also meets the pixel size of eq. (2.10).
                           Not applied to problems with pixel weights.          */
    double gamma0;      /* first-step scale; <= 0 picks 0.3 (2D), 0.2 N^(1/3) (3D) */
    double coarse_eps;  /* apd_fit_weights only: > 0 starts with a coarse-to-fine
                           step: Algorithm 2 on the grid halved along every
                           axis (rounded up) to this looser tolerance, in at
                           most max_evals / 4 passes, whose weights (reached or
                           best) are W_0 of the fit on the problem's grid.
                           0: off (W_0 as opts->warm says).  Not applied to
                           problems with pixel weights.                     */
} apd_fit_opts;

typedef struct {
    int32_t converged;  /* 1 if max rel. error < eps at the returned w   */
    int32_t iters;      /* accepted steps                                */
    int32_t evals;      /* passes                                        */
    int32_t rechecked;  /* pixels re-evaluated in double in the last pass */
    double max_rel_err; /* at the returned w                             */
    double g;           /* g~ at the returned w                          */
    double seconds;     /* wall time of the call                         */
    int32_t grid[3];    /* grid of the last fit (differs from the problem's
                           after refinement)                              */
    int32_t refinements;/* grid refinements made                          */
    int32_t coarse_evals;/* passes of the coarse-to-fine start (included in
                           evals; 0 without one)                          */
} apd_fit_report;

/* Algorithm 2: maximise g~ of eq. (2.7) over w by L-BFGS until
 * |v_i - m_i |P|| < eps v_i for all i.  w_inout [n] device: the start
 * (if opts->warm) and the result.  The solver minimises -g~ with the
 * two-loop recursion, Armijo backtracking from the unit step, gradients
 * projected on sum = 0, and a restart from the scaled steepest step when a
 * search fails.
 * With opts->refine > 0 a fit that cannot reach eps restarts on a refined
 * grid (report->grid, report->refinements).  With opts->coarse_eps > 0 the
 * fit starts from the weights of a fit on the grid halved along every axis
 * (report->coarse_evals): its passes cost a fraction of the fine ones and
 * leave the fine fit a short way to go (a start of Algorithm 2 on a coarser
 * discretisation, in the spirit of the adaptable pixel sizes of Section 4;
 * the stopping rule is still checked on the problem's grid).  After its first, eager
 * evaluation a fit replays the evaluation as a captured HIP graph (unless
 * per-pass profiling is on).
 * Errors: NOT_CONVERGED (w_inout = best iterate, report filled; the message
 * suggests the resolution of eq. (2.10), the paper's "increase J and
 * restart"), LINESEARCH, and those of apd_dual_objective_grad. */
apd_status apd_fit_weights(apd_ctx *ctx, const apd_problem *prob, double *w_inout,
                           const apd_fit_opts *opts, apd_fit_report *report);

/* One pass of the loop of Algorithm 3 (generalised Lloyd): fit w warm from
 * w_inout, then move every seed to the discrete centroid of its cell (an
 * empty cell keeps its seed).  The seeds are read from and written to
 * x_inout [n][dim] (device); prob->x is ignored.  w_inout [n] device. */
apd_status apd_lloyd_step(apd_ctx *ctx, const apd_problem *prob, double *x_inout,
                          double *w_inout, const apd_fit_opts *opts, apd_fit_report *report);

/* Algorithm 2 for B independent problems at once (all of one dim, any n
 * and grid each).  probs: host array [B]; w_inout: host array of B device
 * pointers, each [probs[b].n] (start if opts->warm, result); reports: host
 * array [B] or NULL.  The whole batch advances one evaluation per instance
 * per step (a captured HIP graph of a persistent multi-instance pass and a
 * device L-BFGS with the specification of apd_fit_weights); converged
 * instances drop out.  opts->prec must be APD_FP32 or APD_BF16 (its
 * kernel: apd_set_batch_kernel, apd_autotune_batched); the problems take no
 * pixel weights (INVALID_ARG) and opts->refine is ignored.
 * Errors: as apd_fit_weights (per instance; NOT_CONVERGED if any instance
 * did not converge, the others are still returned). */
apd_status apd_fit_weights_batched(apd_ctx *ctx, const apd_problem *probs, int32_t B,
                                   double *const *w_inout, const apd_fit_opts *opts,
                                   apd_fit_report *reports);

/* ---- learned warm start (2D) ----------------------------------------
 * Algorithm 2 starts from W_0 = 0; these calls predict a better W_0 with a
 * small per-seed network and fit from there, the cold start staying the
 * fallback.  Features of seed i (20 floats): x_i, the upper triangle of
 * A_i, N v_i, and the mean over its 16 nearest seeds of sqrt(N)(x_j - x_i),
 * the upper triangle of A_j, N v_j, N|x_j - x_i|^2_{A_i}, N|x_j - x_i|^2_{A_j},
 * then the distance of x_i to the box boundary along each axis times
 * sqrt(N / |Omega|), the volume deficit d_i = N (v_i - |C_i|) of the cells
 * at W = 0 (eq. (2.8) at zero weights: one assignment pass), and the 1-, 2-
 * and 3-fold repeated means of d over the 16 nearest seeds.  Network
 * 20 -> 128 -> 128 -> 128 -> 1 with ReLU; the parameters are one flat float
 * vector (per layer W[in][out] row-major, then b), 35 841 numbers.  Targets
 * t_i = N (w*_i - mean w*); prediction w_i = (y_i - mean y) / N. */
typedef struct apd_ws_model apd_ws_model;

/* Create a network on ctx's device from host parameters params[n_params]
 * (n_params must be 35 841).  Adam moments start at zero. */
apd_status apd_ws_create(apd_ctx *ctx, apd_ws_model **out, const float *params, int64_t n_params);
void apd_ws_destroy(apd_ws_model *model);
/* Copy the parameters to host params[n_params]. */
apd_status apd_ws_get_params(apd_ctx *ctx, const apd_ws_model *model, float *params, int64_t n_params);
/* Features of prob (dim 2) into F [n][20] (device); runs one FP32-tier
 * pass at W = 0 on prob's grid (errors as apd_dual_objective_grad). */
apd_status apd_ws_features(apd_ctx *ctx, const apd_problem *prob, float *F);
/* Training targets t_i = N (w_i - mean w) (float, device) of solver weights
 * w [n] (device). */
apd_status apd_ws_targets(apd_ctx *ctx, int64_t n, const double *w, float *t);
/* Network output y [S] (device) for features F [S][20] (device), in FP32
 * (the training path). */
apd_status apd_ws_forward(apd_ctx *ctx, apd_ws_model *model, const float *F, int64_t S, float *y);
/* The same output computed for inference: BF16 operands on the matrix cores
 * (weights and activations rounded to BF16 per layer), FP32 accumulation,
 * bias and ReLU in FP32.  apd_ws_predict uses this path. */
apd_status apd_ws_infer(apd_ctx *ctx, apd_ws_model *model, const float *F, int64_t S, float *y);
/* Mean squared error against t [S] (device) into *loss (host, may be NULL)
 * and its gradient with respect to the parameters into grad [35 841]
 * (device, may be NULL); the parameters are not changed. */
apd_status apd_ws_loss_grad(apd_ctx *ctx, apd_ws_model *model, const float *F, const float *t,
                            int64_t S, double *loss, float *grad);
/* One Adam step (beta 0.9 / 0.999, eps 1e-8) on the minibatch (F, t). */
apd_status apd_ws_train_step(apd_ctx *ctx, apd_ws_model *model, const float *F, const float *t,
                             int64_t S, float lr, double *loss);
/* One epoch over the S samples (F [S][20], t [S], device) in storage order:
 * an Adam step (as apd_ws_train_step, rate lr) per minibatch of 4096
 * consecutive samples, the last one shorter when 4096 does not divide S
 * (shuffle between epochs by permuting F and t).  *loss (host, may be NULL)
 * = the sample-weighted mean of the minibatch losses, each taken before its
 * step. */
apd_status apd_ws_train_epoch(apd_ctx *ctx, apd_ws_model *model, const float *F, const float *t,
                              int64_t S, float lr, double *loss);
/* Predicted weights w_out [n] (device) of prob (dim 2): features (one pass at
 * W = 0), BF16 inference, w = (y - mean y) / N. */
apd_status apd_ws_predict(apd_ctx *ctx, apd_ws_model *model, const apd_problem *prob, double *w_out);
/* Predict, then Algorithm 2 warm from the prediction; if that does not
 * converge within opts' budget, Algorithm 2 again from W_0 = 0.
 * *used_warm = 1 if the warm fit was kept; report->evals counts the
 * feature pass at W = 0. */
apd_status apd_fit_weights_ws(apd_ctx *ctx, apd_ws_model *model, const apd_problem *prob,
                              double *w_out, const apd_fit_opts *opts, apd_fit_report *report,
                              int32_t *used_warm);

/* eq. (2.10): *M = the smallest integer with |Omega| / M^dim <
 * (eps / 2^dim) vmin.  A tie within a relative 1e-12 counts as equality
 * (so eps = 0.01, vmin = 1e-4, dim = 2 gives 2001).  Host only. */
apd_status apd_choose_resolution(int32_t dim, double eps, double vmin, double omega,
                                 int32_t *M);

/* Assignment kernels, as apd_pass_stats and apd_autotune_batched name
 * them. */
typedef enum {
    APD_KERNEL_FP32_MATRIX = 0,  /* FP32 matrix cores over every seed          */
    APD_KERNEL_FP32_VECTOR = 1,  /* FP32 vector ALU over every seed            */
    APD_KERNEL_FP32_LISTS = 2,   /* FP32 vector ALU over tile candidate lists  */
    APD_KERNEL_BF16_MATRIX = 3,  /* bf16 matrix cores over every seed          */
    APD_KERNEL_BF16_LISTS = 4,   /* bf16 matrix cores over candidate lists     */
    APD_KERNEL_FP64 = 5,         /* the FP64 tier                              */
    APD_KERNEL_FP32_HYBRID = 6   /* FP32 over every seed: matrix cores form each
                                    position's quadratic in u0, the vector ALU
                                    evaluates it (apd_set_variant 2 or 3)      */
} apd_kernel;

/* Statistics of the last pass (or batched fit) on ctx.  The kernel times
 * are HIP-event times on the ctx stream, filled only while profiling is on
 * (zero after a batched fit). */
typedef struct {
    int64_t pixels;      /* J (0 after a batched fit) */
    int64_t pairs;       /* N J (0 after a batched fit) */
    int64_t rechecked;   /* pixels re-evaluated in double */
    double assign_ms;    /* the O(NJ) assignment kernel */
    double pass_ms;      /* the whole pass: prep .. finalize */
    int64_t tiles_credited; /* tiles credited whole (apd_set_adaptive) */
    int32_t kernel;      /* apd_kernel that ran */
    int32_t pixels_per_lane; /* its pixels (bf16: pixel rows) per lane along
                                axis 0; 0 for the matrix-core FP32 kernel
                                and FP64 */
} apd_pass_stats;
apd_status apd_last_pass_stats(const apd_ctx *ctx, apd_pass_stats *out);

/* Turn HIP-event timing of every pass on (1) or off (0).  With it off,
 * apd_fit_weights evaluates its first point eagerly and then replays that
 * evaluation as a captured HIP graph (same kernels, same results); with it
 * on, every evaluation is enqueued eagerly so that each pass is timed. */
apd_status apd_set_profiling(apd_ctx *ctx, int32_t on);

/* Kernel of the APD_FP32 tier over every seed: 0 = matrix cores
 * (v_mfma_f32_32x32x2f32 forms every cost, the ALU keeps the argmin),
 * 1 = vector ALU, 3 = hybrid (the matrix cores form each position's
 * quadratic in u0 for 32 seeds at a time, the vector ALU evaluates it for
 * rows placed symmetrically about the tile anchor, 16 per position in 3D
 * tiles of 16 x 16 x 8, 8 in 2D tiles of 32 x 32), 2 = the default: the
 * hybrid kernel for problems of at least 1536 seeds on grids of at least
 * 128 hybrid tiles, the vector one otherwise (where the hybrid kernel's
 * per-wave winner search does not pay, or its tiles leave compute units
 * idle).  With candidate lists (apd_set_culling)
 * variants 1 and 2 run the listed vector kernel.  All give identical
 * labels. */
apd_status apd_set_variant(apd_ctx *ctx, int32_t variant);

/* Per-tile candidate lists for the vector APD_FP32 kernel and the APD_BF16
 * kernel, single passes and the batched solver (1 = on, the default; 0 =
 * every seed at every pixel).  A seed is skipped in a tile when a lower
 * bound of its cost over the tile (smallest eigenvalue of A_i times the
 * squared distance to the tile, minus w_i) exceeds the smallest upper bound
 * of any seed's cost there; the labels are unchanged. */
apd_status apd_set_culling(apd_ctx *ctx, int32_t on);

/* Boundary-aware refinement (1 = on, the default; 0 = off), with the
 * candidate lists: a tile whose list holds a single seed lies inside that
 * seed's cell, so its pixels are labelled at once and its moments added in
 * closed form; only tiles that meet a cell boundary are evaluated pixel by
 * pixel (the adaptive refinement the paper's discussion (Section 4)
 * proposes, here on the lists' tiles of 32 x 32 pixels (2D, 4 pixels per
 * lane) or 16 x 8 x 8 voxels (3D)).  Labels, counts, objective and gradient
 * are unchanged.  Not applied with pixel weights or when apd_assign is
 * asked for rel_gap. */
apd_status apd_set_adaptive(apd_ctx *ctx, int32_t on);

/* Tile shape of the vector APD_FP32 kernel: pixels per lane along axis 0
 * (4 or 8; in 2D a wave is 4 x 16 lanes and a tile 2 x 2 waves, 8 times
 * that many rows x 32 columns; in 3D a tile is 4 waves x that many rows x
 * 8 x 8).  0 (the default) picks 4 with candidate lists, and over every
 * seed 8 on grids of at least 2^21 pixels, else 4.  The single-instance
 * APD_BF16 kernel takes half of a set value as its rows per lane (default
 * 4 in 2D, 2 in 3D).  The labels do not depend on it. */
apd_status apd_set_pixels_per_lane(apd_ctx *ctx, int32_t p);

/* Kernel choice for a class of problems: times every exact kernel of the
 * tier (APD_FP32: vector with candidate lists at 4 and at 8 pixels per
 * lane, vector over every seed at 4 and at 8, matrix cores, hybrid) over
 * `reps` passes of prob at weights w (device) with HIP events, sets ctx to
 * the fastest and reports the mean pass times (ms) in the order above.  All
 * candidates return identical results. */
typedef struct {
    int32_t variant;          /* apd_set_variant value of the fastest */
    int32_t culling;          /* apd_set_culling value of the fastest */
    int32_t pixels_per_lane;  /* apd_set_pixels_per_lane value of the fastest */
    int32_t reserved;
    double pass_ms[6];
} apd_tune_result;
apd_status apd_autotune(apd_ctx *ctx, const apd_problem *prob, const double *w,
                        apd_precision prec, int32_t reps, apd_tune_result *res);

/* Kernel choice for apd_fit_weights_batched: runs the batched solve of
 * probs[B] (as apd_fit_weights_batched: one dim, squared norm, no pixel
 * weights) from W_0 = 0 for `evals` evaluations per instance with each
 * candidate assignment kernel of either single-precision tier, times its
 * graph replays with HIP events, sets ctx to the fastest and reports the
 * times (ms).  Candidates, in the order of fit_ms: FP32 vector with
 * candidate lists at 4 and at 8 pixels per lane, FP32 vector over every
 * seed (8), FP32 matrix cores, bf16 matrix cores with candidate lists, bf16
 * matrix cores over every seed.  Every candidate yields the same certified
 * labels, hence the same weights, so from then on apd_fit_weights_batched
 * runs the chosen kernel for either tier asked for (apd_set_batch_kernel
 * with kernel -1 returns to the rule by tier).  The trial weights live in
 * buffers of this call; the problems are not changed.  Errors: as
 * apd_fit_weights_batched, and INVALID_ARG for evals < 1. */
typedef struct {
    int32_t kernel;           /* apd_kernel of the fastest */
    int32_t pixels_per_lane;  /* its pixels (bf16: pixel rows) per lane */
    double fit_ms[6];         /* replay time of each candidate, in the order above */
} apd_tune_batched_result;
apd_status apd_autotune_batched(apd_ctx *ctx, const apd_problem *probs, int32_t B, int32_t evals,
                                apd_tune_batched_result *res);

/* Assignment kernel of apd_fit_weights_batched: kernel -1 (the default)
 * picks by the tier asked for (APD_BF16: bf16 with candidate lists, or over
 * every seed with culling off; APD_FP32: the apd_set_variant /
 * apd_set_culling / apd_set_pixels_per_lane choice, at 8 pixels per lane
 * unless 4 is set); APD_KERNEL_FP32_MATRIX .. APD_KERNEL_BF16_LISTS fix it,
 * with pixels_per_lane 4 or 8 for APD_KERNEL_FP32_LISTS (ignored for the
 * others).  INVALID_ARG for any other value. */
apd_status apd_set_batch_kernel(apd_ctx *ctx, int32_t kernel, int32_t pixels_per_lane);

/* Measurement support: the sustained issue rate of the vector ALU on
 * device `device`, the ceiling of the single-precision assignment kernels
 * (which are bound by it).  op 0 times fused multiply-adds (v_fma_f32), op 1
 * additions (v_add_f32): eight independent register chains per thread,
 * eight waves on every SIMD, one timed launch of about 5 ms on the device's
 * null stream.  *lane_ops_per_s receives instructions x 64 lanes / second.
 * Allocates and frees a small device buffer.
 * Errors: INVALID_ARG (bad op or NULL), DEVICE, OOM. */
apd_status apd_measure_valu_rate(int32_t device, int32_t op, double *lane_ops_per_s);

#ifdef __cplusplus
}
#endif

#endif /* APD_H */
