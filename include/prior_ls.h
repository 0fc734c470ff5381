/*
 * prior_ls.h -- C ABI of the MI355X (gfx950) Priori L+S reconstruction library.
 *
 * The library computes the iteration of Algorithm 1 of Zonoobi, Faghih Roohi and
 * Kassim, "Low-Rank and Sparse Matrix Decomposition with a-priori knowledge for
 * Dynamic 3D MRI reconstruction" (arXiv 1411.6206):
 *
 *   (0) X_0 = A^H(d), S_0 = 0                         (initialisation)
 *   (1) L = SVT(X - S, lambda_L)                      (singular-value soft threshold)
 *   (2) L: sigma <- sigma - lambda_p (sigma - sigma_prev)   (singular-value prior)
 *   (3) S = T^{-1} soft(T(X - L_prev), lambda_S (1 - w))    (support-aware shrink)
 *   (4) X = L + S - A^H(A(L + S) - d)                 (data consistency)
 *
 * where A is the undersampled multi-coil Cartesian Fourier operator of Section 2
 * (frame-by-frame k-space undersampling with a mask, coil sensitivities C_c), the
 * adjoint is written A^{-1} in the paper's Notations, the Casorati matrix has the
 * voxels of one volume as rows and the nt time frames as columns, T is an
 * orthonormal Haar wavelet (nonstandard pyramid over the spatial axes of size > 1,
 * J levels), and the a-priori support of T(S^(t-1)) enters as per-coefficient
 * weights w = q/255 (w = 1 on the support: the coefficient is not shrunk; w = 0:
 * plain L+S threshold).
 *
 * Memory.  Every array argument is DEVICE memory owned by the caller, except
 * `sigma_prev` (host or device memory, nt doubles, read during the call).  Complex
 * arrays are interleaved complex64 (float re, float im), C order, x fastest:
 *     images (L0, S0, L, S, X, M)   [nt][nz][ny][nx]
 *     k-space                       [nc][nt][nz][ny][nx]  (kz, ky, kx; unshifted, DC at 0)
 *     mask                          uint8 [nt][nz][ny], nonzero = that (kz, ky) phase-encode
 *                                   line is sampled for every kx (readout fully sampled)
 *     coil sensitivities            [nc][nz][ny][nx]; NULL means nc == 1 with unit coil
 *     prior weights                 uint8 [nt][nz][ny][nx] in canonical (Mallat) Haar
 *                                   coefficient layout, weight q/255; NULL means all zero
 * The DFT is unitary (1/sqrt(n) on each axis).  k-space entries off the mask are ignored.
 *
 * Streams and threads.  All device work is enqueued on the hipStream_t given to
 * prior_ls_create (NULL = the default stream).  solve/step return after that stream
 * has completed the requested work (they read the convergence statistics).  A handle
 * is used by one host thread at a time; distinct handles are independent.
 *
 * Errors.  Functions return 0 (PRIOR_LS_OK) or a negative status.  The handle keeps
 * a message for the last error (prior_ls_last_error).  Non-convergence is not an
 * error (stats.converged = 0).
 */
#ifndef PRIOR_LS_H
#define PRIOR_LS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PRIOR_LS_OK          0
#define PRIOR_LS_EINVAL     -1  /* NULL required pointer, host pointer where device memory is
                                   required, lambda < 0, lambda_p outside [0,1], struct_size
                                   mismatch, L0 without S0, n_iter < 0, step before solve */
#define PRIOR_LS_ESHAPE     -2  /* unsupported shape: see prior_ls_dims */
#define PRIOR_LS_ENOMEM     -3  /* device allocation failed or plan exceeds hbm_budget */
#define PRIOR_LS_EHIP       -4  /* HIP runtime error (no device, launch failure, ...) */
#define PRIOR_LS_ENONFINITE -5  /* NaN/Inf reached the iterate (stats.nonfinite = 1) */

#define PRIOR_LS_GRAM_FP64   0  /* Casorati Gram on FP64 MFMA from FP32 data: exact products,
                                   FP64 sums (default) */
#define PRIOR_LS_GRAM_FP32   1  /* Gram on FP32 MFMA, FP64 across blocks */
#define PRIOR_LS_GRAM_BF16X3 2  /* Gram on BF16 MFMA with hi+lo split (3 products), FP32
                                   accumulate, FP64 across blocks */

#define PRIOR_LS_T_HAAR      0  /* orthonormal Haar, J = wavelet_levels levels over space */
#define PRIOR_LS_T_TFFT      1  /* unitary DFT along the frames of every voxel (coefficient
                                   f of voxel v is its temporal frequency f); prior weights
                                   are then [nt (frequency)][nz][ny][nx] and wavelet_levels
                                   is not used */
#define PRIOR_LS_T_DB4       2  /* orthonormal four-tap Daubechies wavelet, periodic, J =
                                   wavelet_levels levels along every spatial axis of size > 1
                                   (standard decomposition); coefficients in canonical Mallat
                                   order along each axis, [a_J | d_J | ... | d_1] */

/* Frames per window at most.  Windows of 33..64 frames take the wide Gram (its tiles split
 * over the waves of a block), the 64-frame eigensolver (one LDS copy of the matrix) and the
 * 128 x 128 back-projection operand; the temporal transform takes at most 32. */
#define PRIOR_LS_MAX_NT 64

typedef struct prior_ls_handle prior_ls_handle;   /* opaque; owns all device state */

/* Problem geometry, fixed for the life of a handle.
 * Supported: ny in {16,24,32,48,64,96,128,192,256} with nz in {1,4,8,16,32} (nz = 1 is the
 * 2D case), or nz = 14 with ny in {16,32,64,128,256} (radix 7 along z);
 * nx in {16,24,32,48,64,96,128,192,256}, 1 <= nt <= 64 (<= 32 with the temporal transform),
 * 1 <= nc <= 64,
 * wavelet_levels J in [0,3] with, for the Haar and Daubechies transforms, every spatial axis
 * of size > 1 divisible by 2^J (J = 0 means T is the identity).  Anything else returns
 * PRIOR_LS_ESHAPE. */
typedef struct {
    size_t   struct_size;       /* = sizeof(prior_ls_dims) */
    int32_t  nx, ny, nz, nt, nc;
    int32_t  wavelet_levels;    /* J */
    int32_t  gram_mode;         /* PRIOR_LS_GRAM_* */
    int32_t  transform;         /* sparsifying transform T: PRIOR_LS_T_HAAR (0),
                                   PRIOR_LS_T_TFFT (1) or PRIOR_LS_T_DB4 (2) */
    uint64_t hbm_budget;        /* bytes of device memory the handle may own; 0 = unlimited */
} prior_ls_dims;

/* Per-solve settings (Algorithm 1 inputs lambda_L (= the paper's lambda_T), lambda_S, and
 * the step size lambda_p of step (2); stopping rule of Section 3). */
typedef struct {
    size_t  struct_size;        /* = sizeof(prior_ls_params) */
    double  lambda_L;           /* >= 0; relative to sigma_1 of the current X - S if
                                   lambda_L_relative != 0, else absolute */
    double  lambda_S;           /* >= 0, absolute, in transform-domain units */
    double  lambda_p;           /* in [0,1]; 0 switches step (2) off */
    double  tol;                /* stop when ||Y_k - Y_{k-1}|| / ||Y_{k-1}|| < tol, Y = L + S,
                                   tested at the end of every chunk of check_every
                                   iterations; 0 = run exactly max_iter iterations */
    int32_t lambda_L_relative;
    int32_t max_iter;           /* >= 0; 0 only loads the problem and forms X_0 */
    int32_t check_every;        /* >= 1; iterations per device chunk (one hipGraph) */
    int32_t use_graph;          /* nonzero: replay chunks as captured hipGraphs */
} prior_ls_params;

typedef struct {
    const void    *kspace;      /* complex64 [nc][nt][nz][ny][nx], required */
    const uint8_t *mask;        /* uint8 [nt][nz][ny], required */
    const void    *sens;        /* complex64 [nc][nz][ny][nx]; NULL only when nc == 1 */
    const uint8_t *prior_w;     /* uint8 [nt][nz][ny][nx] canonical Haar layout, or NULL */
    const double  *sigma_prev;  /* host or device memory, nt doubles (singular values of
                                   L^(t-1), any order), read during the call (it is sorted
                                   and padded on the host); required when lambda_p > 0, else
                                   ignored */
    const void    *L0, *S0;     /* complex64 [nt][nz][ny][nx] warm start: both or neither.
                                   Cold: L = X_0 = A^H d, S = 0.  Warm: L = L0, S = S0 and
                                   X_0 = Y - A^H(A Y - d) with Y = L0 + S0 */
} prior_ls_inputs;

/* Output buffers, complex64 [nt][nz][ny][nx] device memory; any may be NULL (skipped).
 * X = L + S (the reconstructed image), M = the data-consistent iterate X_it of step (4). */
typedef struct {
    void *L, *S, *X, *M;
} prior_ls_outputs;

typedef struct {
    size_t  struct_size;        /* = sizeof(prior_ls_stats), set by the caller */
    int32_t iters;              /* iterations run since the last solve (cumulative with step) */
    int32_t converged;          /* rel_change < tol at the last check */
    int32_t nonfinite;
    int32_t sigma_count;        /* = nt */
    int32_t eig_sweeps;         /* Jacobi sweeps of the last eigensolve (warm-started) */
    int32_t reserved;
    double  rel_change;         /* ||Y_k - Y_{k-1}|| / ||Y_{k-1}|| at the last iteration */
    double  resid_norm;         /* ||A(L_k + S_k) - d|| over the sampled entries (FP64) */
    double  nuclear_norm;       /* sum of the singular values of L_k */
    double  l1_weighted;        /* sum over coefficients of (1 - w) |T(S_k)| */
    double  objective;          /* 0.5 resid^2 + tau_L nuclear + lambda_S l1_weighted */
    double  tau_L;              /* singular-value threshold used at the last iteration */
    double  sigma[PRIOR_LS_MAX_NT];  /* singular values of X_{k-1} - S_{k-1}, descending */
    double  ms;                 /* wall time of the call, milliseconds */
} prior_ls_stats;

/* Create a handle for one problem geometry; allocates the device state on the current
 * HIP device.  On failure *out is set to NULL.  `stream` is a hipStream_t (NULL = default). */
int prior_ls_create(const prior_ls_dims *dims, void *stream, prior_ls_handle **out);

/* Load the problem (k-space, mask, sensitivities, prior weights, sigma_prev, optional warm
 * start), form X_0 (step (0)), then run up to params->max_iter iterations of Algorithm 1
 * (steps (1)-(4)).  Writes the requested outputs and, if stats != NULL, the statistics.
 * Inputs may be freed after the call returns. */
int prior_ls_solve(prior_ls_handle *h, const prior_ls_inputs *in, const prior_ls_params *params,
                   const prior_ls_outputs *out, prior_ls_stats *stats);

/* Continue the resident iteration for n_iter more iterations (same parameters as the last
 * solve; n_iter = 0 only writes outputs).  solve(K1) followed by step(K2) computes exactly
 * what solve(K1 + K2) computes. */
int prior_ls_step(prior_ls_handle *h, int32_t n_iter, const prior_ls_outputs *out,
                  prior_ls_stats *stats);

/* The priori L+S scheme over a time sequence (Section 3, Fig. 2), as a sliding window.
 * After prior_ls_solve (the first time instance: plain L+S, i.e. no prior_w and
 * lambda_p = 0) or a previous append, the handle holds the result of a window of nt frames.
 * prior_ls_append drops the window's oldest frame, takes the new frame as the newest, and
 * runs params->max_iter iterations of Algorithm 1 on the new window:
 *   - warm start: L and S shifted by one frame, the new frame starting from the previous
 *     newest frame, then one data-consistency step (step (0) of a warm start);
 *   - a-priori knowledge from the previous window's result: the support T^(t-1) of T(S)
 *     (the coefficients that survived the last shrinkage; shifted the same way, the new
 *     frame taking the previous newest frame's support) as weights w = 1, and the singular
 *     values of L as sigma_prev for step (2) (used when params->lambda_p > 0).
 * kspace_frame: device, complex64 [nc][nz][ny][nx] (entries off the mask are ignored);
 * mask_frame: device, uint8 [nz][ny].  Both may be freed when the call returns.  Outputs
 * and stats as for prior_ls_step; stats.iters counts this window's iterations.  The
 * compact k-space keeps one slot per frame and grows when a frame has more samples than
 * any frame of the window before it.
 * Errors: EINVAL (NULL or host pointers, no window loaded, bad params), ESHAPE (sampled
 * data beyond 2^31 entries), ENOMEM (growing the compact k-space failed), EHIP,
 * ENONFINITE. */
int prior_ls_append(prior_ls_handle *h, const void *kspace_frame, const uint8_t *mask_frame,
                    const prior_ls_params *params, const prior_ls_outputs *out,
                    prior_ls_stats *stats);

/* Launch shapes and schedule of the iteration, chosen by measurement (prior_ls_tune) or
 * set by the caller (for instance from a cache of earlier tunings).  Every choice computes
 * the same iteration; only the Gram split changes its summation order (results agree to
 * rounding; each choice is deterministic). */
typedef struct {
    size_t  struct_size;        /* = sizeof(prior_ls_tuning) */
    int32_t gram_blocks;        /* the Casorati Gram is split over about this many workgroups
                                   of voxels: 0 (default 512) or 64..2048 */
    int32_t bp_grid;            /* back-projection workgroups at most: 0 (default 2048) or
                                   64..65536 */
    int32_t sparse_fork;        /* 0: the sparse update runs beside the reduction / eigensolve
                                   / back-projection (forked after the Gram pass); 1: beside
                                   the whole chain (forked before the Gram pass); 2: on the
                                   main stream after the Gram pass, every kernel alone (the
                                   serial schedule, also used for per-kernel timing) */
    int32_t sparse_grid;        /* Haar sparse update: workgroups at most, each looping over
                                   tiles (fewer leave more bandwidth to the chain it runs
                                   beside): 0 (one per tile) or 64..65536 */
    double  ms_per_iteration;   /* prior_ls_tune: measured time per iteration of the choice */
} prior_ls_tuning;

/* Autotuner.  Loads the problem as prior_ls_solve does, then times params->check_every
 * iterations (replayed as a hipGraph chunk, after one untimed chunk) for candidate launch
 * shapes and schedules: the sparse fork point, the Gram split (256 ... 2048 blocks), the
 * back-projection grid (1024 ... 8192) and, with the Haar transform, the sparse-update grid
 * (256 ... 2048), one knob at a time starting from the current choice.  It reloads the
 * problem before each trial and at the end, so the handle is left exactly as
 * prior_ls_solve(max_iter = 0) leaves it, with the fastest choice applied; *best (may be
 * NULL) receives it.  Errors as for prior_ls_solve. */
int prior_ls_tune(prior_ls_handle *h, const prior_ls_inputs *in, const prior_ls_params *params,
                  prior_ls_tuning *best);

/* Apply a tuning (EINVAL when out of range) / read the one in use. */
int prior_ls_set_tuning(prior_ls_handle *h, const prior_ls_tuning *t);
int prior_ls_get_tuning(const prior_ls_handle *h, prior_ls_tuning *t);

/* Release every resource of the handle.  NULL is a no-op. */
void prior_ls_destroy(prior_ls_handle *h);

/* Static description of a status code. */
const char *prior_ls_strerror(int status);

/* Message of the last error on this handle ("" if none); NULL handle -> the last error of
 * a failed prior_ls_create or prior_ls_server_* call on this thread. */
const char *prior_ls_last_error(const prior_ls_handle *h);

/* Device bytes a handle of these dimensions allocates at create time (excluding the
 * compact k-space, which is sized at solve from the mask).  0 for invalid dims. */
uint64_t prior_ls_plan_bytes(const prior_ls_dims *dims);

/* Benchmark support.  Runs n_iter iterations as one chunk of prior_ls_step (statistics on
 * the last iteration only), but launches the kernels directly (no hipGraph) with a hipEvent
 * recorded before and after each one on the stream it runs on.  kernel_ms (host,
 * PRIOR_LS_NKERNELS doubles) receives, per kernel, the sum of its launch durations over the
 * n_iter iterations, in the order
 *   0 Gram, 1 Gram reduction, 2 eigensolve, 3 sparse update, 4 back-projection,
 *   5 data consistency, 6 statistics, 7 change of the iterate (stopping test).
 * kernel_launches (host, PRIOR_LS_NKERNELS ints, may be NULL) receives the launch counts
 * (1 for the last two). */
#define PRIOR_LS_NKERNELS 8
int prior_ls_step_timed(prior_ls_handle *h, int32_t n_iter, double *kernel_ms,
                        int32_t *kernel_launches, prior_ls_stats *stats);

/* ---- Step-level entry points.  They act on the problem loaded by the last solve and do
 * not change the resident iterate.  Arrays are complex64 device memory in image layout
 * [nt][nz][ny][nx]. ---- */

/* Step (4), data consistency: M = Y - A^H(A(Y) - d).  *resid_norm (host, may be NULL)
 * receives ||A(Y) - d||. */
int prior_ls_op_dc(prior_ls_handle *h, const void *Y, void *M, double *resid_norm);

/* Steps (1)-(2) on the Casorati matrix of C (voxels x frames): L = U diag(sigma_tilde) V^H
 * with the handle's lambda_L / lambda_p / sigma_prev.  sigma (host, nt doubles, may be
 * NULL) receives the singular values of C, descending. */
int prior_ls_op_svt(prior_ls_handle *h, const void *C, void *L, double *sigma);

/* Step (3): S = T^{-1} soft(T(Xm - Lp), lambda_S (1 - w)) with the handle's weights. */
int prior_ls_op_sparse(prior_ls_handle *h, const void *Xm, const void *Lp, void *S);

/* ---- Allocation-free steps (1)-(2), for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc). ----
 *
 * prior_ls_op_svt without a handle: L = U diag(sigma_tilde) V^H for the Casorati matrix of C
 * (n_vox voxels x nt frames), through the same kernels (Gram on MFMA in gram_mode, FP64
 * reduction and Jacobi eigensolve, back-projection L = C W).  Every intermediate (Gram
 * partials, reduced Gram, eigenvectors, W and its MFMA operand, the statistics record) lives
 * in one static device array of PRIOR_LS_NOALLOC_SCRATCH_BYTES per GPU, held until the
 * process ends; the call allocates nothing, does not synchronise and only enqueues work on
 * `stream` (a hipStream_t, NULL = the default stream).
 *   C, L        device complex64 [nt][n_vox] (each frame contiguous, e.g. the image layout
 *               [nt][nz][ny][nx] with n_vox = nx ny nz); L must not overlap C
 *   n_vox       a positive multiple of 64, n_vox * nt < 2^31
 *   nt          1 ... PRIOR_LS_NOALLOC_MAX_NT (larger sizes return ESHAPE: the scratch array
 *               is sized for 32 frames)
 *   lambda_L, lambda_L_relative, lambda_p   as prior_ls_params
 *   sigma_prev  device, nt doubles in descending order; required when lambda_p > 0
 *   sigma       device, nt doubles (may be NULL): the singular values of C, descending
 * Every call on one GPU shares that GPU's scratch array: calls that overlap in time on one
 * GPU (on different streams) race; calls on one stream are ordered.  Errors (EINVAL, ESHAPE,
 * EHIP: message in prior_ls_last_error(NULL) on this thread) are found before anything is
 * enqueued, except kernel-launch failures. */
#define PRIOR_LS_NOALLOC_MAX_NT 32
#define PRIOR_LS_NOALLOC_SCRATCH_BYTES 5313024
int prior_ls_svt_noalloc(const void *C, int64_t n_vox, int32_t nt, int32_t gram_mode,
                         double lambda_L, int32_t lambda_L_relative, double lambda_p,
                         const double *sigma_prev, void *L, double *sigma, void *stream);

/* ---- Batches: several problems advanced together (one launch per kernel of an iteration
 * for all of them), the amortised form of the iteration for problems too small to fill the
 * GPU alone. ----
 *
 * A batch groups `count` existing handles (1 ... 4096) that share the phase-encode plane
 * (ny, nz), transform, wavelet_levels (Haar), gram_mode, the Gram tile class (all nt <= 16,
 * all in 17..32 or all in 33..64; with the temporal transform one nt) and device; nx, nt and nc may
 * differ from problem to problem.  It does not own them: they stay usable on their own, and
 * must outlive the batch.  Each kernel of an iteration of Algorithm 1 is launched once with
 * the problems along the grid's z axis and the largest problem's grid along x; a problem's
 * workgroups read its own arrays, so its masks, coil maps, prior weights, parameters and
 * data are its own, and its workgroups beyond its own grid return at once.  The launch
 * shapes (Gram split, back-projection grid, sparse fork point) are those of the first
 * handle's tuning when the batch is created.  Every problem computes exactly what it
 * computes alone with that tuning: the same kernels in the same order on its data, and it
 * stops where it would alone (after params.max_iter iterations, or at convergence tested
 * after every check_every of its own iterations).  Stopped problems' workgroups return at
 * once.  Calls on a batch and on its handles must not overlap (one thread at a time).
 * Errors: EINVAL (NULL, count out of range, a handle twice, problems that cannot share the
 * kernel instances, mixed devices) with the message in prior_ls_last_error(NULL) on this
 * thread; ENOMEM, EHIP. */
typedef struct prior_ls_batch prior_ls_batch;
int prior_ls_batch_create(prior_ls_handle *const *handles, int32_t count, prior_ls_batch **out);

/* prior_ls_solve of every problem of the batch: in[i], params[i] (their own max_iter, tol,
 * check_every; use_graph of params[0] applies to all), out[i] (out may be NULL), stats[i]
 * (may be NULL; stats[i].ms is the wall time of the whole call).  Each handle's work is
 * ordered after its own stream, like prior_ls_solve.  Returns the first error; a problem
 * that reaches a non-finite iterate stops (stats[i].nonfinite) while the others go on. */
int prior_ls_batch_solve(prior_ls_batch *b, const prior_ls_inputs *in,
                         const prior_ls_params *params, const prior_ls_outputs *out,
                         prior_ls_stats *stats);

/* prior_ls_step of every problem (all loaded): n_iter more iterations under each problem's
 * own parameters of its last solve or append. */
int prior_ls_batch_step(prior_ls_batch *b, int32_t n_iter, const prior_ls_outputs *out,
                        prior_ls_stats *stats);

/* Message of the batch's last error ("" if none). */
const char *prior_ls_batch_last_error(const prior_ls_batch *b);

/* Release the batch (not its handles).  NULL is a no-op. */
void prior_ls_batch_destroy(prior_ls_batch *b);

/* ---- Serving: continuous batching of recursive reconstructions (the priori L+S scheme of
 * Section 3 / Fig. 2 applied to many sequences at once).
 *
 * A request is one sequence: its first window of nt frames is reconstructed by plain L+S
 * (prior_ls_solve with no prior weights and lambda_p = 0), then n_append frames are appended
 * one at a time (prior_ls_append).  Up to max_active sequences of one batch class (see
 * prior_ls_batch_create: the same plane, transform, Gram mode and tile class; nx, nt and nc
 * may differ) are in flight together as a group, each on its own handle: one dispatcher
 * thread starts every member's next window (load or shift) and then advances all members
 * with one batch (prior_ls_batch_*: one launch per kernel of an iteration for all of them),
 * each running its own window's iterations and stopping rule.  Requests join a running
 * group at window boundaries while the oldest pending request is of the group's class; a
 * request of another class waits until the group drains and then starts the next group,
 * which also gathers every request of its class already waiting (they overtake older
 * requests of other classes: they share that group's launches).  A request
 * is admitted when the device bytes it needs (prior_ls_plan_bytes plus the compact k-space
 * of its most sampled frame, in nt slots) fit in hbm_budget beside every resident handle.
 * Handles of finished sequences stay resident and are reused by later requests of the same
 * geometry; idle ones are destroyed, oldest first, when an admission needs their room.  A
 * new group starts with the oldest pending request that fits.  Results do not depend on
 * what else runs: a member of a group computes exactly what it computes alone.
 * Threads: submit, wait and info may be called from any thread. ---- */
typedef struct prior_ls_server prior_ls_server;

typedef struct {
    size_t   struct_size;       /* = sizeof(prior_ls_server_config) */
    uint64_t hbm_budget;        /* device bytes for resident sequence state; 0 = 90% of the
                                   free device memory at create */
    int32_t  max_active;        /* sequences of one geometry in flight at once (one batched
                                   group), 1..64.  Sequences are never driven independently on
                                   streams of their own: a run with four large ones in flight
                                   that way ended in a host segmentation fault whose cause was
                                   not found */
    int32_t  reserved;          /* must be 0 */
} prior_ls_server_config;

typedef struct {
    size_t            struct_size;    /* = sizeof(prior_ls_request) */
    prior_ls_dims     dims;           /* window geometry; dims.hbm_budget is ignored */
    prior_ls_params   first;          /* first window (lambda_p is taken as 0) */
    prior_ls_params   next;           /* every appended frame */
    int32_t           n_append;       /* >= 0 */
    int32_t           reserved;       /* must be 0 */
    const void       *kspace0;        /* device complex64 [nc][nt][nz][ny][nx] */
    const uint8_t    *mask0;          /* device uint8 [nt][nz][ny] */
    const void       *kspace_frames;  /* device complex64 [n_append][nc][nz][ny][nx] */
    const uint8_t    *mask_frames;    /* device uint8 [n_append][nz][ny] */
    const void       *sens;           /* device complex64 [nc][nz][ny][nx]; NULL iff nc == 1 */
    prior_ls_outputs  out;            /* the final window's outputs (device, NULL = skip) */
    prior_ls_stats   *stats;          /* host [n_append + 1] per-window statistics, or NULL */
    double           *latency_ms;     /* host [n_append + 1] per-window call latency, or NULL */
} prior_ls_request;

typedef struct {
    size_t   struct_size;       /* = sizeof(prior_ls_result), set by the caller */
    int32_t  status;            /* PRIOR_LS_OK or the error that ended the sequence */
    int32_t  reused_plan;       /* 1 when a resident handle of the same geometry was reused */
    double   queue_ms;          /* submit -> admission */
    double   run_ms;            /* admission -> last window done */
    double   total_ms;          /* submit -> last window done */
    uint64_t state_bytes;       /* device bytes held while running */
    char     message[160];      /* error message, "" on success */
} prior_ls_result;

typedef struct {
    size_t   struct_size;       /* = sizeof(prior_ls_server_stats), set by the caller */
    uint64_t budget, used, peak_used;   /* bytes: admission budget, resident now, peak */
    int64_t  submitted, completed, failed, reused, evicted;
    int32_t  queued, active, peak_active, resident_idle;
} prior_ls_server_stats;

/* Start the workers on the current HIP device.  EINVAL (bad config), EHIP (no device). */
int prior_ls_server_create(const prior_ls_server_config *cfg, prior_ls_server **out);

/* Queue a request; returns at once with a ticket, without calling the HIP runtime.  Every
 * array of the request must stay valid, and its contents ready (producing work complete),
 * until prior_ls_server_wait returns for the ticket.  Returns EINVAL (NULL required array,
 * struct sizes, n_append < 0) or ESHAPE (dims).  A request whose arrays are not device
 * memory ends with status EINVAL in its result, one whose state alone exceeds the budget
 * with ENOMEM. */
int prior_ls_server_submit(prior_ls_server *s, const prior_ls_request *req, int64_t *ticket);

/* Block until the request of `ticket` has finished, then fill *result and forget the ticket
 * (each ticket is waited for once).  EINVAL for an unknown ticket. */
int prior_ls_server_wait(prior_ls_server *s, int64_t ticket, prior_ls_result *result);

/* Counters of the server (a consistent snapshot). */
int prior_ls_server_info(prior_ls_server *s, prior_ls_server_stats *info);

/* Finish every queued request, then release the workers and resident handles. */
void prior_ls_server_destroy(prior_ls_server *s);

#ifdef __cplusplus
}
#endif
#endif /* PRIOR_LS_H */
