/*
 * tomo.h — C ABI of libtomo, a gfx950 (MI355X) implementation of the Toeplitz
 * MBIR hot path of "Fast Large-Scale Model-Based Iterative Tomography via
 * Exploiting Mathematical Structure, Hierarchical Optimization, Smart
 * Initialization, and Distributed GPU Computing" (arXiv 2603.28756).
 *
 * Problem (Sec. 2, Eq. 5): minimise over the image f
 *     F(f) = 1/2 || R f - g ||^2 + beta * Phi(f)
 * for parallel-beam projections g, with R f evaluated through its Fourier
 * form (Eqs. 3-4), R*R applied as a padded-FFT Toeplitz convolution with a
 * precomputed point-spread function (Sec. 2.1, Eqs. 7-11), an edge-preserving
 * qGGMRF prior Phi coupling each voxel to 8 (2D) or 26 (3D) neighbours
 * (Sec. 2 and Sec. 2.4), an accelerated gradient method with restart
 * (Sec. 2), a ramp-filtered back-projection start (Sec. 2.2) and a
 * coarse-to-fine grid hierarchy with Lanczos prolongation (Sec. 2.3).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Units are pixels; a detector bin is one pixel wide.  Pixel (m_y, m_x) of an
 * N x N slice has centre (m_x - N/2, m_y - N/2); detector bin j sits at
 * t_j = j - c (c = rotation-centre bin); the projection at angle theta
 * integrates along x cos(theta) + y sin(theta) = t.
 *
 * Device arrays are row-major, contiguous, float32, and at least 256-byte
 * aligned:
 *   image / volume   [n_slices][N][N]           (row = y, column = x)
 *   sinogram         [n_slices][n_angles][n_det]
 * The caller owns every device buffer, including the workspace (typically
 * allocated with PyTorch).  The library never allocates or frees device
 * memory.  Host arrays passed in are copied before the call returns.
 *
 * All work is enqueued on the plan's HIP stream and is asynchronous with
 * respect to the host unless stated otherwise.  A plan is not thread-safe;
 * distinct plans are independent.
 *
 * Errors are reported by status code only (no exceptions, no abort);
 * tomo_last_error() returns a per-plan message for the last failure.
 */
#ifndef TOMO_H
#define TOMO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TOMO_OK = 0,
  TOMO_ERR_INVALID_ARG = 1,        /* bad size, pointer, alignment or parameter       */
  TOMO_ERR_NO_DEVICE = 2,          /* no HIP device visible                           */
  TOMO_ERR_UNSUPPORTED_ARCH = 3,   /* current device is not gfx950                    */
  TOMO_ERR_NO_WORKSPACE = 4,       /* tomo_plan_set_workspace() not called            */
  TOMO_ERR_WORKSPACE_TOO_SMALL = 5,/* workspace smaller than tomo_plan_workspace_size */
  TOMO_ERR_NOT_READY = 6,          /* call order: PSF not precomputed yet             */
  TOMO_ERR_HIP = 7,                /* a HIP runtime call failed                       */
  TOMO_ERR_NONFINITE = 8,          /* NaN/Inf met in the input or the iteration       */
  TOMO_ERR_INTERNAL = 9
} tomo_status;

typedef struct tomo_plan_s* tomo_plan;

/* Initial estimate of the coarsest level (tomo_recon_opts_t.init). */
enum {
  TOMO_INIT_FBP = 0,   /* ramp-filtered back-projection, Sec. 2.2                    */
  TOMO_INIT_ZERO = 1,  /* constant zero image                                       */
  TOMO_INIT_USER = 2,  /* caller's image, read from x before iterating              */
  TOMO_INIT_LEARNED = 3 /* network start from the FBP image (tomo_nn.h), FBP fallback  */
};

/* Outcome of a learned start (tomo_recon_stats_t.learned_state). */
enum {
  TOMO_LEARNED_NOT_REQUESTED = 0, /* init was not TOMO_INIT_LEARNED                         */
  TOMO_LEARNED_TESTED = 1,        /* the objective test chose per slice (learned_slices)    */
  TOMO_LEARNED_OUT_OF_DOMAIN = 2  /* the plan's coarsest level is outside the network's
                                     training domain: the FBP start was used              */
};

struct tomo_unet_s;  /* the network of tomo_nn.h */

/* Geometry, discretisation and prior of one reconstruction problem.  All
 * fields are host values; the angle array is copied by tomo_plan_create(). */
typedef struct {
  int32_t n;              /* N: slice width in pixels, even, 16 <= N <= 2048               */
  int32_t n_slices;       /* number of slices along the rotation axis, >= 1               */
  int32_t n_angles;       /* projections per slice, >= 1                                  */
  int32_t n_det;          /* detector bins per projection, even, >= 4                     */
  const double* angles;   /* host [n_angles] radians; NULL -> theta_i = i*pi/n_angles      */
  double center;          /* rotation-centre bin c; NaN -> n_det/2                         */
  int32_t pad;            /* FFT size P of the Toeplitz product: 0 -> the smallest power of
                             two >= 2N; otherwise a power of two >= 2N (Sec. 2.1 asks for
                             >= 2N-1; every such P gives the same result)                 */
  int32_t n_levels;       /* grid levels of the hierarchy (Sec. 2.3), 1..6; level l has
                             N/2^(L-1-l) pixels and n_det/2^(L-1-l) bins; 0 -> 1          */
  int32_t kb_width;       /* Kaiser-Bessel gridding kernel width W in grid cells, 2..16;
                             0 -> 6                                                        */
  double kb_oversamp;     /* gridding oversampling sigma >= 1.25 (the grid is the next
                             power of two >= sigma*N); 0 -> 2                              */
  double kb_beta;         /* KB shape; 0 -> pi*sqrt((W/s)^2 (s-1/2)^2 - 0.8) with s the
                             effective oversampling (Beatty et al. 2005)                   */
  double beta;            /* prior weight beta >= 0                                        */
  double p, q;            /* qGGMRF exponents, 1 <= p <= q = 2                             */
  double sigma;           /* qGGMRF scale sigma > 0                                        */
  double T;               /* qGGMRF threshold T > 0                                        */
  int32_t neighbours;     /* 8 (in-plane) or 26 (3D)                                       */
  uint32_t flags;         /* TOMO_FLAG_* bits; other bits must be 0                        */
} tomo_geometry_t;

/* tomo_geometry_t.flags: run every iteration with direct launches instead of replaying
 * captured three-iteration HIP graphs (which tomo_reconstruct uses for levels with at
 * least 7 iterations, on an internal stream ordered after the plan's stream). */
#define TOMO_FLAG_NO_GRAPH 1u
/* tomo_geometry_t.flags: evaluate the qGGMRF gradient inside the inverse-row epilogue over a
 * neighbour tile (each pair evaluated from both of its voxels) instead of the default
 * separate z-marching kernel that evaluates each neighbour pair once.  Same results to
 * rounding; the default is faster on gfx950. */
#define TOMO_FLAG_FUSED_PRIOR 2u
/* tomo_geometry_t.flags: launch the separate prior kernel on an internal stream beside the
 * forward-row and column passes instead of in sequence on the plan's stream.  In sequence
 * the prior kernel of a FISTA step also writes y and its gradient minus b for the two row
 * passes; on its own stream it does not, and the row passes form y themselves.  Same
 * results to rounding; within about 1% of the sequential schedule at 64 x 512^2, and kernel
 * durations then overlap. */
#define TOMO_FLAG_CONCURRENT_PRIOR 4u

/* Options of tomo_reconstruct(). */
typedef struct {
  const int32_t* iters;   /* host [n_levels]: iterations per level, coarse -> fine, >= 0  */
  int32_t init;           /* TOMO_INIT_*                                                   */
  int32_t restart;        /* 1: gradient-mapping restart test on; 0: plain FISTA           */
  double L_override;      /* > 0: use this step constant on every level instead of the
                             computed one                                                  */
  double* objective_dev;  /* nullable device float64[sum(iters)]: F(y_k) per iteration,
                             the objective at the point where iteration k evaluates its
                             gradient (computing it costs extra prior work)                */
  int32_t* restart_dev;   /* nullable device int32[sum(iters)]: 1 where restart fired     */
  /* TOMO_INIT_LEARNED only (ignored otherwise): */
  struct tomo_unet_s* unet; /* network with parameters set (tomo_nn.h); its images must be
                             N_0 x N_0 (the coarsest level)                                */
  float unet_scale;       /* input scale of the network, > 0 (tomo_unet_forward)           */
  int32_t* init_choice_dev; /* nullable device int32[n_slices]: 1 where the network's start
                             was kept, 0 where the FBP start was                           */
} tomo_recon_opts_t;

/* Host-side summary filled by tomo_reconstruct() when non-NULL. */
typedef struct {
  double L[6];            /* step constant used on each level                               */
  double lambda_pow[6];   /* power-iteration estimate of the largest eigenvalue of R*R     */
  int32_t n_restarts;     /* restarts over all levels                                       */
  int32_t nonfinite_iter; /* first global iteration with a non-finite value, or -1          */
  int32_t learned_state;  /* TOMO_LEARNED_*                                                 */
  int32_t learned_slices; /* slices started from the network's image                        */
} tomo_recon_stats_t;

/* Validate `geom`, bind the plan to the current HIP device and to `hip_stream`
 * (a hipStream_t; NULL = the default stream), and size its workspace.
 * Sec. 2 (problem statement) and Sec. 2.3 (levels).  Nothing is enqueued.
 * Errors: INVALID_ARG (any field out of range, NULL geom/out), NO_DEVICE,
 * UNSUPPORTED_ARCH, HIP.  On error *out is set to NULL. */
tomo_status tomo_plan_create(const tomo_geometry_t* geom, void* hip_stream, tomo_plan* out);

/* Bytes of device workspace the plan needs (all levels, all buffers). */
tomo_status tomo_plan_workspace_size(tomo_plan plan, size_t* bytes);

/* Attach caller-owned device memory of `bytes` bytes (>= workspace size,
 * 256-byte aligned).  The plan keeps the pointer until destroyed or re-attached;
 * re-attaching invalidates precomputed data (call tomo_precompute_psf again).
 * Errors: INVALID_ARG (NULL, misaligned), WORKSPACE_TOO_SMALL. */
tomo_status tomo_plan_set_workspace(tomo_plan plan, void* dev, size_t bytes);

/* Precompute, once per geometry and for every level, the spectrum F K of the
 * point-spread function K = NUFFT1(1) (Sec. 2.1, Eqs. 8-9; the spreading of
 * the all-ones function onto the oversampled grid, the grid FFT, the crop and
 * deapodisation, and the padded FFT all run in float64), and the step constant
 * L = 1.01 * lambda_pow + 2 beta rho''(0), lambda_pow from 30 power iterations
 * of R*R from the all-ones image with float64 norms (Sec. 2, Eq. 6).
 * Asynchronous: the work runs on a stream of the plan's own (default priority) that
 * starts after everything already enqueued on the plan's stream, with scratch and
 * iterate buffers of its own, so that a following tomo_reconstruct's back-projections
 * (R* g and the FBP start) run beside it; every call that needs F K or L (the
 * iterations, tomo_apply_normal, tomo_gradient, tomo_autotune, batches) first orders its
 * stream after it.  Nothing waits for the host.  A non-finite or non-positive
 * lambda_pow is reported by the first call that reads L on the host (tomo_psf_info with
 * L_host or lambda_host, tomo_reconstruct with stats_host) as NONFINITE.
 * Errors: NO_WORKSPACE, HIP. */
tomo_status tomo_precompute_psf(tomo_plan plan);

/* out = R* g (ramp = 0) or the ramp-filtered back-projection
 * (pi/n_angles) R* h g (ramp = 1, Sec. 2.2, Eqs. 12-14) on the finest grid:
 * radial DFT of each projection, optional |omega| ramp, Kaiser-Bessel gridding
 * onto the oversampled grid (Eq. 4), inverse grid FFT, crop and deapodisation.
 * sino: device [n_slices][n_angles][n_det]; out: device [n_slices][N][N].
 * Errors: INVALID_ARG (NULL/misaligned), NO_WORKSPACE, HIP. */
tomo_status tomo_backproject(tomo_plan plan, const float* sino, float* out, int ramp);

/* out = R*R x = Res(F^-1(F K . F Pad x)) on the finest grid (Sec. 2.1, Eq. 9).
 * x, out: device [n_slices][N][N], distinct.
 * Errors: INVALID_ARG, NO_WORKSPACE, NOT_READY (PSF not precomputed), HIP. */
tomo_status tomo_apply_normal(tomo_plan plan, const float* x, float* out);

/* grad = R*R x - b + beta grad Phi(x) on the finest grid (Sec. 2.1, Eq. 11,
 * plus the prior term of Eq. 5).  b is normally R* g from tomo_backproject.
 * x, b, grad: device [n_slices][N][N]; grad must not alias x or b.
 * obj_dev: nullable device float64[1] receiving
 *   1/2 <x, R*R x> - <x, b> + beta Phi(x)
 * (Eq. 10 without its constant 1/2 <g, g>).
 * Errors: INVALID_ARG, NO_WORKSPACE, NOT_READY, HIP. */
tomo_status tomo_gradient(tomo_plan plan, const float* x, const float* b, float* grad,
                          double* obj_dev);

/* sino_out = R x (Sec. 2, Eq. 3: R f = F^-1 NUFFT2 f) on the finest grid, the direct forward
 * projection: the image is deapodised and embedded in the oversampled Kaiser-Bessel grid, the
 * grid is forward-FFT'd, interpolated at the polar samples k_il = (l / n_det)(cos, sin)(theta_i)
 * (the transpose of the back-projection's gridding), and each angle's radial spectrum is
 * inverse-transformed along the detector, keeping the real part.  R and tomo_backproject's R*
 * are adjoint up to float32 rounding.  Needs no PSF.
 * x: device [n_slices][N][N]; sino_out: device [n_slices][n_angles][n_det].
 * Errors: INVALID_ARG, NO_WORKSPACE, HIP. */
tomo_status tomo_forward_project(tomo_plan plan, const float* x, float* sino_out);

/* grad = R*(R x - g) + beta grad Phi(x) on the finest grid, evaluated directly with both
 * non-uniform transforms (Sec. 2, Eqs. 3-4 and 7) instead of the Toeplitz product of Sec. 2.1,
 * for comparison with tomo_gradient (which needs b = R* g and the PSF).
 * x, grad: device [n_slices][N][N] (grad must not alias x); sino: device
 * [n_slices][n_angles][n_det].  obj_dev: nullable device float64[1] receiving
 * 1/2 ||R x - g||^2 + beta Phi(x) (Eq. 5).
 * Errors: INVALID_ARG, NO_WORKSPACE, HIP. */
tomo_status tomo_gradient_direct(tomo_plan plan, const float* x, const float* sino, float* grad,
                                 double* obj_dev);

/* Full reconstruction of `sino` into `x` through the grid hierarchy: per level
 * (coarse to fine) the projections are subsampled (every s-th bin, divided by
 * s), b = R* g is formed, the start is FBP / zero / the caller's image / the
 * learned start on the coarsest level and the Lanczos-3 prolongation of the
 * previous level above it, and `iters[l]` accelerated gradient iterations with
 * optional restart are run (Sec. 2, Sec. 2.2, Sec. 2.3).  Computes the PSF
 * first if it is not ready.
 * Learned start (extension of the FBP start of Sec. 2.2): the network maps the
 * FBP image to a start; if the coarsest level lies outside the network's
 * training domain (tomo_unet_set_domain; a network without one is outside) the
 * FBP start is used.  Otherwise the float64 objective
 *   1/2 <x, R*R x> - <x, R* g> + beta Phi(x)
 * of both candidate starts is evaluated on the device and the FBP start is
 * kept where the network's is larger (or not finite): per slice with the
 * 8-neighbour prior (slices are then independent problems), for the whole
 * volume with the 26-neighbour prior.  The network runs on its own stream,
 * ordered after and before the plan's work by events.
 * sino: device [n_slices][n_angles][n_det].
 * x: device [n_slices][N][N] output; with TOMO_INIT_USER it is first read as
 *    the coarsest-level start image [n_slices][N_0][N_0] (contiguous).
 * stats_host: nullable; when given the call synchronises the plan's stream
 *    and fills it.  Without it, a non-finite iteration is not detected.
 * Errors: INVALID_ARG (also: TOMO_INIT_LEARNED without a network or with
 * unet_scale <= 0), NO_WORKSPACE, NOT_READY (network without parameters or
 * workspace), HIP, NONFINITE (only with stats_host). */
tomo_status tomo_reconstruct(tomo_plan plan, const float* sino, float* x,
                             const tomo_recon_opts_t* opts, tomo_recon_stats_t* stats_host);

/* The plan's geometry as validated at creation (n_slices, n, n_angles, n_det, ...; the
 * centre and KB shape as given), its HIP stream and device (each nullable).
 * Errors: INVALID_ARG (NULL plan). */
tomo_status tomo_plan_geometry(tomo_plan plan, tomo_geometry_t* geom, void** hip_stream,
                               int32_t* device);

/* Copy level `level`'s PSF spectrum F K (float32, unnormalised) into the
 * caller's device array [P_l][P_l/2 + 1] (row = vertical frequency v,
 * column = horizontal frequency u = 0..P_l/2), and its step constants into
 * host doubles (each nullable; reading them waits for the precompute).
 * Errors: INVALID_ARG, NOT_READY, HIP, NONFINITE (lambda_pow not finite and > 0). */
tomo_status tomo_psf_info(tomo_plan plan, int32_t level, float* fk_dev, double* L_host,
                          double* lambda_host);

/* Level geometry: N_l, n_det_l and P_l of level `level` (host out-params). */
tomo_status tomo_level_dims(tomo_plan plan, int32_t level, int32_t* n, int32_t* n_det,
                            int32_t* pad);

/* Plan-free utility: separable 2x Lanczos-3 prolongation of each slice
 * (Sec. 2.3, Eqs. 16-17, normalised by the tap sum), enqueued on hip_stream.
 * in: device [n_slices][n][n]; out: device [n_slices][2n][2n].
 * Errors: INVALID_ARG, HIP. */
tomo_status tomo_lanczos_prolong(const float* in, float* out, int32_t n, int32_t n_slices,
                                 void* hip_stream);

/* Kernel classes timed by tomo_timing_enable(). */
enum {
  TOMO_T_ROWS_FWD = 0,     /* Toeplitz pass R: row FFTs of the padded iterate            */
  TOMO_T_COLS_CONV = 1,    /* pass C: column FFT, PSF-spectrum multiply, inverse FFT     */
  TOMO_T_ROWS_INV = 2,     /* pass R': inverse row FFTs, crop, prior, update epilogue    */
  TOMO_T_FINALIZE = 3,     /* float64 reduction and momentum/restart update              */
  TOMO_T_BACKPROJECT = 4,  /* one whole back-projection / FBP                            */
  TOMO_T_PSF = 5,          /* one whole PSF spectrum + step-constant precompute          */
  TOMO_T_PRIOR = 6,        /* qGGMRF gradient kernel (pair-shared, z-marching)           */
  TOMO_T_COUNT = 7
};

/* Diagnostics: record a pair of HIP events on the plan's stream around every
 * launch of the kernel classes set in `class_mask` (bit i = class i; 0 turns
 * timing off) and reset the accumulators.  Event recording adds a few
 * microseconds of stream overhead per timed launch and nothing else.
 * Errors: INVALID_ARG, HIP. */
tomo_status tomo_timing_enable(tomo_plan plan, uint32_t class_mask);

/* Synchronise the plan's stream and return, per class, the summed event time
 * in milliseconds (host float64[TOMO_T_COUNT]) and the number of timed launches
 * (host int64[TOMO_T_COUNT]); either pointer may be NULL.  Accumulators keep
 * running.  Errors: INVALID_ARG, HIP. */
tomo_status tomo_timing_read(tomo_plan plan, double* total_ms, int64_t* counts);

/* ---- tile autotuner ------------------------------------------------------------------- */
/* Tile schedule of the three Toeplitz passes of one level (Sec. 2.1, Eq. 9: the padded 2D
 * FFT product is carried out as row transforms, column transforms with the PSF-spectrum
 * multiply, and inverse row transforms).  Each pass has variants 0, 1 (default), 2 that
 * halve, keep or double the row pairs (passes R, R') or columns (pass C) one workgroup
 * transforms, within 1024 threads and 128 KiB of LDS; FFT sizes below 256 have the default
 * only.  All variants give bit-identical transforms. */
typedef struct {
  int32_t rows_fwd;       /* variant 0..2 of pass R                                        */
  int32_t cols_conv;      /* variant 0..2 of pass C                                        */
  int32_t rows_inv;       /* variant 0..2 of pass R' (separate-prior path only; the fused
                             and power-iteration forms use the default)                    */
  int32_t fwd_pairs;      /* out: row pairs per workgroup of pass R                        */
  int32_t col_tile;       /* out: columns per workgroup of pass C                          */
  int32_t inv_pairs;      /* out: row pairs per workgroup of pass R'                       */
  float ms[3][3];         /* out (tomo_autotune): mean launch time [pass R, C, R'][variant]
                             in milliseconds on the plan's full volume                     */
  int32_t chunks;         /* slices are split into this many chunks (1, 2, 4; 0 -> 1) that
                             passes R, C, R' run through one after the other, reusing one
                             chunk's half-spectrum buffers (which then stay in the Infinity
                             Cache); not with the fused or concurrent prior                 */
  float ms_chunks[3];     /* out (tomo_autotune): time of the prior kernel and the three
                             passes with 1, 2, 4 chunks (0 where not tried)                 */
} tomo_tiles_t;

/* Time every variant of the three passes on each level at the plan's own shapes (reps
 * launches each, after one warm-up; reps <= 0 means 5) and keep the fastest per pass and
 * level (a variant replaces the default only when at least 3% faster); then, with those tiles,
 * time a whole step (prior kernel and the three passes) with 1, 2 and 4 slice chunks and keep
 * the fastest by the same rule.  Synchronises the plan's stream; overwrites the iterate and spectrum scratch of the
 * workspace (not b, the PSF spectrum or the step constants), so call it before
 * tomo_reconstruct or between reconstructions.  Captured iteration graphs are rebuilt on the
 * next reconstruction.  chosen: nullable host [n_levels], receives the choice and timings.
 * Errors: INVALID_ARG, NO_WORKSPACE, HIP. */
tomo_status tomo_autotune(tomo_plan plan, int32_t reps, tomo_tiles_t* chosen);

/* Set (tiles != NULL: host [n_levels], only the three variant fields and chunks are read)
 * and/or read back (out != NULL: host [n_levels], variant, shape and chunk fields written, ms
 * zero) the tile schedule.  Errors: INVALID_ARG (variant outside 0..2, chunks not 0, 1, 2, 4). */
tomo_status tomo_tiles(tomo_plan plan, const tomo_tiles_t* tiles, tomo_tiles_t* out);

/* ---- batches of independent problems ------------------------------------------------- */
typedef struct tomo_batch_s* tomo_batch;

typedef struct {
  int32_t n_nonfinite;    /* problems with a non-finite iteration                          */
  int32_t n_restarts;     /* restarts summed over all problems                             */
  int32_t wait_timeouts;  /* 1 if a tile of the persistent kernel gave up waiting (results
                             invalid; reported as TOMO_ERR_INTERNAL)                        */
} tomo_batch_stats_t;

/* Group `n` single-level plans (each with its workspace attached, FFT size 256..2048, i.e.
 * 128 <= N <= 1024 at the default padding) into a batch advanced together: every iteration
 * of every problem runs in ONE persistent kernel launch that takes tiles from a phase-ordered
 * queue: the pair-shared prior (which also forms y and beta grad Phi(y) - b), then the three
 * Toeplitz passes, of all problems (Sec. 2.1 and the accelerated method of Sec. 2 applied to
 * each problem independently).  Problems keep their own geometry, prior, step constant, momentum
 * and restart state.  The plans must outlive the batch and must not be used concurrently
 * with it.  Errors: INVALID_ARG, NO_DEVICE, HIP. */
tomo_status tomo_batch_create(const tomo_plan* plans, int32_t n, void* hip_stream, tomo_batch* out);
tomo_status tomo_batch_workspace_size(tomo_batch batch, size_t* bytes);
/* Caller-owned device memory (>= tomo_batch_workspace_size, 256-byte aligned) for the
 * problem descriptors, the work queue and its counters. */
tomo_status tomo_batch_set_workspace(tomo_batch batch, void* dev, size_t bytes);
/* For every problem j: R* g_j and the FBP start from sinos[j] (device, that plan's sinogram
 * layout), the PSF spectrum if not ready, then `iters` iterations of all problems together
 * (captured three-iteration graphs replayed on the batch's internal stream), result into
 * xs[j] (device, [n_slices][N][N]).  sinos and xs are host arrays of n device pointers.
 * Synchronises the batch stream when stats is non-NULL.
 * Errors: INVALID_ARG, NO_WORKSPACE, HIP, NONFINITE / INTERNAL (with stats). */
tomo_status tomo_batch_reconstruct(tomo_batch batch, const float* const* sinos, float* const* xs,
                                   int32_t iters, int32_t restart, tomo_batch_stats_t* stats);
/* Transform schedule of a batch per FFT size P: each problem's passes R, C and R' use
 * `elems` elements per thread (radix-elems Stockham stages, P / elems threads per transform,
 * 256 / (P / elems) transforms per tile), 8 or 16 (default), and a queue item holds `group`
 * consecutive tiles.  Every schedule computes the same transforms (the radix decomposition
 * changes only their rounding). */
#define TOMO_BATCH_MAX_SIZES 8
typedef struct {
  int32_t n_sizes;                      /* distinct FFT sizes in the batch                      */
  int32_t pad[TOMO_BATCH_MAX_SIZES];    /* the sizes, increasing                                */
  int32_t elems[TOMO_BATCH_MAX_SIZES];  /* elements per thread of each size: 8 or 16            */
  int32_t group[TOMO_BATCH_MAX_SIZES];  /* tiles of passes R, C, R' per queue item, 1..64 (8)   */
  int32_t fused_prior;                  /* 0: the pair-shared prior phase (default); 1: problems
                                           with the 8-neighbour prior evaluate it inside pass R'
                                           (each pair from both voxels, no prior phase, fewer
                                           bytes moved); 26-neighbour problems keep the phase    */
  float iter_ms;                        /* out (autotune): one batched iteration, chosen schedule */
  float base_ms;                        /* out (autotune): the starting schedule above            */
  int32_t phase_launches;               /* 0: one persistent launch per iteration whose blocks take
                                           items from the phase-ordered queue and wait for the
                                           items they depend on (default); 1: one launch per phase
                                           and transform size, each block one tile (group is 1),
                                           and a per-problem finalize launch: launch boundaries
                                           order the phases                                      */
} tomo_batch_schedule_t;
/* Time batched iterations (reps launches after a warm-up; reps <= 0 means 5) with the prior
 * phase, the persistent launch, 16 elements per thread and 8 tiles per item everywhere, then
 * try the prior inside pass R' (when a problem has the 8-neighbour prior), one launch per
 * phase (then the prior scheme once more), and for the persistent launch 1, 2, 8, 16, 32 or
 * 64 tiles per item for all sizes and per FFT size half or twice that, then per size 8
 * elements per thread, keeping each change that makes the whole iteration at least 3% faster
 * (Sec. 2.1's padded FFTs, scheduled per size).
 * Computes missing PSF spectra; overwrites every problem's iterates, b and scalars (call it
 * before tomo_batch_reconstruct, which prepares them again).  Synchronises the batch stream.
 * out: nullable.  Errors: INVALID_ARG, NO_WORKSPACE, HIP, INTERNAL. */
tomo_status tomo_batch_autotune(tomo_batch batch, int32_t reps, tomo_batch_schedule_t* out);
/* Set (set != NULL: fused_prior, phase_launches and pad/elems/group triples, sizes not listed
 * keep their choice) and/or read back (out != NULL) the schedule.  Errors: INVALID_ARG (a size
 * not in the batch, elems not 8 or 16, group outside 1..64, fused_prior or phase_launches not
 * 0 or 1). */
tomo_status tomo_batch_schedule(tomo_batch batch, const tomo_batch_schedule_t* set,
                                tomo_batch_schedule_t* out);
tomo_status tomo_batch_destroy(tomo_batch batch);  /* NULL ok */

/* Destroy a plan (NULL is accepted).  Does not free the caller's workspace. */
tomo_status tomo_plan_destroy(tomo_plan plan);

/* Static description of a status code: any int is accepted (a tomo_status value, or
 * "unknown status" for other values). */
const char* tomo_status_string(int32_t status);

/* Message of the plan's last failure ("" if none; NULL plan -> last global error). */
const char* tomo_last_error(tomo_plan plan);

#ifdef __cplusplus
}
#endif

#endif /* TOMO_H */
