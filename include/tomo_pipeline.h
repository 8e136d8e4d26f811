/*
 * tomo_pipeline.h — streaming a volume that does not fit in device memory through one plan
 * (Sec. 2.4: within a node, three cooperating threads joined by bounded work queues move
 * input from host to device, run the reconstruction kernels, and move results back, so that
 * transfers overlap computation).
 *
 * The volume's sinogram and image stay in host memory.  They are cut along the rotation axis
 * into windows of the plan's n_slices slices: window k keeps the result of the interior
 * slices [k C, min((k + 1) C, n_total)), C = n_slices - 2 halo, and is solved with `halo`
 * extra slices of context on each side where the volume has them (the window is shifted
 * inward at the two ends of the volume, so every window has exactly n_slices slices).
 *
 * Each window is an independent call of tomo_reconstruct on its slices, with its own step
 * sizes, restart decisions and objective.  With the 8-neighbour prior the slices of a volume
 * do not interact through the prior; without the restart test (opts->restart = 0) the
 * iteration of every slice is then exactly the iteration of that slice in a whole-volume
 * solve, so the streamed volume equals the whole-volume reconstruction bit for bit.  With the
 * restart test the restart decisions are taken per window.  With the 26-neighbour prior the
 * slices interact: each window sees `halo` slices of context beyond its interior, and the
 * interior approaches the whole-volume solution as halo grows (a one-pass stream cannot
 * exchange halos every iteration as the distributed solver of Sec. 2.4 does).
 *
 * Threads and memory: the upload thread copies a window's sinogram into a pinned staging
 * buffer and on to one of `depth` device slots (its own stream); the compute thread runs
 * tomo_reconstruct on the plan's stream; the download thread copies the window's interior
 * back through a pinned staging buffer into the host image (its own stream).  A slot is
 * reused only after its download has finished, so at most `depth` windows are in flight.
 * Device memory comes from the caller (tomo_pipeline_set_workspace); the pinned host staging
 * buffers (2 x depth windows) are allocated by tomo_pipeline_create and freed by
 * tomo_pipeline_destroy.  Every stream has the default priority.
 */
#ifndef TOMO_PIPELINE_H
#define TOMO_PIPELINE_H

#include "tomo.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tomo_pipeline_s* tomo_pipeline;

/* Host-side summary of one tomo_pipeline_run. */
typedef struct {
  int32_t n_windows;        /* windows solved                                               */
  int32_t nonfinite_window; /* first window whose solve met a non-finite value, or -1       */
  int32_t n_restarts;       /* restarts summed over the windows                             */
  int32_t reserved;
  double wall_ms;           /* the whole call                                               */
  double upload_ms;         /* upload thread, start to last window queued: staging copies,
                               host-to-device transfers and waits for a free slot           */
  double compute_ms;        /* compute thread: tomo_reconstruct calls (and, with stats,
                               their completion)                                            */
  double download_ms;       /* download thread: device-to-host transfers and copies out     */
} tomo_pipeline_stats_t;

/* Window arithmetic (host only): window k of a volume of n_total slices solved n_slices at a
 * time with `halo` context slices on each side starts at slice *first and keeps slices
 * [*keep0, *keep1).  *n_windows (nullable) receives the number of windows.
 * Errors: INVALID_ARG (n_slices - 2 halo < 1, n_total < n_slices, k out of range, NULL). */
tomo_status tomo_pipeline_window(int32_t n_total, int32_t n_slices, int32_t halo, int32_t k,
                                 int32_t* first, int32_t* keep0, int32_t* keep1,
                                 int32_t* n_windows);

/* A pipeline that streams a volume of n_total slices through `plan` (its n_slices is the
 * window size) with `halo` context slices per side and `depth` (1..8) windows in flight.
 * The plan must have its workspace attached; it must not be used by other threads while
 * tomo_pipeline_run runs.  Errors: INVALID_ARG, HIP (pinned staging allocation). */
tomo_status tomo_pipeline_create(tomo_plan plan, int32_t n_total, int32_t halo, int32_t depth,
                                 tomo_pipeline* out);

/* Device bytes of the window slots: depth x (sinogram window + image window). */
tomo_status tomo_pipeline_workspace_size(tomo_pipeline pipe, size_t* bytes);

/* Attach caller-owned device memory (>= workspace size, 256-byte aligned).
 * Errors: INVALID_ARG, WORKSPACE_TOO_SMALL. */
tomo_status tomo_pipeline_set_workspace(tomo_pipeline pipe, void* dev, size_t bytes);

/* Reconstruct the whole volume: sino_host [n_total][n_angles][n_det] and x_host
 * [n_total][N][N] are host float32 arrays (pageable or pinned; the call reads and writes them
 * only through its staging buffers and returns when every window's result is in x_host).
 * opts as for tomo_reconstruct, except: init TOMO_INIT_USER, objective_dev, restart_dev and
 * init_choice_dev are not supported (INVALID_ARG).  With stats non-NULL each window's solve
 * is checked (tomo_reconstruct with stats), and the first window with a non-finite value
 * ends the run with NONFINITE after the windows already in flight have drained.
 * Errors: INVALID_ARG, NO_WORKSPACE, HIP, NONFINITE, and any error of tomo_reconstruct (the
 * message names the window). */
tomo_status tomo_pipeline_run(tomo_pipeline pipe, const float* sino_host, float* x_host,
                              const tomo_recon_opts_t* opts, tomo_pipeline_stats_t* stats);

/* Message of the pipeline's last failure. */
const char* tomo_pipeline_last_error(tomo_pipeline pipe);

tomo_status tomo_pipeline_destroy(tomo_pipeline pipe);  /* NULL ok */

#ifdef __cplusplus
}
#endif

#endif  /* TOMO_PIPELINE_H */
