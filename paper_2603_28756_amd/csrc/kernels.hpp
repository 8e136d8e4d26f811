// Internal launcher interface between the C-ABI layer (tomo_api.cpp) and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "common.hpp"

namespace tomo {

// Device scalar block (float64 slots) shared by the iteration kernels.
enum ScalarSlot {
  SC_MU = 0,         // momentum coefficient: y_k = x_k + mu (x_k - x_{k-1})
  SC_T = 1,          // FISTA t_k
  SC_INVL = 2,       // 1 / L
  SC_GG = 3,         // <g, g> of the current level's projections
  SC_PSCALE = 4,     // power iteration: scale applied to the stored iterate
  SC_LAMBDA = 5,     // power iteration: ||T v|| / ||v||
  SC_VNORM = 6,      // power iteration: ||v|| of the current (scaled) iterate
  SC_RESTART_ON = 7, // 1.0 when the restart test is enabled
  SC_ITER = 8,       // global iteration counter (history index)
  SC_NONFINITE = 9,  // first iteration with a non-finite reduction, -1 if none
  SC_NRESTART = 10,  // restart count
  SC_LASTOBJ = 11,   // last objective value
  SC_BETA = 12,      // prior weight (objective assembly)
  SC_GSUM = 13,      // generic reduction result
  SC_COUNT = 16
};

// MODE_FISTA_Y: a FISTA step whose extrapolated point y and prior term gp - b were written by
// the prior kernel (launch_prior with b and yout): pass R reads y (xk = y), pass R' reads
// x_k, y (in the x_{k-1} slot) and gp - b (in the gpv slot) and not b; <y, b> comes from the
// prior kernel's partial sums.
enum Mode { MODE_FISTA = 0, MODE_GRAD = 1, MODE_POWER = 2, MODE_FISTA_Y = 3 };

// Launch geometry of the hot-path kernels for a padded size P (used for partials sizing).
// v: tile variant 0, 1 (default), 2 of a transform pass.
int rows_inv_rows_per_block(int P, int v);
int cols_tile_width(int P);
// Resolved block shapes of the variants: row pairs of pass R, columns of pass C, row pairs
// of pass R' (0 for an unsupported P).
void tile_shapes(int P, int v_fwd, int v_cc, int v_inv, int* fwd, int* cc, int* inv);

// ---- hot path (float32 data, float64 reductions) --------------------------------------
// Pass R: y = x_k + mu (x_k - x_{k-1}) (or scale * x_k in power mode) -> row R2C -> S1.
// Power mode with pprev: scale = 1 / sqrt(sum of slot 0 of the nprev partial sums pprev[4 b])
// (the previous power step's pass R'), else scal[SC_PSCALE].
hipError_t launch_rows_fwd(int P, int v, int mode, const float* xk, const float* xkm1,
                           const double* scal, cpx<float>* S1, const cpx<float>* tw,
                           int N, int nz, hipStream_t st, const double* pprev = nullptr,
                           int nprev = 0);
// Pass C: column FFT, x FK, inverse column FFT, keep N rows: S1 -> S2.
hipError_t launch_cols_conv(int P, int v, const cpx<float>* S1, cpx<float>* S2, const float* fk,
                            const float* fkn, const cpx<float>* tw, int N, int nz, hipStream_t st);
// Pass R': inverse row C2R + crop + epilogue; writes partial sums [nblocks][4].
// gpv: prior gradient beta grad Phi(y) from launch_prior, or NULL to evaluate the prior
// inside the epilogue over a neighbour tile.
hipError_t launch_rows_inv(int P, int v, int mode, int neighbours, bool with_obj,
                           const cpx<float>* S2, const float* xk, const float* xkm1,
                           const float* b, const float* gpv, float* out, double* partials,
                           const double* scal, const cpx<float>* tw, int N, int nz,
                           const PriorParams& pp, int* nblocks_out, hipStream_t st);
// Prior gradient (and Phi partial sums [blocks][4], slot 0, when with_obj) over z-marching tiles.
int prior_blocks(int N, int nz);
// gp = beta grad Phi(y); with b and yout (both non-null, MODE_FISTA only) gp - b is written
// to gp and y to yout, and the partial sums carry <y, b> in slot 1 (with_obj).
hipError_t launch_prior(int mode, int neighbours, bool with_obj, const float* xk,
                        const float* xkm1, const double* scal, float* gp, const float* b,
                        float* yout, double* partials, int N, int nz, const PriorParams& pp,
                        hipStream_t st);
// Deterministic float64 reduction of the partials + scalar update.
hipError_t launch_finalize(int mode, const double* partials, int nblocks,
                           const double* prior_partials, int nprior, double* scal,
                           double* obj_hist, int32_t* restart_hist, double* obj_out,
                           hipStream_t st);

// ---- batched iteration over independent problems ------------------------------------------
// One problem of a batch; every pointer lives in that problem's own plan workspace.
struct BatchProb {
  int N, P, nz, neighbours;
  int nPr, nR, nC, nRp;     // tiles of the prior phase, pass R, pass C, pass R'
  int el;                   // elements per thread of the transforms (8 or 16)
  int fused;                // 1: the prior inside pass R' (8 neighbours, no prior phase)
  int grp;                  // tiles per queue item of passes R, C, R'
  int iR, iC, iRp;          // queue items of pass R, pass C, pass R'
  int pad0;
  float* x[3];              // rotating iterates
  float* y;                 // extrapolated point y (written by the prior phase)
  float* gp;                // beta grad Phi(y) - b (written by the prior phase)
  const float* b;
  const float* fk;
  const float* fkn;
  cpx<float>* S1;
  cpx<float>* S2;
  double* partials;         // [nRp][4]
  double* scal;             // scalar block (SC_*)
  const cpx<float>* tw;     // twiddles for P
  double* hist;             // nullable objective history (indexed by SC_ITER)
  int32_t* rhist;           // nullable restart flags
  PriorParams pp;
};
constexpr int kBatchThreads = 256;
// Tile counts of problem (N, P, nz) in the batched kernel with `el` elements per thread.
void batch_tile_counts(int N, int P, int nz, int el, int* nPr, int* nR, int* nC, int* nRp);
bool batch_supports(int P);
// Resident blocks of the persistent batch kernel per compute unit (`fused`: the instantiation
// that may evaluate the in-plane prior inside pass R').
int batch_blocks_per_cu(bool fused);
// items: int2 {prob | phase << 24, tile}, ordered by phase (prior, R, C, R'); ctl[0] = queue
// head, ctl[1] = finished blocks, ctl[2] = error flag; cnt[4][nprob] = finished tiles per phase.
hipError_t launch_batch_iteration(bool fused, const BatchProb* probs, const int2* items, int n_items,
                                  int* ctl, int* cnt, int nprob, int ik, int ikm1, int inext,
                                  int grid, hipStream_t st);
// The same iteration as one launch per (phase, transform size) segment of the work list
// (host int4[nseg]: phase, P | EL << 16, first item, item count; phases in order) and a per-problem
// finalize launch; no tile waits.
hipError_t launch_batch_phases(bool fused, const BatchProb* probs, const int2* items,
                               const int4* segs, int nseg, int nprob, int ik, int ikm1, int inext,
                               hipStream_t st);
hipError_t launch_fill_int(int* x, idx_t n, int v, hipStream_t st);

// ---- start selection (learned start with FBP fallback) -----------------------------------
// qGGMRF constants in float64 for the objective of a candidate start.
struct ObjParams {
  double beta;        // prior weight
  double p;           // exponent p
  double qmp;         // q - p
  double lw0;         // (q - p) log2(1 / (T sigma))
  double c_rho2;      // 1 / (p sigma^p (T sigma)^(2 - p))
  double w1, w2, w3;  // normalised neighbour weights: axis, face diagonal, body diagonal
  int neighbours;     // 8 or 26
  int quadratic;      // 1 when p == q
};
constexpr int kObjBlocks = 64;  // blocks per slice of the start objective
// part [nz][kObjBlocks]: per-block float64 sums of F(xb) - F(xa), F(x) = 1/2 x T x - x b +
// beta (forward-pair rho), from ts = T (xa + xb).
hipError_t launch_slice_objective_diff(const float* xa, const float* xb, const float* ts,
                                       const float* b, int N, int nz, const ObjParams& op,
                                       double* part, hipStream_t st);
// out[i] = a[i] + b[i], i < n
hipError_t launch_add(const float* a, const float* b, float* out, idx_t n, hipStream_t st);
// Per slice (per_slice = 1) or for the whole volume: keep xb where the objective difference
// F(xb) - F(xa) (partials pd) is finite and not positive, copying it over xa; choice[z] (and
// choice_user[z], nullable) receive 1 where xb was kept.
hipError_t launch_select_start(const double* pd, int nz, int per_slice, float* xa,
                               const float* xb, int N, int32_t* choice, int32_t* choice_user,
                               hipStream_t st);

// ---- direct (non-Toeplitz) forward projection ----------------------------------------------
// grid[z][cell], slices z0 .. z0+nzb-1: deapodised image embedded at offset -N/2 (mod M).
hipError_t launch_embed_deapod(const float* f, cpx<float>* grid, const float* inv, int N, int M,
                               int z0, int nzb, hipStream_t st);
// fhat[z][p] = KB interpolation of the forward-FFT'd grid at sample p (transpose of the gather).
hipError_t launch_interp(const cpx<float>* grid, const int2* g0, const float* wx, const float* wy,
                         cpx<float>* fhat, int npts, int M, int W, int z0, int nzb, hipStream_t st);
// out[row][j] = Re (1/nd) sum_l fhat[row][l] exp(+2 pi i l (j - c)/nd) (- sino[row][j] when given,
// then part[blocks] = partial sums of out^2).
int radial_idft_blocks(int nd, int rows);
hipError_t launch_radial_idft(const cpx<float>* fhat, const float* sino, float* out, double* part,
                              int nd, int rows, const cpx<float>* tab, const cpx<float>* post,
                              hipStream_t st);
hipError_t launch_add(float* a, const float* b, idx_t n, hipStream_t st);
// out[0] = 1/2 sum rpart + beta sum_k ppart[k][0]
hipError_t launch_direct_objective(const double* rpart, int nr, const double* ppart, int np,
                                   double beta, double* out, hipStream_t st);

// ---- tables and utilities ---------------------------------------------------------------
hipError_t launch_twiddles_f32(cpx<float>* tw, int P, hipStream_t st);
hipError_t launch_twiddles_f64(cpx<double>* tw, int P, hipStream_t st);
hipError_t launch_fill(float* x, idx_t n, float v, hipStream_t st);
hipError_t launch_set_scalars(double* scal, int first, int count, const double* vals_dev_or_null,
                              double v, hipStream_t st);
// out[0..2] = {lambda, a lambda + c, 1 / (a lambda + c)}, lambda = scal[SC_LAMBDA]
hipError_t launch_lipschitz(const double* scal, double a, double c, double* out, hipStream_t st);
hipError_t launch_sumsq_strided(const float* g, idx_t rows, int n_out, int stride, double scale,
                                double* partials, double* out, hipStream_t st);
hipError_t launch_lanczos_prolong(const float* in, float* out, int n, int nz, hipStream_t st);

// ---- back-projection and PSF (gridding) ---------------------------------------------------
struct GridGeom {
  int n;          // output image width N_l (back-projection) or 2 N_l (PSF region)
  int n_det;      // detector bins of the level
  int n_angles;
  int M;          // oversampled grid size
  int W;          // kernel width
  double beta;    // KB shape
  double c;       // rotation-centre bin of the level
  int stride;     // detector subsampling stride of the level (1 = finest)
};

hipError_t launch_radial_tables(cpx<float>* dft_tab, cpx<float>* post, float* rampf,
                                const GridGeom& gg, int ramp, hipStream_t st);
// Radial DFT by chirp-z: L = czt_length(n_det) (the smallest power of two >= max(256,
// 2 n_det - 1)); tables chirp [n_det], fac [n_det - 1], bspec [L] per level (float64-evaluated,
// launch_czt_tables); tw = the float32 twiddle table of length L.  Same output as
// launch_radial_dft (post without the ramp).
int czt_length(int nd);
hipError_t launch_czt_tables(cpx<float>* chirp, cpx<float>* fac, cpx<float>* bspec,
                             const GridGeom& gg, hipStream_t st);
hipError_t launch_radial_czt(const float* sino, int n_det_full, cpx<float>* ghat,
                             const cpx<float>* chirp, const cpx<float>* bspec,
                             const cpx<float>* fac, const cpx<float>* tw, const GridGeom& gg,
                             int nz, hipStream_t st);
hipError_t launch_radial_dft(const float* sino, int n_det_full, cpx<float>* ghat,
                             const cpx<float>* dft_tab, const cpx<float>* post,
                             const GridGeom& gg, int nz, hipStream_t st);
template <typename T>
hipError_t launch_point_table(const double* angle_tab /* [n_angles][2] cos,sin */, int2* g0, T* wx,
                              T* wy, const GridGeom& gg, hipStream_t st);
hipError_t launch_angle_table(const double* angles_dev, double* tab, int n_angles, hipStream_t st);
// Cell-sorted contribution lists of a geometry: cnt [M*M] scratch, row_ptr [M*M+1],
// idx/wts [n_samples * W^2], scan_sums [M*M/4096 + 1].
hipError_t launch_csr_build(const double* atab, const int2* g0, const float* wx, const float* wy,
                            const GridGeom& gg, int* cnt, int* row_ptr, int* idx, float* wts,
                            int* scan_sums, hipStream_t st);
// Lists of the point-spread grid (float64 weights, no sample indices: every sample carries
// the value 1 / n_det): cnt [M*M] scratch, row_ptr [M*M+1], wts [n_samples * W^2].
hipError_t launch_psf_lists(const double* atab, const int2* g0, const double* wx,
                            const double* wy, const GridGeom& gg, int* cnt, int* row_ptr,
                            double* wts, int* scan_sums, hipStream_t st);
// grid [M*M] complex128 = the point-spread grid summed over those lists (imaginary part 0).
hipError_t launch_psf_grid(const int* row_ptr, const double* wts, cpx<double>* grid,
                           const GridGeom& gg, hipStream_t st);
// grid[z][cell] for slices z0 .. z0+nzb-1 (nzb <= 64) from samples [p][nz] complex64.
hipError_t launch_gather(const cpx<float>* ghat, cpx<float>* grid, const int* row_ptr,
                         const int* idx, const float* wts, const GridGeom& gg, int nz, int z0,
                         int nzb, hipStream_t st);
// out[k] = wts[k] rampf[idx[k] mod (n_det - 1)]: the lists' ramp-filtered weights.
hipError_t launch_csr_ramp(const int* idx, const float* wts, const float* rampf, idx_t nnz,
                           const GridGeom& gg, float* out, hipStream_t st);
// Both grids of one list walk: grid (weights wts: R* g) and grid_ramp (weights wts_ramp: the
// ramp filter); the sums equal those of two launch_gather calls.  nzb 1..64.
hipError_t launch_gather_dual(const cpx<float>* ghat, cpx<float>* grid, cpx<float>* grid_ramp,
                              const int* row_ptr, const int* idx, const float* wts,
                              const float* wts_ramp, const GridGeom& gg, int nz, int z0, int nzb,
                              hipStream_t st);
hipError_t launch_deapod_table(float* inv, const GridGeom& gg, hipStream_t st);
hipError_t launch_fft2d_f32(cpx<float>* data, int M, int batch, int dir,
                            const cpx<float>* tw, hipStream_t st);
hipError_t launch_fft2d_f64(cpx<double>* data, int M, int batch, int dir,
                            const cpx<double>* tw, hipStream_t st);
// The 2D inverse-direction transform of a back-projection grid [batch][M][M] followed by the
// crop to N x N and the deapodisation into out [batch][N][N]: the row pass stores only the
// columns the crop keeps, the column pass transforms only those and writes the cropped rows.
// Overwrites the kept columns of data.  Same values as launch_fft2d_f32 (+1) then
// launch_crop_deapod.
hipError_t launch_fft2d_crop_f32(cpx<float>* data, int M, int batch, const cpx<float>* tw,
                                 float* out, const float* inv, int N, hipStream_t st);
hipError_t launch_crop_deapod(const cpx<float>* grid, float* out, const float* inv,
                              const GridGeom& gg, int nzb, hipStream_t st);
hipError_t launch_psf_embed(const cpx<double>* grid, cpx<double>* emb, const GridGeom& gg,
                            int N, int P, hipStream_t st);
hipError_t launch_fk_store(const cpx<double>* spec, float* fk, float* fkn, int P,
                           hipStream_t st);
hipError_t launch_fk_export(const float* fk, const float* fkn, float* out, int P,
                            hipStream_t st);

}  // namespace tomo
