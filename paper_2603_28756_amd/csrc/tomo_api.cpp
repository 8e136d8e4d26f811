// C-ABI layer of libtomo: plan lifecycle, validation, workspace carving and the
// orchestration of the HIP kernels.  Host code only; every numerical step runs in
// the kernels of toeplitz_kernels.hip and gridding_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/tomo.h"
#include "../../include/tomo_nn.h"
#include "kernels.hpp"
#include "unet_view.hpp"

using namespace tomo;

namespace {

thread_local std::string g_last_error;

constexpr size_t kAlign = 256;
constexpr int kMaxLevels = 6;
constexpr int kPowerIters = 30;
constexpr size_t kMaxGraphs = 24;  // cached three-iteration graph executables per plan
constexpr int kBatchDefaultGroup = 8;  // tiles per queue item of a batch before autotuning
constexpr int kBatchMaxGroup = 64;
constexpr int kMinFft = 32, kMaxHot = 4096, kMaxGrid = 8192;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
int next_pow2(long long x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}
bool is_pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }
int ilog2i(int x) {
  int l = 0;
  while ((1 << l) < x) ++l;
  return l;
}

struct Level {
  int n = 0, nd = 0, P = 0, M = 0, Mpsf = 0, stride = 1;
  double c = 0.0;
  double beta_bp = 0.0, beta_psf = 0.0;
  double L = 0.0, lambda = 0.0;
  size_t off_fk = 0, off_fkn = 0, off_b = 0;
  size_t off_rowptr = 0, off_cidx = 0, off_cw = 0, off_deapod = 0;  // gridding lists
  size_t off_cwr = 0;  // the lists' ramp-filtered weights (FBP)
  size_t off_prow = 0, off_pw = 0;  // point-spread grid lists (row pointers, float64 weights)
  size_t off_czc = 0, off_czf = 0, off_czb = 0;  // radial chirp-z tables (chirp, factor, B)
  int v_fwd = 1, v_cc = 1, v_inv = 1;  // tile variants of passes R, C, R'
  // the level's PSF precompute as one graph, captured with tile variants psf_key
  hipGraphExec_t psf_exec = nullptr;
  int psf_key = -1;
  int chunks = 1;  // slice chunks that passes R, C, R' run through one after the other
};

}  // namespace

struct tomo_plan_s {
  tomo_geometry_t g{};
  std::vector<double> angles;
  hipStream_t stream = nullptr;
  int device = 0;
  int nz = 0, n_levels = 1;
  std::vector<Level> lv;
  PriorParams pp{};
  ObjParams op{};       // the same prior in float64 (objective of candidate starts)
  double rho2_0 = 0.0;  // rho''(0)

  // workspace
  char* ws = nullptr;
  size_t ws_bytes = 0, need = 0;
  size_t off_scal = 0, off_partials = 0, n_partials = 0;
  size_t off_tw32[14] = {}, off_tw64[14] = {};
  size_t off_angles = 0, off_atab = 0;
  size_t off_x[3] = {};
  size_t off_ghat = 0, off_dfttab = 0, off_post = 0;
  size_t off_g0 = 0, off_wx = 0, off_wy = 0;
  size_t off_scratch = 0, scratch_bytes = 0;
  size_t off_gp = 0, off_ppartials = 0, off_y = 0;
  size_t off_cnt = 0, off_scan = 0, off_rampf = 0;
  size_t off_objpart = 0, off_choice = 0;  // learned start: objective partials, choice
  size_t off_resid = 0, off_rpart = 0;      // direct gradient: residual sinogram, its partials
  // PSF precompute: its own scratch and power-iteration buffers (it runs on fstream, beside
  // the back-projections on the plan's stream), and per level lambda, L, 1 / L on the device
  size_t off_psf = 0, off_pv[2] = {}, off_pS1 = 0, off_pS2 = 0, off_ppart = 0, off_pscal = 0;
  size_t off_lvl = 0;
  bool fused_prior = false, grids_ready = false;
  bool tables_ready = false, psf_ready = false;
  bool psf_host = false;  // lambda and L of every level copied to the host
  std::string err;

  // iteration graphs: replayed on an internal stream ordered against `stream` by events
  hipStream_t gstream = nullptr;
  hipEvent_t gev_in = nullptr, gev_out = nullptr;
  // prior kernel on its own stream, concurrent with the forward-row and column passes
  bool concurrent_prior = false;
  hipStream_t pstream = nullptr;
  hipEvent_t pev_fork = nullptr, pev_join = nullptr;
  // PSF precompute stream: forked from the plan's stream; consumers of the PSF spectrum and
  // of L wait for fev_done
  hipStream_t fstream = nullptr;
  hipEvent_t fev_fork = nullptr, fev_done = nullptr;
  // learned start: the network's stream ordered after / before the plan's stream
  hipEvent_t nev_fork = nullptr, nev_join = nullptr;
  struct GraphKey { int level, ik, nz; double* hist; int32_t* rhist; bool obj; };
  struct GraphEnt { GraphKey key; hipGraphExec_t exec; };
  std::vector<GraphEnt> graphs;
  bool use_graphs = true;

  // diagnostics: event pairs around timed kernel classes
  uint32_t tmask = 0;
  struct Pending { hipEvent_t a, b; int cls; };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  double tms[TOMO_T_COUNT] = {};
  int64_t tcnt[TOMO_T_COUNT] = {};

  template <typename T>
  T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
  double* scal() const { return at<double>(off_scal); }
  double* partials() const { return at<double>(off_partials); }
  cpx<float>* tw32(int P) const { return at<cpx<float>>(off_tw32[ilog2i(P)]); }
  cpx<double>* tw64(int P) const { return at<cpx<double>>(off_tw64[ilog2i(P)]); }
  float* xbuf(int i) const { return at<float>(off_x[i]); }
  cpx<float>* S1() const { return at<cpx<float>>(off_scratch); }
  cpx<float>* S2(const Level& l) const {
    return at<cpx<float>>(off_scratch + align_up((size_t)nz * l.n * (l.P / 2) * 8));
  }
};

namespace {

tomo_status fail(tomo_plan p, tomo_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (p) p->err = buf;
  g_last_error = buf;
  return s;
}

#define HIPCHK(plan, call)                                                              \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(plan, TOMO_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_));   \
  } while (0)

bool aligned(const void* p) { return (reinterpret_cast<uintptr_t>(p) % kAlign) == 0; }

double beatty_beta(int W, double s) {
  const double v = (W / s) * (W / s) * (s - 0.5) * (s - 0.5) - 0.8;
  return M_PI * std::sqrt(v > 0.0 ? v : 0.0);
}

// Carve the workspace: every region 256-byte aligned, offsets relative to the base.
void layout(tomo_plan p) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align_up(bytes);
    return o;
  };
  const Level& fin = p->lv.back();
  p->off_scal = take(SC_COUNT * sizeof(double));
  size_t maxblocks = 512;
  for (const Level& l : p->lv) {
    const int rb = rows_inv_rows_per_block(l.P, 0);  // smallest variant: most blocks
    const size_t nb = (size_t)p->nz * ((l.n + rb - 1) / rb);
    if (nb > maxblocks) maxblocks = nb;
  }
  p->n_partials = maxblocks;
  p->off_partials = take(maxblocks * 4 * sizeof(double));
  for (int k = ilog2i(kMinFft); k <= ilog2i(kMaxGrid); ++k) {
    p->off_tw32[k] = take((size_t(1) << k) * sizeof(cpx<float>));
    p->off_tw64[k] = take((size_t(1) << k) * sizeof(cpx<double>));
  }
  const int na = p->g.n_angles;
  p->off_angles = take(na * sizeof(double));
  p->off_atab = take(2 * na * sizeof(double));
  size_t maxcells = 0;
  for (Level& l : p->lv) {
    l.off_fk = take((size_t)l.P * (l.P / 2) * sizeof(float));
    l.off_fkn = take((size_t)l.P * sizeof(float));
    l.off_b = take((size_t)p->nz * l.n * l.n * sizeof(float));
    const size_t cells = (size_t)l.M * l.M;
    const size_t nnz = (size_t)p->g.n_angles * (l.nd - 1) * p->g.kb_width * p->g.kb_width;
    l.off_rowptr = take((cells + 1) * sizeof(int));
    l.off_cidx = take(nnz * sizeof(int));
    l.off_cw = take(nnz * sizeof(float));
    l.off_cwr = take(nnz * sizeof(float));
    l.off_deapod = take((size_t)l.n * sizeof(float));
    l.off_czc = take((size_t)l.nd * sizeof(cpx<float>));
    l.off_czf = take((size_t)l.nd * sizeof(cpx<float>));
    l.off_czb = take((size_t)czt_length(l.nd) * sizeof(cpx<float>));
    const size_t pcells = (size_t)l.Mpsf * l.Mpsf;
    l.off_prow = take((pcells + 1) * sizeof(int));
    l.off_pw = take(nnz * sizeof(double));
    maxcells = std::max(maxcells, std::max(cells, pcells));
  }
  p->off_cnt = take(maxcells * sizeof(int));
  p->off_scan = take((maxcells / 4096 + 2) * sizeof(int));
  for (int i = 0; i < 3; ++i) p->off_x[i] = take((size_t)p->nz * fin.n * fin.n * sizeof(float));
  p->off_gp = take((size_t)p->nz * fin.n * fin.n * sizeof(float));
  p->off_y = take((size_t)p->nz * fin.n * fin.n * sizeof(float));
  size_t maxprior = 1;
  for (const Level& l : p->lv) maxprior = std::max(maxprior, (size_t)prior_blocks(l.n, p->nz));
  p->off_ppartials = take(maxprior * 4 * sizeof(double));
  p->off_objpart = take((size_t)p->nz * kObjBlocks * sizeof(double));
  p->off_resid = take((size_t)p->nz * na * fin.nd * sizeof(float));
  p->off_rpart = take((size_t)radial_idft_blocks(fin.nd, p->nz * na) * sizeof(double));
  p->off_choice = take((size_t)p->nz * sizeof(int32_t));
  const size_t npts_max = (size_t)na * (fin.nd - 1);
  p->off_ghat = take((size_t)p->nz * npts_max * sizeof(cpx<float>));
  p->off_dfttab = take((size_t)fin.nd * sizeof(cpx<float>));
  p->off_post = take((size_t)fin.nd * sizeof(cpx<float>));
  p->off_rampf = take((size_t)fin.nd * sizeof(float));
  const int W = p->g.kb_width;
  p->off_g0 = take(npts_max * sizeof(int2));
  p->off_wx = take(npts_max * W * sizeof(float));
  p->off_wy = take(npts_max * W * sizeof(float));
  size_t scratch = 0;
  for (const Level& l : p->lv) {
    const size_t s1 = align_up((size_t)p->nz * l.n * (l.P / 2) * 8);
    const size_t hot = 2 * s1;
    // R* g and FBP grids of up to 32 slices: the back-projection walks its lists once per
    // chunk of slices, and 32 slices per walk read 256-byte lines per sample (16: 128 bytes)
    const size_t bp = 2 * (size_t)std::min(p->nz, 32) * l.M * l.M * sizeof(cpx<float>);
    const size_t npts = (size_t)na * (l.nd - 1);
    scratch = std::max(scratch, std::max(hot, bp));
  }
  p->scratch_bytes = scratch;
  p->off_scratch = take(scratch);
  size_t psf = 0, pn = 0, pspec = 0;
  for (const Level& l : p->lv) {
    const size_t npts = (size_t)na * (l.nd - 1);
    psf = std::max(psf, align_up((size_t)l.Mpsf * l.Mpsf * sizeof(cpx<double>)) +
                            align_up((size_t)l.P * l.P * sizeof(cpx<double>)) +
                            align_up(npts * sizeof(int2)) + 2 * align_up(npts * W * sizeof(double)));
    pn = std::max(pn, (size_t)l.n * l.n);
    pspec = std::max(pspec, (size_t)l.n * (l.P / 2));
  }
  p->off_psf = take(psf);
  for (int i = 0; i < 2; ++i) p->off_pv[i] = take(pn * sizeof(float));
  p->off_pS1 = take(pspec * sizeof(cpx<float>));
  p->off_pS2 = take(pspec * sizeof(cpx<float>));
  p->off_ppart = take(maxblocks * 4 * sizeof(double));
  p->off_pscal = take(SC_COUNT * sizeof(double));
  p->off_lvl = take(3 * (size_t)p->n_levels * sizeof(double));
  p->need = off;
}

tomo_status check_ws(tomo_plan p) {
  if (!p->ws) return fail(p, TOMO_ERR_NO_WORKSPACE, "no workspace attached");
  return TOMO_OK;
}

hipEvent_t take_event(tomo_plan p) {
  if (!p->pool.empty()) {
    hipEvent_t e = p->pool.back();
    p->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Opens a timed region for kernel class `cls` when it is enabled; returns the pending index.
int tbegin(tomo_plan p, int cls, hipStream_t s) {
  if (!(p->tmask & (1u << cls))) return -1;
  hipEvent_t a = take_event(p), b = take_event(p);
  if (!a || !b) return -1;
  (void)hipEventRecord(a, s);
  p->pending.push_back({a, b, cls});
  return (int)p->pending.size() - 1;
}
int tbegin(tomo_plan p, int cls) { return tbegin(p, cls, p->stream); }
void tend(tomo_plan p, int idx, hipStream_t s) {
  if (idx >= 0) (void)hipEventRecord(p->pending[idx].b, s);
}
void tend(tomo_plan p, int idx) { tend(p, idx, p->stream); }

// Stream and events of the concurrent prior kernel, created once per plan (before any capture).
tomo_status ensure_prior_stream(tomo_plan p) {
  if (!p->concurrent_prior || p->fused_prior || p->pstream) return TOMO_OK;
  HIPCHK(p, hipStreamCreateWithFlags(&p->pstream, hipStreamNonBlocking));
  HIPCHK(p, hipEventCreateWithFlags(&p->pev_fork, hipEventDisableTiming));
  HIPCHK(p, hipEventCreateWithFlags(&p->pev_join, hipEventDisableTiming));
  return TOMO_OK;
}

tomo_status tresolve(tomo_plan p) {
  HIPCHK(p, hipStreamSynchronize(p->stream));
  if (p->fstream) HIPCHK(p, hipStreamSynchronize(p->fstream));  // PSF launches are timed there
  for (auto& e : p->pending) {
    float ms = 0.f;
    HIPCHK(p, hipEventElapsedTime(&ms, e.a, e.b));
    p->tms[e.cls] += ms;
    p->tcnt[e.cls] += 1;
    p->pool.push_back(e.a);
    p->pool.push_back(e.b);
  }
  p->pending.clear();
  return TOMO_OK;
}

tomo_status ensure_tables(tomo_plan p) {
  if (p->tables_ready) return TOMO_OK;
  hipStream_t st = p->stream;
  for (int k = ilog2i(kMinFft); k <= ilog2i(kMaxGrid); ++k) {
    HIPCHK(p, launch_twiddles_f32(p->at<cpx<float>>(p->off_tw32[k]), 1 << k, st));
    HIPCHK(p, launch_twiddles_f64(p->at<cpx<double>>(p->off_tw64[k]), 1 << k, st));
  }
  HIPCHK(p, hipMemcpyAsync(p->at<double>(p->off_angles), p->angles.data(),
                           p->angles.size() * sizeof(double), hipMemcpyHostToDevice, st));
  HIPCHK(p, launch_angle_table(p->at<double>(p->off_angles), p->at<double>(p->off_atab),
                               p->g.n_angles, st));
  HIPCHK(p, launch_set_scalars(p->scal(), 0, SC_COUNT, nullptr, 0.0, st));
  HIPCHK(p, launch_set_scalars(p->scal(), SC_BETA, 1, nullptr, p->g.beta, st));
  HIPCHK(p, launch_set_scalars(p->scal(), SC_NONFINITE, 1, nullptr, -1.0, st));
  p->tables_ready = true;
  return TOMO_OK;
}

GridGeom bp_geom(tomo_plan p, const Level& l) {
  GridGeom gg;
  gg.n = l.n;
  gg.n_det = l.nd;
  gg.n_angles = p->g.n_angles;
  gg.M = l.M;
  gg.W = p->g.kb_width;
  gg.beta = l.beta_bp;
  gg.c = l.c;
  gg.stride = l.stride;
  return gg;
}

// Geometry-only gridding data of every level: the cell-sorted contribution lists of the
// back-projection grid and the deapodisation factors (built once per attached workspace).
// Geometry of level l's point-spread grid: the image doubled (2N, so that every lag of an
// N x N image is on it), oversampled grid M_psf, the PSF's own Kaiser-Bessel shape.
GridGeom psf_geom(tomo_plan p, const Level& l) {
  GridGeom gg;
  gg.n = 2 * l.n;
  gg.n_det = l.nd;
  gg.n_angles = p->g.n_angles;
  gg.M = l.Mpsf;
  gg.W = p->g.kb_width;
  gg.beta = l.beta_psf;
  gg.c = l.c;
  gg.stride = 1;
  return gg;
}

// The PSF precompute's scratch: grid [M_psf^2] and embedding [P^2] (complex128), and the
// sample table of the PSF geometry (footprint origins, float64 1D weights).
struct PsfScratch {
  cpx<double>* grid;
  cpx<double>* emb;
  int2* g0;
  double *wx, *wy;
};
PsfScratch psf_scratch(tomo_plan p, const Level& l) {
  const size_t npts = (size_t)p->g.n_angles * (l.nd - 1);
  size_t off = p->off_psf;
  PsfScratch s;
  s.grid = p->at<cpx<double>>(off);
  off += align_up((size_t)l.Mpsf * l.Mpsf * sizeof(cpx<double>));
  s.emb = p->at<cpx<double>>(off);
  off += align_up((size_t)l.P * l.P * sizeof(cpx<double>));
  s.g0 = p->at<int2>(off);
  off += align_up(npts * sizeof(int2));
  s.wx = p->at<double>(off);
  off += align_up(npts * p->g.kb_width * sizeof(double));
  s.wy = p->at<double>(off);
  return s;
}

// Cell-sorted lists of every level, once per geometry: the back-projection grid's (sample
// indices and float32 weights) and the point-spread grid's (float64 weights).  Runs on the
// plan's stream before any PSF precompute of this workspace.
tomo_status ensure_grids(tomo_plan p) {
  if (p->grids_ready) return TOMO_OK;
  hipStream_t st = p->stream;
  for (Level& l : p->lv) {
    const GridGeom gg = bp_geom(p, l);
    int2* g0 = p->at<int2>(p->off_g0);
    float* wx = p->at<float>(p->off_wx);
    float* wy = p->at<float>(p->off_wy);
    HIPCHK(p, launch_point_table<float>(p->at<double>(p->off_atab), g0, wx, wy, gg, st));
    HIPCHK(p, launch_csr_build(p->at<double>(p->off_atab), g0, wx, wy, gg, p->at<int>(p->off_cnt),
                               p->at<int>(l.off_rowptr), p->at<int>(l.off_cidx),
                               p->at<float>(l.off_cw), p->at<int>(p->off_scan), st));
    HIPCHK(p, launch_deapod_table(p->at<float>(l.off_deapod), gg, st));
    {
      // ramp weights of the level (radial_tables also writes the level's DFT tables, which
      // every back-projection rewrites before use)
      const size_t nnz = (size_t)p->g.n_angles * (l.nd - 1) * p->g.kb_width * p->g.kb_width;
      HIPCHK(p, launch_radial_tables(p->at<cpx<float>>(p->off_dfttab), p->at<cpx<float>>(p->off_post),
                                     p->at<float>(p->off_rampf), gg, 0, st));
      HIPCHK(p, launch_csr_ramp(p->at<int>(l.off_cidx), p->at<float>(l.off_cw),
                                p->at<float>(p->off_rampf), (idx_t)nnz, gg, p->at<float>(l.off_cwr), st));
    }
    if (czt_length(l.nd) <= kMaxGrid)
      HIPCHK(p, launch_czt_tables(p->at<cpx<float>>(l.off_czc), p->at<cpx<float>>(l.off_czf),
                                  p->at<cpx<float>>(l.off_czb), gg, st));
    const GridGeom pg = psf_geom(p, l);
    const PsfScratch ps = psf_scratch(p, l);
    HIPCHK(p, launch_point_table<double>(p->at<double>(p->off_atab), ps.g0, ps.wx, ps.wy, pg, st));
    HIPCHK(p, launch_psf_lists(p->at<double>(p->off_atab), ps.g0, ps.wx, ps.wy, pg,
                               p->at<int>(p->off_cnt), p->at<int>(l.off_prow),
                               p->at<double>(l.off_pw), p->at<int>(p->off_scan), st));
  }
  p->grids_ready = true;
  return TOMO_OK;
}

// out[nz][N_l][N_l] = R*_l g_l (ramp = 0) or FBP (ramp = 1) of level l.  With reuse the
// radial spectrum of the previous call (same level and sinogram) is used again.
tomo_status backproject_level_impl(tomo_plan p, const Level& l, const float* sino, float* out,
                                   int ramp, bool reuse);
tomo_status backproject_level(tomo_plan p, const Level& l, const float* sino, float* out,
                              int ramp, bool reuse = false) {
  const int ti = tbegin(p, TOMO_T_BACKPROJECT);
  const tomo_status s = backproject_level_impl(p, l, sino, out, ramp, reuse);
  tend(p, ti);
  return s;
}

// Radial spectrum of level l's projections into ghat (and the ramp weights into rampf).
tomo_status radial_spectrum(tomo_plan p, const Level& l, const float* sino) {
  hipStream_t st = p->stream;
  const GridGeom gg = bp_geom(p, l);
  cpx<float>* ghat = p->at<cpx<float>>(p->off_ghat);
  cpx<float>* tab = p->at<cpx<float>>(p->off_dfttab);
  cpx<float>* post = p->at<cpx<float>>(p->off_post);
  HIPCHK(p, launch_radial_tables(tab, post, p->at<float>(p->off_rampf), gg, 0, st));
  // the radial DFT by chirp-z (two FFTs of length L per row); the direct sum where L would
  // exceed the largest transform
  const int L = czt_length(l.nd);
  if (L <= kMaxGrid)
    HIPCHK(p, launch_radial_czt(sino, p->g.n_det, ghat, p->at<cpx<float>>(l.off_czc),
                                p->at<cpx<float>>(l.off_czb), p->at<cpx<float>>(l.off_czf),
                                p->tw32(L), gg, p->nz, st));
  else
    HIPCHK(p, launch_radial_dft(sino, p->g.n_det, ghat, tab, post, gg, p->nz, st));
  return TOMO_OK;
}

// R* g (out_b) and the FBP (out_fbp) of level l from one radial spectrum and one walk of the
// gridding lists per slice chunk (the scratch holds both grids of a chunk).
tomo_status backproject_level_dual_impl(tomo_plan p, const Level& l, const float* sino,
                                        float* out_b, float* out_fbp) {
  hipStream_t st = p->stream;
  tomo_status s = ensure_grids(p);
  if (s == TOMO_OK) s = radial_spectrum(p, l, sino);
  if (s != TOMO_OK) return s;
  const GridGeom gg = bp_geom(p, l);
  const size_t slice_grid = (size_t)l.M * l.M * sizeof(cpx<float>);
  int chunk = (int)std::min<size_t>((size_t)p->nz, p->scratch_bytes / (2 * slice_grid));
  if (chunk > 64) chunk = 64;
  if (chunk < 1) return fail(p, TOMO_ERR_INTERNAL, "scratch too small for two grid slices");
  cpx<float>* grid = p->at<cpx<float>>(p->off_scratch);
  cpx<float>* grid2 = grid + (size_t)chunk * l.M * l.M;
  for (int z0 = 0; z0 < p->nz; z0 += chunk) {
    const int zc = std::min(chunk, p->nz - z0);
    HIPCHK(p, launch_gather_dual(p->at<cpx<float>>(p->off_ghat), grid, grid2, p->at<int>(l.off_rowptr),
                                 p->at<int>(l.off_cidx), p->at<float>(l.off_cw),
                                 p->at<float>(l.off_cwr), gg, p->nz, z0, zc, st));
    HIPCHK(p, launch_fft2d_crop_f32(grid, l.M, zc, p->tw32(l.M), out_b + (size_t)z0 * l.n * l.n,
                                    p->at<float>(l.off_deapod), l.n, st));
    HIPCHK(p, launch_fft2d_crop_f32(grid2, l.M, zc, p->tw32(l.M), out_fbp + (size_t)z0 * l.n * l.n,
                                    p->at<float>(l.off_deapod), l.n, st));
  }
  return TOMO_OK;
}
tomo_status backproject_level_dual(tomo_plan p, const Level& l, const float* sino, float* out_b,
                                   float* out_fbp) {
  const int ti = tbegin(p, TOMO_T_BACKPROJECT);
  const tomo_status s = backproject_level_dual_impl(p, l, sino, out_b, out_fbp);
  tend(p, ti);
  return s;
}

tomo_status backproject_level_impl(tomo_plan p, const Level& l, const float* sino, float* out,
                                   int ramp, bool reuse) {
  hipStream_t st = p->stream;
  tomo_status s = ensure_grids(p);
  if (s != TOMO_OK) return s;
  const GridGeom gg = bp_geom(p, l);
  cpx<float>* ghat = p->at<cpx<float>>(p->off_ghat);
  if (!reuse && (s = radial_spectrum(p, l, sino)) != TOMO_OK) return s;
  const size_t slice_grid = (size_t)l.M * l.M * sizeof(cpx<float>);
  int chunk = (int)std::min<size_t>((size_t)p->nz, p->scratch_bytes / slice_grid);
  if (chunk < 1) return fail(p, TOMO_ERR_INTERNAL, "scratch too small for one grid slice");
  cpx<float>* grid = p->at<cpx<float>>(p->off_scratch);
  for (int z0 = 0; z0 < p->nz; z0 += chunk) {
    const int zc = std::min(chunk, p->nz - z0);
    for (int zb = 0; zb < zc; zb += 64) {
      const int nzb = std::min(64, zc - zb);
      HIPCHK(p, launch_gather(ghat, grid + (size_t)zb * l.M * l.M, p->at<int>(l.off_rowptr),
                              p->at<int>(l.off_cidx), p->at<float>(ramp ? l.off_cwr : l.off_cw), gg,
                              p->nz, z0 + zb, nzb, st));
    }
    HIPCHK(p, launch_fft2d_crop_f32(grid, l.M, zc, p->tw32(l.M), out + (size_t)z0 * l.n * l.n,
                                    p->at<float>(l.off_deapod), l.n, st));
  }
  return TOMO_OK;
}

// One application of the Toeplitz passes on level l (and, outside power mode, of the prior
// kernel unless the fused-prior epilogue is selected).  *nprior receives the number of prior
// partial sums the finalize must add (0 when none).  In sequence, a FISTA step's prior
// kernel also writes y and gp - b for passes R and R'.  With the concurrent flag the prior
// kernel reads only x_k, x_{k-1} and mu and runs on its own stream beside the forward-row
// and column passes (which then form y themselves); the inverse-row pass, the only reader
// of its output, waits for it.
tomo_status toeplitz_passes(tomo_plan p, const Level& l, int mode, int nz, const float* xk,
                            const float* xkm1, const float* b, float* out, bool obj,
                            int* nblocks, int* nprior = nullptr) {
  hipStream_t st = p->stream;
  cpx<float>* S1 = p->S1();
  cpx<float>* S2 = p->S2(l);
  const float* gpv = nullptr;
  if (nprior) *nprior = 0;
  const bool conc = mode != MODE_POWER && !p->fused_prior && p->concurrent_prior;
  // In sequence, a FISTA step lets the prior kernel (which forms y anyway and is bound by
  // its arithmetic, not by memory) also write y and gp - b: pass R then reads y alone and
  // pass R' reads y and gp - b instead of x_{k-1}, b and gp (4 bytes per voxel less for each
  // of the two memory-bound passes).
  const bool yg = mode == MODE_FISTA && !p->fused_prior && !conc;
  float* ybuf = yg ? p->at<float>(p->off_y) : nullptr;
  if (mode != MODE_POWER && !p->fused_prior) {
    hipStream_t ps = st;
    if (conc) {
      tomo_status s = ensure_prior_stream(p);
      if (s != TOMO_OK) return s;
      ps = p->pstream;
      HIPCHK(p, hipEventRecord(p->pev_fork, st));
      HIPCHK(p, hipStreamWaitEvent(ps, p->pev_fork, 0));
    }
    const int tp = tbegin(p, TOMO_T_PRIOR, ps);
    HIPCHK(p, launch_prior(mode, p->g.neighbours, obj, xk, xkm1, p->scal(), p->at<float>(p->off_gp),
                           yg ? b : nullptr, ybuf, p->at<double>(p->off_ppartials), l.n, nz,
                           p->pp, ps));
    tend(p, tp, ps);
    if (conc) HIPCHK(p, hipEventRecord(p->pev_join, ps));
    gpv = p->at<float>(p->off_gp);
    if (nprior && obj) *nprior = prior_blocks(l.n, nz);
  }
  // per-class timing covers the iteration and gradient launches, not the power iteration
  const bool timed = mode != MODE_POWER;
  // With the prior in sequence (or computed inside pass R'), passes R, C and R' may run through
  // the slices in chunks that reuse the same S1 and S2 buffers: a chunk's half spectra then
  // stay in the 256 MB Infinity Cache between the passes (the autotuner picks the count).  Each
  // chunk's pass-R' partial sums follow the previous chunk's in the partials buffer.
  const int nch = (conc || mode == MODE_POWER || p->fused_prior) ? 1
                                                                  : std::max(1, std::min(l.chunks, nz));
  const size_t plane = (size_t)l.n * l.n;
  int nbtot = 0;
  for (int c = 0; c < nch; ++c) {
    const int z0 = (int)((long long)c * nz / nch), zc = (int)((long long)(c + 1) * nz / nch) - z0;
    const size_t o = (size_t)z0 * plane;
    int ti = timed ? tbegin(p, TOMO_T_ROWS_FWD) : -1;
    if (yg)
      HIPCHK(p, launch_rows_fwd(l.P, l.v_fwd, MODE_FISTA_Y, ybuf + o, ybuf + o, p->scal(), S1,
                                p->tw32(l.P), l.n, zc, st));
    else
      HIPCHK(p, launch_rows_fwd(l.P, l.v_fwd, mode, xk + o, xkm1 + o, p->scal(), S1, p->tw32(l.P),
                                l.n, zc, st));
    tend(p, ti);
    ti = timed ? tbegin(p, TOMO_T_COLS_CONV) : -1;
    HIPCHK(p, launch_cols_conv(l.P, l.v_cc, S1, S2, p->at<float>(l.off_fk), p->at<float>(l.off_fkn),
                               p->tw32(l.P), l.n, zc, st));
    tend(p, ti);
    // the prior on its own stream (one chunk): pass R' is the only reader of its output
    if (conc) HIPCHK(p, hipStreamWaitEvent(st, p->pev_join, 0));
    ti = timed ? tbegin(p, TOMO_T_ROWS_INV) : -1;
    int nbc = 0;
    double* part = p->partials() + (size_t)nbtot * 4;
    if (yg)
      HIPCHK(p, launch_rows_inv(l.P, l.v_inv, MODE_FISTA_Y, p->g.neighbours, obj, S2, xk + o,
                                ybuf + o, nullptr, gpv + o, out + o, part, p->scal(), p->tw32(l.P),
                                l.n, zc, p->pp, &nbc, st));
    else if (nch == 1)
      HIPCHK(p, launch_rows_inv(l.P, l.v_inv, mode, p->g.neighbours, obj, S2, xk, xkm1, b, gpv, out,
                                part, p->scal(), p->tw32(l.P), l.n, nz, p->pp, &nbc, st));
    else  // separate prior (gpv set): every operand is slice-local
      HIPCHK(p, launch_rows_inv(l.P, l.v_inv, mode, p->g.neighbours, obj, S2, xk + o, xkm1 + o,
                                b ? b + o : nullptr, gpv + o, out + o, part, p->scal(), p->tw32(l.P),
                                l.n, zc, p->pp, &nbc, st));
    tend(p, ti);
    nbtot += nbc;
  }
  *nblocks = nbtot;
  return TOMO_OK;
}

// PSF spectrum F K of level li (Sec. 2.1, Eq. 9) and the largest eigenvalue of T by power
// iteration, on the PSF stream with the PSF's own scratch, iterate and spectrum buffers (so
// that it can run beside the back-projections of the plan's stream).  lambda, L and 1 / L
// stay on the device (off_lvl); nothing here waits for the host.
tomo_status psf_level_launches(tomo_plan p, Level& l, int li) {
  hipStream_t st = p->fstream;
  const GridGeom gg = psf_geom(p, l);
  const PsfScratch ps = psf_scratch(p, l);
  cpx<double>* grid = ps.grid;
  cpx<double>* emb = ps.emb;
  // spreading of the all-ones function over the level's cell-sorted lists
  HIPCHK(p, launch_psf_grid(p->at<int>(l.off_prow), p->at<double>(l.off_pw), grid, gg, st));
  HIPCHK(p, launch_fft2d_f64(grid, l.Mpsf, 1, +1, p->tw64(l.Mpsf), st));
  HIPCHK(p, launch_psf_embed(grid, emb, gg, l.n, l.P, st));
  HIPCHK(p, launch_fft2d_f64(emb, l.P, 1, -1, p->tw64(l.P), st));
  const float* fk = p->at<float>(l.off_fk);
  const float* fkn = p->at<float>(l.off_fkn);
  HIPCHK(p, launch_fk_store(emb, const_cast<float*>(fk), const_cast<float*>(fkn), l.P, st));

  // Power iteration on one slice: v0 = 1, lambda = ||T v|| / ||v||; each step applies the
  // three Toeplitz passes to the scaled iterate and normalises in the float64 finalize.
  float* v = p->at<float>(p->off_pv[0]);
  float* w = p->at<float>(p->off_pv[1]);
  cpx<float>* S1 = p->at<cpx<float>>(p->off_pS1);
  cpx<float>* S2 = p->at<cpx<float>>(p->off_pS2);
  double* part = p->at<double>(p->off_ppart);
  double* sc = p->at<double>(p->off_pscal);
  HIPCHK(p, launch_fill(v, (idx_t)l.n * l.n, 1.0f, st));
  HIPCHK(p, launch_set_scalars(sc, SC_PSCALE, 1, nullptr, 1.0, st));
  HIPCHK(p, launch_set_scalars(sc, SC_VNORM, 1, nullptr, (double)l.n, st));
  // each step after the first takes its scale 1 / ||T v|| from the previous step's pass R'
  // partial sums inside pass R; one finalize after the last step gives lambda (the iterate
  // then has unit norm)
  int nb_prev = 0;
  for (int it = 0; it < kPowerIters; ++it) {
    int nb = 0;
    HIPCHK(p, launch_rows_fwd(l.P, l.v_fwd, MODE_POWER, v, v, sc, S1, p->tw32(l.P), l.n, 1, st,
                              it > 0 ? part : nullptr, nb_prev));
    HIPCHK(p, launch_cols_conv(l.P, l.v_cc, S1, S2, fk, fkn, p->tw32(l.P), l.n, 1, st));
    HIPCHK(p, launch_rows_inv(l.P, l.v_inv, MODE_POWER, p->g.neighbours, false, S2, v, v, nullptr,
                              nullptr, w, part, sc, p->tw32(l.P), l.n, 1, p->pp, &nb, st));
    nb_prev = nb;
    std::swap(v, w);
  }
  if (kPowerIters > 1) HIPCHK(p, launch_set_scalars(sc, SC_VNORM, 1, nullptr, 1.0, st));
  HIPCHK(p, launch_finalize(MODE_POWER, part, nb_prev, nullptr, 0, sc, nullptr, nullptr, nullptr, st));
  // L = 1.01 lambda + 2 beta rho''(0) (a bound on the Hessian of the whole objective)
  HIPCHK(p, launch_lipschitz(sc, 1.01, 2.0 * p->g.beta * p->rho2_0,
                             p->at<double>(p->off_lvl) + 3 * (size_t)li, st));
  return TOMO_OK;
}

void drop_psf_graphs(tomo_plan p) {
  bool any = false;
  for (auto& l : p->lv) any = any || l.psf_exec;
  if (!any) return;
  if (p->fstream) (void)hipStreamSynchronize(p->fstream);
  for (auto& l : p->lv) {
    if (l.psf_exec) (void)hipGraphExecDestroy(l.psf_exec);
    l.psf_exec = nullptr;
    l.psf_key = -1;
  }
}

// The PSF precompute of level l on the PSF stream: its ~130 launches (spectrum, 30 power
// iterations of four kernels each on one slice, step constant) are captured once into a
// graph and replayed, so the host spends one launch on them instead of keeping the plan's
// own stream waiting behind them.  Launched one by one when kernel timing is on or graphs
// are off.  The graph holds the workspace pointers and the level's tile variants; it is
// captured again when the tiles change and dropped with the workspace.
tomo_status psf_level(tomo_plan p, Level& l, int li) {
  if (!p->use_graphs || p->tmask != 0) return psf_level_launches(p, l, li);
  const int key = l.v_fwd * 9 + l.v_cc * 3 + l.v_inv;
  if (l.psf_exec && l.psf_key != key) {
    HIPCHK(p, hipStreamSynchronize(p->fstream));
    (void)hipGraphExecDestroy(l.psf_exec);
    l.psf_exec = nullptr;
  }
  if (!l.psf_exec) {
    hipGraph_t graph = nullptr;
    HIPCHK(p, hipStreamBeginCapture(p->fstream, hipStreamCaptureModeRelaxed));
    const tomo_status s = psf_level_launches(p, l, li);
    hipError_t e = hipStreamEndCapture(p->fstream, &graph);
    if (s != TOMO_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return s;
    }
    if (e != hipSuccess) return fail(p, TOMO_ERR_HIP, "PSF graph capture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&l.psf_exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      l.psf_exec = nullptr;
      return fail(p, TOMO_ERR_HIP, "PSF graph instantiate: %s", hipGetErrorString(e));
    }
    l.psf_key = key;
  }
  HIPCHK(p, hipGraphLaunch(l.psf_exec, p->fstream));
  return TOMO_OK;
}

// Copy lambda and L of every level to the host (waits for the PSF stream); a non-finite or
// non-positive lambda is reported here.
tomo_status psf_host_values(tomo_plan p) {
  if (!p->psf_ready) return fail(p, TOMO_ERR_NOT_READY, "PSF not precomputed");
  if (p->psf_host) return TOMO_OK;
  std::vector<double> v(3 * (size_t)p->n_levels);
  HIPCHK(p, hipMemcpyAsync(v.data(), p->at<double>(p->off_lvl), v.size() * sizeof(double),
                           hipMemcpyDeviceToHost, p->fstream));
  HIPCHK(p, hipStreamSynchronize(p->fstream));
  for (int li = 0; li < p->n_levels; ++li) {
    const double lam = v[3 * li];
    if (!std::isfinite(lam) || lam <= 0.0)
      return fail(p, TOMO_ERR_NONFINITE, "power iteration gave lambda = %g on level %d", lam, li);
    p->lv[li].lambda = lam;
    p->lv[li].L = v[3 * li + 1];
  }
  p->psf_host = true;
  return TOMO_OK;
}

// Order stream st after the PSF precompute (spectrum, lambda and L of every level).
tomo_status psf_join(tomo_plan p, hipStream_t st) {
  if (!p->psf_ready) return fail(p, TOMO_ERR_NOT_READY, "PSF not precomputed");
  HIPCHK(p, hipStreamWaitEvent(st, p->fev_done, 0));
  return TOMO_OK;
}

// One FISTA iteration on level l with buffers (ik, ikm1, inext).
tomo_status fista_iteration(tomo_plan p, const Level& l, int ik, int ikm1, int inext,
                            const float* b, double* hist, int32_t* rhist, hipStream_t st) {
  int nb = 0;
  hipStream_t keep = p->stream;
  p->stream = st;
  int npr = 0;
  tomo_status s = toeplitz_passes(p, l, MODE_FISTA, p->nz, p->xbuf(ik), p->xbuf(ikm1), b,
                                  p->xbuf(inext), hist != nullptr, &nb, &npr);
  if (s == TOMO_OK) {
    const int tf = tbegin(p, TOMO_T_FINALIZE);
    hipError_t e = launch_finalize(MODE_FISTA, p->partials(), nb, p->at<double>(p->off_ppartials),
                                   npr, p->scal(), hist, rhist, nullptr, st);
    tend(p, tf);
    if (e != hipSuccess) s = fail(p, TOMO_ERR_HIP, "finalize launch: %s", hipGetErrorString(e));
  }
  p->stream = keep;
  return s;
}

// Graph of three consecutive iterations starting from buffers (ik, ik, (ik+1)%3) after the
// first iteration of a level, i.e. the steady rotation (ik, ikm1, inext) -> period 3.
tomo_status get_graph(tomo_plan p, int level, int ik, int ikm1, int inext, const float* b,
                      double* hist, int32_t* rhist, hipGraphExec_t* out) {
  for (auto& g : p->graphs)
    if (g.key.level == level && g.key.ik == ik * 9 + ikm1 * 3 + inext && g.key.nz == p->nz &&
        g.key.hist == hist && g.key.rhist == rhist) {
      *out = g.exec;
      return TOMO_OK;
    }
  if (!p->gstream) {
    HIPCHK(p, hipStreamCreateWithFlags(&p->gstream, hipStreamNonBlocking));
    HIPCHK(p, hipEventCreateWithFlags(&p->gev_in, hipEventDisableTiming));
    HIPCHK(p, hipEventCreateWithFlags(&p->gev_out, hipEventDisableTiming));
  }
  const Level& l = p->lv[level];
  if (tomo_status ps = ensure_prior_stream(p); ps != TOMO_OK) return ps;
  hipGraph_t graph = nullptr;
  HIPCHK(p, hipStreamBeginCapture(p->gstream, hipStreamCaptureModeRelaxed));
  tomo_status s = TOMO_OK;
  int a = ik, b0 = ikm1, c = inext;
  for (int k = 0; k < 3 && s == TOMO_OK; ++k) {
    s = fista_iteration(p, l, a, b0, c, b, hist, rhist, p->gstream);
    b0 = a;
    a = c;
    c = 3 - a - b0;
  }
  hipError_t e = hipStreamEndCapture(p->gstream, &graph);
  if (s != TOMO_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return s;
  }
  if (e != hipSuccess) return fail(p, TOMO_ERR_HIP, "graph capture: %s", hipGetErrorString(e));
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return fail(p, TOMO_ERR_HIP, "graph instantiate: %s", hipGetErrorString(e));
  // The key holds the caller's history pointers, so a caller passing fresh history buffers
  // would grow the cache without bound: keep the most recent kMaxGraphs executables (the
  // evicted one may still be queued on the internal stream, which is drained first).
  if (p->graphs.size() >= kMaxGraphs) {
    HIPCHK(p, hipStreamSynchronize(p->gstream));
    (void)hipGraphExecDestroy(p->graphs.front().exec);
    p->graphs.erase(p->graphs.begin());
  }
  p->graphs.push_back({{level, ik * 9 + ikm1 * 3 + inext, p->nz, hist, rhist, hist != nullptr}, exec});
  *out = exec;
  return TOMO_OK;
}

// Is the coarsest level inside the network's training domain (tomo_unet_domain_t)?
bool in_domain(tomo_plan p, const Level& l, const UnetView& v) {
  if (v.height != l.n || v.width != l.n || !v.has_domain) return false;
  const tomo_unet_domain_t& d = v.domain;
  auto close = [](double a, double b) { return std::fabs(a - b) <= 1e-9 * std::max(std::fabs(a), std::fabs(b)); };
  const double dc = std::isnan(d.center) ? 0.5 * d.n_det : d.center;
  return d.n == l.n && d.n_det == l.nd && std::fabs(l.c - dc) <= 1e-6 &&
         p->g.n_angles >= d.n_angles_min && p->g.n_angles <= d.n_angles_max &&
         close(d.beta, p->g.beta) && close(d.p, p->g.p) && close(d.sigma, p->g.sigma) &&
         close(d.T, p->g.T) && d.neighbours == p->g.neighbours;
}

// Learned start on level l: the FBP image in xbuf(cur) is mapped by the network into
// xbuf(alt); the float64 difference of the two starts' objectives (from T of their sum, into
// the y volume) decides, per slice with the 8-neighbour prior or for the whole volume with the
// 26-neighbour prior, which one xbuf(cur) holds afterwards (FBP unless the network's objective
// is not larger).
tomo_status learned_start(tomo_plan p, const Level& l, const float* b, int cur, const UnetView& net,
                          const tomo_recon_opts_t* o) {
  hipStream_t st = p->stream;
  float* xa = p->xbuf(cur);
  float* xb = p->xbuf((cur + 1) % 3);
  float* ty = p->at<float>(p->off_y);
  const size_t plane = (size_t)l.n * l.n;
  const bool fork = net.stream != st;
  if (fork) {
    if (!p->nev_fork) HIPCHK(p, hipEventCreateWithFlags(&p->nev_fork, hipEventDisableTiming));
    if (!p->nev_join) HIPCHK(p, hipEventCreateWithFlags(&p->nev_join, hipEventDisableTiming));
    HIPCHK(p, hipEventRecord(p->nev_fork, st));
    HIPCHK(p, hipStreamWaitEvent(net.stream, p->nev_fork, 0));
  }
  for (int z0 = 0; z0 < p->nz; z0 += net.max_batch) {
    const int m = std::min(net.max_batch, p->nz - z0);
    const tomo_status s = tomo_unet_forward(o->unet, xa + z0 * plane, xb + z0 * plane, m, o->unet_scale);
    if (s != TOMO_OK) return fail(p, s, "learned start: %s", tomo_unet_last_error(o->unet));
  }
  if (fork) {
    HIPCHK(p, hipEventRecord(p->nev_join, net.stream));
    HIPCHK(p, hipStreamWaitEvent(st, p->nev_join, 0));
  }
  // F(xb) - F(xa) from one Toeplitz product, T (xa + xb) (the third iterate buffer holds the
  // sum), instead of one product per candidate
  double* pd = p->at<double>(p->off_objpart);
  float* sum = p->xbuf((cur + 2) % 3);
  HIPCHK(p, launch_add(xa, xb, sum, (idx_t)p->nz * plane, st));
  HIPCHK(p, launch_set_scalars(p->scal(), SC_PSCALE, 1, nullptr, 1.0, st));
  int nb = 0;
  tomo_status s = toeplitz_passes(p, l, MODE_POWER, p->nz, sum, sum, nullptr, ty, false, &nb);
  if (s != TOMO_OK) return s;
  HIPCHK(p, launch_slice_objective_diff(xa, xb, ty, b, l.n, p->nz, p->op, pd, st));
  HIPCHK(p, launch_select_start(pd, p->nz, p->g.neighbours == 8 ? 1 : 0, xa, xb, l.n,
                                p->at<int32_t>(p->off_choice), o->init_choice_dev, st));
  return TOMO_OK;
}

// out = R x on the finest level (Sec. 2, Eq. 3); with sino, out = R x - sino and the partial
// sums of its squares go to rpart.  The radial spectra reuse the back-projection's sample
// buffer ([slice][sample] here) and the grids its scratch.
tomo_status forward_project_impl(tomo_plan p, const float* x, float* out, const float* sino,
                                 double* rpart) {
  hipStream_t st = p->stream;
  tomo_status s = ensure_tables(p);
  if (s == TOMO_OK) s = ensure_grids(p);
  if (s != TOMO_OK) return s;
  const Level& l = p->lv.back();
  const GridGeom gg = bp_geom(p, l);
  int2* g0 = p->at<int2>(p->off_g0);
  float* wx = p->at<float>(p->off_wx);
  float* wy = p->at<float>(p->off_wy);
  cpx<float>* tab = p->at<cpx<float>>(p->off_dfttab);
  cpx<float>* post = p->at<cpx<float>>(p->off_post);
  HIPCHK(p, launch_point_table<float>(p->at<double>(p->off_atab), g0, wx, wy, gg, st));
  HIPCHK(p, launch_radial_tables(tab, post, p->at<float>(p->off_rampf), gg, 0, st));
  cpx<float>* fhat = p->at<cpx<float>>(p->off_ghat);
  const int npts = p->g.n_angles * (l.nd - 1);
  const size_t slice_grid = (size_t)l.M * l.M * sizeof(cpx<float>);
  const int chunk = (int)std::min<size_t>((size_t)p->nz, p->scratch_bytes / slice_grid);
  if (chunk < 1) return fail(p, TOMO_ERR_INTERNAL, "scratch too small for one grid slice");
  cpx<float>* grid = p->at<cpx<float>>(p->off_scratch);
  for (int z0 = 0; z0 < p->nz; z0 += chunk) {
    const int zc = std::min(chunk, p->nz - z0);
    HIPCHK(p, launch_embed_deapod(x, grid, p->at<float>(l.off_deapod), l.n, l.M, z0, zc, st));
    HIPCHK(p, launch_fft2d_f32(grid, l.M, zc, -1, p->tw32(l.M), st));
    HIPCHK(p, launch_interp(grid, g0, wx, wy, fhat, npts, l.M, p->g.kb_width, z0, zc, st));
  }
  HIPCHK(p, launch_radial_idft(fhat, sino, out, rpart, l.nd, p->nz * p->g.n_angles, tab, post, st));
  return TOMO_OK;
}

tomo_status validate_geom(const tomo_geometry_t* g) {
  if (!g) return fail(nullptr, TOMO_ERR_INVALID_ARG, "geometry is NULL");
  if (g->n < 16 || g->n > 2048 || (g->n & 1))
    return fail(nullptr, TOMO_ERR_INVALID_ARG, "n = %d must be even and in [16, 2048]", g->n);
  if (g->n_slices < 1) return fail(nullptr, TOMO_ERR_INVALID_ARG, "n_slices must be >= 1");
  if (g->n_angles < 1) return fail(nullptr, TOMO_ERR_INVALID_ARG, "n_angles must be >= 1");
  if (g->n_det < 4 || (g->n_det & 1))
    return fail(nullptr, TOMO_ERR_INVALID_ARG, "n_det = %d must be even and >= 4", g->n_det);
  if (g->n_det > 16384) return fail(nullptr, TOMO_ERR_INVALID_ARG, "n_det too large");
  const int L = g->n_levels == 0 ? 1 : g->n_levels;
  if (L < 1 || L > kMaxLevels)
    return fail(nullptr, TOMO_ERR_INVALID_ARG, "n_levels must be in [1, %d]", kMaxLevels);
  const int s = 1 << (L - 1);
  if (g->n % s || (g->n / s) < 16 || ((g->n / s) & 1))
    return fail(nullptr, TOMO_ERR_INVALID_ARG,
                "n must be divisible by 2^(n_levels-1) with an even coarsest width >= 16");
  if (g->n_det % (2 * s))
    return fail(nullptr, TOMO_ERR_INVALID_ARG,
                "n_det must be divisible by 2^n_levels (even bins on every level)");
  if (g->pad != 0 && (!is_pow2(g->pad) || g->pad < 2 * g->n || g->pad > kMaxHot))
    return fail(nullptr, TOMO_ERR_INVALID_ARG, "pad must be 0 or a power of two in [2N, %d]",
                kMaxHot);
  const int W = g->kb_width == 0 ? 6 : g->kb_width;
  if (W < 2 || W > 16) return fail(nullptr, TOMO_ERR_INVALID_ARG, "kb_width must be in [2, 16]");
  const double sg = g->kb_oversamp == 0.0 ? 2.0 : g->kb_oversamp;
  if (!(sg >= 1.25 && sg <= 4.0))
    return fail(nullptr, TOMO_ERR_INVALID_ARG, "kb_oversamp must be in [1.25, 4]");
  if (!(g->kb_beta >= 0.0) || !std::isfinite(g->kb_beta))
    return fail(nullptr, TOMO_ERR_INVALID_ARG, "kb_beta must be >= 0");
  if (!(g->beta >= 0.0) || !std::isfinite(g->beta))
    return fail(nullptr, TOMO_ERR_INVALID_ARG, "beta must be >= 0");
  if (!(g->p >= 1.0 && g->p <= 2.0)) return fail(nullptr, TOMO_ERR_INVALID_ARG, "p must be in [1, 2]");
  if (g->q != 2.0) return fail(nullptr, TOMO_ERR_INVALID_ARG, "q must be 2");
  if (!(g->sigma > 0.0) || !std::isfinite(g->sigma))
    return fail(nullptr, TOMO_ERR_INVALID_ARG, "sigma must be > 0");
  if (!(g->T > 0.0) || !std::isfinite(g->T)) return fail(nullptr, TOMO_ERR_INVALID_ARG, "T must be > 0");
  if (g->neighbours != 8 && g->neighbours != 26)
    return fail(nullptr, TOMO_ERR_INVALID_ARG, "neighbours must be 8 or 26");
  if (g->flags & ~(uint32_t)(TOMO_FLAG_NO_GRAPH | TOMO_FLAG_FUSED_PRIOR | TOMO_FLAG_CONCURRENT_PRIOR))
    return fail(nullptr, TOMO_ERR_INVALID_ARG, "unknown flag bits 0x%x", g->flags);
  if (g->angles)
    for (int i = 0; i < g->n_angles; ++i)
      if (!std::isfinite(g->angles[i]))
        return fail(nullptr, TOMO_ERR_INVALID_ARG, "angle %d is not finite", i);
  if (!std::isnan(g->center) && !std::isfinite(g->center))
    return fail(nullptr, TOMO_ERR_INVALID_ARG, "center must be finite or NaN");
  return TOMO_OK;
}

}  // namespace

// ===================================================================================== ABI
extern "C" {

tomo_status tomo_plan_create(const tomo_geometry_t* geom, void* hip_stream, tomo_plan* out) {
  if (!out) return fail(nullptr, TOMO_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  tomo_status s = validate_geom(geom);
  if (s != TOMO_OK) return s;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0)
    return fail(nullptr, TOMO_ERR_NO_DEVICE, "no HIP device visible");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(nullptr, TOMO_ERR_NO_DEVICE, "hipGetDevice failed");
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return fail(nullptr, TOMO_ERR_HIP, "hipGetDeviceProperties failed");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(nullptr, TOMO_ERR_UNSUPPORTED_ARCH, "device arch %s is not gfx950", prop.gcnArchName);

  tomo_plan p = new tomo_plan_s();
  p->g = *geom;
  p->device = dev;
  p->stream = static_cast<hipStream_t>(hip_stream);
  p->nz = geom->n_slices;
  p->use_graphs = (geom->flags & TOMO_FLAG_NO_GRAPH) == 0;
  p->fused_prior = (geom->flags & TOMO_FLAG_FUSED_PRIOR) != 0;
  p->concurrent_prior = (geom->flags & TOMO_FLAG_CONCURRENT_PRIOR) != 0;
  p->n_levels = geom->n_levels == 0 ? 1 : geom->n_levels;
  if (p->g.kb_width == 0) p->g.kb_width = 6;
  if (p->g.kb_oversamp == 0.0) p->g.kb_oversamp = 2.0;
  p->angles.resize(geom->n_angles);
  for (int i = 0; i < geom->n_angles; ++i)
    p->angles[i] = geom->angles ? geom->angles[i] : i * M_PI / geom->n_angles;
  p->g.angles = nullptr;
  const double center = std::isnan(geom->center) ? geom->n_det / 2.0 : geom->center;

  const int L = p->n_levels;
  p->lv.resize(L);
  for (int l = 0; l < L; ++l) {
    Level& lv = p->lv[l];
    const int s = 1 << (L - 1 - l);
    lv.stride = s;
    lv.n = geom->n / s;
    lv.nd = geom->n_det / s;
    lv.c = center / s;
    lv.P = geom->pad ? geom->pad / s : next_pow2(2LL * lv.n);
    if (lv.P < kMinFft) lv.P = kMinFft;
    lv.M = next_pow2((long long)std::ceil(p->g.kb_oversamp * lv.n - 1e-9));
    if (lv.M < kMinFft) lv.M = kMinFft;
    lv.Mpsf = next_pow2((long long)std::ceil(p->g.kb_oversamp * 2 * lv.n - 1e-9));
    if (lv.Mpsf < kMinFft) lv.Mpsf = kMinFft;
    if (lv.P > kMaxHot || lv.M > kMaxGrid || lv.Mpsf > kMaxGrid) {
      delete p;
      return fail(nullptr, TOMO_ERR_INVALID_ARG, "sizes exceed the supported FFT range");
    }
    lv.beta_bp = geom->kb_beta > 0.0 ? geom->kb_beta
                                     : beatty_beta(p->g.kb_width, (double)lv.M / lv.n);
    lv.beta_psf = geom->kb_beta > 0.0 ? geom->kb_beta
                                      : beatty_beta(p->g.kb_width, (double)lv.Mpsf / (2.0 * lv.n));
  }

  // qGGMRF constants (q = 2)
  const double pe = geom->p, q = geom->q, sg = geom->sigma, T = geom->T;
  PriorParams& pp = p->pp;
  pp.beta = (float)geom->beta;
  pp.p = (float)pe;
  pp.qmp = (float)(q - pe);
  pp.q_over_p = (float)(q / pe);
  pp.inv_Tsigma = (float)(1.0 / (T * sg));
  pp.c_grad = (float)(std::pow(T * sg, pe - q) / std::pow(sg, pe));
  pp.c_val = (float)(std::pow(T * sg, pe) / (pe * std::pow(sg, pe)));
  pp.qm1 = (float)(q - 1.0);
  pp.lw0 = (float)((q - pe) * std::log2(1.0 / (T * sg)));
  pp.qop_m1 = (float)(q / pe - 1.0);
  pp.c_val2 = (float)(std::pow(T * sg, pe) / (pe * std::pow(sg, pe)) / ((T * sg) * (T * sg)));
  const double r1 = 1.0, r2 = 1.0 / std::sqrt(2.0), r3 = 1.0 / std::sqrt(3.0);
  const double sum = geom->neighbours == 26 ? 6 * r1 + 12 * r2 + 8 * r3 : 4 * r1 + 4 * r2;
  pp.wts[0] = 0.f;
  pp.wts[1] = (float)(r1 / sum);
  pp.wts[2] = (float)(r2 / sum);
  pp.wts[3] = (float)(r3 / sum);
  pp.neighbours = geom->neighbours;
  pp.quadratic = pe == q ? 1 : 0;
  ObjParams& op = p->op;
  op.beta = geom->beta;
  op.p = pe;
  op.qmp = q - pe;
  op.lw0 = (q - pe) * std::log2(1.0 / (T * sg));
  op.c_rho2 = 1.0 / (pe * std::pow(sg, pe) * std::pow(T * sg, 2.0 - pe));
  op.w1 = r1 / sum;
  op.w2 = r2 / sum;
  op.w3 = r3 / sum;
  op.neighbours = geom->neighbours;
  op.quadratic = pe == q ? 1 : 0;
  p->rho2_0 = pe == q ? 1.0 / (2.0 * sg * sg) : 2.0 / (pe * std::pow(T, 2.0 - pe) * sg * sg);

  layout(p);
  *out = p;
  return TOMO_OK;
}

tomo_status tomo_plan_workspace_size(tomo_plan p, size_t* bytes) {
  if (!p || !bytes) return fail(p, TOMO_ERR_INVALID_ARG, "NULL argument");
  *bytes = p->need;
  return TOMO_OK;
}

tomo_status tomo_plan_set_workspace(tomo_plan p, void* dev, size_t bytes) {
  if (!p || !dev) return fail(p, TOMO_ERR_INVALID_ARG, "NULL argument");
  if (!aligned(dev)) return fail(p, TOMO_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  if (bytes < p->need)
    return fail(p, TOMO_ERR_WORKSPACE_TOO_SMALL, "workspace %zu B < required %zu B", bytes, p->need);
  for (auto& g : p->graphs) (void)hipGraphExecDestroy(g.exec);  // captured with the old pointers
  p->graphs.clear();
  if (p->fstream) HIPCHK(p, hipStreamSynchronize(p->fstream));  // a PSF precompute may still write
  drop_psf_graphs(p);
  p->ws = static_cast<char*>(dev);
  p->ws_bytes = bytes;
  p->tables_ready = false;
  p->psf_ready = false;
  p->grids_ready = false;
  return TOMO_OK;
}

tomo_status tomo_precompute_psf(tomo_plan p) {
  if (!p) return fail(nullptr, TOMO_ERR_INVALID_ARG, "plan is NULL");
  tomo_status s = check_ws(p);
  if (s != TOMO_OK) return s;
  HIPCHK(p, hipSetDevice(p->device));
  if ((s = ensure_tables(p)) != TOMO_OK) return s;
  if ((s = ensure_grids(p)) != TOMO_OK) return s;
  if (!p->fstream) {
    HIPCHK(p, hipStreamCreateWithFlags(&p->fstream, hipStreamNonBlocking));
    HIPCHK(p, hipEventCreateWithFlags(&p->fev_fork, hipEventDisableTiming));
    HIPCHK(p, hipEventCreateWithFlags(&p->fev_done, hipEventDisableTiming));
  }
  p->psf_ready = false;
  p->psf_host = false;
  // after everything already enqueued on the plan's stream (tables, gridding lists, and any
  // earlier use of the spectrum this overwrites)
  HIPCHK(p, hipEventRecord(p->fev_fork, p->stream));
  HIPCHK(p, hipStreamWaitEvent(p->fstream, p->fev_fork, 0));
  for (int li = 0; li < p->n_levels; ++li) {
    const int ti = tbegin(p, TOMO_T_PSF, p->fstream);
    s = psf_level(p, p->lv[li], li);
    tend(p, ti, p->fstream);
    if (s != TOMO_OK) return s;
  }
  HIPCHK(p, hipEventRecord(p->fev_done, p->fstream));
  p->psf_ready = true;
  return TOMO_OK;
}

tomo_status tomo_backproject(tomo_plan p, const float* sino, float* out, int ramp) {
  if (!p || !sino || !out) return fail(p, TOMO_ERR_INVALID_ARG, "NULL argument");
  if (!aligned(sino) || !aligned(out)) return fail(p, TOMO_ERR_INVALID_ARG, "arrays must be 256-byte aligned");
  tomo_status s = check_ws(p);
  if (s != TOMO_OK) return s;
  HIPCHK(p, hipSetDevice(p->device));
  if ((s = ensure_tables(p)) != TOMO_OK) return s;
  return backproject_level(p, p->lv.back(), sino, out, ramp ? 1 : 0);
}

tomo_status tomo_apply_normal(tomo_plan p, const float* x, float* out) {
  if (!p || !x || !out) return fail(p, TOMO_ERR_INVALID_ARG, "NULL argument");
  if (!aligned(x) || !aligned(out)) return fail(p, TOMO_ERR_INVALID_ARG, "arrays must be 256-byte aligned");
  if (x == out) return fail(p, TOMO_ERR_INVALID_ARG, "x and out must be distinct");
  tomo_status s = check_ws(p);
  if (s != TOMO_OK) return s;
  if (!p->psf_ready) return fail(p, TOMO_ERR_NOT_READY, "PSF not precomputed");
  HIPCHK(p, hipSetDevice(p->device));
  if ((s = psf_join(p, p->stream)) != TOMO_OK) return s;
  HIPCHK(p, launch_set_scalars(p->scal(), SC_PSCALE, 1, nullptr, 1.0, p->stream));
  int nb = 0;
  return toeplitz_passes(p, p->lv.back(), MODE_POWER, p->nz, x, x, nullptr, out, false, &nb);
}

tomo_status tomo_gradient(tomo_plan p, const float* x, const float* b, float* grad,
                          double* obj_dev) {
  if (!p || !x || !b || !grad) return fail(p, TOMO_ERR_INVALID_ARG, "NULL argument");
  if (!aligned(x) || !aligned(b) || !aligned(grad))
    return fail(p, TOMO_ERR_INVALID_ARG, "arrays must be 256-byte aligned");
  if (grad == x || grad == b) return fail(p, TOMO_ERR_INVALID_ARG, "grad must not alias x or b");
  tomo_status s = check_ws(p);
  if (s != TOMO_OK) return s;
  if (!p->psf_ready) return fail(p, TOMO_ERR_NOT_READY, "PSF not precomputed");
  HIPCHK(p, hipSetDevice(p->device));
  if ((s = psf_join(p, p->stream)) != TOMO_OK) return s;
  int nb = 0, npr = 0;
  if ((s = toeplitz_passes(p, p->lv.back(), MODE_GRAD, p->nz, x, x, b, grad, obj_dev != nullptr,
                           &nb, &npr)) != TOMO_OK)
    return s;
  HIPCHK(p, launch_finalize(MODE_GRAD, p->partials(), nb, p->at<double>(p->off_ppartials), npr,
                            p->scal(), nullptr, nullptr, obj_dev, p->stream));
  return TOMO_OK;
}

tomo_status tomo_forward_project(tomo_plan p, const float* x, float* sino_out) {
  if (!p || !x || !sino_out) return fail(p, TOMO_ERR_INVALID_ARG, "NULL argument");
  if (!aligned(x) || !aligned(sino_out)) return fail(p, TOMO_ERR_INVALID_ARG, "arrays must be 256-byte aligned");
  tomo_status s = check_ws(p);
  if (s != TOMO_OK) return s;
  HIPCHK(p, hipSetDevice(p->device));
  return forward_project_impl(p, x, sino_out, nullptr, nullptr);
}

tomo_status tomo_gradient_direct(tomo_plan p, const float* x, const float* sino, float* grad,
                                 double* obj_dev) {
  if (!p || !x || !sino || !grad) return fail(p, TOMO_ERR_INVALID_ARG, "NULL argument");
  if (!aligned(x) || !aligned(sino) || !aligned(grad))
    return fail(p, TOMO_ERR_INVALID_ARG, "arrays must be 256-byte aligned");
  if (grad == x) return fail(p, TOMO_ERR_INVALID_ARG, "grad must not alias x");
  tomo_status s = check_ws(p);
  if (s != TOMO_OK) return s;
  HIPCHK(p, hipSetDevice(p->device));
  hipStream_t st = p->stream;
  const Level& l = p->lv.back();
  float* resid = p->at<float>(p->off_resid);
  double* rpart = p->at<double>(p->off_rpart);
  if ((s = forward_project_impl(p, x, resid, sino, rpart)) != TOMO_OK) return s;
  if ((s = backproject_level(p, l, resid, grad, 0)) != TOMO_OK) return s;
  float* gp = p->at<float>(p->off_gp);
  double* pp = p->at<double>(p->off_ppartials);
  HIPCHK(p, launch_prior(MODE_GRAD, p->g.neighbours, obj_dev != nullptr, x, x, p->scal(), gp, nullptr,
                         nullptr, pp, l.n, p->nz, p->pp, st));
  HIPCHK(p, launch_add(grad, gp, (idx_t)p->nz * l.n * l.n, st));
  if (obj_dev)
    HIPCHK(p, launch_direct_objective(rpart, radial_idft_blocks(l.nd, p->nz * p->g.n_angles), pp,
                                      prior_blocks(l.n, p->nz), p->g.beta, obj_dev, st));
  return TOMO_OK;
}

tomo_status tomo_reconstruct(tomo_plan p, const float* sino, float* x,
                             const tomo_recon_opts_t* opts, tomo_recon_stats_t* stats) {
  if (!p || !sino || !x || !opts || !opts->iters) return fail(p, TOMO_ERR_INVALID_ARG, "NULL argument");
  if (!aligned(sino) || !aligned(x)) return fail(p, TOMO_ERR_INVALID_ARG, "arrays must be 256-byte aligned");
  if (opts->init < TOMO_INIT_FBP || opts->init > TOMO_INIT_LEARNED)
    return fail(p, TOMO_ERR_INVALID_ARG, "unknown init");
  UnetView net;
  if (opts->init == TOMO_INIT_LEARNED) {
    if (!unet_view(opts->unet, &net)) return fail(p, TOMO_ERR_INVALID_ARG, "learned start without a network");
    if (!(opts->unet_scale > 0.f) || !std::isfinite(opts->unet_scale))
      return fail(p, TOMO_ERR_INVALID_ARG, "unet_scale must be > 0");
    if (!net.ready) return fail(p, TOMO_ERR_NOT_READY, "network has no workspace or parameters");
  }
  int learned_state = TOMO_LEARNED_NOT_REQUESTED;
  if (opts->L_override < 0.0 || !std::isfinite(opts->L_override))
    return fail(p, TOMO_ERR_INVALID_ARG, "L_override must be >= 0");
  for (int l = 0; l < p->n_levels; ++l)
    if (opts->iters[l] < 0) return fail(p, TOMO_ERR_INVALID_ARG, "iters must be >= 0");
  tomo_status s = check_ws(p);
  if (s != TOMO_OK) return s;
  HIPCHK(p, hipSetDevice(p->device));
  if ((s = ensure_tables(p)) != TOMO_OK) return s;
  if (!p->psf_ready && (s = tomo_precompute_psf(p)) != TOMO_OK) return s;
  hipStream_t st = p->stream;
  double* sc = p->scal();
  HIPCHK(p, launch_set_scalars(sc, SC_ITER, 1, nullptr, 0.0, st));
  HIPCHK(p, launch_set_scalars(sc, SC_NRESTART, 1, nullptr, 0.0, st));
  HIPCHK(p, launch_set_scalars(sc, SC_NONFINITE, 1, nullptr, -1.0, st));
  HIPCHK(p, launch_set_scalars(sc, SC_BETA, 1, nullptr, p->g.beta, st));
  HIPCHK(p, launch_set_scalars(sc, SC_RESTART_ON, 1, nullptr, opts->restart ? 1.0 : 0.0, st));

  int cur = 0;  // buffer holding the current iterate
  for (int li = 0; li < p->n_levels; ++li) {
    const Level& l = p->lv[li];
    const size_t vol = (size_t)p->nz * l.n * l.n;
    float* b = p->at<float>(l.off_b);
    const bool fbp = li == 0 && (opts->init == TOMO_INIT_FBP || opts->init == TOMO_INIT_LEARNED);
    if (fbp) s = backproject_level_dual(p, l, sino, b, p->xbuf(cur));  // b and the FBP start
    else s = backproject_level(p, l, sino, b, 0);
    if (s != TOMO_OK) return s;
    HIPCHK(p, launch_sumsq_strided(sino, (idx_t)p->nz * p->g.n_angles, l.nd, l.stride,
                                   1.0 / l.stride, p->partials(), sc + SC_GG, st));
    if (li == 0) {
      if (fbp) {
        if (opts->init == TOMO_INIT_LEARNED) {
          learned_state = in_domain(p, l, net) ? TOMO_LEARNED_TESTED : TOMO_LEARNED_OUT_OF_DOMAIN;
          if (learned_state == TOMO_LEARNED_TESTED &&
              ((s = psf_join(p, st)) != TOMO_OK || (s = learned_start(p, l, b, cur, net, opts)) != TOMO_OK))
            return s;
        }
      } else if (opts->init == TOMO_INIT_ZERO) {
        HIPCHK(p, launch_fill(p->xbuf(cur), (idx_t)vol, 0.0f, st));
      } else {
        HIPCHK(p, hipMemcpyAsync(p->xbuf(cur), x, vol * sizeof(float), hipMemcpyDeviceToDevice, st));
      }
    } else {
      const int nxt = (cur + 1) % 3;
      HIPCHK(p, launch_lanczos_prolong(p->xbuf(cur), p->xbuf(nxt), p->lv[li - 1].n, p->nz, st));
      cur = nxt;
    }
    // the iterations need the level's PSF spectrum and 1 / L: wait for the PSF stream here, so
    // that the back-projections above overlap the precompute
    if ((s = psf_join(p, st)) != TOMO_OK) return s;
    HIPCHK(p, launch_set_scalars(sc, SC_MU, 1, nullptr, 0.0, st));
    HIPCHK(p, launch_set_scalars(sc, SC_T, 1, nullptr, 1.0, st));
    if (opts->L_override > 0.0)
      HIPCHK(p, launch_set_scalars(sc, SC_INVL, 1, nullptr, 1.0 / opts->L_override, st));
    else
      HIPCHK(p, launch_set_scalars(sc, SC_INVL, 1, p->at<double>(p->off_lvl) + 3 * (size_t)li + 2,
                                   0.0, st));
    int ik = cur, ikm1 = cur, inext = (cur + 1) % 3;
    const int n_it = opts->iters[li];
    // Graph replay of 3-iteration blocks once the buffer rotation is periodic; the events
    // order the internal stream after everything already enqueued on the plan's stream.
    const bool graphs = p->use_graphs && p->tmask == 0 && n_it >= 7;
    int k = 0;
    while (k < n_it) {
      if (graphs && k >= 1 && n_it - k >= 3) {
        hipGraphExec_t exec = nullptr;
        if ((s = get_graph(p, li, ik, ikm1, inext, b, opts->objective_dev, opts->restart_dev,
                           &exec)) != TOMO_OK)
          return s;
        HIPCHK(p, hipEventRecord(p->gev_in, st));
        HIPCHK(p, hipStreamWaitEvent(p->gstream, p->gev_in, 0));
        while (n_it - k >= 3) {
          HIPCHK(p, hipGraphLaunch(exec, p->gstream));
          k += 3;
        }
        HIPCHK(p, hipEventRecord(p->gev_out, p->gstream));
        HIPCHK(p, hipStreamWaitEvent(st, p->gev_out, 0));
        continue;  // three iterations restore the buffer assignment
      }
      if ((s = fista_iteration(p, l, ik, ikm1, inext, b, opts->objective_dev, opts->restart_dev,
                               st)) != TOMO_OK)
        return s;
      // x_{k-1} <- x_k, x_k <- x_{k+1}; the freed buffer receives the next iterate
      ikm1 = ik;
      ik = inext;
      inext = 3 - ik - ikm1;
      ++k;
    }
    cur = ik;
  }
  const size_t vol = (size_t)p->nz * p->lv.back().n * p->lv.back().n;
  HIPCHK(p, hipMemcpyAsync(x, p->xbuf(cur), vol * sizeof(float), hipMemcpyDeviceToDevice, st));
  if (stats) {
    double sv[SC_COUNT];
    HIPCHK(p, hipMemcpyAsync(sv, sc, sizeof sv, hipMemcpyDeviceToHost, st));
    HIPCHK(p, hipStreamSynchronize(st));
    if ((s = psf_host_values(p)) != TOMO_OK) return s;
    std::memset(stats, 0, sizeof *stats);
    for (int l = 0; l < p->n_levels && l < 6; ++l) {
      stats->L[l] = opts->L_override > 0.0 ? opts->L_override : p->lv[l].L;
      stats->lambda_pow[l] = p->lv[l].lambda;
    }
    stats->n_restarts = (int32_t)sv[SC_NRESTART];
    stats->nonfinite_iter = (int32_t)sv[SC_NONFINITE];
    stats->learned_state = learned_state;
    stats->learned_slices = 0;
    if (learned_state == TOMO_LEARNED_TESTED) {
      std::vector<int32_t> ch((size_t)p->nz);
      HIPCHK(p, hipMemcpy(ch.data(), p->at<int32_t>(p->off_choice), ch.size() * sizeof(int32_t),
                          hipMemcpyDeviceToHost));
      for (int32_t c : ch) stats->learned_slices += c;
    }
    if (stats->nonfinite_iter >= 0)
      return fail(p, TOMO_ERR_NONFINITE, "non-finite value at iteration %d", stats->nonfinite_iter);
  }
  return TOMO_OK;
}

tomo_status tomo_psf_info(tomo_plan p, int32_t level, float* fk_dev, double* L_host,
                          double* lambda_host) {
  if (!p || level < 0 || level >= p->n_levels) return fail(p, TOMO_ERR_INVALID_ARG, "bad level");
  if (!p->psf_ready) return fail(p, TOMO_ERR_NOT_READY, "PSF not precomputed");
  const Level& l = p->lv[level];
  tomo_status s = TOMO_OK;
  if (fk_dev) {
    HIPCHK(p, hipSetDevice(p->device));
    if ((s = psf_join(p, p->stream)) != TOMO_OK) return s;
    HIPCHK(p, launch_fk_export(p->at<float>(l.off_fk), p->at<float>(l.off_fkn), fk_dev, l.P,
                               p->stream));
  }
  if ((L_host || lambda_host) && (s = psf_host_values(p)) != TOMO_OK) return s;
  if (L_host) *L_host = l.L;
  if (lambda_host) *lambda_host = l.lambda;
  return TOMO_OK;
}

tomo_status tomo_plan_geometry(tomo_plan p, tomo_geometry_t* geom, void** hip_stream,
                               int32_t* device) {
  if (!p) return fail(nullptr, TOMO_ERR_INVALID_ARG, "plan is NULL");
  if (geom) *geom = p->g;
  if (hip_stream) *hip_stream = p->stream;
  if (device) *device = p->device;
  return TOMO_OK;
}

tomo_status tomo_level_dims(tomo_plan p, int32_t level, int32_t* n, int32_t* n_det, int32_t* pad) {
  if (!p || level < 0 || level >= p->n_levels) return fail(p, TOMO_ERR_INVALID_ARG, "bad level");
  const Level& l = p->lv[level];
  if (n) *n = l.n;
  if (n_det) *n_det = l.nd;
  if (pad) *pad = l.P;
  return TOMO_OK;
}

tomo_status tomo_lanczos_prolong(const float* in, float* out, int32_t n, int32_t n_slices,
                                 void* hip_stream) {
  if (!in || !out || n < 1 || n_slices < 1) return fail(nullptr, TOMO_ERR_INVALID_ARG, "bad argument");
  hipError_t e = launch_lanczos_prolong(in, out, n, n_slices, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return fail(nullptr, TOMO_ERR_HIP, "prolongation launch: %s", hipGetErrorString(e));
  return TOMO_OK;
}

// ============================================================================== batches
}  // extern "C"

struct tomo_batch_s {
  std::vector<tomo_plan> plans;
  hipStream_t stream = nullptr;
  int device = 0, grid = 0, grid_fused = 0;
  bool fused = false;          // 8-neighbour problems take the prior inside pass R'
  bool phases = false;         // one launch per phase and size (and a finalize launch)
  std::vector<int4> segs;      // work-list segments of one phase and transform size
  std::vector<BatchProb> probs;
  std::vector<int2> items;
  std::vector<int> order;      // problems by decreasing FFT size (queue order within a phase)
  std::vector<int> sizes;      // distinct FFT sizes, increasing
  std::vector<int> size_el;    // elements per thread chosen for each size
  std::vector<int> size_grp;   // tiles per queue item chosen for each size
  size_t items_cap = 0;        // items the workspace holds (every size at 8 elements per thread)
  char* ws = nullptr;
  size_t need = 0, off_probs = 0, off_items = 0, off_ctl = 0, off_cnt = 0;
  hipStream_t gstream = nullptr;
  hipEvent_t gev_in = nullptr, gev_out = nullptr;
  hipGraphExec_t gexec = nullptr;
  int graph_rot = -1;
  std::string err;
};

namespace {

tomo_status bfail(tomo_batch b, tomo_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (b) b->err = buf;
  g_last_error = buf;
  return s;
}

#define BHIPCHK(b, call)                                                                 \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return bfail(b, TOMO_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_));      \
  } while (0)

// Per-problem setup on the batch stream: PSF (if needed), b, FBP start, scalars.
tomo_status batch_prepare(tomo_batch bt, int j, const float* sino, int restart) {
  tomo_plan p = bt->plans[j];
  hipStream_t keep = p->stream;
  p->stream = bt->stream;
  tomo_status s = ensure_tables(p);
  if (s == TOMO_OK && !p->psf_ready) s = tomo_precompute_psf(p);
  const Level& l = p->lv[0];
  if (s == TOMO_OK) s = backproject_level(p, l, sino, p->at<float>(l.off_b), 0);
  if (s == TOMO_OK) s = backproject_level(p, l, sino, p->xbuf(0), 1, true);
  hipStream_t st = bt->stream;
  if (s == TOMO_OK) s = psf_join(p, st);
  double* sc = p->scal();
  hipError_t e = hipSuccess;
  if (s == TOMO_OK) {
    e = launch_sumsq_strided(sino, (idx_t)p->nz * p->g.n_angles, l.nd, 1, 1.0, p->partials(),
                             sc + SC_GG, st);
    if (e == hipSuccess) e = launch_set_scalars(sc, SC_MU, 1, nullptr, 0.0, st);
    if (e == hipSuccess) e = launch_set_scalars(sc, SC_T, 1, nullptr, 1.0, st);
    if (e == hipSuccess)
      e = launch_set_scalars(sc, SC_INVL, 1, p->at<double>(p->off_lvl) + 2, 0.0, st);
    if (e == hipSuccess) e = launch_set_scalars(sc, SC_RESTART_ON, 1, nullptr, restart ? 1.0 : 0.0, st);
    if (e == hipSuccess) e = launch_set_scalars(sc, SC_ITER, 1, nullptr, 0.0, st);
    if (e == hipSuccess) e = launch_set_scalars(sc, SC_NRESTART, 1, nullptr, 0.0, st);
    if (e == hipSuccess) e = launch_set_scalars(sc, SC_NONFINITE, 1, nullptr, -1.0, st);
    if (e != hipSuccess) s = bfail(bt, TOMO_ERR_HIP, "batch setup launch: %s", hipGetErrorString(e));
  } else {
    bfail(bt, s, "problem %d: %s", j, p->err.c_str());
  }
  p->stream = keep;
  return s;
}

// Tile counts and the phase-ordered work list for the current per-size schedule.
void batch_build_items(tomo_batch b) {
  const int n = (int)b->plans.size();
  for (int j = 0; j < n; ++j) {
    BatchProb& d = b->probs[j];
    const size_t si = std::lower_bound(b->sizes.begin(), b->sizes.end(), d.P) - b->sizes.begin();
    d.el = b->size_el[si];
    d.fused = b->fused && d.neighbours == 8 ? 1 : 0;
    d.grp = b->phases ? 1 : b->size_grp[si];  // one launch per phase: one tile per item
    batch_tile_counts(d.N, d.P, d.nz, d.el, &d.nPr, &d.nR, &d.nC, &d.nRp);
    if (d.fused) d.nPr = 0;
    d.iR = (d.nR + d.grp - 1) / d.grp;
    d.iC = (d.nC + d.grp - 1) / d.grp;
    d.iRp = (d.nRp + d.grp - 1) / d.grp;
  }
  b->items.clear();
  b->segs.clear();
  for (int ph = 0; ph < 4; ++ph)
    for (int j : b->order) {  // decreasing transform size: each size is one segment
      const BatchProb& d = b->probs[j];
      const int cntp = ph == 0 ? d.nPr : ph == 1 ? d.iR : ph == 2 ? d.iC : d.iRp;
      const int key = ph == 0 ? 0 : (d.P | (d.el << 16));
      if (b->segs.empty() || b->segs.back().x != ph || b->segs.back().y != key)
        b->segs.push_back(make_int4(ph, key, (int)b->items.size(), 0));
      for (int t = 0; t < cntp; ++t) b->items.push_back(make_int2(j | (ph << 24), t));
      b->segs.back().w += cntp;
    }
}

// Copy the work list and the problem descriptors (whose tile counts and element choice must
// match the list) to the workspace; a captured graph holds the old item count.
tomo_status batch_upload_items(tomo_batch b) {
  if (b->items.size() > b->items_cap) return bfail(b, TOMO_ERR_INTERNAL, "work list exceeds its capacity");
  BHIPCHK(b, hipMemcpyAsync(b->ws + b->off_items, b->items.data(), b->items.size() * sizeof(int2),
                            hipMemcpyHostToDevice, b->stream));
  BHIPCHK(b, hipMemcpyAsync(b->ws + b->off_probs, b->probs.data(), b->probs.size() * sizeof(BatchProb),
                            hipMemcpyHostToDevice, b->stream));
  // the host vectors are rebuilt by the next schedule change: finish the copies first
  BHIPCHK(b, hipStreamSynchronize(b->stream));
  if (b->gexec) {
    (void)hipGraphExecDestroy(b->gexec);
    b->gexec = nullptr;
  }
  return TOMO_OK;
}

// Device pointers of every problem (its plan's workspace).
void batch_fill_descriptors(tomo_batch b) {
  for (size_t j = 0; j < b->plans.size(); ++j) {
    tomo_plan p = b->plans[j];
    const Level& l = p->lv[0];
    BatchProb& d = b->probs[j];
    for (int i = 0; i < 3; ++i) d.x[i] = p->xbuf(i);
    d.y = p->at<float>(p->off_y);
    d.gp = p->at<float>(p->off_gp);
    d.b = p->at<float>(l.off_b);
    d.fk = p->at<float>(l.off_fk);
    d.fkn = p->at<float>(l.off_fkn);
    d.S1 = p->S1();
    d.S2 = p->S2(l);
    d.partials = p->partials();
    d.scal = p->scal();
    d.tw = p->tw32(l.P);
    d.hist = nullptr;
    d.rhist = nullptr;
    d.pp = p->pp;
  }
}

tomo_status batch_launch(tomo_batch bt, int ik, int ikm1, int inext, hipStream_t st);

// Mean time of one batched iteration over `reps` launches (after one warm-up) with the current
// schedule, on state prepared by tomo_batch_autotune.
tomo_status batch_time(tomo_batch b, int reps, hipEvent_t e0, hipEvent_t e1, float* ms) {
  hipStream_t st = b->stream;
  const int n = (int)b->plans.size();
  BHIPCHK(b, launch_fill_int(reinterpret_cast<int*>(b->ws + b->off_ctl), 4, 0, st));
  BHIPCHK(b, launch_fill_int(reinterpret_cast<int*>(b->ws + b->off_cnt), 4 * (idx_t)n, 0, st));
  int ik = 0, ikm1 = 0, inext = 1;
  for (int r = -1; r < reps; ++r) {
    if (r == 0) BHIPCHK(b, hipEventRecord(e0, st));
    if (tomo_status s = batch_launch(b, ik, ikm1, inext, st); s != TOMO_OK) return s;
    ikm1 = ik;
    ik = inext;
    inext = 3 - ik - ikm1;
  }
  BHIPCHK(b, hipEventRecord(e1, st));
  BHIPCHK(b, hipEventSynchronize(e1));
  float t = 0.f;
  BHIPCHK(b, hipEventElapsedTime(&t, e0, e1));
  int ctl[4];
  BHIPCHK(b, hipMemcpy(ctl, b->ws + b->off_ctl, sizeof ctl, hipMemcpyDeviceToHost));
  if (ctl[2]) return bfail(b, TOMO_ERR_INTERNAL, "a tile wait timed out while timing");
  *ms = t / (float)reps;
  return TOMO_OK;
}

void batch_report(tomo_batch b, tomo_batch_schedule_t* out) {
  std::memset(out, 0, sizeof *out);
  out->n_sizes = (int32_t)b->sizes.size();
  out->fused_prior = b->fused ? 1 : 0;
  out->phase_launches = b->phases ? 1 : 0;
  for (size_t i = 0; i < b->sizes.size() && i < TOMO_BATCH_MAX_SIZES; ++i) {
    out->pad[i] = b->sizes[i];
    out->elems[i] = b->size_el[i];
    out->group[i] = b->phases ? 1 : b->size_grp[i];
  }
}

tomo_status batch_launch(tomo_batch bt, int ik, int ikm1, int inext, hipStream_t st) {
  const int nprob = (int)bt->plans.size();
  if (bt->phases) {
    BHIPCHK(bt, launch_batch_phases(bt->fused, reinterpret_cast<const BatchProb*>(bt->ws + bt->off_probs),
                                    reinterpret_cast<const int2*>(bt->ws + bt->off_items), bt->segs.data(),
                                    (int)bt->segs.size(), nprob, ik, ikm1, inext, st));
    return TOMO_OK;
  }
  BHIPCHK(bt, launch_batch_iteration(bt->fused, reinterpret_cast<const BatchProb*>(bt->ws + bt->off_probs),
                                     reinterpret_cast<const int2*>(bt->ws + bt->off_items),
                                     (int)bt->items.size(), reinterpret_cast<int*>(bt->ws + bt->off_ctl),
                                     reinterpret_cast<int*>(bt->ws + bt->off_cnt), nprob, ik, ikm1,
                                     inext, bt->fused ? bt->grid_fused : bt->grid, st));
  return TOMO_OK;
}

}  // namespace

extern "C" {

tomo_status tomo_batch_create(const tomo_plan* plans, int32_t n, void* hip_stream, tomo_batch* out) {
  if (!out) return bfail(nullptr, TOMO_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!plans || n < 1 || n > (1 << 20)) return bfail(nullptr, TOMO_ERR_INVALID_ARG, "need 1..2^20 plans");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return bfail(nullptr, TOMO_ERR_NO_DEVICE, "hipGetDevice failed");
  for (int j = 0; j < n; ++j) {
    tomo_plan p = plans[j];
    if (!p) return bfail(nullptr, TOMO_ERR_INVALID_ARG, "plan %d is NULL", j);
    if (p->n_levels != 1) return bfail(nullptr, TOMO_ERR_INVALID_ARG, "plan %d has several levels", j);
    if (!p->ws) return bfail(nullptr, TOMO_ERR_INVALID_ARG, "plan %d has no workspace", j);
    if (!batch_supports(p->lv[0].P))
      return bfail(nullptr, TOMO_ERR_INVALID_ARG, "plan %d: FFT size %d outside 256..2048", j, p->lv[0].P);
    if (p->device != dev) return bfail(nullptr, TOMO_ERR_INVALID_ARG, "plan %d is on another device", j);
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return bfail(nullptr, TOMO_ERR_HIP, "hipGetDeviceProperties failed");
  tomo_batch b = new tomo_batch_s();
  b->plans.assign(plans, plans + n);
  b->stream = static_cast<hipStream_t>(hip_stream);
  b->device = dev;
  // every resident 256-thread block takes tiles until the queue is empty
  b->grid = prop.multiProcessorCount * batch_blocks_per_cu(false);
  b->grid_fused = prop.multiProcessorCount * batch_blocks_per_cu(true);
  // work list: all prior tiles, then pass R, pass C and pass R'; larger transforms first
  b->order.resize(n);
  for (int j = 0; j < n; ++j) b->order[j] = j;
  std::stable_sort(b->order.begin(), b->order.end(),
                   [&](int a, int c) { return plans[a]->lv[0].P > plans[c]->lv[0].P; });
  b->probs.resize(n);
  for (int j = 0; j < n; ++j) {
    const Level& l = plans[j]->lv[0];
    BatchProb& d = b->probs[j];
    std::memset(&d, 0, sizeof d);
    d.N = l.n;
    d.P = l.P;
    d.nz = plans[j]->nz;
    d.neighbours = plans[j]->g.neighbours;
    b->sizes.push_back(l.P);
  }
  std::sort(b->sizes.begin(), b->sizes.end());
  b->sizes.erase(std::unique(b->sizes.begin(), b->sizes.end()), b->sizes.end());
  // capacity: 8 elements per thread and one tile per item give the most items
  b->size_el.assign(b->sizes.size(), 8);
  b->size_grp.assign(b->sizes.size(), 1);
  batch_build_items(b);
  b->items_cap = b->items.size();
  b->size_el.assign(b->sizes.size(), 16);
  b->size_grp.assign(b->sizes.size(), kBatchDefaultGroup);
  batch_build_items(b);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align_up(bytes);
    return o;
  };
  b->off_probs = take(n * sizeof(BatchProb));
  b->off_items = take(b->items_cap * sizeof(int2));
  b->off_ctl = take(4 * sizeof(int));
  b->off_cnt = take(4 * (size_t)n * sizeof(int));
  b->need = off;
  *out = b;
  return TOMO_OK;
}

tomo_status tomo_batch_workspace_size(tomo_batch b, size_t* bytes) {
  if (!b || !bytes) return bfail(b, TOMO_ERR_INVALID_ARG, "NULL argument");
  *bytes = b->need;
  return TOMO_OK;
}

tomo_status tomo_batch_set_workspace(tomo_batch b, void* dev, size_t bytes) {
  if (!b || !dev) return bfail(b, TOMO_ERR_INVALID_ARG, "NULL argument");
  if (!aligned(dev)) return bfail(b, TOMO_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  if (bytes < b->need) return bfail(b, TOMO_ERR_WORKSPACE_TOO_SMALL, "workspace too small");
  if (b->gexec) {
    (void)hipGraphExecDestroy(b->gexec);
    b->gexec = nullptr;
  }
  b->ws = static_cast<char*>(dev);
  if (tomo_status s = batch_upload_items(b); s != TOMO_OK) return s;
  BHIPCHK(b, launch_fill_int(reinterpret_cast<int*>(b->ws + b->off_ctl), 4, 0, b->stream));
  BHIPCHK(b, launch_fill_int(reinterpret_cast<int*>(b->ws + b->off_cnt), 4 * (idx_t)b->plans.size(), 0,
                             b->stream));
  BHIPCHK(b, hipStreamSynchronize(b->stream));
  return TOMO_OK;
}

tomo_status tomo_batch_reconstruct(tomo_batch b, const float* const* sinos, float* const* xs,
                                   int32_t iters, int32_t restart, tomo_batch_stats_t* stats) {
  if (!b || !sinos || !xs || iters < 0) return bfail(b, TOMO_ERR_INVALID_ARG, "bad argument");
  if (!b->ws) return bfail(b, TOMO_ERR_NO_WORKSPACE, "no workspace attached");
  const int n = (int)b->plans.size();
  for (int j = 0; j < n; ++j)
    if (!sinos[j] || !xs[j] || !aligned(sinos[j]) || !aligned(xs[j]))
      return bfail(b, TOMO_ERR_INVALID_ARG, "problem %d: NULL or misaligned array", j);
  BHIPCHK(b, hipSetDevice(b->device));
  tomo_status s;
  for (int j = 0; j < n; ++j)
    if ((s = batch_prepare(b, j, sinos[j], restart)) != TOMO_OK) return s;
  batch_fill_descriptors(b);
  hipStream_t st = b->stream;
  BHIPCHK(b, hipMemcpyAsync(b->ws + b->off_probs, b->probs.data(), n * sizeof(BatchProb),
                            hipMemcpyHostToDevice, st));
  BHIPCHK(b, launch_fill_int(reinterpret_cast<int*>(b->ws + b->off_ctl), 4, 0, st));
  BHIPCHK(b, launch_fill_int(reinterpret_cast<int*>(b->ws + b->off_cnt), 4 * (idx_t)n, 0, st));
  int ik = 0, ikm1 = 0, inext = 1, k = 0;
  while (k < iters) {
    if (k >= 1 && iters - k >= 3) {
      // steady rotation: replay a captured graph of three persistent launches
      const int rot = ik * 9 + ikm1 * 3 + inext;
      if (!b->gstream) {
        BHIPCHK(b, hipStreamCreateWithFlags(&b->gstream, hipStreamNonBlocking));
        BHIPCHK(b, hipEventCreateWithFlags(&b->gev_in, hipEventDisableTiming));
        BHIPCHK(b, hipEventCreateWithFlags(&b->gev_out, hipEventDisableTiming));
      }
      if (!b->gexec || b->graph_rot != rot) {
        if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
        b->gexec = nullptr;
        hipGraph_t g = nullptr;
        BHIPCHK(b, hipStreamBeginCapture(b->gstream, hipStreamCaptureModeRelaxed));
        int a = ik, c = ikm1, d = inext;
        for (int r = 0; r < 3; ++r) {
          s = batch_launch(b, a, c, d, b->gstream);
          if (s != TOMO_OK) break;
          c = a;
          a = d;
          d = 3 - a - c;
        }
        const hipError_t e = hipStreamEndCapture(b->gstream, &g);
        if (s != TOMO_OK) {
          if (g) (void)hipGraphDestroy(g);
          return s;
        }
        if (e != hipSuccess) return bfail(b, TOMO_ERR_HIP, "batch graph capture: %s", hipGetErrorString(e));
        const hipError_t e2 = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e2 != hipSuccess) return bfail(b, TOMO_ERR_HIP, "batch graph instantiate: %s", hipGetErrorString(e2));
        b->graph_rot = rot;
      }
      BHIPCHK(b, hipEventRecord(b->gev_in, st));
      BHIPCHK(b, hipStreamWaitEvent(b->gstream, b->gev_in, 0));
      while (iters - k >= 3) {
        BHIPCHK(b, hipGraphLaunch(b->gexec, b->gstream));
        k += 3;
      }
      BHIPCHK(b, hipEventRecord(b->gev_out, b->gstream));
      BHIPCHK(b, hipStreamWaitEvent(st, b->gev_out, 0));
      continue;
    }
    if ((s = batch_launch(b, ik, ikm1, inext, st)) != TOMO_OK) return s;
    ikm1 = ik;
    ik = inext;
    inext = 3 - ik - ikm1;
    ++k;
  }
  for (int j = 0; j < n; ++j) {
    tomo_plan p = b->plans[j];
    const size_t vol = (size_t)p->nz * p->lv[0].n * p->lv[0].n;
    BHIPCHK(b, hipMemcpyAsync(xs[j], p->xbuf(ik), vol * sizeof(float), hipMemcpyDeviceToDevice, st));
  }
  if (stats) {
    std::memset(stats, 0, sizeof *stats);
    int ctl[4];
    BHIPCHK(b, hipMemcpyAsync(ctl, b->ws + b->off_ctl, sizeof ctl, hipMemcpyDeviceToHost, st));
    std::vector<double> sv((size_t)n * SC_COUNT);
    for (int j = 0; j < n; ++j)
      BHIPCHK(b, hipMemcpyAsync(&sv[(size_t)j * SC_COUNT], b->plans[j]->scal(), SC_COUNT * sizeof(double),
                                hipMemcpyDeviceToHost, st));
    BHIPCHK(b, hipStreamSynchronize(st));
    for (int j = 0; j < n; ++j) {
      stats->n_restarts += (int32_t)sv[(size_t)j * SC_COUNT + SC_NRESTART];
      if (sv[(size_t)j * SC_COUNT + SC_NONFINITE] >= 0.0) stats->n_nonfinite += 1;
    }
    stats->wait_timeouts = ctl[2] != 0;
    if (stats->wait_timeouts) return bfail(b, TOMO_ERR_INTERNAL, "a batch tile gave up waiting");
    if (stats->n_nonfinite) return bfail(b, TOMO_ERR_NONFINITE, "%d problems went non-finite", stats->n_nonfinite);
  }
  return TOMO_OK;
}

tomo_status tomo_batch_schedule(tomo_batch b, const tomo_batch_schedule_t* set,
                                tomo_batch_schedule_t* out) {
  if (!b) return bfail(b, TOMO_ERR_INVALID_ARG, "batch is NULL");
  if (set) {
    // earlier asynchronous copies may still read the host descriptors rebuilt below
    if (b->ws) BHIPCHK(b, hipStreamSynchronize(b->stream));
    if (set->fused_prior != 0 && set->fused_prior != 1)
      return bfail(b, TOMO_ERR_INVALID_ARG, "fused_prior must be 0 or 1");
    if (set->phase_launches != 0 && set->phase_launches != 1)
      return bfail(b, TOMO_ERR_INVALID_ARG, "phase_launches must be 0 or 1");
    std::vector<int> el = b->size_el, grp = b->size_grp;
    for (int i = 0; i < set->n_sizes && i < TOMO_BATCH_MAX_SIZES; ++i) {
      const auto it = std::find(b->sizes.begin(), b->sizes.end(), set->pad[i]);
      if (it == b->sizes.end()) return bfail(b, TOMO_ERR_INVALID_ARG, "no problem with FFT size %d", set->pad[i]);
      if (set->elems[i] != 8 && set->elems[i] != 16)
        return bfail(b, TOMO_ERR_INVALID_ARG, "elements per thread must be 8 or 16");
      if (set->group[i] < 1 || set->group[i] > kBatchMaxGroup)
        return bfail(b, TOMO_ERR_INVALID_ARG, "tiles per item must be in 1..%d", kBatchMaxGroup);
      el[it - b->sizes.begin()] = set->elems[i];
      grp[it - b->sizes.begin()] = set->group[i];
    }
    b->size_el = el;
    b->size_grp = grp;
    b->fused = set->fused_prior == 1;
    b->phases = set->phase_launches == 1;
    batch_build_items(b);
    if (b->ws) {
      BHIPCHK(b, hipSetDevice(b->device));
      if (tomo_status s = batch_upload_items(b); s != TOMO_OK) return s;
    }
  }
  if (out) batch_report(b, out);
  return TOMO_OK;
}

tomo_status tomo_batch_autotune(tomo_batch b, int32_t reps, tomo_batch_schedule_t* out) {
  if (!b) return bfail(b, TOMO_ERR_INVALID_ARG, "batch is NULL");
  if (!b->ws) return bfail(b, TOMO_ERR_NO_WORKSPACE, "no workspace attached");
  if (reps <= 0) reps = 5;
  BHIPCHK(b, hipSetDevice(b->device));
  hipStream_t st = b->stream;
  BHIPCHK(b, hipStreamSynchronize(st));  // earlier copies may still read the host descriptors
  // state to iterate on: tables and PSF of every problem, zero iterates, b and prior buffers
  for (tomo_plan p : b->plans) {
    hipStream_t keep = p->stream;
    p->stream = st;
    tomo_status s = ensure_tables(p);
    if (s == TOMO_OK && !p->psf_ready) s = tomo_precompute_psf(p);
    p->stream = keep;
    if (s == TOMO_OK) s = psf_join(p, st);
    if (s != TOMO_OK) return bfail(b, s, "autotune setup: %s", p->err.c_str());
    const Level& l = p->lv[0];
    const idx_t vol = (idx_t)p->nz * l.n * l.n;
    float* bufs[6] = {p->xbuf(0), p->xbuf(1), p->xbuf(2), p->at<float>(p->off_y),
                      p->at<float>(p->off_gp), p->at<float>(l.off_b)};
    for (float* f : bufs) BHIPCHK(b, launch_fill(f, vol, 0.0f, st));
    double* sc = p->scal();
    BHIPCHK(b, launch_set_scalars(sc, 0, SC_COUNT, nullptr, 0.0, st));
    BHIPCHK(b, launch_set_scalars(sc, SC_T, 1, nullptr, 1.0, st));
    BHIPCHK(b, launch_set_scalars(sc, SC_INVL, 1, p->at<double>(p->off_lvl) + 2, 0.0, st));
    BHIPCHK(b, launch_set_scalars(sc, SC_NONFINITE, 1, nullptr, -1.0, st));
  }
  batch_fill_descriptors(b);
  BHIPCHK(b, hipMemcpyAsync(b->ws + b->off_probs, b->probs.data(), b->plans.size() * sizeof(BatchProb),
                            hipMemcpyHostToDevice, st));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  BHIPCHK(b, hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return bfail(b, TOMO_ERR_HIP, "hipEventCreate failed");
  }
  // coordinate descent: the prior scheme first (the pair-shared prior phase, or for
  // 8-neighbour problems the prior inside pass R'), then one size at a time 8 instead of 16
  // elements per thread, each change kept where the whole batched iteration gets at least 3%
  // faster
  tomo_status s = TOMO_OK;
  float best = 0.f, base = 0.f;
  b->size_el.assign(b->sizes.size(), 16);
  b->size_grp.assign(b->sizes.size(), kBatchDefaultGroup);
  b->fused = false;
  b->phases = false;
  batch_build_items(b);
  s = batch_upload_items(b);
  if (s == TOMO_OK) s = batch_time(b, reps, e0, e1, &best);
  base = best;
  bool any8 = false;
  for (tomo_plan p : b->plans) any8 = any8 || p->g.neighbours == 8;
  if (s == TOMO_OK && any8) {
    b->fused = true;
    batch_build_items(b);
    float t = 0.f;
    s = batch_upload_items(b);
    if (s == TOMO_OK) s = batch_time(b, reps, e0, e1, &t);
    if (s == TOMO_OK && t < 0.97f * best) best = t;
    else b->fused = false;
  }
  // one launch per phase (one tile per block) instead of the persistent queue
  if (s == TOMO_OK) {
    const std::vector<int> prev = b->size_grp;
    b->phases = true;
    b->size_grp.assign(b->sizes.size(), 1);
    batch_build_items(b);
    float t = 0.f;
    s = batch_upload_items(b);
    if (s == TOMO_OK) s = batch_time(b, reps, e0, e1, &t);
    if (s == TOMO_OK && t < 0.97f * best) {
      best = t;
    } else {
      b->phases = false;
      b->size_grp = prev;
    }
  }
  // with one launch per phase, the prior scheme again
  if (s == TOMO_OK && b->phases && any8) {
    b->fused = !b->fused;
    batch_build_items(b);
    float t = 0.f;
    s = batch_upload_items(b);
    if (s == TOMO_OK) s = batch_time(b, reps, e0, e1, &t);
    if (s == TOMO_OK && t < 0.97f * best) best = t;
    else b->fused = !b->fused;
  }
  // tiles per queue item: the same for every size first, then each size halved or doubled
  auto try_groups = [&](const std::vector<int>& g) {
    const std::vector<int> prev = b->size_grp;
    b->size_grp = g;
    batch_build_items(b);
    float t = 0.f;
    s = batch_upload_items(b);
    if (s == TOMO_OK) s = batch_time(b, reps, e0, e1, &t);
    if (s == TOMO_OK && t < 0.97f * best) best = t;
    else b->size_grp = prev;
  };
  // (one launch per phase always takes one tile per item)
  for (int g : {1, 2, 8, 16, 32, 64})
    if (s == TOMO_OK && !b->phases) try_groups(std::vector<int>(b->sizes.size(), g));
  for (size_t i = 0; s == TOMO_OK && !b->phases && i < b->sizes.size(); ++i)
    for (int f : {2, -2}) {
      std::vector<int> g = b->size_grp;
      g[i] = f > 0 ? g[i] * 2 : g[i] / 2;
      if (s == TOMO_OK && g[i] >= 1 && g[i] <= kBatchMaxGroup) try_groups(g);
    }
  for (size_t i = 0; s == TOMO_OK && i < b->sizes.size(); ++i) {
    b->size_el[i] = 8;
    batch_build_items(b);
    float t = 0.f;
    s = batch_upload_items(b);
    if (s == TOMO_OK) s = batch_time(b, reps, e0, e1, &t);
    if (s == TOMO_OK && t < 0.97f * best) {
      best = t;
    } else {
      b->size_el[i] = 16;
    }
  }
  if (s == TOMO_OK) {
    batch_build_items(b);
    s = batch_upload_items(b);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (s != TOMO_OK) return s;
  if (out) {
    batch_report(b, out);
    out->iter_ms = best;
    out->base_ms = base;
  }
  return TOMO_OK;
}

tomo_status tomo_batch_destroy(tomo_batch b) {
  if (!b) return TOMO_OK;
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->gstream) {
    (void)hipStreamSynchronize(b->gstream);
    (void)hipStreamDestroy(b->gstream);
  }
  if (b->gev_in) (void)hipEventDestroy(b->gev_in);
  if (b->gev_out) (void)hipEventDestroy(b->gev_out);
  delete b;
  return TOMO_OK;
}

tomo_status tomo_timing_enable(tomo_plan p, uint32_t class_mask) {
  if (!p) return fail(nullptr, TOMO_ERR_INVALID_ARG, "plan is NULL");
  if (!p->pending.empty()) {
    tomo_status s = tresolve(p);
    if (s != TOMO_OK) return s;
  }
  p->tmask = class_mask & ((1u << TOMO_T_COUNT) - 1);
  for (int i = 0; i < TOMO_T_COUNT; ++i) {
    p->tms[i] = 0.0;
    p->tcnt[i] = 0;
  }
  return TOMO_OK;
}

tomo_status tomo_timing_read(tomo_plan p, double* total_ms, int64_t* counts) {
  if (!p) return fail(nullptr, TOMO_ERR_INVALID_ARG, "plan is NULL");
  tomo_status s = tresolve(p);
  if (s != TOMO_OK) return s;
  for (int i = 0; i < TOMO_T_COUNT; ++i) {
    if (total_ms) total_ms[i] = p->tms[i];
    if (counts) counts[i] = p->tcnt[i];
  }
  return TOMO_OK;
}

namespace {
void fill_tiles(const Level& l, tomo_tiles_t* o) {
  o->chunks = l.chunks;
  o->rows_fwd = l.v_fwd;
  o->cols_conv = l.v_cc;
  o->rows_inv = l.v_inv;
  tile_shapes(l.P, l.v_fwd, l.v_cc, l.v_inv, &o->fwd_pairs, &o->col_tile, &o->inv_pairs);
}
void drop_graphs(tomo_plan p) {
  if (p->graphs.empty()) return;
  if (p->gstream) (void)hipStreamSynchronize(p->gstream);
  for (auto& g : p->graphs) (void)hipGraphExecDestroy(g.exec);
  p->graphs.clear();
}
}  // namespace

tomo_status tomo_tiles(tomo_plan p, const tomo_tiles_t* tiles, tomo_tiles_t* out) {
  if (!p) return fail(nullptr, TOMO_ERR_INVALID_ARG, "plan is NULL");
  if (tiles) {
    for (int i = 0; i < p->n_levels; ++i) {
      const tomo_tiles_t& t = tiles[i];
      if (t.rows_fwd < 0 || t.rows_fwd > 2 || t.cols_conv < 0 || t.cols_conv > 2 ||
          t.rows_inv < 0 || t.rows_inv > 2)
        return fail(p, TOMO_ERR_INVALID_ARG, "tile variant of level %d outside 0..2", i);
      if (t.chunks != 0 && t.chunks != 1 && t.chunks != 2 && t.chunks != 4)
        return fail(p, TOMO_ERR_INVALID_ARG, "slice chunks of level %d must be 1, 2 or 4", i);
    }
    drop_graphs(p);
    for (int i = 0; i < p->n_levels; ++i) {
      p->lv[i].v_fwd = tiles[i].rows_fwd;
      p->lv[i].v_cc = tiles[i].cols_conv;
      p->lv[i].v_inv = tiles[i].rows_inv;
      p->lv[i].chunks = tiles[i].chunks == 0 ? 1 : tiles[i].chunks;
    }
  }
  if (out)
    for (int i = 0; i < p->n_levels; ++i) {
      std::memset(&out[i], 0, sizeof out[i]);
      fill_tiles(p->lv[i], &out[i]);
    }
  return TOMO_OK;
}

tomo_status tomo_autotune(tomo_plan p, int32_t reps, tomo_tiles_t* chosen) {
  if (!p) return fail(nullptr, TOMO_ERR_INVALID_ARG, "plan is NULL");
  if (reps > 1000) return fail(p, TOMO_ERR_INVALID_ARG, "reps = %d too large", reps);
  if (reps <= 0) reps = 5;
  if (tomo_status s = check_ws(p); s != TOMO_OK) return s;
  hipStream_t st = p->stream;
  drop_graphs(p);
  // the timings must not overlap a PSF precompute still running beside the plan's stream
  if (p->fstream) HIPCHK(p, hipStreamSynchronize(p->fstream));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(p, hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(p, TOMO_ERR_HIP, "event create failed");
  }
  tomo_status s = TOMO_OK;
  for (int li = 0; li < p->n_levels && s == TOMO_OK; ++li) {
    Level& l = p->lv[li];
    const idx_t vol = (idx_t)p->nz * l.n * l.n;
    float* x = p->xbuf(0);
    float* bb = p->xbuf(1);
    float* out = p->xbuf(2);
    float* gp = p->at<float>(p->off_gp);
    cpx<float>* S1 = p->S1();
    cpx<float>* S2 = p->S2(l);
    const float* fk = p->at<float>(l.off_fk);
    const float* fkn = p->at<float>(l.off_fkn);
    // defined inputs: the timings do not depend on the values
    if (launch_set_scalars(p->scal(), SC_MU, 1, nullptr, 0.0, st) != hipSuccess ||
        launch_fill(x, vol, 1.0f, st) != hipSuccess || launch_fill(bb, vol, 0.5f, st) != hipSuccess ||
        launch_fill(gp, vol, 0.0f, st) != hipSuccess) {
      s = fail(p, TOMO_ERR_HIP, "autotune fill failed");
      break;
    }
    float ms[3][3] = {};
    for (int pass = 0; pass < 3 && s == TOMO_OK; ++pass) {
      for (int v = 0; v < 3 && s == TOMO_OK; ++v) {
        auto launch = [&]() -> hipError_t {
          int nb = 0;
          // the modes a FISTA step uses: y and gp - b precomputed unless the prior runs
          // fused or on its own stream
          const bool yg = !p->fused_prior && !p->concurrent_prior;
          if (pass == 0)
            return launch_rows_fwd(l.P, v, yg ? MODE_FISTA_Y : MODE_FISTA, x, x, p->scal(), S1,
                                   p->tw32(l.P), l.n, p->nz, st);
          if (pass == 1)
            return launch_cols_conv(l.P, v, S1, S2, fk, fkn, p->tw32(l.P), l.n, p->nz, st);
          return launch_rows_inv(l.P, v, yg ? MODE_FISTA_Y : MODE_GRAD, p->g.neighbours, false, S2,
                                 x, x, bb, gp, out, p->partials(), p->scal(), p->tw32(l.P), l.n,
                                 p->nz, p->pp, &nb, st);
        };
        hipError_t e = launch();
        if (e == hipSuccess) e = hipEventRecord(e0, st);
        for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch();
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float t = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
        if (e != hipSuccess) s = fail(p, TOMO_ERR_HIP, "autotune: %s", hipGetErrorString(e));
        ms[pass][v] = t / reps;
      }
    }
    if (s != TOMO_OK) break;
    // a variant replaces the default only when at least 3% faster, so that timing noise
    // does not flip schedules between runs
    auto best = [&](int pass) {
      int b = 1;
      for (int v = 0; v < 3; ++v)
        if (v != 1 && ms[pass][v] < 0.97f * ms[pass][1] && ms[pass][v] < ms[pass][b]) b = v;
      return b;
    };
    l.v_fwd = best(0);
    l.v_cc = best(1);
    l.v_inv = best(2);
    // slice chunks of passes R, C, R' (1, 2 or 4; a count replaces 1 only when at least 3%
    // faster): the whole step of the prior kernel and the three passes, timed with the chosen
    // tiles on the plan's own volume
    float msc[3] = {};
    const int counts[3] = {1, 2, 4};
    l.chunks = 1;
    if (!p->fused_prior && !p->concurrent_prior) {
      const int keep_mask = p->tmask;
      p->tmask = 0;
      for (int ci = 0; ci < 3 && s == TOMO_OK; ++ci) {
        if (counts[ci] > p->nz) { msc[ci] = 0.f; continue; }
        l.chunks = counts[ci];
        int nb = 0;
        tomo_status ts = toeplitz_passes(p, l, MODE_FISTA, p->nz, x, x, bb, out, false, &nb);
        hipError_t e = ts == TOMO_OK ? hipEventRecord(e0, st) : hipErrorUnknown;
        for (int r = 0; r < reps && e == hipSuccess && ts == TOMO_OK; ++r)
          ts = toeplitz_passes(p, l, MODE_FISTA, p->nz, x, x, bb, out, false, &nb);
        if (e == hipSuccess && ts == TOMO_OK) e = hipEventRecord(e1, st);
        if (e == hipSuccess && ts == TOMO_OK) e = hipEventSynchronize(e1);
        float t = 0.f;
        if (e == hipSuccess && ts == TOMO_OK) e = hipEventElapsedTime(&t, e0, e1);
        if (ts != TOMO_OK) s = ts;
        else if (e != hipSuccess) s = fail(p, TOMO_ERR_HIP, "autotune: %s", hipGetErrorString(e));
        msc[ci] = t / reps;
      }
      p->tmask = keep_mask;
      int bc = 0;
      for (int ci = 1; ci < 3; ++ci)
        if (msc[ci] > 0.f && msc[ci] < 0.97f * msc[0] && msc[ci] < msc[bc]) bc = ci;
      l.chunks = counts[bc];
    }
    if (chosen) {
      std::memset(&chosen[li], 0, sizeof chosen[li]);
      fill_tiles(l, &chosen[li]);
      std::memcpy(chosen[li].ms, ms, sizeof ms);
      std::memcpy(chosen[li].ms_chunks, msc, sizeof msc);
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return s;
}

tomo_status tomo_plan_destroy(tomo_plan p) {
  if (!p) return TOMO_OK;
  if (!p->pending.empty()) (void)hipStreamSynchronize(p->stream);
  for (auto& e : p->pending) {
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  for (hipEvent_t e : p->pool) (void)hipEventDestroy(e);
  for (auto& g : p->graphs) (void)hipGraphExecDestroy(g.exec);
  drop_psf_graphs(p);
  if (p->gstream) {
    (void)hipStreamSynchronize(p->gstream);
    (void)hipStreamDestroy(p->gstream);
  }
  if (p->pstream) {
    (void)hipStreamSynchronize(p->pstream);
    (void)hipStreamDestroy(p->pstream);
  }
  if (p->pev_fork) (void)hipEventDestroy(p->pev_fork);
  if (p->pev_join) (void)hipEventDestroy(p->pev_join);
  if (p->fstream) {
    (void)hipStreamSynchronize(p->fstream);
    (void)hipStreamDestroy(p->fstream);
  }
  if (p->fev_fork) (void)hipEventDestroy(p->fev_fork);
  if (p->fev_done) (void)hipEventDestroy(p->fev_done);
  if (p->gev_in) (void)hipEventDestroy(p->gev_in);
  if (p->gev_out) (void)hipEventDestroy(p->gev_out);
  if (p->nev_fork) (void)hipEventDestroy(p->nev_fork);
  if (p->nev_join) (void)hipEventDestroy(p->nev_join);
  delete p;
  return TOMO_OK;
}

const char* tomo_status_string(int32_t s) {
  switch (s) {
    case TOMO_OK: return "ok";
    case TOMO_ERR_INVALID_ARG: return "invalid argument";
    case TOMO_ERR_NO_DEVICE: return "no HIP device";
    case TOMO_ERR_UNSUPPORTED_ARCH: return "unsupported GPU architecture (needs gfx950)";
    case TOMO_ERR_NO_WORKSPACE: return "no workspace attached";
    case TOMO_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
    case TOMO_ERR_NOT_READY: return "PSF not precomputed";
    case TOMO_ERR_HIP: return "HIP runtime error";
    case TOMO_ERR_NONFINITE: return "non-finite value";
    case TOMO_ERR_INTERNAL: return "internal error";
  }
  return "unknown status";
}

const char* tomo_last_error(tomo_plan p) { return p ? p->err.c_str() : g_last_error.c_str(); }

}  // extern "C"
