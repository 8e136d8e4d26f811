// Streaming of a volume that does not fit in device memory through one plan (Sec. 2.4: three
// cooperating host threads joined by bounded work queues move input to the device, run the
// kernels and move results back, overlapping transfers with computation).  Only the public
// C ABI of the plan is used here; the window solves are ordinary tomo_reconstruct calls.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "tomo.h"
#include "tomo_pipeline.h"

namespace {

constexpr size_t kAlign = 256;
constexpr int kMaxDepth = 8;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

thread_local std::string g_pipe_error;

// Blocking FIFO of bounded capacity.  close() wakes every waiter: push then fails, pop keeps
// returning queued items until the queue is empty and then fails (drain on close).
template <class T>
class BoundedQueue {
 public:
  explicit BoundedQueue(size_t cap) : cap_(cap) {}
  bool push(const T& v) {
    std::unique_lock<std::mutex> lk(m_);
    not_full_.wait(lk, [&] { return closed_ || q_.size() < cap_; });
    if (closed_) return false;
    q_.push_back(v);
    not_empty_.notify_one();
    return true;
  }
  bool pop(T* v) {
    std::unique_lock<std::mutex> lk(m_);
    not_empty_.wait(lk, [&] { return closed_ || !q_.empty(); });
    if (q_.empty()) return false;
    *v = q_.front();
    q_.pop_front();
    not_full_.notify_one();
    return true;
  }
  void close() {
    std::lock_guard<std::mutex> lk(m_);
    closed_ = true;
    not_full_.notify_all();
    not_empty_.notify_all();
  }

 private:
  size_t cap_;
  std::deque<T> q_;
  bool closed_ = false;
  std::mutex m_;
  std::condition_variable not_full_, not_empty_;
};

struct Window {
  int k, slot, first, keep0, keep1;
};

// Window k: interior [k C, min((k + 1) C, n_total)), solved on [first, first + nz) with first
// = clamp(k C - halo, 0, n_total - nz); the clamped window still contains the interior.
bool window_of(int n_total, int nz, int halo, int k, int* first, int* keep0, int* keep1,
               int* n_windows) {
  const int C = nz - 2 * halo;
  if (C < 1 || n_total < nz || halo < 0) return false;
  const int W = (n_total + C - 1) / C;
  if (n_windows) *n_windows = W;
  if (k < 0 || k >= W) return false;
  const int k0 = k * C, k1 = std::min(k0 + C, n_total);
  const int f = std::min(std::max(k0 - halo, 0), n_total - nz);
  if (first) *first = f;
  if (keep0) *keep0 = k0;
  if (keep1) *keep1 = k1;
  return true;
}

double ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct tomo_pipeline_s {
  tomo_plan plan = nullptr;
  tomo_geometry_t g{};
  hipStream_t pstream = nullptr;  // the plan's stream (not owned)
  int device = 0;
  int n_total = 0, halo = 0, depth = 0, n_windows = 0;
  size_t sino_win = 0, x_win = 0;  // floats per window
  size_t need = 0;
  char* ws = nullptr;
  std::vector<float*> pin_in, pin_out;  // pinned host staging per slot
  std::vector<hipEvent_t> ev_up, ev_comp;
  hipStream_t ustream = nullptr, dstream = nullptr;
  std::string err;
  float* dev_sino(int s) const {
    return reinterpret_cast<float*>(ws + (size_t)s * (align_up(sino_win * 4) + align_up(x_win * 4)));
  }
  float* dev_x(int s) const { return reinterpret_cast<float*>(reinterpret_cast<char*>(dev_sino(s)) + align_up(sino_win * 4)); }
};

namespace {

tomo_status pfail(tomo_pipeline p, tomo_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (p) p->err = buf;
  g_pipe_error = buf;
  return s;
}

void release(tomo_pipeline p) {
  for (float* h : p->pin_in) if (h) (void)hipHostFree(h);
  for (float* h : p->pin_out) if (h) (void)hipHostFree(h);
  for (hipEvent_t e : p->ev_up) if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : p->ev_comp) if (e) (void)hipEventDestroy(e);
  if (p->ustream) (void)hipStreamDestroy(p->ustream);
  if (p->dstream) (void)hipStreamDestroy(p->dstream);
}

// State shared by the three threads of one run.  The first failure wins: it records its
// status and message, and closes every queue so that blocked threads wake up and leave.
struct RunState {
  BoundedQueue<int> free_slots;
  BoundedQueue<Window> work, done;
  std::atomic<bool> abort{false};
  std::mutex m;
  tomo_status status = TOMO_OK;
  std::string msg;
  int nonfinite_window = -1;
  std::atomic<int> restarts{0}, finished{0};
  double up_ms = 0.0, comp_ms = 0.0, down_ms = 0.0;
  explicit RunState(int depth) : free_slots(depth), work(depth), done(depth) {}
  void fail(tomo_status s, const std::string& text) {
    {
      std::lock_guard<std::mutex> lk(m);
      if (status == TOMO_OK) {
        status = s;
        msg = text;
      }
    }
    abort = true;
    free_slots.close();
    work.close();
    done.close();
  }
};

std::string hip_msg(const char* what, int k, hipError_t e) {
  char buf[256];
  snprintf(buf, sizeof buf, "window %d: %s failed: %s", k, what, hipGetErrorString(e));
  return buf;
}

void upload_thread(tomo_pipeline p, RunState* rs, const float* sino_host) {
  if (hipSetDevice(p->device) != hipSuccess) return rs->fail(TOMO_ERR_HIP, "upload: hipSetDevice failed");
  const auto t0 = std::chrono::steady_clock::now();
  const size_t per_slice = (size_t)p->g.n_angles * p->g.n_det;
  for (int k = 0; k < p->n_windows && !rs->abort; ++k) {
    Window w{k, -1, 0, 0, 0};
    if (!rs->free_slots.pop(&w.slot)) break;
    window_of(p->n_total, p->g.n_slices, p->halo, k, &w.first, &w.keep0, &w.keep1, nullptr);
    std::memcpy(p->pin_in[w.slot], sino_host + (size_t)w.first * per_slice, p->sino_win * sizeof(float));
    hipError_t e = hipMemcpyAsync(p->dev_sino(w.slot), p->pin_in[w.slot], p->sino_win * sizeof(float),
                                  hipMemcpyHostToDevice, p->ustream);
    if (e == hipSuccess) e = hipEventRecord(p->ev_up[w.slot], p->ustream);
    if (e != hipSuccess) return rs->fail(TOMO_ERR_HIP, hip_msg("upload", k, e));
    if (!rs->work.push(w)) break;
  }
  rs->up_ms = ms_since(t0);
  rs->work.close();  // no more windows: the compute thread drains the queue and ends
}

void compute_thread(tomo_pipeline p, RunState* rs, const tomo_recon_opts_t* opts, bool check) {
  if (hipSetDevice(p->device) != hipSuccess) return rs->fail(TOMO_ERR_HIP, "compute: hipSetDevice failed");
  double busy = 0.0;
  Window w;
  while (rs->work.pop(&w)) {
    if (rs->abort) break;
    const auto t0 = std::chrono::steady_clock::now();
    hipError_t e = hipStreamWaitEvent(p->pstream, p->ev_up[w.slot], 0);
    if (e != hipSuccess) return rs->fail(TOMO_ERR_HIP, hip_msg("hipStreamWaitEvent", w.k, e));
    tomo_recon_stats_t st;
    const tomo_status s = tomo_reconstruct(p->plan, p->dev_sino(w.slot), p->dev_x(w.slot), opts,
                                           check ? &st : nullptr);
    if (s != TOMO_OK) {
      if (s == TOMO_ERR_NONFINITE) {
        std::lock_guard<std::mutex> lk(rs->m);
        if (rs->nonfinite_window < 0) rs->nonfinite_window = w.k;
      }
      char buf[640];
      snprintf(buf, sizeof buf, "window %d (slices %d..%d): %s", w.k, w.first,
               w.first + p->g.n_slices - 1, tomo_last_error(p->plan));
      return rs->fail(s, buf);
    }
    if (check) rs->restarts += st.n_restarts;
    e = hipEventRecord(p->ev_comp[w.slot], p->pstream);
    if (e != hipSuccess) return rs->fail(TOMO_ERR_HIP, hip_msg("hipEventRecord", w.k, e));
    busy += ms_since(t0);
    if (!rs->done.push(w)) break;
  }
  rs->comp_ms = busy;
  rs->done.close();
}

void download_thread(tomo_pipeline p, RunState* rs, float* x_host) {
  if (hipSetDevice(p->device) != hipSuccess) return rs->fail(TOMO_ERR_HIP, "download: hipSetDevice failed");
  const size_t plane = (size_t)p->g.n * p->g.n;
  double busy = 0.0;
  Window w;
  while (rs->done.pop(&w)) {
    if (rs->abort) break;
    const auto t0 = std::chrono::steady_clock::now();
    const size_t cnt = (size_t)(w.keep1 - w.keep0) * plane;
    hipError_t e = hipStreamWaitEvent(p->dstream, p->ev_comp[w.slot], 0);
    if (e == hipSuccess)
      e = hipMemcpyAsync(p->pin_out[w.slot], p->dev_x(w.slot) + (size_t)(w.keep0 - w.first) * plane,
                         cnt * sizeof(float), hipMemcpyDeviceToHost, p->dstream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->dstream);
    if (e != hipSuccess) return rs->fail(TOMO_ERR_HIP, hip_msg("download", w.k, e));
    std::memcpy(x_host + (size_t)w.keep0 * plane, p->pin_out[w.slot], cnt * sizeof(float));
    busy += ms_since(t0);
    rs->finished += 1;
    if (!rs->free_slots.push(w.slot)) break;  // the slot (device and staging) is free again
  }
  rs->down_ms = busy;
}

}  // namespace

extern "C" {

tomo_status tomo_pipeline_window(int32_t n_total, int32_t n_slices, int32_t halo, int32_t k,
                                 int32_t* first, int32_t* keep0, int32_t* keep1,
                                 int32_t* n_windows) {
  if (!first || !keep0 || !keep1)
    return pfail(nullptr, TOMO_ERR_INVALID_ARG, "NULL output");
  if (!window_of(n_total, n_slices, halo, k, first, keep0, keep1, n_windows))
    return pfail(nullptr, TOMO_ERR_INVALID_ARG,
                 "need halo >= 0, n_slices - 2 halo >= 1, n_total >= n_slices and a window index "
                 "in range (n_total %d, n_slices %d, halo %d, k %d)", n_total, n_slices, halo, k);
  return TOMO_OK;
}

tomo_status tomo_pipeline_create(tomo_plan plan, int32_t n_total, int32_t halo, int32_t depth,
                                 tomo_pipeline* out) {
  if (!out) return pfail(nullptr, TOMO_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!plan) return pfail(nullptr, TOMO_ERR_INVALID_ARG, "plan is NULL");
  if (depth < 1 || depth > kMaxDepth) return pfail(nullptr, TOMO_ERR_INVALID_ARG, "depth must be 1..%d", kMaxDepth);
  tomo_pipeline p = new tomo_pipeline_s();
  p->plan = plan;
  void* st = nullptr;
  tomo_plan_geometry(plan, &p->g, &st, &p->device);
  p->pstream = static_cast<hipStream_t>(st);
  int W = 0;
  if (!window_of(n_total, p->g.n_slices, halo, 0, nullptr, nullptr, nullptr, &W)) {
    delete p;
    return pfail(nullptr, TOMO_ERR_INVALID_ARG,
                 "need halo >= 0, n_slices - 2 halo >= 1 and n_total >= n_slices (n_total %d, "
                 "n_slices %d, halo %d)", n_total, p->g.n_slices, halo);
  }
  p->n_total = n_total;
  p->halo = halo;
  p->depth = depth;
  p->n_windows = W;
  p->sino_win = (size_t)p->g.n_slices * p->g.n_angles * p->g.n_det;
  p->x_win = (size_t)p->g.n_slices * p->g.n * p->g.n;
  p->need = (size_t)depth * (align_up(p->sino_win * 4) + align_up(p->x_win * 4));
  p->pin_in.assign(depth, nullptr);
  p->pin_out.assign(depth, nullptr);
  p->ev_up.assign(depth, nullptr);
  p->ev_comp.assign(depth, nullptr);
  hipError_t e = hipSetDevice(p->device);
  for (int s = 0; s < depth && e == hipSuccess; ++s) {
    e = hipHostMalloc(reinterpret_cast<void**>(&p->pin_in[s]), p->sino_win * sizeof(float));
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&p->pin_out[s]), p->x_win * sizeof(float));
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_up[s], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_comp[s], hipEventDisableTiming);
  }
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->ustream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->dstream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    release(p);
    delete p;
    return pfail(nullptr, TOMO_ERR_HIP, "pipeline setup failed: %s", hipGetErrorString(e));
  }
  *out = p;
  return TOMO_OK;
}

tomo_status tomo_pipeline_workspace_size(tomo_pipeline p, size_t* bytes) {
  if (!p || !bytes) return pfail(p, TOMO_ERR_INVALID_ARG, "NULL argument");
  *bytes = p->need;
  return TOMO_OK;
}

tomo_status tomo_pipeline_set_workspace(tomo_pipeline p, void* dev, size_t bytes) {
  if (!p || !dev) return pfail(p, TOMO_ERR_INVALID_ARG, "NULL argument");
  if (reinterpret_cast<uintptr_t>(dev) % kAlign) return pfail(p, TOMO_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  if (bytes < p->need)
    return pfail(p, TOMO_ERR_WORKSPACE_TOO_SMALL, "workspace %zu B < required %zu B", bytes, p->need);
  p->ws = static_cast<char*>(dev);
  return TOMO_OK;
}

tomo_status tomo_pipeline_run(tomo_pipeline p, const float* sino_host, float* x_host,
                              const tomo_recon_opts_t* opts, tomo_pipeline_stats_t* stats) {
  if (!p || !sino_host || !x_host || !opts || !opts->iters) return pfail(p, TOMO_ERR_INVALID_ARG, "NULL argument");
  if (opts->init == TOMO_INIT_USER)
    return pfail(p, TOMO_ERR_INVALID_ARG, "a user start image is not streamed (TOMO_INIT_USER)");
  if (opts->objective_dev || opts->restart_dev || opts->init_choice_dev)
    return pfail(p, TOMO_ERR_INVALID_ARG, "per-iteration device outputs are not streamed");
  if (!p->ws) return pfail(p, TOMO_ERR_NO_WORKSPACE, "no workspace attached");
  if (hipSetDevice(p->device) != hipSuccess) return pfail(p, TOMO_ERR_HIP, "hipSetDevice failed");
  const auto t0 = std::chrono::steady_clock::now();
  RunState rs(p->depth);
  for (int s = 0; s < p->depth; ++s) rs.free_slots.push(s);
  std::thread tu(upload_thread, p, &rs, sino_host);
  std::thread tc(compute_thread, p, &rs, opts, stats != nullptr);
  std::thread td(download_thread, p, &rs, x_host);
  tu.join();
  tc.join();
  td.join();
  // after a failure, windows already on the device may still be running: let them end
  (void)hipStreamSynchronize(p->pstream);
  (void)hipStreamSynchronize(p->ustream);
  (void)hipStreamSynchronize(p->dstream);
  if (stats) {
    std::memset(stats, 0, sizeof *stats);
    stats->n_windows = rs.finished;
    stats->nonfinite_window = rs.nonfinite_window;
    stats->n_restarts = rs.restarts;
    stats->wall_ms = ms_since(t0);
    stats->upload_ms = rs.up_ms;
    stats->compute_ms = rs.comp_ms;
    stats->download_ms = rs.down_ms;
  }
  if (rs.status != TOMO_OK) return pfail(p, rs.status, "%s", rs.msg.c_str());
  if (rs.finished != p->n_windows)
    return pfail(p, TOMO_ERR_INTERNAL, "%d of %d windows finished", (int)rs.finished, p->n_windows);
  return TOMO_OK;
}

const char* tomo_pipeline_last_error(tomo_pipeline p) {
  return p ? p->err.c_str() : g_pipe_error.c_str();
}

tomo_status tomo_pipeline_destroy(tomo_pipeline p) {
  if (!p) return TOMO_OK;
  (void)hipSetDevice(p->device);
  if (p->ustream) (void)hipStreamSynchronize(p->ustream);
  if (p->dstream) (void)hipStreamSynchronize(p->dstream);
  release(p);
  delete p;
  return TOMO_OK;
}

}  // extern "C"
