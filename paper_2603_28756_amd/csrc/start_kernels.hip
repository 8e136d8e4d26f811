// Choice of the start image when a learned start is offered (Sec. 2.2 takes the ramp-filtered
// back-projection as the start; Sec. 3.2 counts a better start as iterations saved): the
// float64 difference of the two candidate starts' objectives per slice, and the per-slice (or
// whole-volume) choice between the network's start and the FBP start.
//
// Objective of a candidate x (Eq. 10 without the constant 1/2 <g, g>, plus the prior of
// Eq. 5):  1/2 <x, T x> - <x, b> + beta Phi(x), Phi summed over unordered neighbour pairs,
// each pair counted once at the voxel that precedes it (forward offsets), so that the sums
// of all slices give the whole volume's objective also with the 26-neighbourhood.
#include "kernels.hpp"

namespace tomo {
namespace {

constexpr int SO_NT = 256;

// rho(d) = |d|^p / (p sigma^p) * w / (1 + w),  w = (|d| / (T sigma))^(q - p); for q = 2 this is
// c d^2 / (1 + w) with c = 1 / (p sigma^p (T sigma)^(2 - p)).  d, d^2 and the sums are float64; w
// comes from the hardware exp2/log2 in float32 (relative error ~1e-7 in each term, as in the
// iteration's own objective).
TOMO_DEV double rho64(double d, const ObjParams& op) {
  if (d == 0.0) return 0.0;
  double r = 0.5;
  if (!op.quadratic) {
    const float w = __builtin_amdgcn_exp2f(
        __builtin_fmaf((float)op.qmp, __builtin_amdgcn_logf((float)fabs(d)), (float)op.lw0));
    r = 1.0 / (1.0 + (double)w);
  }
  return op.c_rho2 * d * d * r;
}

TOMO_DEV double block_sum(double v, double* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = SO_NT / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] += sh[t + s];
    __syncthreads();
  }
  return sh[0];
}

// The difference of the objectives of xb and xa in one pass, with t = T (xa + xb) (T is
// symmetric, so <xb, T xb> - <xa, T xa> = <xb - xa, T (xa + xb)>):
//   F(xb) - F(xa) = 1/2 <xb - xa, t> - <xb - xa, b> + beta (Phi(xb) - Phi(xa)),
// part[z][blk]: this block's share of slice z's terms (a fixed assignment of pixels to threads
// and a fixed reduction tree: deterministic).
__global__ __launch_bounds__(SO_NT) void slice_objective_diff_kernel(
    const float* __restrict__ xa, const float* __restrict__ xb, const float* __restrict__ ts,
    const float* __restrict__ b, int N, int nz, ObjParams op, double* __restrict__ part) {
  __shared__ double sh[SO_NT];
  const int z = blockIdx.y;
  const idx_t plane = (idx_t)N * N;
  const float* az = xa + z * plane;
  const float* bz_ = xb + z * plane;
  const float* tz = ts + z * plane;
  const float* gz = b + z * plane;
  const bool up = op.neighbours == 26 && z + 1 < nz;
  double data = 0.0, prior = 0.0;
  auto pair = [&](double w, double va, double vb, const float* na, const float* nb) {
    prior += w * (rho64(vb - *nb, op) - rho64(va - *na, op));
  };
  for (int i = blockIdx.x * SO_NT + threadIdx.x; i < N * N; i += gridDim.x * SO_NT) {
    const int r = i / N, c = i - r * N;
    const double va = az[i], vb = bz_[i], dv = vb - va;
    data += 0.5 * dv * (double)tz[i] - dv * (double)gz[i];
    if (c + 1 < N) pair(op.w1, va, vb, az + i + 1, bz_ + i + 1);
    if (r + 1 < N) {
      pair(op.w1, va, vb, az + i + N, bz_ + i + N);
      if (c > 0) pair(op.w2, va, vb, az + i + N - 1, bz_ + i + N - 1);
      if (c + 1 < N) pair(op.w2, va, vb, az + i + N + 1, bz_ + i + N + 1);
    }
    if (up) {
      for (int dy = -1; dy <= 1; ++dy) {
        if (r + dy < 0 || r + dy >= N) continue;
        for (int dx = -1; dx <= 1; ++dx) {
          if (c + dx < 0 || c + dx >= N) continue;
          const int k = (dy != 0) + (dx != 0);
          const double w = k == 0 ? op.w1 : (k == 1 ? op.w2 : op.w3);
          const idx_t o = plane + i + dy * N + dx;
          pair(w, va, vb, az + o, bz_ + o);
        }
      }
    }
  }
  const double s = block_sum(data + op.beta * prior, sh);
  if (threadIdx.x == 0) part[(idx_t)z * gridDim.x + blockIdx.x] = s;
}

__global__ __launch_bounds__(SO_NT) void add_kernel(const float* __restrict__ a,
                                                    const float* __restrict__ b,
                                                    float* __restrict__ out, idx_t n) {
  for (idx_t i = (idx_t)blockIdx.x * SO_NT + threadIdx.x; i < n; i += (idx_t)gridDim.x * SO_NT)
    out[i] = a[i] + b[i];
}

// Thread z decides for slice z (per_slice) or for the whole volume (every thread takes the
// same decision from the same fixed-order sums): the network's start is kept unless the
// objective difference F(xb) - F(xa) (partials pd) is positive or not finite.
__global__ __launch_bounds__(64) void start_choice_kernel(
    const double* __restrict__ pd, int nblk, int nz, int per_slice,
    int32_t* __restrict__ choice, int32_t* __restrict__ choice_user) {
  const int z = blockIdx.x * 64 + threadIdx.x;
  if (z >= nz) return;
  const int z0 = per_slice ? z : 0, z1 = per_slice ? z + 1 : nz;
  double fd = 0.0;
  for (int zz = z0; zz < z1; ++zz)
    for (int k = 0; k < nblk; ++k) fd += pd[(idx_t)zz * nblk + k];
  const int keep = (isfinite(fd) && !(fd > 0.0)) ? 1 : 0;
  choice[z] = keep;
  if (choice_user) choice_user[z] = keep;
}

// A kept slice z (choice[z]) is copied from xb over xa with gridDim.x blocks per slice,
// 16 bytes per access when every slice starts 16-byte aligned (N^2 % 4 == 0; the volumes
// start 256-byte aligned), else 4.
__global__ __launch_bounds__(SO_NT) void start_copy_kernel(float* __restrict__ xa,
                                                           const float* __restrict__ xb, int N,
                                                           const int32_t* __restrict__ choice) {
  const int z = blockIdx.y;
  if (!choice[z]) return;
  const idx_t plane = (idx_t)N * N;
  float* dst = xa + z * plane;
  const float* src = xb + z * plane;
  const idx_t i0 = (idx_t)blockIdx.x * SO_NT + threadIdx.x, step = (idx_t)gridDim.x * SO_NT;
  if (plane % 4 == 0) {
    for (idx_t i = i0; i < plane / 4; i += step)
      reinterpret_cast<float4*>(dst)[i] = reinterpret_cast<const float4*>(src)[i];
  } else {
    for (idx_t i = i0; i < plane; i += step) dst[i] = src[i];
  }
}

}  // namespace

hipError_t launch_slice_objective_diff(const float* xa, const float* xb, const float* ts,
                                       const float* b, int N, int nz, const ObjParams& op,
                                       double* part, hipStream_t st) {
  hipLaunchKernelGGL(slice_objective_diff_kernel, dim3(kObjBlocks, nz), dim3(SO_NT), 0, st, xa, xb,
                     ts, b, N, nz, op, part);
  return hipGetLastError();
}

hipError_t launch_add(const float* a, const float* b, float* out, idx_t n, hipStream_t st) {
  const idx_t nb = (n + SO_NT - 1) / SO_NT;
  hipLaunchKernelGGL(add_kernel, dim3((unsigned)(nb < 8192 ? nb : 8192)), dim3(SO_NT), 0, st, a, b,
                     out, n);
  return hipGetLastError();
}

hipError_t launch_select_start(const double* pd, int nz, int per_slice, float* xa,
                               const float* xb, int N, int32_t* choice, int32_t* choice_user,
                               hipStream_t st) {
  hipLaunchKernelGGL(start_choice_kernel, dim3((nz + 63) / 64), dim3(64), 0, st, pd, kObjBlocks, nz,
                     per_slice, choice, choice_user);
  hipLaunchKernelGGL(start_copy_kernel, dim3(64, nz), dim3(SO_NT), 0, st, xa, xb, N, choice);
  return hipGetLastError();
}

}  // namespace tomo
