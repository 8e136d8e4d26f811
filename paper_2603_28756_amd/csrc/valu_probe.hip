// Issue-rate probe for the vector ALU of gfx950: dependent chains of full-rate FP32 fused
// multiply-adds against chains of the transcendental instructions the prior uses
// (v_log_f32, v_exp_f32, v_rcp_f32).  The ratio of the two times is the issue weight of a
// transcendental relative to a full-rate operation, which the prior's ALU roofline uses.
// Standalone executable; every thread writes one float of an output buffer sized to the grid.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

namespace {

constexpr int kChains = 8;  // independent chains per thread (latency hidden within a wave)

template <int KIND>
__global__ void __launch_bounds__(256) chains(float* out, int iters, float a, float b) {
  float x[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) x[c] = 1.0f + 0.01f * c + 1e-6f * threadIdx.x;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
      if constexpr (KIND == 0) {
        x[c] = __builtin_fmaf(x[c], a, b);
        x[c] = __builtin_fmaf(x[c], a, b);
      } else if constexpr (KIND == 1) {
        x[c] = __builtin_amdgcn_exp2f(x[c]);
        x[c] = __builtin_amdgcn_logf(x[c]);
      } else {
        x[c] = __builtin_amdgcn_rcpf(x[c]);
        x[c] = __builtin_amdgcn_rcpf(x[c]);
      }
    }
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += x[c];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

#define CHECK(e)                                                              \
  do {                                                                        \
    const hipError_t err_ = (e);                                              \
    if (err_ != hipSuccess) {                                                 \
      std::fprintf(stderr, "%s: %s\n", #e, hipGetErrorString(err_));         \
      std::exit(1);                                                           \
    }                                                                         \
  } while (0)

}  // namespace

int main() {
  const int blocks = 4096, threads = 256, iters = 2048;
  float* out = nullptr;
  CHECK(hipMalloc(&out, (size_t)blocks * threads * sizeof(float)));
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  const char* names[3] = {"fma+fma", "exp2+log2", "rcp+rcp"};
  float best[3] = {0, 0, 0};
  for (int k = 0; k < 3; ++k) {
    for (int rep = 0; rep < 5; ++rep) {
      CHECK(hipEventRecord(e0));
      if (k == 0) chains<0><<<blocks, threads>>>(out, iters, 0.999f, 0.001f);
      if (k == 1) chains<1><<<blocks, threads>>>(out, iters, 0.f, 0.f);
      if (k == 2) chains<2><<<blocks, threads>>>(out, iters, 0.f, 0.f);
      CHECK(hipGetLastError());
      CHECK(hipEventRecord(e1));
      CHECK(hipEventSynchronize(e1));
      float ms = 0.f;
      CHECK(hipEventElapsedTime(&ms, e0, e1));
      if (rep == 0 || ms < best[k]) best[k] = ms;
    }
  }
  const double lane_ops = 2.0 * blocks * threads * kChains * iters;
  for (int k = 0; k < 3; ++k)
    std::printf("%-10s %8.3f ms  %.2f T lane-instructions/s  weight vs fma %.2f\n", names[k],
                best[k], lane_ops / (best[k] * 1e-3) / 1e12, best[k] / best[0]);
  CHECK(hipFree(out));
  return 0;
}
