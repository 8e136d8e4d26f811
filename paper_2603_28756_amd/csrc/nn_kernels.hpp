// Launchers of the U-Net kernels (bfloat16 NHWC tensors as uint16_t, float32 parameters).
// A tensor argument is a pointer to its first channel plus the channel count `ld` of the
// buffer that holds it; channel counts of the matrix-core convolutions are multiples of 32.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace tomo {

// 3x3 convolution, zero padding: y = act(bias + conv(x, w)) (* (mask > 0) when mask != NULL).
// w: bfloat16 [cout][3][3][cin].  Supported forms: ReLU with bias, plain with bias, plain
// without bias (optionally masked).
// With xu != NULL (ReLU form only) the input is the concatenation [up2(xu), x]: channels
// 0..cu-1 come from xu (half resolution, channel stride ldu), the rest from x.  With
// pool != NULL (ReLU form, even H and W) the 2x2 average of the output is also written to
// pool (half resolution, channel stride ldp).
// With head != NULL (ReLU form with bias, no concatenation or pooling, cout 32 or 64) the
// output is not stored: the 1x1 head r = hb + sum_c hw[c] y[c] and x0 = fbp + s r are written
// instead (r nullable), per pixel.
struct NnHead {
  const float* hw;
  const float* hb;
  const float* fbp;
  float s;
  float* r;
  float* x0;
};
hipError_t nn_conv3x3(const uint16_t* x, int ldx, const uint16_t* w, const float* bias,
                      uint16_t* y, int ldy, const uint16_t* mask, int ldm, int cin, int cout,
                      int B, int H, int W, bool relu, hipStream_t st,
                      const uint16_t* xu = nullptr, int ldu = 0, int cu = 0,
                      uint16_t* pool = nullptr, int ldp = 0, const NnHead* head = nullptr);

struct WgradPlan {
  int ntn = 0, ntc = 0, nsplit = 0, px_per_split = 0;
  size_t scratch_floats = 0;
};
WgradPlan nn_wgrad_plan(int cin, int cout, int npx);
size_t nn_wgrad_scratch_bound(int cin, int cout, int max_npx);
// dw [cout][3][3][cin] = sum_p dz[p, co] x[p + tap, ci]; db [cout] = sum_p dz[p, co].
hipError_t nn_conv3x3_wgrad(const uint16_t* dz, int ldz, const uint16_t* x, int ldx, float* dw,
                            float* db, int cin, int cout, int B, int H, int W, float* scratch,
                            size_t scratch_floats, hipStream_t st);

// First layer (one input channel u = fbp * inv_s), float32 arithmetic: ReLU output.
hipError_t nn_conv_in(const float* fbp, float inv_s, const float* w, const float* bias,
                      uint16_t* y, int cout, int B, int H, int W, hipStream_t st);
int nn_conv_in_wgrad_blocks(int npx);
hipError_t nn_conv_in_wgrad(const uint16_t* dz, const float* fbp, float inv_s, float* dw,
                            float* db, int cout, int B, int H, int W, float* scratch,
                            size_t scratch_floats, hipStream_t st);

hipError_t nn_avgpool2(const uint16_t* in, int ldi, uint16_t* out, int ldo, int C, int B, int H,
                       int W, hipStream_t st);
// de += 0.25 up2(dp) where e > 0 (H, W: the full-resolution size)
hipError_t nn_avgpool2_back(const uint16_t* dp, int ldp, const uint16_t* e, int lde, uint16_t* de,
                            int ldd, int C, int B, int H, int W, hipStream_t st);
// H, W: the full-resolution (output of up2, input of up2_back) size
hipError_t nn_up2(const uint16_t* in, int ldi, uint16_t* out, int ldo, int C, int B, int H, int W,
                  hipStream_t st);
hipError_t nn_up2_back(const uint16_t* in, int ldi, uint16_t* out, int ldo, int C, int B, int H,
                       int W, hipStream_t st);

hipError_t nn_head(const uint16_t* d, const float* hw, const float* hb, const float* fbp, float s,
                   float* r, float* x0, int C, int npx, hipStream_t st);
int nn_head_back_blocks(int npx);
hipError_t nn_head_back(const float* r, const float* fbp, const float* target, float inv_s,
                        const uint16_t* d, const float* hw, uint16_t* dd, double* part, float* ghw,
                        float* ghb, double* loss, int C, int npx, hipStream_t st);

hipError_t nn_adam(float* th, const float* g, float* m, float* v, size_t n, float lr, float b1,
                   float b2, float c1, float c2, float eps, hipStream_t st);
hipError_t nn_weight_prep(const float* w, uint16_t* wbf, uint16_t* wflip, int cin, int cout,
                          hipStream_t st);
hipError_t nn_f32_to_bf16(const float* in, uint16_t* out, size_t n, hipStream_t st);

}  // namespace tomo
