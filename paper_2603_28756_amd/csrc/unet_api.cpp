// C ABI of the learned start (include/tomo_nn.h): a U-Net that maps the FBP image to a
// start close to the converged reconstruction, trained and evaluated on the GPU by the
// kernels of unet_kernels.hip.  The host code only sequences launches and carves the
// caller-owned workspace.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "tomo_nn.h"
#include "nn_kernels.hpp"
#include "unet_view.hpp"

using namespace tomo;

namespace {
constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
thread_local std::string g_nn_err;
}  // namespace

struct tomo_unet_s {
  int L = 4, C0 = 32, maxB = 1, H = 0, W = 0;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  size_t ws_bytes = 0, need = 0;
  struct Conv {
    int cin = 0, cout = 0;
    size_t w = 0, b = 0;            // float offsets of weights and bias in the parameter vector
    size_t wbf = 0, wflip = 0;      // byte offsets of the bfloat16 copies (not for the first)
  };
  std::vector<Conv> convs;  // order: E0a, E0b, ..., E(L-1)b, D(L-2)a, D(L-2)b, ..., D0a, D0b
  size_t head_w = 0, head_b = 0, n_params = 0;
  size_t off_theta = 0, off_m = 0, off_v = 0, off_grad = 0;
  struct Lvl {
    int h = 0, w = 0, c = 0;
    size_t Ea = 0, cat = 0, P = 0, Da = 0, D = 0, Elast = 0;     // activations
    size_t dEa = 0, dcat = 0, dP = 0, dDa = 0, dD = 0, dElast = 0;  // gradients
  };
  std::vector<Lvl> lv;
  size_t off_r = 0, off_scratch = 0, scratch_floats = 0, off_hpart = 0, off_loss = 0;
  int64_t step = 0;
  bool params_ready = false;
  bool has_domain = false;
  tomo_unet_domain_t domain{};
  std::string err;

  template <typename T>
  T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
  float* theta() const { return at<float>(off_theta); }
  float* grad() const { return at<float>(off_grad); }
  int ch(int l) const { return C0 << l; }
  int catld(int l) const { return ch(l + 1) + ch(l); }
  // E_l as (pointer, ld): the skip half of cat_l, or the bottleneck buffer
  uint16_t* E(int l, int* ld) const {
    if (l < L - 1) { *ld = catld(l); return at<uint16_t>(lv[l].cat) + ch(l + 1); }
    *ld = ch(l);
    return at<uint16_t>(lv[l].Elast);
  }
  uint16_t* dE(int l, int* ld) const {
    if (l < L - 1) { *ld = catld(l); return at<uint16_t>(lv[l].dcat) + ch(l + 1); }
    *ld = ch(l);
    return at<uint16_t>(lv[l].dElast);
  }
  // D_l (decoder output; D_{L-1} is E_{L-1}) with ld = ch(l)
  uint16_t* D(int l) const { return l == L - 1 ? at<uint16_t>(lv[l].Elast) : at<uint16_t>(lv[l].D); }
  uint16_t* dD(int l) const { return l == L - 1 ? at<uint16_t>(lv[l].dElast) : at<uint16_t>(lv[l].dD); }
};

namespace {

tomo_status nfail(tomo_unet u, tomo_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (u) u->err = buf;
  g_nn_err = buf;
  return s;
}

#define NCHK(u, expr)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return nfail(u, TOMO_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

void layout(tomo_unet u) {
  size_t off = 0;
  auto take = [&](size_t bytes) { const size_t o = off; off += align_up(bytes); return o; };
  // parameters, in the order of the flat vector
  u->convs.clear();
  size_t o = 0;
  auto add = [&](int cin, int cout) {
    tomo_unet_s::Conv c;
    c.cin = cin;
    c.cout = cout;
    c.w = o;
    o += (size_t)cout * 9 * cin;
    c.b = o;
    o += cout;
    u->convs.push_back(c);
  };
  for (int l = 0; l < u->L; ++l) {
    add(l == 0 ? 1 : u->ch(l - 1), u->ch(l));
    add(u->ch(l), u->ch(l));
  }
  for (int l = u->L - 2; l >= 0; --l) {
    add(u->catld(l), u->ch(l));
    add(u->ch(l), u->ch(l));
  }
  u->head_w = o;
  o += u->C0;
  u->head_b = o;
  o += 1;
  u->n_params = o;
  u->off_theta = take(o * 4);
  u->off_m = take(o * 4);
  u->off_v = take(o * 4);
  u->off_grad = take(o * 4);
  for (size_t i = 1; i < u->convs.size(); ++i) {
    const size_t n = (size_t)u->convs[i].cout * 9 * u->convs[i].cin * 2;
    u->convs[i].wbf = take(n);
    u->convs[i].wflip = take(n);
  }
  // activations and gradients
  u->lv.assign(u->L, tomo_unet_s::Lvl{});
  size_t scratch = 0;
  for (int l = 0; l < u->L; ++l) {
    auto& v = u->lv[l];
    v.h = u->H >> l;
    v.w = u->W >> l;
    v.c = u->ch(l);
    const size_t px = (size_t)u->maxB * v.h * v.w;
    auto t16 = [&](int c) { return take(px * c * 2); };
    v.Ea = t16(v.c);
    v.dEa = t16(v.c);
    if (l < u->L - 1) {
      v.cat = t16(u->catld(l));
      v.dcat = t16(u->catld(l));
      v.Da = t16(v.c);
      v.dDa = t16(v.c);
      v.D = t16(v.c);
      v.dD = t16(v.c);
    } else {
      v.Elast = t16(v.c);
      v.dElast = t16(v.c);
    }
    if (l > 0) {
      v.P = t16(u->ch(l - 1));
      v.dP = t16(u->ch(l - 1));
    }
  }
  for (size_t i = 1; i < u->convs.size(); ++i) {
    // the level of conv i: encoder convs 2l, 2l+1; decoder convs follow
    int l;
    if (i < (size_t)2 * u->L) l = (int)i / 2;
    else l = u->L - 2 - (int)(i - 2 * u->L) / 2;
    // every batch 1..maxB must fit: bound over all pixel counts up to the largest
    const size_t npx = (size_t)u->maxB * (u->H >> l) * (u->W >> l);
    const size_t need = nn_wgrad_scratch_bound(u->convs[i].cin, u->convs[i].cout, (int)npx);
    if (need > scratch) scratch = need;
  }
  const int npx0 = u->maxB * u->H * u->W;
  const size_t in_scr = (size_t)nn_conv_in_wgrad_blocks(npx0) * u->C0 * 10;
  if (in_scr > scratch) scratch = in_scr;
  u->scratch_floats = scratch;
  u->off_scratch = take(scratch * 4);
  u->off_r = take((size_t)npx0 * 4);
  u->off_hpart = take((size_t)nn_head_back_blocks(npx0) * (u->C0 + 2) * 8);
  u->off_loss = take(8);
  u->need = off;
}

tomo_status ready(tomo_unet u, bool need_params) {
  if (!u) return nfail(nullptr, TOMO_ERR_INVALID_ARG, "network is NULL");
  if (!u->ws) return nfail(u, TOMO_ERR_NO_WORKSPACE, "no workspace attached");
  if (need_params && !u->params_ready) return nfail(u, TOMO_ERR_NOT_READY, "parameters not set");
  return TOMO_OK;
}

tomo_status prep_weights(tomo_unet u) {
  for (size_t i = 1; i < u->convs.size(); ++i) {
    const auto& c = u->convs[i];
    NCHK(u, nn_weight_prep(u->theta() + c.w, u->at<uint16_t>(c.wbf), u->at<uint16_t>(c.wflip),
                           c.cin, c.cout, u->stream));
  }
  return TOMO_OK;
}

// keep_cat: materialise the concatenation buffers (the backward pass reads them); without
// it the decoder convolutions read the upsampled half of their input directly.
tomo_status forward(tomo_unet u, const float* fbp, float* x0, int B, float s, bool keep_cat) {
  hipStream_t st = u->stream;
  const float* th = u->theta();
  const int L = u->L;
  const auto& cv = u->convs;
  NCHK(u, nn_conv_in(fbp, 1.f / s, th + cv[0].w, th + cv[0].b, u->at<uint16_t>(u->lv[0].Ea), u->C0,
                     B, u->H, u->W, st));
  for (int l = 0; l < L; ++l) {
    const auto& v = u->lv[l];
    if (l > 0) {
      // P_l was written by the epilogue of the conv that produced E_{l-1}
      const auto& c = cv[2 * l];
      NCHK(u, nn_conv3x3(u->at<uint16_t>(v.P), u->ch(l - 1), u->at<uint16_t>(c.wbf), th + c.b,
                         u->at<uint16_t>(v.Ea), v.c, nullptr, 0, c.cin, c.cout, B, v.h, v.w, true, st));
    }
    int lde;
    uint16_t* ep = u->E(l, &lde);
    const auto& c = cv[2 * l + 1];
    uint16_t* pnext = l + 1 < L ? u->at<uint16_t>(u->lv[l + 1].P) : nullptr;
    NCHK(u, nn_conv3x3(u->at<uint16_t>(v.Ea), v.c, u->at<uint16_t>(c.wbf), th + c.b, ep, lde,
                       nullptr, 0, c.cin, c.cout, B, v.h, v.w, true, st, nullptr, 0, 0, pnext, v.c));
  }
  int k = 2 * L;
  for (int l = L - 2; l >= 0; --l, k += 2) {
    const auto& v = u->lv[l];
    const int cu = u->ch(l + 1), ld = u->catld(l);
    const auto& ca = cv[k];
    if (keep_cat) {
      NCHK(u, nn_up2(u->D(l + 1), cu, u->at<uint16_t>(v.cat), ld, cu, B, v.h, v.w, st));
      NCHK(u, nn_conv3x3(u->at<uint16_t>(v.cat), ld, u->at<uint16_t>(ca.wbf), th + ca.b,
                         u->at<uint16_t>(v.Da), v.c, nullptr, 0, ca.cin, ca.cout, B, v.h, v.w, true, st));
    } else {
      int lde;
      const uint16_t* ep = u->E(l, &lde);
      NCHK(u, nn_conv3x3(ep, lde, u->at<uint16_t>(ca.wbf), th + ca.b, u->at<uint16_t>(v.Da), v.c,
                         nullptr, 0, ca.cin, ca.cout, B, v.h, v.w, true, st, u->D(l + 1), cu, cu));
    }
    const auto& cb = cv[k + 1];
    if (l == 0 && !keep_cat && (cb.cout == 32 || cb.cout == 64)) {
      // inference: the last convolution writes the head's output instead of D_0
      const NnHead hd{th + u->head_w, th + u->head_b, fbp, s, nullptr, x0};
      NCHK(u, nn_conv3x3(u->at<uint16_t>(v.Da), v.c, u->at<uint16_t>(cb.wbf), th + cb.b, nullptr, 0,
                         nullptr, 0, cb.cin, cb.cout, B, v.h, v.w, true, st, nullptr, 0, 0, nullptr, 0,
                         &hd));
      return TOMO_OK;
    }
    NCHK(u, nn_conv3x3(u->at<uint16_t>(v.Da), v.c, u->at<uint16_t>(cb.wbf), th + cb.b,
                       u->at<uint16_t>(v.D), v.c, nullptr, 0, cb.cin, cb.cout, B, v.h, v.w, true, st));
  }
  NCHK(u, nn_head(u->D(0), th + u->head_w, th + u->head_b, fbp, s, u->at<float>(u->off_r), x0, u->C0,
                  B * u->H * u->W, st));
  return TOMO_OK;
}

tomo_status wgrad(tomo_unet u, const tomo_unet_s::Conv& c, const uint16_t* dz, int ldz,
                  const uint16_t* x, int ldx, int B, int h, int w) {
  NCHK(u, nn_conv3x3_wgrad(dz, ldz, x, ldx, u->grad() + c.w, u->grad() + c.b, c.cin, c.cout, B, h, w,
                           u->at<float>(u->off_scratch), u->scratch_floats, u->stream));
  return TOMO_OK;
}

// input gradient of conv c: dx = conv(dz, flip(w)^T), masked by the forward input when given
tomo_status dgrad(tomo_unet u, const tomo_unet_s::Conv& c, const uint16_t* dz, int ldz,
                  uint16_t* dx, int lddx, const uint16_t* mask, int ldm, int B, int h, int w) {
  NCHK(u, nn_conv3x3(dz, ldz, u->at<uint16_t>(c.wflip), nullptr, dx, lddx, mask, ldm, c.cout, c.cin,
                     B, h, w, false, u->stream));
  return TOMO_OK;
}

tomo_status backward(tomo_unet u, const float* fbp, const float* target, int B, float s,
                     double* loss) {
  hipStream_t st = u->stream;
  const int L = u->L;
  const auto& cv = u->convs;
  const int npx = B * u->H * u->W;
  NCHK(u, nn_head_back(u->at<float>(u->off_r), fbp, target, 1.f / s, u->D(0), u->theta() + u->head_w,
                       u->dD(0), u->at<double>(u->off_hpart), u->grad() + u->head_w,
                       u->grad() + u->head_b, loss, u->C0, npx, st));
  tomo_status r;
  // decoder, from the head upwards
  for (int l = 0; l <= L - 2; ++l) {
    const auto& v = u->lv[l];
    const int kb = 2 * L + 2 * (L - 2 - l) + 1, ka = kb - 1;
    const int ld = u->catld(l);
    if ((r = wgrad(u, cv[kb], u->dD(l), v.c, u->at<uint16_t>(v.Da), v.c, B, v.h, v.w)) != TOMO_OK) return r;
    if ((r = dgrad(u, cv[kb], u->dD(l), v.c, u->at<uint16_t>(v.dDa), v.c, u->at<uint16_t>(v.Da), v.c,
                   B, v.h, v.w)) != TOMO_OK) return r;
    if ((r = wgrad(u, cv[ka], u->at<uint16_t>(v.dDa), v.c, u->at<uint16_t>(v.cat), ld, B, v.h, v.w)) != TOMO_OK)
      return r;
    if ((r = dgrad(u, cv[ka], u->at<uint16_t>(v.dDa), v.c, u->at<uint16_t>(v.dcat), ld,
                   u->at<uint16_t>(v.cat), ld, B, v.h, v.w)) != TOMO_OK) return r;
    const int cu = u->ch(l + 1);
    NCHK(u, nn_up2_back(u->at<uint16_t>(v.dcat), ld, u->dD(l + 1), cu, cu, B, v.h, v.w, st));
  }
  // encoder, from the bottleneck down
  for (int l = L - 1; l >= 0; --l) {
    const auto& v = u->lv[l];
    int lde;
    uint16_t* de = u->dE(l, &lde);
    const auto& cb = cv[2 * l + 1];
    if ((r = wgrad(u, cb, de, lde, u->at<uint16_t>(v.Ea), v.c, B, v.h, v.w)) != TOMO_OK) return r;
    if ((r = dgrad(u, cb, de, lde, u->at<uint16_t>(v.dEa), v.c, u->at<uint16_t>(v.Ea), v.c, B, v.h,
                   v.w)) != TOMO_OK) return r;
    const auto& ca = cv[2 * l];
    if (l == 0) {
      NCHK(u, nn_conv_in_wgrad(u->at<uint16_t>(v.dEa), fbp, 1.f / s, u->grad() + ca.w,
                               u->grad() + ca.b, u->C0, B, u->H, u->W, u->at<float>(u->off_scratch),
                               u->scratch_floats, st));
    } else {
      const int cp = u->ch(l - 1);
      if ((r = wgrad(u, ca, u->at<uint16_t>(v.dEa), v.c, u->at<uint16_t>(v.P), cp, B, v.h, v.w)) != TOMO_OK)
        return r;
      if ((r = dgrad(u, ca, u->at<uint16_t>(v.dEa), v.c, u->at<uint16_t>(v.dP), cp, nullptr, 0, B, v.h,
                     v.w)) != TOMO_OK) return r;
      int ldp, ldpd;
      const uint16_t* ep = u->E(l - 1, &ldp);
      uint16_t* dep = u->dE(l - 1, &ldpd);
      const auto& vp = u->lv[l - 1];
      NCHK(u, nn_avgpool2_back(u->at<uint16_t>(v.dP), cp, ep, ldp, dep, ldpd, cp, B, vp.h, vp.w, st));
    }
  }
  return TOMO_OK;
}

tomo_status check_call(tomo_unet u, const void* a, const void* b, int B, float s) {
  if (!a || !b) return nfail(u, TOMO_ERR_INVALID_ARG, "NULL array");
  if (B < 1 || B > u->maxB) return nfail(u, TOMO_ERR_INVALID_ARG, "batch %d outside 1..%d", B, u->maxB);
  if (!(s > 0.f) || !std::isfinite(s)) return nfail(u, TOMO_ERR_INVALID_ARG, "scale must be > 0");
  return TOMO_OK;
}

}  // namespace

extern "C" {

const char* tomo_unet_last_error(tomo_unet u) { return u ? u->err.c_str() : g_nn_err.c_str(); }

tomo_status tomo_unet_create(int32_t levels, int32_t base_channels, int32_t max_batch,
                             int32_t height, int32_t width, void* hip_stream, tomo_unet* out) {
  if (!out) return nfail(nullptr, TOMO_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (levels < 1 || levels > 6) return nfail(nullptr, TOMO_ERR_INVALID_ARG, "levels %d outside 1..6", levels);
  if (base_channels < 32 || base_channels > 256 || base_channels % 32 ||
      (base_channels << (levels - 1)) > 1024)
    return nfail(nullptr, TOMO_ERR_INVALID_ARG,
                 "base channels %d: a multiple of 32 in 32..256, at most 1024 at the bottom", base_channels);
  if (max_batch < 1) return nfail(nullptr, TOMO_ERR_INVALID_ARG, "max_batch must be >= 1");
  const int div = 1 << (levels - 1);
  if (height < div || width < div || height % div || width % div)
    return nfail(nullptr, TOMO_ERR_INVALID_ARG, "image %dx%d must be a positive multiple of %d", height,
                 width, div);
  if ((int64_t)max_batch * height * width > (int64_t)1 << 30 || height > 32767 || width > 32767)
    return nfail(nullptr, TOMO_ERR_INVALID_ARG, "batch x image too large (height, width <= 32767)");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
    return nfail(nullptr, TOMO_ERR_NO_DEVICE, "no HIP device");
  auto* u = new tomo_unet_s();
  u->L = levels;
  u->C0 = base_channels;
  u->maxB = max_batch;
  u->H = height;
  u->W = width;
  u->stream = static_cast<hipStream_t>(hip_stream);
  layout(u);
  *out = u;
  return TOMO_OK;
}

tomo_status tomo_unet_workspace_size(tomo_unet u, size_t* bytes) {
  if (!u || !bytes) return nfail(u, TOMO_ERR_INVALID_ARG, "NULL argument");
  *bytes = u->need;
  return TOMO_OK;
}

tomo_status tomo_unet_set_workspace(tomo_unet u, void* dev, size_t bytes) {
  if (!u || !dev) return nfail(u, TOMO_ERR_INVALID_ARG, "NULL argument");
  if (reinterpret_cast<uintptr_t>(dev) % kAlign) return nfail(u, TOMO_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  if (bytes < u->need) return nfail(u, TOMO_ERR_WORKSPACE_TOO_SMALL, "workspace %zu < %zu bytes", bytes, u->need);
  u->ws = static_cast<char*>(dev);
  u->ws_bytes = bytes;
  u->params_ready = false;
  return TOMO_OK;
}

tomo_status tomo_unet_num_params(tomo_unet u, int64_t* n) {
  if (!u || !n) return nfail(u, TOMO_ERR_INVALID_ARG, "NULL argument");
  *n = (int64_t)u->n_params;
  return TOMO_OK;
}

tomo_status tomo_unet_set_params(tomo_unet u, const float* theta) {
  if (tomo_status s = ready(u, false); s != TOMO_OK) return s;
  if (!theta) return nfail(u, TOMO_ERR_INVALID_ARG, "theta is NULL");
  const size_t n = u->n_params * 4;
  NCHK(u, hipMemcpyAsync(u->theta(), theta, n, hipMemcpyDeviceToDevice, u->stream));
  NCHK(u, hipMemsetAsync(u->at<float>(u->off_m), 0, n, u->stream));
  NCHK(u, hipMemsetAsync(u->at<float>(u->off_v), 0, n, u->stream));
  u->step = 0;
  if (tomo_status s = prep_weights(u); s != TOMO_OK) return s;
  u->params_ready = true;
  return TOMO_OK;
}

tomo_status tomo_unet_get_params(tomo_unet u, float* theta) {
  if (tomo_status s = ready(u, true); s != TOMO_OK) return s;
  if (!theta) return nfail(u, TOMO_ERR_INVALID_ARG, "theta is NULL");
  NCHK(u, hipMemcpyAsync(theta, u->theta(), u->n_params * 4, hipMemcpyDeviceToDevice, u->stream));
  return TOMO_OK;
}

tomo_status tomo_unet_forward(tomo_unet u, const float* fbp, float* x0, int32_t batch, float scale) {
  if (tomo_status s = ready(u, true); s != TOMO_OK) return s;
  if (tomo_status s = check_call(u, fbp, x0, batch, scale); s != TOMO_OK) return s;
  return forward(u, fbp, x0, batch, scale, false);
}

tomo_status tomo_unet_loss_grad(tomo_unet u, const float* fbp, const float* target, int32_t batch,
                                float scale, float* grad, double* loss) {
  if (tomo_status s = ready(u, true); s != TOMO_OK) return s;
  if (tomo_status s = check_call(u, fbp, target, batch, scale); s != TOMO_OK) return s;
  tomo_status s = forward(u, fbp, nullptr, batch, scale, true);
  if (s == TOMO_OK) s = backward(u, fbp, target, batch, scale, loss ? loss : u->at<double>(u->off_loss));
  if (s == TOMO_OK && grad)
    NCHK(u, hipMemcpyAsync(grad, u->grad(), u->n_params * 4, hipMemcpyDeviceToDevice, u->stream));
  return s;
}

tomo_status tomo_unet_train_step(tomo_unet u, const float* fbp, const float* target, int32_t batch,
                                 float scale, float lr, double* loss) {
  if (tomo_status s = ready(u, true); s != TOMO_OK) return s;
  if (tomo_status s = check_call(u, fbp, target, batch, scale); s != TOMO_OK) return s;
  if (!(lr > 0.f) || !std::isfinite(lr)) return nfail(u, TOMO_ERR_INVALID_ARG, "learning rate must be > 0");
  tomo_status s = forward(u, fbp, nullptr, batch, scale, true);
  if (s == TOMO_OK) s = backward(u, fbp, target, batch, scale, loss ? loss : u->at<double>(u->off_loss));
  if (s != TOMO_OK) return s;
  u->step += 1;
  const double b1 = 0.9, b2 = 0.999;
  const float c1 = (float)(1.0 / (1.0 - std::pow(b1, (double)u->step)));
  const float c2 = (float)(1.0 / (1.0 - std::pow(b2, (double)u->step)));
  NCHK(u, nn_adam(u->theta(), u->grad(), u->at<float>(u->off_m), u->at<float>(u->off_v), u->n_params,
                  lr, (float)b1, (float)b2, c1, c2, 1e-8f, u->stream));
  return prep_weights(u);
}

tomo_status tomo_unet_set_domain(tomo_unet u, const tomo_unet_domain_t* d) {
  if (!u) return nfail(nullptr, TOMO_ERR_INVALID_ARG, "network is NULL");
  if (!d) {
    u->has_domain = false;
    return TOMO_OK;
  }
  if (d->n < 1 || d->n_det < 2 || d->n_angles_min < 1 || d->n_angles_max < d->n_angles_min ||
      !(d->beta >= 0.0) || !(d->p >= 1.0) || !(d->sigma > 0.0) || !(d->T > 0.0) ||
      (d->neighbours != 8 && d->neighbours != 26))
    return nfail(u, TOMO_ERR_INVALID_ARG, "invalid training domain");
  u->domain = *d;
  u->has_domain = true;
  return TOMO_OK;
}

tomo_status tomo_unet_destroy(tomo_unet u) {
  delete u;
  return TOMO_OK;
}

tomo_status tomo_nn_conv3x3(const uint16_t* x, int32_t ldx, const uint16_t* w, const float* bias,
                            uint16_t* y, int32_t ldy, const uint16_t* mask, int32_t ldm, int32_t cin,
                            int32_t cout, int32_t batch, int32_t height, int32_t width, int32_t relu,
                            void* hip_stream) {
  if (!x || !w || !y) return nfail(nullptr, TOMO_ERR_INVALID_ARG, "NULL array");
  if (cin % 32 || cout % 32 || cin < 32 || cout < 32 || ldx < cin || ldy < cout || ldx % 8 || ldy % 8 ||
      (mask && (ldm < cout || ldm % 8)) || batch < 1 || height < 1 || width < 1 || height > 32767 ||
      width > 32767)
    return nfail(nullptr, TOMO_ERR_INVALID_ARG, "unsupported shape");
  if ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(w)) % 16)
    return nfail(nullptr, TOMO_ERR_INVALID_ARG, "x and w must be 16-byte aligned");
  if (relu && (!bias || mask)) return nfail(nullptr, TOMO_ERR_INVALID_ARG, "ReLU form needs a bias and no mask");
  if (bias && mask) return nfail(nullptr, TOMO_ERR_INVALID_ARG, "a masked form has no bias");
  const hipError_t e = nn_conv3x3(x, ldx, w, bias, y, ldy, mask, ldm, cin, cout, batch, height, width,
                                  relu != 0, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return nfail(nullptr, TOMO_ERR_HIP, "conv3x3: %s", hipGetErrorString(e));
  return TOMO_OK;
}

tomo_status tomo_nn_wgrad_scratch(int32_t cin, int32_t cout, int32_t npx, size_t* floats) {
  if (!floats || cin < 32 || cout < 32 || cin % 32 || cout % 32 || npx < 1)
    return nfail(nullptr, TOMO_ERR_INVALID_ARG, "unsupported shape");
  *floats = nn_wgrad_plan(cin, cout, npx).scratch_floats;
  return TOMO_OK;
}

tomo_status tomo_nn_conv3x3_wgrad(const uint16_t* dz, int32_t ldz, const uint16_t* x, int32_t ldx,
                                  float* dw, float* db, int32_t cin, int32_t cout, int32_t batch,
                                  int32_t height, int32_t width, float* scratch,
                                  size_t scratch_floats, void* hip_stream) {
  if (!dz || !x || !dw || !db || !scratch) return nfail(nullptr, TOMO_ERR_INVALID_ARG, "NULL array");
  if (cin % 32 || cout % 32 || cin < 32 || cout < 32 || ldz < cout || ldx < cin || ldz % 8 || ldx % 8 ||
      batch < 1 || height < 1 || width < 1)
    return nfail(nullptr, TOMO_ERR_INVALID_ARG, "unsupported shape");
  if ((reinterpret_cast<uintptr_t>(dz) | reinterpret_cast<uintptr_t>(x)) % 16)
    return nfail(nullptr, TOMO_ERR_INVALID_ARG, "dz and x must be 16-byte aligned");
  if (nn_wgrad_plan(cin, cout, batch * height * width).scratch_floats > scratch_floats)
    return nfail(nullptr, TOMO_ERR_WORKSPACE_TOO_SMALL, "scratch too small");
  const hipError_t e = nn_conv3x3_wgrad(dz, ldz, x, ldx, dw, db, cin, cout, batch, height, width,
                                        scratch, scratch_floats, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return nfail(nullptr, TOMO_ERR_HIP, "conv3x3 wgrad: %s", hipGetErrorString(e));
  return TOMO_OK;
}

}  // extern "C"

namespace tomo {
bool unet_view(tomo_unet u, UnetView* v) {
  if (!u || !v) return false;
  v->height = u->H;
  v->width = u->W;
  v->max_batch = u->maxB;
  v->ready = u->ws != nullptr && u->params_ready;
  v->has_domain = u->has_domain;
  v->domain = u->domain;
  v->stream = u->stream;
  return true;
}
}  // namespace tomo

extern "C" {

// ---- weight gradient without caller scratch ------------------------------------------------
// The split partial sums of tomo_nn_conv3x3_wgrad_noalloc live in this file-scope device array
// (one copy per GPU, held until the process ends).  Host code never passes its name to a
// kernel: the device address is looked up once per device with hipGetSymbolAddress and kept.
// Every split partial is written before it is summed, so nothing needs clearing between calls.
static __device__ __align__(256) float wgrad_scratch[TOMO_NN_WGRAD_NOALLOC_MAX_FLOATS];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_dev[kMaxDevices] = {};

hipError_t scratch_on_current_device(float** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(wgrad_scratch));
    if (e != hipSuccess) return e;
    g_scratch_dev[dev] = static_cast<float*>(ptr);
  }
  *out = g_scratch_dev[dev];
  return hipSuccess;
}
}  // namespace

tomo_status tomo_nn_conv3x3_wgrad_noalloc(const uint16_t* dz, int32_t ldz, const uint16_t* x,
                                          int32_t ldx, float* dw, float* db, int32_t cin,
                                          int32_t cout, int32_t batch, int32_t height,
                                          int32_t width, void* hip_stream) {
  if (!dz || !x || !dw || !db) return nfail(nullptr, TOMO_ERR_INVALID_ARG, "NULL array");
  if (cin % 32 || cout % 32 || cin < 32 || cout < 32 || ldz < cout || ldx < cin || ldz % 8 || ldx % 8 ||
      batch < 1 || height < 1 || width < 1)
    return nfail(nullptr, TOMO_ERR_INVALID_ARG, "unsupported shape");
  if ((reinterpret_cast<uintptr_t>(dz) | reinterpret_cast<uintptr_t>(x)) % 16)
    return nfail(nullptr, TOMO_ERR_INVALID_ARG, "dz and x must be 16-byte aligned");
  const size_t need = nn_wgrad_plan(cin, cout, batch * height * width).scratch_floats;
  if (need > (size_t)TOMO_NN_WGRAD_NOALLOC_MAX_FLOATS)
    return nfail(nullptr, TOMO_ERR_WORKSPACE_TOO_SMALL,
                 "split sums need %zu floats, more than the %d of the static scratch", need,
                 TOMO_NN_WGRAD_NOALLOC_MAX_FLOATS);
  float* scr = nullptr;
  hipError_t e = scratch_on_current_device(&scr);
  if (e != hipSuccess)
    return nfail(nullptr, TOMO_ERR_HIP, "static scratch address: %s", hipGetErrorString(e));
  e = nn_conv3x3_wgrad(dz, ldz, x, ldx, dw, db, cin, cout, batch, height, width, scr,
                       (size_t)TOMO_NN_WGRAD_NOALLOC_MAX_FLOATS, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return nfail(nullptr, TOMO_ERR_HIP, "conv3x3 wgrad: %s", hipGetErrorString(e));
  return TOMO_OK;
}

}  // extern "C"
