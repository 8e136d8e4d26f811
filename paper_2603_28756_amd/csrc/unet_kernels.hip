// Kernels of the learned start: a 2D U-Net in bfloat16 with float32 accumulation on the
// gfx950 matrix cores (v_mfma_f32_16x16x32_bf16), its backward pass and an Adam update.
//
// Tensors are NHWC ([batch][row][column][channel]) bfloat16 stored as uint16_t; a tensor
// argument is a pointer to its first channel plus `ld`, the channel count of the buffer
// it lives in (a skip concatenation is a channel range of a wider buffer).
//
// MFMA 16x16x32 bf16 operand layout (lane l of a wave): A (16 x 32) row l%16, k values
// 8*(l/16) .. 8*(l/16)+7; B (32 x 16) column l%16, the same k values; D (16 x 16) rows
// 4*(l/16) .. +3 of column l%16.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "nn_kernels.hpp"

namespace tomo {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// float -> bfloat16, round to nearest, ties to even (NaN kept quiet)
TOMO_DEV uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
TOMO_DEV float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

TOMO_DEV u16x8 ld8(const uint16_t* p) { return *reinterpret_cast<const u16x8*>(p); }
TOMO_DEV void st8(uint16_t* p, u16x8 v) { *reinterpret_cast<u16x8*>(p) = v; }
TOMO_DEV f32x4 mfma(u16x8 a, u16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                 __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

// ------------------------------------------------------------------ 3x3 conv, forward
// y[p, co] = act(bias[co] + sum_{tap, ci} w[co][tap][ci] x[p + tap, ci]) (zero padding), then
// multiplied by (mask[p, co] > 0) when a mask is given (the ReLU derivative of the forward
// activation when this kernel computes an input gradient).
// 3x3 conv on 2D pixel tiles staged through LDS.  A block owns a tile 16 pixels wide and
// 4*RPW rows high (wave w: rows w*RPW .. w*RPW+RPW-1) x BN output channels.  For each chunk
// of 32 input channels it stages (a) the input tile with a one-pixel halo, 64 bytes per
// pixel, and (b) the weights of all 9 taps for its BN channels; every staging load of a chunk
// is issued before the first LDS store, so their latencies overlap.  Then every wave runs
// 9 taps x RPW rows x BN/16 MFMAs reading both operands from LDS (each 16-pixel fragment and
// each 16-channel weight fragment is one contiguous kilobyte).  The weights are the MFMA's
// first operand, so a lane's accumulator holds 4 consecutive output channels of one pixel
// and the results leave as 8-byte stores.
template <int BN, int RPW>
struct ConvTile {
  static constexpr int TW = 16, TH = 4 * RPW, HW_ = TW + 2, HH = TH + 2;
  static constexpr int A_PIX = HH * HW_;                 // halo pixels
  static constexpr int A_BYTES = A_PIX * 64;              // 32 bf16 channels per pixel
  static constexpr int B_BYTES = 9 * BN * 64;             // [tap][co][32 channels]
  static constexpr int BYTES = A_BYTES + B_BYTES;
  static constexpr int A_EL = A_PIX * 4, B_EL = 9 * BN * 4;  // 16-byte staging elements
  static constexpr int NA = (A_EL + 255) / 256, NB = (B_EL + 255) / 256;  // per thread
};

// generic pointer into shared memory -> LDS address space (the destination operand of
// global_load_lds)
TOMO_DEV __attribute__((address_space(3))) void* lds_ptr(uint16_t* p) {
  return (__attribute__((address_space(3))) void*)(p);
}

TOMO_DEV void st4bf(uint16_t* p, const uint16_t (&v)[4]) {
  *reinterpret_cast<uint2*>(p) = make_uint2((uint32_t)v[0] | ((uint32_t)v[1] << 16),
                                            (uint32_t)v[2] | ((uint32_t)v[3] << 16));
}

// UPCAT: the input is the concatenation [up2(xu), x]: channels below cu are read from the
// half-resolution tensor xu at (row/2, column/2), the others from x (channel c - cu).
// POOL: also write the 2x2 average of the (bfloat16-rounded) output to pool (channel
// stride ldp, half resolution); a 2x2 block spans two rows of one lane and the lane pair
// (2m, 2m+1).
// HEAD: the output is not stored; the 1x1 head over the block's BN (= all) channels is
// written instead (r = hb + sum_c hw[c] y[c], x0 = fbp + s r).
template <int BN, int RPW, bool RELU, bool BIAS, bool MASK, bool UPCAT, bool POOL, bool HEAD>
// waves per SIMD: what the LDS tile allows (4 blocks of BN = 32, 2 of BN = 64 per CU), 3 for
// the concatenating and head forms, which spill at 4
__global__ void __launch_bounds__(256, BN == 32 ? ((UPCAT || HEAD) ? 3 : 4) : 2)
conv3x3_tile_kernel(const uint16_t* __restrict__ x, int ldx, const uint16_t* __restrict__ w,
                    const float* __restrict__ bias, uint16_t* __restrict__ y, int ldy,
                    const uint16_t* __restrict__ mask, int ldm, int cin, int H, int W, int ntx,
                    int nty, const uint16_t* __restrict__ xu, int ldu, int cu,
                    uint16_t* __restrict__ pool, int ldp, NnHead hd) {
  using T = ConvTile<BN, RPW>;
  constexpr int NJ = BN / 16;
  __shared__ __align__(16) unsigned char smem[T::BYTES];
  uint16_t* sa = reinterpret_cast<uint16_t*>(smem);
  uint16_t* sb = reinterpret_cast<uint16_t*>(smem + T::A_BYTES);
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  int bx = blockIdx.x;
  const int tx = bx % ntx;
  bx /= ntx;
  const int ty = bx % nty;
  const int cot = bx / nty;
  const int x0 = tx * T::TW, y0 = ty * T::TH, co0 = cot * BN;
  const size_t img = (size_t)blockIdx.y * H * W;
  const int kq = (lane >> 4) * 8, lc = lane & 15;
  f32x4 acc[RPW][NJ];
#pragma unroll
  for (int r = 0; r < RPW; ++r)
#pragma unroll
    for (int j = 0; j < NJ; ++j) acc[r][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  // HEAD: the FBP values and head weights of this lane, read before the convolution so that
  // their latency is hidden behind it
  float fbv[RPW], hwv[NJ][4];
  if constexpr (HEAD) {
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
      const int gy = y0 + wave * RPW + r, gx = x0 + lc;
      fbv[r] = (gy < H && gx < W) ? hd.fbp[img + (size_t)gy * W + gx] : 0.f;
    }
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
      for (int i = 0; i < 4; ++i) hwv[j][i] = hd.hw[16 * j + 4 * (lane >> 4) + i];
  }
  // staging element e: input pixel e / 4 (halo tile, row-major) channels 8 (e % 4) .. +7,
  // or weight row e / 4 = tap * BN + co, channels 8 (e % 4) .. +7; LDS byte offset 16 e.
  // Elements t + 256 i of one wave are 64 consecutive 16-byte slots, so each goes straight
  // from memory to LDS (global_load_lds_dwordx4: lane l of the wave writes its wave base
  // + 16 l), with no registers in between.  A halo pixel outside the image loads a pixel
  // inside it and is overwritten with zeros once the copies have landed.
  bool zero_a[T::NA];
  int src_a[T::NA];  // clamped pixel of each element, as (row, column) packed
#pragma unroll
  for (int i = 0; i < T::NA; ++i) {
    const int e = t + 256 * i;
    const int pix = e >> 2;
    const int hy = pix / T::HW_, hx = pix - hy * T::HW_;
    const int gy = y0 + hy - 1, gx = x0 + hx - 1;
    zero_a[i] = e < T::A_EL && !(gy >= 0 && gy < H && gx >= 0 && gx < W);
    src_a[i] = (min(max(gy, 0), H - 1) << 16) | min(max(gx, 0), W - 1);
  }
  auto stage = [&](int c0, uint16_t* da, uint16_t* db) {
#pragma unroll
    for (int i = 0; i < T::NA; ++i) {
      const int e = t + 256 * i;
      if (e < T::A_EL) {
        const int q = (e & 3) * 8, gy = src_a[i] >> 16, gx = src_a[i] & 0xffff;
        const uint16_t* src =
            (UPCAT && c0 < cu)
                ? xu + (((size_t)blockIdx.y * (H / 2) + gy / 2) * (W / 2) + gx / 2) * ldu + c0 + q
                : x + (img + (size_t)gy * W + gx) * ldx + c0 - (UPCAT ? cu : 0) + q;
        __builtin_amdgcn_global_load_lds(src, lds_ptr(da + (256 * i + 64 * wave) * 8), 16, 0, 0);
      }
    }
#pragma unroll
    for (int i = 0; i < T::NB; ++i) {
      const int e = t + 256 * i;
      if (e < T::B_EL) {
        const int q = (e & 3) * 8, rest = e >> 2;
        const int co = rest % BN, tap = rest / BN;
        __builtin_amdgcn_global_load_lds(w + ((size_t)(co0 + co) * 9 + tap) * cin + c0 + q,
                                         lds_ptr(db + (256 * i + 64 * wave) * 8), 16, 0, 0);
      }
    }
  };
  // wait for this thread's copies, zero its out-of-image halo elements, publish the chunk
  auto land = [&](uint16_t* da) {
    __builtin_amdgcn_s_waitcnt(0);
#pragma unroll
    for (int i = 0; i < T::NA; ++i)
      if (zero_a[i]) st8(da + (t + 256 * i) * 8, u16x8{0, 0, 0, 0, 0, 0, 0, 0});
    __syncthreads();
  };
  auto compute = [&](const uint16_t* ca, const uint16_t* cb) {
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
      const int ky = tap / 3, kx = tap % 3;
      u16x8 b[NJ];
#pragma unroll
      for (int j = 0; j < NJ; ++j) b[j] = ld8(cb + (tap * BN + j * 16 + lc) * 32 + kq);
#pragma unroll
      for (int r = 0; r < RPW; ++r) {
        const u16x8 a = ld8(ca + ((wave * RPW + r + ky) * T::HW_ + lc + kx) * 32 + kq);
#pragma unroll
        for (int j = 0; j < NJ; ++j) acc[r][j] = mfma(b[j], a, acc[r][j]);
      }
    }
  };
  for (int c0 = 0; c0 < cin; c0 += 32) {
    stage(c0, sa, sb);
    land(sa);
    compute(sa, sb);
    __syncthreads();
  }
  // lane holds channels co0 + 16 j + cq + i (i = 0..3) of pixel x0 + lc in row
  // y0 + wave * RPW + r
  const int gx = x0 + lc, cq = 4 * (lane >> 4);
  float bv[NJ][4];
#pragma unroll
  for (int j = 0; j < NJ; ++j)
#pragma unroll
    for (int i = 0; i < 4; ++i) bv[j][i] = BIAS ? bias[co0 + 16 * j + cq + i] : 0.f;
  const float hb = HEAD ? hd.hb[0] : 0.f;
  uint16_t ob[RPW][NJ][4];
#pragma unroll
  for (int r = 0; r < RPW; ++r) {
    const int gy = y0 + wave * RPW + r;
    const bool ok = gy < H && gx < W;
    const size_t pix = img + (size_t)gy * W + gx;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int co = co0 + 16 * j + cq;
      uint2 mk = make_uint2(0u, 0u);
      if (MASK && ok) mk = *reinterpret_cast<const uint2*>(mask + pix * ldm + co);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float v = acc[r][j][i] + bv[j][i];
        if (RELU) v = fmaxf(v, 0.f);
        if (MASK) {
          const uint32_t mw = (i < 2) ? mk.x : mk.y;
          if (!(bf2f((uint16_t)(mw >> (16 * (i & 1)))) > 0.f)) v = 0.f;
        }
        ob[r][j][i] = ok ? f2bf(v) : (uint16_t)0;
      }
      if (!HEAD && ok) st4bf(y + pix * ldy + co, ob[r][j]);
    }
    if constexpr (HEAD) {
      // the pixel's channels lie in lanes lc, lc + 16, lc + 32, lc + 48
      float part = 0.f;
#pragma unroll
      for (int j = 0; j < NJ; ++j)
#pragma unroll
        for (int i = 0; i < 4; ++i) part = fmaf(hwv[j][i], bf2f(ob[r][j][i]), part);
      part += __shfl_xor(part, 16);
      part += __shfl_xor(part, 32);
      if (lane < 16 && ok) {
        const float a = hb + part;
        if (hd.r) hd.r[pix] = a;
        hd.x0[pix] = fbv[r] + hd.s * a;
      }
    }
  }
  if constexpr (POOL) {
    const int h2 = H / 2, w2 = W / 2;
    const int px2 = gx >> 1;
#pragma unroll
    for (int r = 0; r < RPW; r += 2) {
      const int py = (y0 + wave * RPW + r) / 2;
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        uint16_t pv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          // ((top left + top right) + bottom left) + bottom right
          const float a = bf2f(ob[r][j][i]), c = bf2f(ob[r + 1][j][i]);
          const float an = __shfl_xor(a, 1), cn = __shfl_xor(c, 1);
          pv[i] = f2bf(0.25f * (((a + an) + c) + cn));
        }
        if (!(lane & 1) && py < h2 && px2 < w2)
          st4bf(pool + (((size_t)blockIdx.y * h2 + py) * w2 + px2) * ldp + co0 + 16 * j + cq, pv);
      }
    }
  }
}

// ------------------------------------------------------------------ 3x3 conv, weights
// part[s][co][n] = sum over the pixels of split s of dz[p, co] x[p + tap(n), ci(n)],
// n = tap * cin + ci; partb[s][co] = sum over the same pixels of dz[p, co].  This kernel serves
// widths that are not a multiple of 32 (the haloed kernel below takes the others).  A block owns a
// 64 x 64 tile of (co, n) and one pixel split; 32-pixel steps are staged through LDS
// transposed so that the K dimension (pixels) is contiguous for the matrix-core operands.
constexpr int WG_K = 32, WG_PAD = 8;

__global__ void __launch_bounds__(256)
conv3x3_wgrad_kernel(const uint16_t* __restrict__ dz, int ldz, const uint16_t* __restrict__ x,
                     int ldx, float* __restrict__ part, float* __restrict__ partb, int cin,
                     int cout, int H, int W, int npx, int px_per_split) {
  __shared__ __align__(16) uint16_t sa[64][WG_K + WG_PAD];  // [co][pixel]
  __shared__ __align__(16) uint16_t sb[64][WG_K + WG_PAD];  // [n][pixel]
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const int n0 = blockIdx.x * 64, co0 = blockIdx.y * 64, s = blockIdx.z;
  const int nn = 9 * cin;
  const int pb = s * px_per_split, pe = min(npx, pb + px_per_split);
  const int cw = (wave & 1) * 32, nw = (wave >> 1) * 32;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  // staging: threads 0..127 read dz, threads 128..255 read x; each takes two adjacent
  // pixels (2 pp, 2 pp + 1) of one 8-channel group and writes each channel's pair of pixels
  // as one 32-bit LDS word (the tiles are stored [channel][pixel])
  const int half = t >> 7, pp = (t & 127) >> 3, cg = (t & 7) * 8;
  // the column group of the x tile: tap and channel are fixed over the loop
  const int n = n0 + cg;
  const int tap = n < nn ? n / cin : 0, ci = n - tap * cin;
  const int ky = tap / 3 - 1, kx = tap % 3 - 1;
  float bsum = 0.f;
  const int HW = H * W;
  uint16_t(*dst)[WG_K + WG_PAD] = half ? sb : sa;
  // image coordinates (slice, row, column) of the two pixels, stepped by WG_K per chunk so
  // that the loop divides only once
  int cb[2], cy[2], cx[2];
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const int p = pb + 2 * pp + e;
    cb[e] = p / HW;
    const int rem = p - cb[e] * HW;
    cy[e] = rem / W;
    cx[e] = rem - cy[e] * W;
  }
  // the chunk at p0 into registers; the next chunk's loads are issued before the current
  // chunk's products so that their latency is hidden behind them
  u16x8 v[2];
  auto load_chunk = [&](int p0) {
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int p = p0 + 2 * pp + e;
      v[e] = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
      if (p < pe) {
        if (half == 0) {
          if (co0 + cg < cout) v[e] = ld8(dz + (size_t)p * ldz + co0 + cg);
        } else if (n < nn) {
          const int yy = cy[e] + ky, xx = cx[e] + kx;
          if (yy >= 0 && yy < H && xx >= 0 && xx < W)
            v[e] = ld8(x + ((size_t)cb[e] * HW + (size_t)yy * W + xx) * ldx + ci);
        }
      }
      cx[e] += WG_K;
      while (cx[e] >= W) {
        cx[e] -= W;
        if (++cy[e] == H) {
          cy[e] = 0;
          ++cb[e];
        }
      }
    }
  };
  load_chunk(pb);
  for (int p0 = pb; p0 < pe; p0 += WG_K) {
#pragma unroll
    for (int j = 0; j < 8; ++j)
      *reinterpret_cast<uint32_t*>(&dst[cg + j][2 * pp]) =
          (uint32_t)v[0][j] | ((uint32_t)v[1][j] << 16);
    __syncthreads();
    if (p0 + WG_K < pe) load_chunk(p0 + WG_K);
    if (blockIdx.x == 0 && t < 64) {
#pragma unroll 8
      for (int k = 0; k < WG_K; ++k) bsum += bf2f(sa[t][k]);
    }
    const int kq = (lane >> 4) * 8;
    u16x8 a[2], bb[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) a[i] = ld8(&sa[cw + 16 * i + (lane & 15)][kq]);
#pragma unroll
    for (int j = 0; j < 2; ++j) bb[j] = ld8(&sb[nw + 16 * j + (lane & 15)][kq]);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = mfma(a[i], bb[j], acc[i][j]);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = n0 + nw + 16 * j + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int co = co0 + cw + 16 * i + 4 * (lane >> 4) + r;
        if (co < cout && col < nn) part[((size_t)s * cout + co) * nn + col] = acc[i][j][r];
      }
    }
  if (blockIdx.x == 0 && t < 64 && co0 + t < cout) partb[(size_t)s * cout + co0 + t] = bsum;
}

// The same weight gradient over haloed row tiles (W a multiple of 32): a block owns 32 output
// channels x 32 input channels x all 9 taps and one pixel split, walked in 32-pixel chunks
// of one image row.  Per chunk it stages dz [32 co][32 pixels] and the input rows y-1, y, y+1
// at columns x0-1 .. x0+32 of its 32 channels, so that each input value is fetched once per
// row rather than once per tap; a tap's column shift is taken from an aligned 16-byte read
// and the 32-bit word after it.  Wave w: co tile w & 1, ci tile w >> 1, all 9 taps.
constexpr int WH_Q = 40;  // staged columns per row (34 used)

TOMO_DEV u16x8 shift_cols(u16x8 lo, uint32_t next, int s) {
  const uint4 d = __builtin_bit_cast(uint4, lo);
  if (s == 0) return lo;
  if (s == 2) return __builtin_bit_cast(u16x8, make_uint4(d.y, d.z, d.w, next));
  return __builtin_bit_cast(u16x8, make_uint4((d.x >> 16) | (d.y << 16), (d.y >> 16) | (d.z << 16),
                                              (d.z >> 16) | (d.w << 16), (d.w >> 16) | (next << 16)));
}

__global__ void __launch_bounds__(256)
conv3x3_wgrad_halo_kernel(const uint16_t* __restrict__ dz, int ldz, const uint16_t* __restrict__ x,
                          int ldx, float* __restrict__ part, float* __restrict__ partb, int cin,
                          int cout, int H, int W, int npx, int px_per_split) {
  __shared__ __align__(16) uint16_t sa[32][WG_K + WG_PAD];  // [co][pixel]
  __shared__ __align__(16) uint16_t sx[32][3][WH_Q];        // [ci][row][column + 1]
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const int ci0 = blockIdx.x * 32, co0 = blockIdx.y * 32, s = blockIdx.z;
  const int nn = 9 * cin;
  const int pb = s * px_per_split, pe = min(npx, pb + px_per_split);
  const int HW = H * W;
  // chunk position (slice, row, first column), stepped by 32 pixels
  int cb = pb / HW, cy = (pb - cb * HW) / W, cx = pb - cb * HW - cy * W;
  // staging items: dz (threads 0..127: pixel t >> 2, channels 8 (t & 3) ..), input
  // (items t and t + 256 below 408: channel group i & 3, row/column (i >> 2) / 34, % 34)
  u16x8 vd, vx[2];
  auto load_chunk = [&](int p0) {
    if (t < 128) vd = ld8(dz + (size_t)(p0 + (t >> 2)) * ldz + co0 + 8 * (t & 3));
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int i = t + 256 * e;
      vx[e] = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
      if (i < 408) {
        const int rq = i >> 2, r = rq / 34, q = rq - 34 * r;
        const int yy = cy + r - 1, xx = cx + q - 1;
        if (yy >= 0 && yy < H && xx >= 0 && xx < W)
          vx[e] = ld8(x + ((size_t)cb * HW + (size_t)yy * W + xx) * ldx + ci0 + 8 * (i & 3));
      }
    }
    cx += WG_K;
    if (cx == W) {
      cx = 0;
      if (++cy == H) {
        cy = 0;
        ++cb;
      }
    }
  };
  f32x4 acc[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) acc[k] = f32x4{0.f, 0.f, 0.f, 0.f};
  float bsum = 0.f;
  const int cot = wave & 1, cit = wave >> 1, kq = (lane >> 4) * 8;
  load_chunk(pb);
  for (int p0 = pb; p0 < pe; p0 += WG_K) {
    if (t < 128) {
#pragma unroll
      for (int j = 0; j < 8; ++j) sa[8 * (t & 3) + j][t >> 2] = vd[j];
    }
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int i = t + 256 * e;
      if (i < 408) {
        const int rq = i >> 2, r = rq / 34, q = rq - 34 * r;
#pragma unroll
        for (int j = 0; j < 8; ++j) sx[8 * (i & 3) + j][r][q] = vx[e][j];
      }
    }
    __syncthreads();
    if (p0 + WG_K < pe) load_chunk(p0 + WG_K);
    if (blockIdx.x == 0 && t < 32) {
#pragma unroll 8
      for (int k = 0; k < WG_K; ++k) bsum += bf2f(sa[t][k]);
    }
    const u16x8 a = ld8(&sa[16 * cot + (lane & 15)][kq]);
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const uint16_t* row = &sx[16 * cit + (lane & 15)][r][kq];
      const u16x8 lo = ld8(row);
      const uint32_t next = *reinterpret_cast<const uint32_t*>(row + 8);
#pragma unroll
      for (int sh = 0; sh < 3; ++sh) acc[3 * r + sh] = mfma(a, shift_cols(lo, next, sh), acc[3 * r + sh]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int tap = 0; tap < 9; ++tap) {
    const int col = tap * cin + ci0 + 16 * cit + (lane & 15);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int co = co0 + 16 * cot + 4 * (lane >> 4) + r;
      part[((size_t)s * cout + co) * nn + col] = acc[tap][r];
    }
  }
  if (blockIdx.x == 0 && t < 32) partb[(size_t)s * cout + co0 + t] = bsum;
}

// out[i] = sum_s part[s][i] in a fixed order: a block takes 64 outputs; thread group g (of
// SS_G) sums the splits g, g + SS_G, ... in order, then the group sums are added in order.
// Few outputs (the bias, small layers) take 16 groups so that the launch still fills the chip.
template <int SS_G>
__global__ void __launch_bounds__(64 * SS_G)
sum_splits_kernel(const float* __restrict__ part, int nsplit, size_t n, float* __restrict__ out) {
  __shared__ float sg[SS_G][64];
  const int il = threadIdx.x & 63, g = threadIdx.x >> 6;
  const size_t i = (size_t)blockIdx.x * 64 + il;
  float a = 0.f;
  if (i < n)
    for (int s = g; s < nsplit; s += SS_G) a += part[(size_t)s * n + i];
  sg[g][il] = a;
  __syncthreads();
  if (g == 0 && i < n) {
    float t = sg[0][il];
#pragma unroll
    for (int k = 1; k < SS_G; ++k) t += sg[k][il];
    out[i] = t;
  }
}

// ------------------------------------------------- first layer (one input channel), fp32
// y[p, co] = relu(b[co] + sum_tap w[co][tap] u[p + tap]), u = fbp * inv_s; a thread makes
// all channels of one pixel (weights and biases from LDS).
constexpr int CIN_MAXC = 256;
__global__ void __launch_bounds__(256)
conv_in_kernel(const float* __restrict__ fbp, float inv_s, const float* __restrict__ w,
               const float* __restrict__ bias, uint16_t* __restrict__ y, int cout, int H, int W,
               int npx) {
  __shared__ float sw[CIN_MAXC * 10];
  for (int e = threadIdx.x; e < cout * 10; e += blockDim.x)
    sw[e] = (e % 10) < 9 ? w[(e / 10) * 9 + e % 10] : bias[e / 10];
  __syncthreads();
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npx) return;
  const int HW = H * W, b = p / HW, rem = p - b * HW, r = rem / W, c = rem - r * W;
  float u[9];
#pragma unroll
  for (int tap = 0; tap < 9; ++tap) {
    const int yy = r + tap / 3 - 1, xx = c + tap % 3 - 1;
    u[tap] = (yy >= 0 && yy < H && xx >= 0 && xx < W)
                 ? fbp[(size_t)b * HW + (size_t)yy * W + xx] * inv_s : 0.f;
  }
  for (int c0 = 0; c0 < cout; c0 += 8) {
    u16x8 out;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const float* wj = sw + (c0 + j) * 10;
      float a = wj[9];
#pragma unroll
      for (int tap = 0; tap < 9; ++tap) a = fmaf(wj[tap], u[tap], a);
      out[j] = f2bf(fmaxf(a, 0.f));
    }
    st8(y + (size_t)p * cout + c0, out);
  }
}

// The same for a channel count fixed at compile time: weights and biases are read from LDS
// as three 16-byte broadcast words per channel (48-byte rows); same products in the same
// order (bias first, taps 0..8), so the same results.  The
// block's 256 pixels are consecutive, so their outputs form one contiguous run of 512 CO
// bytes: each thread puts its pixel's channels in LDS and the block then writes the run in
// 16-byte pieces with consecutive lanes on consecutive pieces.
template <int CO>
__global__ void __launch_bounds__(256)
conv_in_fixed_kernel(const float* __restrict__ fbp, float inv_s, const float* __restrict__ w,
                     const float* __restrict__ bias, uint16_t* __restrict__ y, int H, int W,
                     int npx) {
  constexpr int NC = CO / 8;  // 16-byte pieces per pixel
  __shared__ u16x8 so[256 * NC];
  __shared__ float4 sf[CO * 3];  // [channel][9 taps, bias, 2 unused]: broadcast reads
  for (int e = threadIdx.x; e < CO * 12; e += 256) {
    const int ch = e / 12, k = e - ch * 12;
    reinterpret_cast<float*>(sf)[e] = k < 9 ? w[ch * 9 + k] : (k == 9 ? bias[ch] : 0.f);
  }
  __syncthreads();
  const int p0 = blockIdx.x * 256, p = p0 + threadIdx.x;
  if (p < npx) {
    const int HW = H * W, b = p / HW, rem = p - b * HW, r = rem / W, c = rem - r * W;
    float u[9];
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
      const int yy = r + tap / 3 - 1, xx = c + tap % 3 - 1;
      u[tap] = (yy >= 0 && yy < H && xx >= 0 && xx < W)
                   ? fbp[(size_t)b * HW + (size_t)yy * W + xx] * inv_s : 0.f;
    }
#pragma unroll
    for (int c0 = 0; c0 < CO; c0 += 8) {
      u16x8 out;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const float4 wa = sf[(c0 + j) * 3], wb = sf[(c0 + j) * 3 + 1], wc = sf[(c0 + j) * 3 + 2];
        const float wt[9] = {wa.x, wa.y, wa.z, wa.w, wb.x, wb.y, wb.z, wb.w, wc.x};
        float a = wc.y;
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) a = fmaf(wt[tap], u[tap], a);
        out[j] = f2bf(fmaxf(a, 0.f));
      }
      // piece index rotated by the pixel so that neighbouring lanes hit different banks
      so[threadIdx.x * NC + ((c0 / 8 + threadIdx.x) % NC)] = out;
    }
  }
  __syncthreads();
  const int nval = min(256, npx - p0) * NC;
#pragma unroll
  for (int k0 = 0; k0 < 256 * NC; k0 += 256) {
    const int k = k0 + threadIdx.x, px = k / NC, pc = k % NC;
    if (k < nval) st8(y + ((size_t)p0 * NC + k) * 8, so[px * NC + ((pc + px) % NC)]);
  }
}

// part[blk][co*10 + k] (k < 9: weight of tap k, k = 9: bias) over the pixels of block blk.
// Thread t takes channels 8 g .. 8 g + 7 (g = t % tpp2, tpp2 = cout / 8 rounded up to a power
// of two; threads with 8 g >= cout hold zeros) of pixel lane t / tpp2: one 16-byte read of dz
// and the 9 neighbours per pixel, whose image, row and column are stepped along (no division
// per pixel).  The lanes of a wave that hold the same channels are combined by butterfly
// shuffles, then the 4 waves in order.
__global__ void __launch_bounds__(256)
conv_in_wgrad_kernel(const uint16_t* __restrict__ dz, const float* __restrict__ fbp, float inv_s,
                     float* __restrict__ part, int cout, int tpp2, int H, int W, int npx,
                     int px_per_blk) {
  extern __shared__ float sred[];  // [4 waves][tpp2][80]
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int g = t & (tpp2 - 1), pl = t / tpp2, lanes = 256 / tpp2;
  const bool has_ch = 8 * g < cout;
  const int pb = blockIdx.x * px_per_blk, pe = min(npx, pb + px_per_blk);
  const int HW = H * W;
  float acc[8][10];
#pragma unroll
  for (int j = 0; j < 8; ++j)
#pragma unroll
    for (int k = 0; k < 10; ++k) acc[j][k] = 0.f;
  if (has_ch && pb + pl < pe) {
    int p = pb + pl;
    int b = p / HW, r = (p - b * HW) / W, c = p - b * HW - r * W;
    for (; p < pe; p += lanes) {
      const u16x8 dv = ld8(dz + (size_t)p * cout + 8 * g);
      const float* img = fbp + (size_t)b * HW;
      float nb9[9];
#pragma unroll
      for (int tap = 0; tap < 9; ++tap) {
        const int yy = r + tap / 3 - 1, xx = c + tap % 3 - 1;
        nb9[tap] = (yy >= 0 && yy < H && xx >= 0 && xx < W) ? img[yy * W + xx] * inv_s : 0.f;
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const float d = bf2f(dv[j]);
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) acc[j][tap] = fmaf(d, nb9[tap], acc[j][tap]);
        acc[j][9] += d;
      }
      c += lanes;
      while (c >= W) {
        c -= W;
        if (++r == H) {
          r = 0;
          ++b;
        }
      }
    }
  }
#pragma unroll
  for (int j = 0; j < 8; ++j)
#pragma unroll
    for (int k = 0; k < 10; ++k)
      for (int off = tpp2; off < 64; off <<= 1) acc[j][k] += __shfl_xor(acc[j][k], off);
  if (lane < tpp2) {
#pragma unroll
    for (int j = 0; j < 8; ++j)
#pragma unroll
      for (int k = 0; k < 10; ++k) sred[(wave * tpp2 + lane) * 80 + j * 10 + k] = acc[j][k];
  }
  __syncthreads();
  for (int o = t; o < cout * 10; o += 256) {
    const int co = o / 10, k = o - co * 10, cg = co >> 3, j = co & 7;
    float a = 0.f;
#pragma unroll
    for (int w = 0; w < 4; ++w) a += sred[(w * tpp2 + cg) * 80 + j * 10 + k];
    part[(size_t)blockIdx.x * cout * 10 + o] = a;
  }
}

// dw[co][tap] = sum_blk part[blk][co*10 + tap], db[co] = sum_blk part[blk][co*10 + 9];
// one block per output, fixed-order strided sums then a fixed-order tree
__global__ void __launch_bounds__(256)
conv_in_reduce_kernel(const float* __restrict__ part, int nblk, int cout, float* __restrict__ dw,
                      float* __restrict__ db) {
  __shared__ float sh[256];
  const int o = blockIdx.x, t = threadIdx.x;
  float a = 0.f;
  for (int b = t; b < nblk; b += 256) a += part[(size_t)b * cout * 10 + o];
  sh[t] = a;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) sh[t] += sh[t + w];
    __syncthreads();
  }
  if (t == 0) {
    const int co = o / 10, k = o - co * 10;
    if (k < 9) dw[co * 9 + k] = sh[0];
    else db[co] = sh[0];
  }
}

// ------------------------------------------------------------ pooling and upsampling
// out[b, i, j, c] = mean of in[b, 2i+a, 2j+e, c]; 8 channels per thread
__global__ void avgpool2_kernel(const uint16_t* __restrict__ in, int ldi, uint16_t* __restrict__ out,
                                int ldo, int C, int B, int H, int W) {
  const int h = H / 2, w = W / 2, g8 = C / 8;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)B * h * w * g8) return;
  const size_t q = idx / g8;
  const int c0 = (int)(idx - q * g8) * 8;
  const int b = (int)(q / ((size_t)h * w)), rem = (int)(q - (size_t)b * h * w), i = rem / w, j = rem - i * w;
  float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const u16x8 v = ld8(in + (((size_t)b * H + 2 * i + a) * W + 2 * j + e) * ldi + c0);
#pragma unroll
      for (int k = 0; k < 8; ++k) s[k] += bf2f(v[k]);
    }
  u16x8 o;
#pragma unroll
  for (int k = 0; k < 8; ++k) o[k] = f2bf(0.25f * s[k]);
  st8(out + q * ldo + c0, o);
}

// dE[b, 2i+a, 2j+e, c] += 0.25 dP[b, i, j, c] where E > 0 (E: the pooled activation)
__global__ void avgpool2_back_kernel(const uint16_t* __restrict__ dp, int ldp,
                                     const uint16_t* __restrict__ e_act, int lde,
                                     uint16_t* __restrict__ de, int ldd, int C, int B, int H, int W) {
  const int h = H / 2, w = W / 2, g8 = C / 8;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)B * H * W * g8) return;
  const size_t q = idx / g8;
  const int c0 = (int)(idx - q * g8) * 8;
  const int b = (int)(q / ((size_t)H * W)), rem = (int)(q - (size_t)b * H * W), r = rem / W, c = rem - r * W;
  const u16x8 g = ld8(dp + (((size_t)b * h + r / 2) * w + c / 2) * ldp + c0);
  const u16x8 ev = ld8(e_act + q * lde + c0);
  u16x8 d = ld8(de + q * ldd + c0);
#pragma unroll
  for (int k = 0; k < 8; ++k)
    if (bf2f(ev[k]) > 0.f) d[k] = f2bf(bf2f(d[k]) + 0.25f * bf2f(g[k]));
  st8(de + q * ldd + c0, d);
}

// out[b, r, c, :C] = in[b, r/2, c/2, :C]
__global__ void up2_kernel(const uint16_t* __restrict__ in, int ldi, uint16_t* __restrict__ out,
                           int ldo, int C, int B, int H, int W) {
  const int g8 = C / 8;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)B * H * W * g8) return;
  const size_t q = idx / g8;
  const int c0 = (int)(idx - q * g8) * 8;
  const int b = (int)(q / ((size_t)H * W)), rem = (int)(q - (size_t)b * H * W), r = rem / W, c = rem - r * W;
  st8(out + q * ldo + c0, ld8(in + (((size_t)b * (H / 2) + r / 2) * (W / 2) + c / 2) * ldi + c0));
}

// out[b, i, j, :C] = sum_{a, e} in[b, 2i+a, 2j+e, :C]
__global__ void up2_back_kernel(const uint16_t* __restrict__ in, int ldi, uint16_t* __restrict__ out,
                                int ldo, int C, int B, int H, int W) {
  const int h = H / 2, w = W / 2, g8 = C / 8;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)B * h * w * g8) return;
  const size_t q = idx / g8;
  const int c0 = (int)(idx - q * g8) * 8;
  const int b = (int)(q / ((size_t)h * w)), rem = (int)(q - (size_t)b * h * w), i = rem / w, j = rem - i * w;
  float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const u16x8 v = ld8(in + (((size_t)b * H + 2 * i + a) * W + 2 * j + e) * ldi + c0);
#pragma unroll
      for (int k = 0; k < 8; ++k) s[k] += bf2f(v[k]);
    }
  u16x8 o;
#pragma unroll
  for (int k = 0; k < 8; ++k) o[k] = f2bf(s[k]);
  st8(out + q * ldo + c0, o);
}

// ---------------------------------------------------------------------------- head, loss
// r = hb + sum_c hw[c] D[p, c]; x0 = fbp + s r
__global__ void head_kernel(const uint16_t* __restrict__ d, const float* __restrict__ hw,
                            const float* __restrict__ hb, const float* __restrict__ fbp, float s,
                            float* __restrict__ r, float* __restrict__ x0, int C, int npx) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npx) return;
  float a = hb[0];
  for (int c0 = 0; c0 < C; c0 += 8) {
    const u16x8 v = ld8(d + (size_t)p * C + c0);
#pragma unroll
    for (int k = 0; k < 8; ++k) a = fmaf(hw[c0 + k], bf2f(v[k]), a);
  }
  if (r) r[p] = a;
  if (x0) x0[p] = fbp[p] + s * a;
}

// dr = 2 (r - (target - fbp)/s) / npx; dD[p, c] = hw[c] dr (D > 0); per block: sum of the
// squared residual (float64), sum dr, sum dr D[:, c] -> part[blk][C + 2].  Each sum is taken
// over a wave by butterfly shuffles, then over the 4 waves in order after one barrier.
__global__ void __launch_bounds__(256)
head_back_kernel(const float* __restrict__ r, const float* __restrict__ fbp,
                 const float* __restrict__ target, float inv_s, const uint16_t* __restrict__ d,
                 const float* __restrict__ hw, uint16_t* __restrict__ dd, double* __restrict__ part,
                 int C, int npx) {
  extern __shared__ double sh[];  // [4 waves][C + 2]
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int p = blockIdx.x * 256 + t;
  double sq = 0.0;
  float dr = 0.f;
  if (p < npx) {
    const float diff = r[p] - (target[p] - fbp[p]) * inv_s;
    sq = (double)diff * diff;
    dr = 2.f * diff / (float)npx;
  }
  // gradient of the last activation, and the sums dr D[:, c] of the 8 channels of each read
  // (all lanes take part in the shuffles; lanes past the end add zeros)
  for (int c0 = 0; c0 < C; c0 += 8) {
    u16x8 v = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
    if (p < npx) {
      v = ld8(d + (size_t)p * C + c0);
      u16x8 o;
#pragma unroll
      for (int k = 0; k < 8; ++k) o[k] = f2bf(bf2f(v[k]) > 0.f ? hw[c0 + k] * dr : 0.f);
      st8(dd + (size_t)p * C + c0, o);
    }
    double a[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = (double)dr * bf2f(v[k]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
      for (int k = 0; k < 8; ++k) a[k] += __shfl_xor(a[k], off);
    if (lane == 0) {
#pragma unroll
      for (int k = 0; k < 8; ++k) sh[wave * (C + 2) + 2 + c0 + k] = a[k];
    }
  }
  double a0 = sq, a1 = dr;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    a0 += __shfl_xor(a0, off);
    a1 += __shfl_xor(a1, off);
  }
  if (lane == 0) {
    sh[wave * (C + 2)] = a0;
    sh[wave * (C + 2) + 1] = a1;
  }
  __syncthreads();
  for (int k = t; k < C + 2; k += 256)
    part[(size_t)blockIdx.x * (C + 2) + k] =
        (sh[k] + sh[(C + 2) + k]) + (sh[2 * (C + 2) + k] + sh[3 * (C + 2) + k]);
}

// fixed-order sums of head_back partials (block k sums column k): loss (mean), head weight
// and bias gradients
__global__ void __launch_bounds__(256)
head_reduce_kernel(const double* __restrict__ part, int nblk, int C, int npx,
                   float* __restrict__ ghw, float* __restrict__ ghb, double* __restrict__ loss) {
  __shared__ double sh[256];
  const int k = blockIdx.x, t = threadIdx.x;
  double a = 0.0;
  for (int b = t; b < nblk; b += 256) a += part[(size_t)b * (C + 2) + k];
  sh[t] = a;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) sh[t] += sh[t + o];
    __syncthreads();
  }
  if (t != 0) return;
  a = sh[0];
  if (k == 0) {
    if (loss) *loss = a / npx;
  } else if (k == 1) {
    if (ghb) ghb[0] = (float)a;
  } else if (ghw) {
    ghw[k - 2] = (float)a;
  }
}

// ---------------------------------------------------------------------- optimiser, weights
__global__ void adam_kernel(float* __restrict__ th, const float* __restrict__ g,
                            float* __restrict__ m, float* __restrict__ v, size_t n, float lr,
                            float b1, float b2, float c1, float c2, float eps) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  th[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// wbf[co][tap][ci] = bf16(w[co][tap][ci]); wflip[ci][tap][co] = bf16(w[co][8 - tap][ci])
__global__ void weight_prep_kernel(const float* __restrict__ w, uint16_t* __restrict__ wbf,
                                   uint16_t* __restrict__ wflip, int cin, int cout) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t n = (size_t)cout * 9 * cin;
  if (i >= n) return;
  const int co = (int)(i / (9 * (size_t)cin)), rem = (int)(i - (size_t)co * 9 * cin);
  const int tap = rem / cin, ci = rem - tap * cin;
  const uint16_t h = f2bf(w[i]);
  wbf[i] = h;
  if (wflip) wflip[((size_t)ci * 9 + (8 - tap)) * cout + co] = h;
}

__global__ void f32_to_bf16_kernel(const float* __restrict__ in, uint16_t* __restrict__ out, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = f2bf(in[i]);
}

unsigned blocks_for(size_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

// ------------------------------------------------------------------------------ launchers
hipError_t nn_conv3x3(const uint16_t* x, int ldx, const uint16_t* w, const float* bias,
                      uint16_t* y, int ldy, const uint16_t* mask, int ldm, int cin, int cout,
                      int B, int H, int W, bool relu, hipStream_t st, const uint16_t* xu, int ldu,
                      int cu, uint16_t* pool, int ldp, const NnHead* head) {
  // the staging packs a clamped (row, column) into 15 bits each
  if (H > 32767 || W > 32767) return hipErrorInvalidValue;
  if (head) {
    if (!relu || !bias || mask || xu || pool || (cout != 32 && cout != 64) || cin % 32 || ldx % 8 ||
        B < 1 || H < 1 || W < 1 || !head->hw || !head->hb || !head->fbp || !head->x0)
      return hipErrorInvalidValue;
    const int ntx = (W + 15) / 16, nty = (H + 15) / 16;
    if (cout == 64)
      hipLaunchKernelGGL((conv3x3_tile_kernel<64, 4, true, true, false, false, false, true>),
                         dim3(ntx * nty, B), dim3(256), 0, st, x, ldx, w, bias, nullptr, 0, nullptr,
                         0, cin, H, W, ntx, nty, nullptr, 0, 0, nullptr, 0, *head);
    else
      hipLaunchKernelGGL((conv3x3_tile_kernel<32, 4, true, true, false, false, false, true>),
                         dim3(ntx * nty, B), dim3(256), 0, st, x, ldx, w, bias, nullptr, 0, nullptr,
                         0, cin, H, W, ntx, nty, nullptr, 0, 0, nullptr, 0, *head);
    return hipGetLastError();
  }
  if (cin % 32 || cout % 32 || ldx % 8 || ldy % 8 || ldy < cout || B < 1 || H < 1 || W < 1)
    return hipErrorInvalidValue;
  if (mask && (ldm % 8 || ldm < cout)) return hipErrorInvalidValue;
  if (xu && (cu % 32 || cu <= 0 || cu >= cin || ldu % 8 || H % 2 || W % 2)) return hipErrorInvalidValue;
  if (pool && (H % 2 || W % 2 || ldp < cout || ldp % 8 || !relu || !bias || mask))
    return hipErrorInvalidValue;
  const bool bi = bias != nullptr, m = mask != nullptr, up = xu != nullptr, pl = pool != nullptr;
  const int ntx = (W + 15) / 16;
  // 64 output channels per block when they divide cout, else 32; 4 rows per wave
#define CV(BN, RPW, R, BI, M, U, PO)                                                              \
  do {                                                                                            \
    const int nty = (H + 4 * RPW - 1) / (4 * RPW);                                                \
    hipLaunchKernelGGL((conv3x3_tile_kernel<BN, RPW, R, BI, M, U, PO, false>),                     \
                       dim3(ntx * nty * (cout / BN), B), dim3(256), 0, st, x, ldx, w, bias, y, ldy, \
                       mask, ldm, cin, H, W, ntx, nty, xu, ldu, cu, pool, ldp, NnHead{});         \
  } while (0)
#define CV_FORMS(BN, RPW)                                                        \
  if (relu && bi && !m && up && !pl) CV(BN, RPW, true, true, false, true, false); \
  else if (up) return hipErrorInvalidValue;                                      \
  else if (relu && bi && !m && pl) CV(BN, RPW, true, true, false, false, true);  \
  else if (relu && bi && !m) CV(BN, RPW, true, true, false, false, false);       \
  else if (!relu && !bi && m) CV(BN, RPW, false, false, true, false, false);     \
  else if (!relu && !bi && !m) CV(BN, RPW, false, false, false, false, false);   \
  else if (!relu && bi && !m) CV(BN, RPW, false, true, false, false, false);     \
  else return hipErrorInvalidValue;
  if (cout % 64 == 0) {
    CV_FORMS(64, 4)
  } else {
    CV_FORMS(32, 4)
  }
#undef CV_FORMS
#undef CV
  return hipGetLastError();
}

static void launch_sum_splits(const float* part, int nsplit, size_t n, float* out, hipStream_t st) {
  const unsigned nb = blocks_for(n, 64);
  if (nb < 512)
    hipLaunchKernelGGL(sum_splits_kernel<16>, dim3(nb), dim3(64 * 16), 0, st, part, nsplit, n, out);
  else
    hipLaunchKernelGGL(sum_splits_kernel<4>, dim3(nb), dim3(64 * 4), 0, st, part, nsplit, n, out);
}

WgradPlan nn_wgrad_plan(int cin, int cout, int npx) {
  WgradPlan pl;
  pl.ntn = (9 * cin + 63) / 64;
  pl.ntc = (cout + 63) / 64;
  // about 960 blocks of the haloed kernel's (cin / 32) x (cout / 32) tiles (5 fit a CU at its
  // register use: 960 to 1280 blocks were fastest, fewer splits also shorten the split sums),
  // at least 256 pixels per split, a multiple of the 32-pixel step
  const int tiles = (cin / 32) * (cout / 32);
  int ns = 960 / (tiles > 0 ? tiles : 1);
  if (ns < 1) ns = 1;
  int per = (npx + ns - 1) / ns;
  if (per < 256) per = 256;
  per = (per + WG_K - 1) / WG_K * WG_K;
  pl.px_per_split = per;
  pl.nsplit = (npx + per - 1) / per;
  pl.scratch_floats = (size_t)pl.nsplit * cout * (9 * cin + 1);
  return pl;
}

// per >= ceil(npx / ns) gives nsplit <= ns, and per >= 256 gives nsplit <= ceil(npx / 256),
// so this bounds the scratch of every pixel count up to max_npx (nsplit is not monotone in
// npx because per is rounded to the 32-pixel step).
size_t nn_wgrad_scratch_bound(int cin, int cout, int max_npx) {
  const int tiles = (cin / 32) * (cout / 32);
  int ns = 960 / (tiles > 0 ? tiles : 1);
  if (ns < 1) ns = 1;
  const int by_px = (max_npx + 255) / 256;
  const int nsplit = by_px < ns ? by_px : ns;
  return (size_t)nsplit * cout * (9 * cin + 1);
}

hipError_t nn_conv3x3_wgrad(const uint16_t* dz, int ldz, const uint16_t* x, int ldx, float* dw,
                            float* db, int cin, int cout, int B, int H, int W, float* scratch,
                            size_t scratch_floats, hipStream_t st) {
  if (cin % 32 || cout % 32 || ldz % 8 || ldx % 8) return hipErrorInvalidValue;
  const int npx = B * H * W;
  const WgradPlan pl = nn_wgrad_plan(cin, cout, npx);
  if (pl.scratch_floats > scratch_floats) return hipErrorInvalidValue;
  float* part = scratch;
  float* partb = scratch + (size_t)pl.nsplit * cout * 9 * cin;
  if (W % WG_K == 0)
    hipLaunchKernelGGL(conv3x3_wgrad_halo_kernel, dim3(cin / 32, cout / 32, pl.nsplit), dim3(256),
                       0, st, dz, ldz, x, ldx, part, partb, cin, cout, H, W, npx, pl.px_per_split);
  else
    hipLaunchKernelGGL(conv3x3_wgrad_kernel, dim3(pl.ntn, pl.ntc, pl.nsplit), dim3(256), 0, st,
                       dz, ldz, x, ldx, part, partb, cin, cout, H, W, npx, pl.px_per_split);
  const size_t nw = (size_t)cout * 9 * cin;
  launch_sum_splits(part, pl.nsplit, nw, dw, st);
  launch_sum_splits(partb, pl.nsplit, (size_t)cout, db, st);
  return hipGetLastError();
}

hipError_t nn_conv_in(const float* fbp, float inv_s, const float* w, const float* bias,
                      uint16_t* y, int cout, int B, int H, int W, hipStream_t st) {
  if (cout % 8 || cout > CIN_MAXC) return hipErrorInvalidValue;
  const size_t n = (size_t)B * H * W;
  if (cout == 32)
    hipLaunchKernelGGL(conv_in_fixed_kernel<32>, dim3(blocks_for(n, 256)), dim3(256), 0, st, fbp,
                       inv_s, w, bias, y, H, W, B * H * W);
  else if (cout == 64)
    hipLaunchKernelGGL(conv_in_fixed_kernel<64>, dim3(blocks_for(n, 256)), dim3(256), 0, st, fbp,
                       inv_s, w, bias, y, H, W, B * H * W);
  else
    hipLaunchKernelGGL(conv_in_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, fbp, inv_s, w,
                       bias, y, cout, H, W, B * H * W);
  return hipGetLastError();
}

constexpr int CIN_WG_PX = 2048;  // pixels per block of the first-layer weight gradient
int nn_conv_in_wgrad_blocks(int npx) { return (npx + CIN_WG_PX - 1) / CIN_WG_PX; }

hipError_t nn_conv_in_wgrad(const uint16_t* dz, const float* fbp, float inv_s, float* dw,
                            float* db, int cout, int B, int H, int W, float* scratch,
                            size_t scratch_floats, hipStream_t st) {
  // 8 channels per thread, cout / 8 threads per pixel rounded up to a power of two (<= 32)
  if (cout < 8 || cout > 256 || cout % 8) return hipErrorInvalidValue;
  int tpp2 = 1;
  while (tpp2 < cout / 8) tpp2 <<= 1;
  const int npx = B * H * W, nb = nn_conv_in_wgrad_blocks(npx);
  if ((size_t)nb * cout * 10 > scratch_floats) return hipErrorInvalidValue;
  hipLaunchKernelGGL(conv_in_wgrad_kernel, dim3(nb), dim3(256), 4 * tpp2 * 80 * sizeof(float),
                     st, dz, fbp, inv_s, scratch, cout, tpp2, H, W, npx, CIN_WG_PX);
  hipLaunchKernelGGL(conv_in_reduce_kernel, dim3(cout * 10), dim3(256), 0, st, scratch, nb, cout,
                     dw, db);
  return hipGetLastError();
}

hipError_t nn_avgpool2(const uint16_t* in, int ldi, uint16_t* out, int ldo, int C, int B, int H,
                       int W, hipStream_t st) {
  const size_t n = (size_t)B * (H / 2) * (W / 2) * (C / 8);
  hipLaunchKernelGGL(avgpool2_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, in, ldi, out, ldo,
                     C, B, H, W);
  return hipGetLastError();
}

hipError_t nn_avgpool2_back(const uint16_t* dp, int ldp, const uint16_t* e, int lde, uint16_t* de,
                            int ldd, int C, int B, int H, int W, hipStream_t st) {
  const size_t n = (size_t)B * H * W * (C / 8);
  hipLaunchKernelGGL(avgpool2_back_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, dp, ldp, e,
                     lde, de, ldd, C, B, H, W);
  return hipGetLastError();
}

hipError_t nn_up2(const uint16_t* in, int ldi, uint16_t* out, int ldo, int C, int B, int H, int W,
                  hipStream_t st) {
  const size_t n = (size_t)B * H * W * (C / 8);
  hipLaunchKernelGGL(up2_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, in, ldi, out, ldo, C,
                     B, H, W);
  return hipGetLastError();
}

hipError_t nn_up2_back(const uint16_t* in, int ldi, uint16_t* out, int ldo, int C, int B, int H,
                       int W, hipStream_t st) {
  const size_t n = (size_t)B * (H / 2) * (W / 2) * (C / 8);
  hipLaunchKernelGGL(up2_back_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, in, ldi, out, ldo,
                     C, B, H, W);
  return hipGetLastError();
}

hipError_t nn_head(const uint16_t* d, const float* hw, const float* hb, const float* fbp, float s,
                   float* r, float* x0, int C, int npx, hipStream_t st) {
  hipLaunchKernelGGL(head_kernel, dim3(blocks_for(npx, 256)), dim3(256), 0, st, d, hw, hb, fbp, s, r,
                     x0, C, npx);
  return hipGetLastError();
}

int nn_head_back_blocks(int npx) { return (npx + 255) / 256; }

hipError_t nn_head_back(const float* r, const float* fbp, const float* target, float inv_s,
                        const uint16_t* d, const float* hw, uint16_t* dd, double* part, float* ghw,
                        float* ghb, double* loss, int C, int npx, hipStream_t st) {
  if (C % 8 || C + 2 > 1024) return hipErrorInvalidValue;
  const int nb = nn_head_back_blocks(npx);
  hipLaunchKernelGGL(head_back_kernel, dim3(nb), dim3(256), 4 * (C + 2) * sizeof(double), st, r,
                     fbp, target, inv_s, d, hw, dd, part, C, npx);
  hipLaunchKernelGGL(head_reduce_kernel, dim3(C + 2), dim3(256), 0, st, part, nb, C, npx, ghw, ghb,
                     loss);
  return hipGetLastError();
}

hipError_t nn_adam(float* th, const float* g, float* m, float* v, size_t n, float lr, float b1,
                   float b2, float c1, float c2, float eps, hipStream_t st) {
  hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, th, g, m, v, n, lr, b1,
                     b2, c1, c2, eps);
  return hipGetLastError();
}

hipError_t nn_weight_prep(const float* w, uint16_t* wbf, uint16_t* wflip, int cin, int cout,
                          hipStream_t st) {
  const size_t n = (size_t)cout * 9 * cin;
  hipLaunchKernelGGL(weight_prep_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, w, wbf, wflip,
                     cin, cout);
  return hipGetLastError();
}

hipError_t nn_f32_to_bf16(const float* in, uint16_t* out, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(f32_to_bf16_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, in, out, n);
  return hipGetLastError();
}

}  // namespace tomo
