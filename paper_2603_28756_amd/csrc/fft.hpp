// Stockham autosort FFT building blocks for gfx950 (register butterflies + LDS exchange).
//
// A length-P transform (P a power of two) is split into stages of radix R_s
// (R_s <= E, the elements each thread holds).  A group of TPF = P/E threads
// owns one transform; thread q of the group handles butterflies
// j = q + m*TPF, m = 0..E/R-1, of every stage.  With span p = R_0*...*R_{s-1},
// stage s reads x[j + r*P/R] (r = 0..R-1), multiplies by W_{pR}^{r*(j mod p)},
// applies a radix-R DFT in registers and writes y[(j/p)*p*R + (j mod p) + r*p].
// After the last stage the outputs sit in registers at the same positions the
// first stage of a transform with that radix reads, which lets a forward
// transform hand its result to an inverse transform without touching LDS.
//
// Direction DIR = -1 computes sum_n x[n] exp(-2 pi i k n / P); DIR = +1 the
// unnormalised inverse.  Twiddles come from a table tw[m] = exp(-2 pi i m / P)
// (float64-computed, rounded to the element type).
#pragma once

#include "common.hpp"

namespace fft {

constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x / 2); }

// cos/sin(2 pi m / 16), m = 0..15, used for the constant twiddles inside a radix-R DFT (R <= 16).
__device__ constexpr double kCos16[16] = {
    1.0, 0.92387953251128673848, 0.70710678118654752440, 0.38268343236508977173,
    0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128673848,
    -1.0, -0.92387953251128673848, -0.70710678118654752440, -0.38268343236508977173,
    0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128673848};
__device__ constexpr double kSin16[16] = {
    0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128673848,
    1.0, 0.92387953251128673848, 0.70710678118654752440, 0.38268343236508977173,
    0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128673848,
    -1.0, -0.92387953251128673848, -0.70710678118654752440, -0.38268343236508977173};

// a * exp(DIR * 2 pi i j / L) for compile-time-foldable j, L (L <= 16).
template <int DIR, typename T>
TOMO_DEV cpx<T> rot_const(cpx<T> a, int j, int L) {
  const int m = (j * (16 / L)) & 15;  // angle 2 pi m / 16
  if (m == 0) return a;
  if (m == 4) return DIR < 0 ? mk(a.im, -a.re) : mk(-a.im, a.re);     // * -i  /  * +i
  if (m == 8) return mk(-a.re, -a.im);
  if (m == 12) return DIR < 0 ? mk(-a.im, a.re) : mk(a.im, -a.re);
  const T c = (T)kCos16[m];
  const T s = DIR < 0 ? -(T)kSin16[m] : (T)kSin16[m];
  if (m == 2 || m == 6 || m == 10 || m == 14) {
    // |c| == |s| == sqrt(1/2): sign flips, two adds and two multiplies
    const T h = (T)0.70710678118654752440;
    const T cr = c > 0 ? a.re : -a.re, ci = c > 0 ? a.im : -a.im;
    const T sr = s > 0 ? a.re : -a.re, si = s > 0 ? a.im : -a.im;
    return mk(h * (cr - si), h * (sr + ci));
  }
  return mk(a.re * c - a.im * s, a.re * s + a.im * c);
}

// In-register radix-R DFT (R = 1, 2, 4, 8, 16), natural order in and out:
// radix-2 decimation in frequency followed by a bit-reversal renaming.  HZ: the upper
// half of the inputs is zero (a zero-padded transform), so the first level only rotates.
template <int R, int DIR, bool HZ = false, typename T>
TOMO_DEV void dft_reg(cpx<T>* v) {
  if constexpr (R > 1) {
    if constexpr (HZ) {
#pragma unroll
      for (int j = 0; j < R / 2; ++j) v[j + R / 2] = rot_const<DIR>(v[j], j, R);
    }
#pragma unroll
    for (int h = HZ ? R / 4 : R / 2; h >= 1; h >>= 1) {
#pragma unroll
      for (int blk = 0; blk < R; blk += 2 * h) {
#pragma unroll
        for (int j = 0; j < h; ++j) {
          const cpx<T> a = v[blk + j], b = v[blk + j + h];
          v[blk + j] = a + b;
          v[blk + j + h] = rot_const<DIR>(a - b, j, 2 * h);
        }
      }
    }
    cpx<T> t[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
      int br = 0;
#pragma unroll
      for (int b = 0; b < ilog2(R); ++b) br |= ((i >> b) & 1) << (ilog2(R) - 1 - b);
      t[br] = v[i];
    }
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] = t[i];
  }
}

// Radix schedule: stages of radix E, the remainder last.
template <int P_, int E_>
struct Plan {
  static constexpr int P = P_;
  static constexpr int E = E_ < P_ ? E_ : P_;
  static constexpr int TPF = P / E;
  static constexpr int LE = ilog2(E), LP = ilog2(P);
  static constexpr int NS = (LP + LE - 1) / LE;
  static constexpr int radix(int s) { return s < NS - 1 ? E : (1 << (LP - LE * (NS - 1))); }
  static constexpr int span(int s) { int p = 1; for (int i = 0; i < s; ++i) p *= radix(i); return p; }
};

// Same stages in reverse order (inverse transform that starts where a forward one ended).
template <class F>
struct RevPlan {
  static constexpr int P = F::P, E = F::E, TPF = F::TPF, NS = F::NS;
  static constexpr int radix(int s) { return F::radix(NS - 1 - s); }
  static constexpr int span(int s) { int p = 1; for (int i = 0; i < s; ++i) p *= radix(i); return p; }
};

// w[r] = W_P^{r*e} for r = 1..R-1 from table lookups of w^1, w^2, w^4, w^8 and products.
template <int R, typename T>
TOMO_DEV void stage_twiddles(const cpx<T>* __restrict__ tw, int e, cpx<T>* w) {
  if constexpr (R >= 2) w[1] = tw[e];
  if constexpr (R >= 4) { w[2] = tw[2 * e]; w[3] = cmul(w[1], w[2]); }
  if constexpr (R >= 8) {
    w[4] = tw[4 * e];
    w[5] = cmul(w[1], w[4]); w[6] = cmul(w[2], w[4]); w[7] = cmul(w[3], w[4]);
  }
  if constexpr (R >= 16) {
    w[8] = tw[8 * e];
#pragma unroll
    for (int r = 9; r < 16; ++r) w[r] = cmul(w[r - 8], w[8]);
  }
}

// Twiddle + radix-R butterfly of every butterfly this thread owns (registers only).
// HZ (first stage only): inputs at positions >= P/2 are zero.
template <class PL, int S, int DIR, bool HZ = false, typename T>
TOMO_DEV void stage_compute(cpx<T>* v, int q, const cpx<T>* __restrict__ tw) {
  constexpr int R = PL::radix(S), p = PL::span(S), E = PL::E, TPF = PL::TPF, P = PL::P;
#pragma unroll
  for (int m = 0; m < E / R; ++m) {
    if constexpr (p > 1) {
      const int j = q + m * TPF;
      const int k = j & (p - 1);
      if (k != 0) {
        cpx<T> w[R];
        stage_twiddles<R>(tw, k * (P / (p * R)), w);
#pragma unroll
        for (int r = 1; r < R; ++r) v[m * R + r] = cmul(v[m * R + r], DIR < 0 ? w[r] : conj(w[r]));
      }
    }
    // position j + r P/R >= P/2 exactly when r >= R/2 (one butterfly per thread, E = R)
    static_assert(!HZ || (S == 0 && E == R), "zero upper half: first stage with E = R only");
    dft_reg<R, DIR, HZ>(&v[m * R]);
  }
}

// Output position of butterfly j of a stage with radix R and span p, before the r * p term:
// the bits of j with log2(R) zero bits inserted at bit log2(p).  The map is bitwise, so for
// j = q + m TPF (q < TPF, disjoint bits) it is the sum of the maps of q and of m TPF.
template <int R, int p>
TOMO_DEV int out_base(int j) { return (j / p) * p * R + (j & (p - 1)); }

// Stores and loads address the LDS view with a per-thread part Q (from q alone) and a part K
// known at compile time, with disjoint bits (i = Q + K = Q | K); views whose layout is
// bitwise in i use the split to keep the per-thread work out of the unrolled accesses.
template <class PL, int S, typename T, class Lds>
TOMO_DEV void stage_store(const cpx<T>* v, int q, Lds& lds) {
  constexpr int R = PL::radix(S), p = PL::span(S), E = PL::E, TPF = PL::TPF;
  const int Q = out_base<R, p>(q);
#pragma unroll
  for (int m = 0; m < E / R; ++m) {
    const int Kb = out_base<R, p>(m * TPF);
#pragma unroll
    for (int r = 0; r < R; ++r) lds.st2(Q, Kb + r * p, v[m * R + r]);
  }
}

// Load the inputs of a stage with radix R (position j + r*P/R into v[m*R + r]).
template <int P, int TPF, int E, int R, typename T, class Lds>
TOMO_DEV void stage_load(cpx<T>* v, int q, Lds& lds) {
#pragma unroll
  for (int m = 0; m < E / R; ++m)
#pragma unroll
    for (int r = 0; r < R; ++r) v[m * R + r] = lds.ld2(q, m * TPF + r * (P / R));
}

// Position held by register v[m*R + r] in the layout of a radix-R stage input/last-stage output.
template <int P, int TPF, int R>
TOMO_DEV int reg_pos(int q, int m, int r) { return q + m * TPF + r * (P / R); }

// Run stages S..NS-1 of plan PL; v enters in the input layout of stage S and leaves in
// the output layout of the last stage.  Every thread of the block must call this
// (it contains block barriers).  HZ: the input's upper half (positions >= P/2) is zero.
template <class PL, int S, int DIR, bool HZ = false, typename T, class Lds>
TOMO_DEV void run_stages(cpx<T>* v, int q, const cpx<T>* __restrict__ tw, Lds& lds) {
  stage_compute<PL, S, DIR, HZ && S == 0>(v, q, tw);
  if constexpr (S + 1 < PL::NS) {
    stage_store<PL, S>(v, q, lds);
    __syncthreads();
    stage_load<PL::P, PL::TPF, PL::E, PL::radix(S + 1)>(v, q, lds);
    __syncthreads();
    run_stages<PL, S + 1, DIR>(v, q, tw, lds);
  }
}

// LDS views.  Column view: element (idx, c) of TC interleaved transforms at slot(idx)*TC + c.
// SWZ = 0: slot = idx.  SWZ = 1: the two low bits of idx are XORed with bits 2-3 and 4-5
// (a permutation within each aligned group of 4 slots).  For P = 1024, 16 elements per
// thread and 8 columns, every stage store and load of a wave then spreads over all banks
// (two passes per 64-lane 8-byte access, the minimum), where the plain layout takes eight
// passes for the stores of the first forward and first inverse stage.
template <typename T, int TC, int SWZ = 0>
struct LdsCols {
  cpx<T>* base;
  int c;
  static TOMO_DEV int slot(int i) {
    if constexpr (SWZ == 1) return i ^ (((i >> 2) ^ (i >> 4)) & 3);
    else return i;
  }
  TOMO_DEV void st(int i, cpx<T> x) { base[slot(i) * TC + c] = x; }
  TOMO_DEV cpx<T> ld(int i) const { return base[slot(i) * TC + c]; }
  // i = Q + K with disjoint bits: slot is XOR-linear, slot(i) = slot(Q) ^ slot(K), and only
  // bits 0-1 of the two can meet, so the address is one of four per-thread bases plus a
  // compile-time offset.
  TOMO_DEV cpx<T>* at2(int Q, int K) const {
    if constexpr (SWZ == 1) {
      const int sk = slot(K);
      return base + ((slot(Q) ^ (sk & 3)) * TC + c) + (sk & ~3) * TC;
    } else {
      return base + (Q * TC + c) + K * TC;
    }
  }
  TOMO_DEV void st2(int Q, int K, cpx<T> x) { *at2(Q, K) = x; }
  TOMO_DEV cpx<T> ld2(int Q, int K) const { return *at2(Q, K); }
};

// Row view: one contiguous transform per region, padded by one element every 16.
template <typename T>
struct LdsRow {
  cpx<T>* base;
  static TOMO_DEV int pad(int i) { return i + (i >> 4); }
  TOMO_DEV void st(int i, cpx<T> x) { base[pad(i)] = x; }
  TOMO_DEV cpx<T> ld(int i) const { return base[pad(i)]; }
  TOMO_DEV void st2(int Q, int K, cpx<T> x) { st(Q + K, x); }
  TOMO_DEV cpx<T> ld2(int Q, int K) const { return ld(Q + K); }
};

template <int P>
constexpr int row_region() { return P + P / 16; }

}  // namespace fft
