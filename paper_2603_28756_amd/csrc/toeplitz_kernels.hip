// Hot path of the Toeplitz MBIR iteration on gfx950 (Sec. 2.1, Eqs. 9-11; Sec. 2, Eqs. 5-6).
//
// R*R y = Res_{NxN} F^-1(F K . F Pad y) is evaluated in three passes over a
// half spectrum S[z][row][u] (u = 0..P/2-1, complex64, the u = 0 slot packing
// the real DC column in its real part and the real Nyquist column u = P/2 in
// its imaginary part):
//   pass R  : rows of y (two real rows per complex transform) -> forward FFT of
//             length P (second half zero) -> Hermitian split -> S1
//   pass C  : per column u: forward FFT of length P (rows >= N zero), multiply
//             by F K / P^2, inverse FFT, keep rows < N -> S2
//   pass R' : rows of S2 -> inverse FFT of length P (two rows per complex
//             transform) -> keep columns < N -> T y, then the fused epilogue:
//             grad = T y - b + beta grad Phi(y) over 8 or 26 neighbours, the
//             gradient step, and float64 partial sums for the objective and
//             the restart test.
// A single-block float64 finalize turns the partial sums into the next momentum
// coefficient, so no host synchronisation is needed between iterations.
#include "common.hpp"
#include "fft.hpp"
#include "kernels.hpp"

namespace tomo {
namespace {

constexpr int kE = 16;  // elements per thread in the float32 transforms

// ----------------------------------------------------------------------------------- prior
// qGGMRF derivative (and value) for q = 2 in the factored form
//   rho'(d) = c_grad d (q/p + w) / (1 + w)^2,  rho(d) = c_val t^2 / (1 + w),
//   t = |d| / (T sigma), w = t^(q - p).
template <bool VAL>
TOMO_DEV void qggmrf(float d, const PriorParams& pp, float& rp, float& rv) {
  const float t = fabsf(d) * pp.inv_Tsigma;
  float w = 1.f;
  if (!pp.quadratic) w = __builtin_amdgcn_exp2f(pp.qmp * __builtin_amdgcn_logf(t));
  const float r = __builtin_amdgcn_rcpf(1.f + w);
  rp = pp.c_grad * d * (pp.q_over_p + w) * r * r;
  if constexpr (VAL) rv = pp.c_val * t * t * r;
}

// Workgroups of a launch are handed to the 8 XCDs round-robin by linear id, and each XCD has
// its own L2.  This maps the hardware id to a logical tile id so that every XCD receives one
// contiguous range of logical ids (a bijection on [0, total)); tiles that share cache lines
// are then adjacent in logical order and meet in one L2.
TOMO_DEV int xcd_contiguous(int hw, int total) {
  constexpr int X = 8;
  const int q = total / X, r = total % X;
  const int xcd = hw % X, local = hw / X;
  return xcd < r ? xcd * (q + 1) + local : r * (q + 1) + (xcd - r) * q + local;
}

template <int NT>
TOMO_DEV void block_sum4(double a0, double a1, double a2, double a3, double* out, double* sbuf) {
  double a[4] = {a0, a1, a2, a3};
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
      if (off < NT) a[i] += __shfl_xor(a[i], off, 64);  // blocks narrower than a wave
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int i = 0; i < 4; ++i) sbuf[wave * 4 + i] = a[i];
  __syncthreads();
  if (threadIdx.x == 0) {
    constexpr int NW = (NT + 63) / 64;
    double s[4] = {0, 0, 0, 0};
    for (int w = 0; w < NW; ++w)
#pragma unroll
      for (int i = 0; i < 4; ++i) s[i] += sbuf[w * 4 + i];
#pragma unroll
    for (int i = 0; i < 4; ++i) out[i] = s[i];
  }
}

// ---------------------------------------------------------------------------------- pass R
template <int P, int PAIRS>
constexpr int rows_fwd_lds() { return PAIRS * fft::row_region<P>() * 8; }

// Block `blk` transforms row pairs blk*PAIRS .. blk*PAIRS+PAIRS-1 (counted over all slices).
// y = x_k + mu (x_k - x_{k-1}), or s * x_k in power mode, or y = xk as given (MODE_FISTA_Y).
template <int P, int PAIRS, int MODE, int EL = kE>
TOMO_DEV void rows_fwd_body(unsigned char* smem, int blk, const float* __restrict__ xk,
                            const float* __restrict__ xkm1, float mu, float s,
                            cpx<float>* __restrict__ S1, const cpx<float>* __restrict__ tw, int N,
                            int n_pairs) {
  using PL = fft::Plan<P, EL>;
  constexpr int TPF = PL::TPF, E = PL::E, R0 = PL::radix(0), RL = PL::radix(PL::NS - 1);
  constexpr int REG = fft::row_region<P>();
  constexpr int H = P / 2;
  cpx<float>* lds = reinterpret_cast<cpx<float>*>(smem);

  const int t = threadIdx.x, pr = t / TPF, q = t - pr * TPF;
  const int gp = blk * PAIRS + pr;
  const bool active = gp < n_pairs;
  const int halfN = N >> 1;
  const int z = active ? gp / halfN : 0;
  const int r1 = active ? 2 * (gp - z * halfN) : 0;
  const idx_t row1 = ((idx_t)z * N + r1) * N;
  const idx_t row2 = row1 + N;

  cpx<float> v[E];
#pragma unroll
  for (int m = 0; m < E / R0; ++m)
#pragma unroll
    for (int r = 0; r < R0; ++r) {
      const int n = fft::reg_pos<P, TPF, R0>(q, m, r);
      cpx<float> zz = mk(0.f, 0.f);
      // positions >= P/2 >= N are the zero padding: r >= R0/2 (E = R0) never loads
      if (2 * r < R0 && active && n < N) {
        const float a1 = xk[row1 + n], a2 = xk[row2 + n];
        if constexpr (MODE == MODE_POWER) {
          zz = mk(s * a1, s * a2);
        } else if constexpr (MODE == MODE_FISTA_Y) {
          zz = mk(a1, a2);  // y written by the prior kernel
        } else {
          const float b1 = xkm1[row1 + n], b2 = xkm1[row2 + n];
          zz = mk(a1 + mu * (a1 - b1), a2 + mu * (a2 - b2));
        }
      }
      v[m * R0 + r] = zz;
    }

  fft::LdsRow<float> L{lds + pr * REG};
  fft::run_stages<PL, 0, -1, true>(v, q, tw, L);
#pragma unroll
  for (int m = 0; m < E / RL; ++m)
#pragma unroll
    for (int r = 0; r < RL; ++r) L.st(fft::reg_pos<P, TPF, RL>(q, m, r), v[m * RL + r]);
  __syncthreads();

  if (active) {
    cpx<float>* o1 = S1 + ((idx_t)z * N + r1) * H;
    cpx<float>* o2 = o1 + H;
    for (int u = q; u < H; u += TPF) {
      const cpx<float> zu = L.ld(u);
      if (u == 0) {
        const cpx<float> zn = L.ld(H);
        o1[0] = mk(zu.re, zn.re);
        o2[0] = mk(zu.im, zn.im);
      } else {
        const cpx<float> zm = L.ld(P - u);
        // X1 = (Z[u] + conj Z[P-u]) / 2,  X2 = (Z[u] - conj Z[P-u]) / (2i)
        o1[u] = mk(0.5f * (zu.re + zm.re), 0.5f * (zu.im - zm.im));
        o2[u] = mk(0.5f * (zu.im + zm.im), -0.5f * (zu.re - zm.re));
      }
    }
  }
}

// MODE_POWER with pprev: the scale is 1 / ||T v|| of the previous power step, formed by every
// block from that step's pass R' partial sums (slot 0, nprev blocks) in one fixed order, in
// place of a separate one-block reduction launch between the steps.
template <int P, int PAIRS, int MODE>
__global__ void __launch_bounds__(PAIRS * (P / kE))
rows_fwd_kernel(const float* __restrict__ xk, const float* __restrict__ xkm1,
                const double* __restrict__ scal, cpx<float>* __restrict__ S1,
                const cpx<float>* __restrict__ tw, int N, int n_pairs,
                const double* __restrict__ pprev, int nprev) {
  __shared__ __align__(16) unsigned char smem[rows_fwd_lds<P, PAIRS>()];
  float mu = 0.f, s = 1.f;
  if constexpr (MODE == MODE_POWER) {
    if (pprev) {
      constexpr int NT = PAIRS * (P / kE);
      __shared__ double red[NT];
      double a = 0.0;
      for (int b = threadIdx.x; b < nprev; b += NT) a += pprev[(idx_t)b * 4];
      red[threadIdx.x] = a;
      __syncthreads();
      for (int h = NT / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
      }
      const double wn = sqrt(red[0]);
      s = wn > 0.0 ? (float)(1.0 / wn) : 0.f;
    } else {
      s = (float)scal[SC_PSCALE];
    }
  } else {
    mu = (float)scal[SC_MU];
  }
  rows_fwd_body<P, PAIRS, MODE>(smem, blockIdx.x, xk, xkm1, mu, s, S1, tw, N, n_pairs);
}

// ---------------------------------------------------------------------------------- pass C
template <int P, int TC>
constexpr int cols_conv_lds() { return P * TC * 8; }

// Column tile `bx` (columns bx*TC .. bx*TC+TC-1) of slice z.
template <int P, int TC, int EL = kE>
TOMO_DEV void cols_conv_body(unsigned char* smem, int bx, int z,
                             const cpx<float>* __restrict__ S1, cpx<float>* __restrict__ S2,
                             const float* __restrict__ fk, const float* __restrict__ fkn,
                             const cpx<float>* __restrict__ tw, int N) {
  using PL = fft::Plan<P, EL>;
  using IPL = fft::RevPlan<PL>;
  constexpr int TPF = PL::TPF, E = PL::E, R0 = PL::radix(0), RL = PL::radix(PL::NS - 1);
  constexpr int H = P / 2;
  cpx<float>* lds = reinterpret_cast<cpx<float>*>(smem);

  const int t = threadIdx.x, c = t % TC, q = t / TC;
  const int u = bx * TC + c;
  const cpx<float>* in = S1 + (idx_t)z * N * H + u;

  cpx<float> v[E];
#pragma unroll
  for (int m = 0; m < E / R0; ++m)
#pragma unroll
    for (int r = 0; r < R0; ++r) {
      const int n = fft::reg_pos<P, TPF, R0>(q, m, r);
      // positions >= P/2 >= N are the zero padding (r >= R0/2)
      v[m * R0 + r] = (2 * r < R0 && n < N) ? in[(idx_t)n * H] : mk(0.f, 0.f);
    }

  fft::LdsCols<float, TC, 1> L{lds, c};
  fft::run_stages<PL, 0, -1, true>(v, q, tw, L);

  if (bx == 0) {
    // Column 0 carries the DC column (real part) and the Nyquist column (imag part); both
    // are real, so their spectra C0, CN are Hermitian and C0 FK0 + i CN FKN is recovered
    // from Z[v] and conj Z[-v].
#pragma unroll
    for (int m = 0; m < E / RL; ++m)
#pragma unroll
      for (int r = 0; r < RL; ++r) L.st(fft::reg_pos<P, TPF, RL>(q, m, r), v[m * RL + r]);
    __syncthreads();
#pragma unroll
    for (int m = 0; m < E / RL; ++m)
#pragma unroll
      for (int r = 0; r < RL; ++r) {
        const int n = fft::reg_pos<P, TPF, RL>(q, m, r);
        const cpx<float> zv = v[m * RL + r];
        if (c == 0) {
          const cpx<float> zm = conj(L.ld((P - n) & (P - 1)));
          const float f0 = fk[fk_index(n, 0, P)], fN = fkn[n];
          const float a = 0.5f * (f0 + fN), b = 0.5f * (f0 - fN);
          v[m * RL + r] = mk(a * zv.re + b * zm.re, a * zv.im + b * zm.im);
        } else {
          v[m * RL + r] = scale(zv, fk[fk_index(n, u, P)]);
        }
      }
    __syncthreads();
  } else {
#pragma unroll
    for (int m = 0; m < E / RL; ++m)
#pragma unroll
      for (int r = 0; r < RL; ++r) {
        const int n = fft::reg_pos<P, TPF, RL>(q, m, r);
        v[m * RL + r] = scale(v[m * RL + r], fk[fk_index(n, u, P)]);
      }
  }

  fft::run_stages<IPL, 0, +1>(v, q, tw, L);

  cpx<float>* out = S2 + (idx_t)z * N * H + u;
#pragma unroll
  for (int m = 0; m < E / R0; ++m)
#pragma unroll
    for (int r = 0; r < R0; ++r) {
      const int n = fft::reg_pos<P, TPF, R0>(q, m, r);
      if (2 * r < R0 && n < N) out[(idx_t)n * H] = v[m * R0 + r];  // rows >= P/2 are cropped
    }
}

template <int P, int TC>
__global__ void __launch_bounds__(TC * (P / kE))
cols_conv_kernel(const cpx<float>* __restrict__ S1, cpx<float>* __restrict__ S2,
                 const float* __restrict__ fk, const float* __restrict__ fkn,
                 const cpx<float>* __restrict__ tw, int N, int nz) {
  __shared__ __align__(16) unsigned char smem[cols_conv_lds<P, TC>()];
  // Logical order: groups of G adjacent column tiles (which share 128-byte lines of S1, S2
  // and F K), then slices, then the group index; each XCD thus works on one band of columns
  // across all slices and holds only that band of F K in its L2.
  constexpr int NCG = (P / 2) / TC, G = NCG < 8 ? NCG : 8;
  const int lam = xcd_contiguous(blockIdx.x, NCG * nz);
  const int rest = lam / G;
  cols_conv_body<P, TC>(smem, (rest / nz) * G + lam % G, rest % nz, S1, S2, fk, fkn, tw, N);
}

// ---------------------------------------------------------------------------- prior (3D)
// gp = beta grad Phi(y), y = x_k + mu (x_k - x_{k-1}), with every neighbour pair evaluated
// once.  A block owns a TX x 16 column of voxels (32 x 16 by default, one per thread) and
// marches through 16 slices, keeping planes z and z+1 (with a one-voxel halo) in LDS.  Per
// plane each thread evaluates the forward pairs of its voxel: 4 in-plane offsets (0,1),
// (1,-1), (1,0), (1,1) and the 9 offsets into plane z+1; the forward pairs that start on the halo ring and end
// inside the tile are spread over the threads as one (position, offset) item each.  A pair's
// value enters its first voxel with + (kept in registers) and its second with - (read back
// from LDS by the voxel at the far end; rho' is odd).  Tiles whose halo ring lies inside the
// volume run without bounds tests; on the others a pair that leaves the volume gets
// difference 0 (rho'(0) = 0) from validity masks computed once per thread.  With OBJ the
// block also sums rho over the forward pairs of its own voxels.
//
// LDS layout: each wave owns an 8 x 8 block of the tile and planes are stored with a row
// stride S (24 for 16-wide tiles, 40 for 32-wide) for which the 8 rows of a wave (offsets
// 0, S, ..., 7 S) fall on disjoint bank ranges for both 32-lane halves (32 banks) and the
// whole wave (64 banks); every access of a wave to its own block shifted by a constant (a
// neighbour offset) is then free of bank conflicts.
constexpr int PR_TX = 32, PR_TY = 16, PR_ZC = 16;  // tile columns (volume kernel), rows, slices
constexpr int PR_NT = PR_TX * PR_TY;                 // one voxel per thread
// Tile shape of width TX (32 for the volume kernel, 16 for the 256-thread batch phase).
template <int TX_>
struct PriorShape {
  static_assert(TX_ == 16 || TX_ == 32, "tile width");
  static constexpr int TX = TX_, TY = PR_TY, NT = TX * TY;
  static constexpr int WX = TX / 8;                                  // 8 x 8 wave blocks per tile row
  static constexpr int HX = TX + 2, HY = TY + 2, HA = HX * HY;       // halo tile
  static constexpr int S = TX == 32 ? 40 : 24, PA = HY * S;          // LDS row stride, plane
};

// rho'(d) / c_grad and rho(d) for q = 2, arranged for few instructions:
//   rho'(d) / c_grad = d r (1 + (q/p - 1) r),  r = 1 / (1 + w),
//   w = (|d| / (T sigma))^(q-p) = exp2((q-p) log2|d| + lw0),  rho(d) = c_val2 d^2 r.
// d = 0 gives w = 0 and a zero derivative and value.  QUAD: p = q, w = 1.
template <bool VAL, bool QUAD>
TOMO_DEV void qggmrf_unit(float d, const PriorParams& pp, float& rp, float& rv) {
  float r = 0.5f;
  if constexpr (!QUAD) {
    const float w =
        __builtin_amdgcn_exp2f(__builtin_fmaf(pp.qmp, __builtin_amdgcn_logf(fabsf(d)), pp.lw0));
    r = __builtin_amdgcn_rcpf(1.f + w);
  }
  rp = d * r * __builtin_fmaf(pp.qop_m1, r, 1.f);
  if constexpr (VAL) rv = pp.c_val2 * d * d * r;
}

template <int NB, int TX = PR_TX>
struct PriorLds {
  using SH = PriorShape<TX>;
  float Y[2][SH::PA];
  float fin[4][SH::PA];
  float fz[NB == 26 ? 9 : 1][SH::PA];
  double sred[(SH::NT / 64) * 4];
};

// YG: also store y and write gp - b in place of gp (b = bvec), and with OBJ sum <y, b>, for
// a FISTA step whose passes R and R' then read y and gp - b instead of x_{k-1}, b and gp.
template <int NB, bool OBJ, bool QUAD, bool EDGE, bool YG, int TXW = PR_TX>
TOMO_DEV void prior_tile(PriorLds<NB, TXW>& L, const float* __restrict__ xk,
                         const float* __restrict__ xkm1, float* __restrict__ gp,
                         const float* __restrict__ bvec, float* __restrict__ yout,
                         double* __restrict__ part_out, int N, int nz, int c0, int r0, int z0,
                         float mu, bool fista, const PriorParams& pp) {
  using SH = PriorShape<TXW>;
  constexpr int HX = SH::HX, HY = SH::HY, HA = SH::HA, S = SH::S, TX = SH::TX, TY = SH::TY;
  const int t = threadIdx.x;
  // own voxel: wave w covers rows 8 (w / WX) .. +7 and columns 8 (w % WX) .. +7 of the tile
  const int wv = t >> 6, ln = t & 63;
  const int tr = 8 * (wv / SH::WX) + (ln >> 3), tc = 8 * (wv % SH::WX) + (ln & 7);
  const int s = (tr + 1) * S + tc + 1;  // own position in a plane buffer
  const int z1 = min(z0 + PR_ZC, nz);
  // neighbour weights with beta and the rho' prefactor folded in
  const float kb = pp.beta * pp.c_grad;
  const float w1 = kb * pp.wts[1], w2 = kb * pp.wts[2], w3 = kb * pp.wts[3];

  auto inside = [&](int a, int b) {  // halo coordinates -> inside the volume
    const int r = r0 - 1 + a, c = c0 - 1 + b;
    return r >= 0 && r < N && c >= 0 && c < N;
  };
  auto in_tile = [&](int a, int b) { return a >= 1 && a <= TY && b >= 1 && b <= TX; };

  // Halo items, as (row a, column b) of the halo ring and an offset index.  In-plane
  // (3 TX + 3 TY + 2): top row x offsets (1,-1),(1,0),(1,1); left column x (0,1),(1,1);
  // right column x (1,-1); two corners.  Cross-plane (6 TX + 6 TY + 4): top row x dy=+1,
  // bottom row x dy=-1, left column x dx=+1, right column x dx=-1 (3 each), four corners.
  // Items whose end leaves the tile are idle.
  int in_a = -1, in_b = 0, in_o = 0;
  {
    constexpr int i0 = 3 * TX, i1 = i0 + 2 * TY, i2 = i1 + TY;
    if (t < i0) { in_a = 0; in_b = t / 3 + 1; in_o = 1 + t % 3; }
    else if (t < i1) { const int k = t - i0; in_a = k / 2 + 1; in_b = 0; in_o = (k & 1) ? 3 : 0; }
    else if (t < i2) { in_a = t - i1 + 1; in_b = HX - 1; in_o = 1; }
    else if (t == i2) { in_a = 0; in_b = 0; in_o = 3; }
    else if (t == i2 + 1) { in_a = 0; in_b = HX - 1; in_o = 1; }
  }
  int x_a = -1, x_b = 0, x_o = 0;
  {
    constexpr int j0 = 3 * TX, j1 = 2 * j0, j2 = j1 + 3 * TY, j3 = j2 + 3 * TY;
    if (t < j0) { x_a = 0; x_b = t / 3 + 1; x_o = 6 + t % 3; }
    else if (t < j1) { x_a = HY - 1; x_b = (t - j0) / 3 + 1; x_o = (t - j0) % 3; }
    else if (t < j2) { x_a = (t - j1) / 3 + 1; x_b = 0; x_o = 3 * ((t - j1) % 3) + 2; }
    else if (t < j3) { x_a = (t - j2) / 3 + 1; x_b = HX - 1; x_o = 3 * ((t - j2) % 3); }
    else if (t == j3) { x_a = 0; x_b = 0; x_o = 8; }
    else if (t == j3 + 1) { x_a = 0; x_b = HX - 1; x_o = 6; }
    else if (t == j3 + 2) { x_a = HY - 1; x_b = 0; x_o = 2; }
    else if (t == j3 + 3) { x_a = HY - 1; x_b = HX - 1; x_o = 0; }
    static_assert(j3 + 4 <= SH::NT && 3 * TX + 3 * TY + 2 <= SH::NT, "one item per thread");
  }
  // resolve the items once: start and end positions, activity and validity
  int in_pos = 0, in_q = 0, x_pos = 0, x_q = 0;
  bool in_act = false, x_act = false, in_ok = true, x_ok = true;
  if (in_a >= 0) {
    const int dy = in_o == 0 ? 0 : 1, dx = in_o == 0 ? 1 : in_o - 2;
    in_act = in_tile(in_a + dy, in_b + dx);
    in_pos = in_a * S + in_b;
    in_q = in_pos + dy * S + dx;
    if constexpr (EDGE) in_ok = inside(in_a, in_b) && inside(in_a + dy, in_b + dx);
  }
  if (x_a >= 0) {
    const int dy = x_o / 3 - 1, dx = x_o % 3 - 1;
    x_act = in_tile(x_a + dy, x_b + dx);
    x_pos = x_a * S + x_b;
    x_q = x_pos + dy * S + dx;
    if constexpr (EDGE) x_ok = inside(x_a, x_b) && inside(x_a + dy, x_b + dx);
  }
  // own-pair validity: bits 0..3 in-plane offsets, bits 4..12 offsets into the next plane
  uint32_t m_own = 0x1fffu;
  if constexpr (EDGE) {
    m_own = 0;
    const int a = tr + 1, b = tc + 1;
    if (inside(a, b)) {
      m_own |= (uint32_t)inside(a, b + 1) | ((uint32_t)inside(a + 1, b - 1) << 1) |
               ((uint32_t)inside(a + 1, b) << 2) | ((uint32_t)inside(a + 1, b + 1) << 3);
#pragma unroll
      for (int o = 0; o < 9; ++o) m_own |= (uint32_t)inside(a + o / 3 - 1, b + o % 3 - 1) << (4 + o);
    }
  }
  // plane loads: the (at most two) halo elements of this thread, read row by row from
  // global memory (coalesced) and placed at their padded plane positions
  const int e1 = t + SH::NT;
  const bool has_e1 = e1 < HA;
  int g0, g1 = 0, l0, l1 = 0;
  bool v0 = true, v1 = true;
  {
    const int a = t / HX, b = t - a * HX;
    g0 = (r0 - 1 + a) * N + (c0 - 1 + b);
    l0 = a * S + b;
    if constexpr (EDGE) v0 = inside(a, b);
    if (has_e1) {
      const int a1 = e1 / HX, b1 = e1 - a1 * HX;
      g1 = (r0 - 1 + a1) * N + (c0 - 1 + b1);
      l1 = a1 * S + b1;
      if constexpr (EDGE) v1 = inside(a1, b1);
    }
  }
  const idx_t plane = (idx_t)N * N;
  auto yval = [&](idx_t o) {
    const float xa = xk[o];
    return fista ? xa + mu * (xa - xkm1[o]) : xa;
  };
  auto load_plane = [&](int z, float* dst) {
    const idx_t zb = (idx_t)z * plane;
    dst[l0] = v0 ? yval(zb + g0) : 0.f;
    if (has_e1) dst[l1] = v1 ? yval(zb + g1) : 0.f;
  };
  // Planes inside the march are read one iteration ahead into registers (issue) and written
  // to LDS at the top of the next iteration (commit), so their memory latency overlaps a
  // whole plane of pair evaluations.
  float ra0 = 0.f, rb0 = 0.f, ra1 = 0.f, rb1 = 0.f;
  auto issue = [&](int z) {
    const idx_t zb = (idx_t)z * plane;
    if (v0) {
      ra0 = xk[zb + g0];
      if (fista) rb0 = xkm1[zb + g0];
    }
    if (has_e1 && v1) {
      ra1 = xk[zb + g1];
      if (fista) rb1 = xkm1[zb + g1];
    }
  };
  auto commit = [&](float* dst) {
    dst[l0] = v0 ? (fista ? ra0 + mu * (ra0 - rb0) : ra0) : 0.f;
    if (has_e1) dst[l1] = v1 ? (fista ? ra1 + mu * (ra1 - rb1) : ra1) : 0.f;
  };
  double phi = 0.0, yb = 0.0;

  // forward pairs from plane buffer `src` to plane buffer `dst` (9 offsets (dy, dx)); the
  // weighted sum for the voxel in `src` is returned, the values go to fz for the far ends
  auto cross_fwd = [&](const float* src, const float* dst, bool count_phi) {
    const float ys = src[s];
    float up = 0.f;
#pragma unroll
    for (int o = 0; o < 9; ++o) {
      const int dy = o / 3 - 1, dx = o % 3 - 1;
      const float w = (dy != 0 && dx != 0) ? w3 : ((dy != 0 || dx != 0) ? w2 : w1);
      float d = ys - dst[s + dy * S + dx];
      if constexpr (EDGE) d = (m_own >> (4 + o)) & 1u ? d : 0.f;
      float rp, rv = 0.f;
      qggmrf_unit<OBJ, QUAD>(d, pp, rp, rv);
      L.fz[o][s] = rp;
      up = __builtin_fmaf(w, rp, up);
      if (OBJ && count_phi) phi += (double)(pp.wts[1 + (dy != 0) + (dx != 0)] * rv);
    }
    if (x_act) {
      float rp, rv;
      qggmrf_unit<false, QUAD>(x_ok ? src[x_pos] - dst[x_q] : 0.f, pp, rp, rv);
      L.fz[x_o][x_pos] = rp;
    }
    return up;
  };
  // the plane-(z+1) voxel's backward sum at this thread's (row, column)
  auto cross_back = [&]() {
    float dn = 0.f;
#pragma unroll
    for (int o = 0; o < 9; ++o) {
      const int dy = o / 3 - 1, dx = o % 3 - 1;
      const float w = (dy != 0 && dx != 0) ? w3 : ((dy != 0 || dx != 0) ? w2 : w1);
      dn = __builtin_fmaf(w, L.fz[o][s - dy * S - dx], dn);
    }
    return -dn;
  };

  int cur = 0;
  load_plane(z0, L.Y[cur]);
  float acc = 0.f, accn = 0.f;
  if (NB == 26 && z0 > 0) {
    load_plane(z0 - 1, L.Y[1 - cur]);
    __syncthreads();
    (void)cross_fwd(L.Y[1 - cur], L.Y[cur], false);
    __syncthreads();
    acc = cross_back();
  }
  // first plane read ahead: z0 + 1 (the next plane of z0, or the second plane of the march)
  if (NB == 26 ? z0 + 1 < nz : z0 + 1 < z1) issue(z0 + 1);
  // YG: b is read one plane ahead as well (bcur for this plane, bnext for the next)
  const int r = r0 + tr, c = c0 + tc;
  const bool store = !EDGE || (r < N && c < N);
  float bcur = 0.f, bnext = 0.f;
  if (YG && store) bcur = bvec[((idx_t)z0 * N + r) * N + c];
  __syncthreads();

  constexpr int offs[4] = {1, S - 1, S, S + 1};
  for (int z = z0; z < z1; ++z) {
    const bool has_next = NB == 26 && z + 1 < nz;
    if (NB != 26 && z > z0) {
      commit(L.Y[cur]);
      if (z + 1 < z1) issue(z + 1);
      __syncthreads();
    }
    if (has_next) {
      commit(L.Y[1 - cur]);
      // the plane after next, or (past the march) plane z again, an L2 hit whose values are
      // not used: the reads stay unconditional, which keeps the memory-counter waits exact
      issue(z + 2 <= z1 && z + 2 < nz ? z + 2 : z);
    }
    const idx_t go = ((idx_t)z * N + r) * N + c;
    if (YG && store) bnext = bvec[go + (z + 1 < z1 ? plane : 0)];  // b of the next plane
    float own = 0.f, ys_own;
    {
      const float* y = L.Y[cur];
      const float ys = y[s];
      ys_own = ys;
#pragma unroll
      for (int o = 0; o < 4; ++o) {
        float d = ys - y[s + offs[o]];
        if constexpr (EDGE) d = (m_own >> o) & 1u ? d : 0.f;
        float rp, rv = 0.f;
        qggmrf_unit<OBJ, QUAD>(d, pp, rp, rv);
        L.fin[o][s] = rp;
        own = __builtin_fmaf((o == 0 || o == 2) ? w1 : w2, rp, own);
        if (OBJ) phi += (double)(((o == 0 || o == 2) ? pp.wts[1] : pp.wts[2]) * rv);
      }
      if (in_act) {
        float rp, rv;
        qggmrf_unit<false, QUAD>(in_ok ? y[in_pos] - y[in_q] : 0.f, pp, rp, rv);
        L.fin[in_o][in_pos] = rp;
      }
    }
    __syncthreads();
    acc += own - (w1 * L.fin[0][s - offs[0]] + w2 * L.fin[1][s - offs[1]] +
                  w1 * L.fin[2][s - offs[2]] + w2 * L.fin[3][s - offs[3]]);
    if (has_next) {
      acc += cross_fwd(L.Y[cur], L.Y[1 - cur], true);
      __syncthreads();
      accn = cross_back();
    }
    if (store) {
      if constexpr (YG) {
        gp[go] = acc - bcur;
        yout[go] = ys_own;
        if (OBJ) yb += (double)ys_own * (double)bcur;
      } else {
        gp[go] = acc;
      }
    }
    bcur = bnext;
    acc = accn;
    accn = 0.f;
    if (NB == 26) cur = 1 - cur;
    __syncthreads();
  }
  if (part_out) block_sum4<SH::NT>(phi, yb, 0.0, 0.0, part_out, L.sred);
}

template <int NB, bool OBJ, bool QUAD, bool YG>
__global__ void __launch_bounds__(PR_NT)
prior_kernel(const float* __restrict__ xk, const float* __restrict__ xkm1,
             const double* __restrict__ scal, float* __restrict__ gp,
             const float* __restrict__ bvec, float* __restrict__ yout,
             double* __restrict__ partials, int N, int nz, int mode_fista, PriorParams pp) {
  __shared__ PriorLds<NB> L;
  // logical tile: x fastest, then y, then the slice chunk; XCD-contiguous so that tiles
  // sharing halo lines meet in one L2
  const int ntx = (N + PR_TX - 1) / PR_TX, nty = (N + PR_TY - 1) / PR_TY;
  const int lam = xcd_contiguous(blockIdx.x, ntx * nty * ((nz + PR_ZC - 1) / PR_ZC));
  const int c0 = (lam % ntx) * PR_TX, r0 = ((lam / ntx) % nty) * PR_TY;
  const int z0 = (lam / (ntx * nty)) * PR_ZC;
  const float mu = mode_fista ? (float)scal[SC_MU] : 0.f;
  double* part = partials ? partials + (idx_t)blockIdx.x * 4 : nullptr;
  const bool interior = r0 >= 1 && c0 >= 1 && r0 + PR_TY + 1 <= N && c0 + PR_TX + 1 <= N;
  if (interior)
    prior_tile<NB, OBJ, QUAD, false, YG>(L, xk, xkm1, gp, bvec, yout, part, N, nz, c0, r0, z0, mu,
                                         mode_fista != 0, pp);
  else
    prior_tile<NB, OBJ, QUAD, true, YG>(L, xk, xkm1, gp, bvec, yout, part, N, nz, c0, r0, z0, mu,
                                        mode_fista != 0, pp);
}

// --------------------------------------------------------------------------------- pass R'
template <int P, int PAIRS, int NB, int EL = kE>
struct RowsInvLds {
  static constexpr int TPF = P / EL, NT = PAIRS * TPF, RB = 2 * PAIRS, H = P / 2;
  static constexpr int CW = 64;
  static constexpr int ZD = (NB == 26) ? 3 : 1;
  static constexpr int YT = NB == 0 ? 1 : ZD * (RB + 2) * (CW + 2);
  static constexpr int FFT_BYTES = PAIRS * fft::row_region<P>() * 8;
  static constexpr int YT_BYTES = YT * 4;
  static constexpr int A_BYTES = FFT_BYTES > YT_BYTES ? FFT_BYTES : YT_BYTES;
  // Without the fused prior the transformed rows of pair pr overlay that pair's own FFT
  // region (2 H floats fit in P + P/16 complex); the fused prior needs region A for its tile.
  static constexpr bool OVER = NB == 0;
  static constexpr int REGF = 2 * fft::row_region<P>();  // floats per pair region
  static constexpr int TY_BYTES = OVER ? 0 : RB * H * 4;
  static TOMO_DEV int ty(int ry, int col) {
    return OVER ? (ry >> 1) * REGF + (ry & 1) * H + col : ry * H + col;
  }
  static constexpr int RED_BYTES = ((NT + 63) / 64) * 4 * 8;
  static constexpr int BYTES = A_BYTES + TY_BYTES + RED_BYTES;
};

// Block `blk` handles rows r0 .. r0+2*PAIRS-1 of one slice (blk counted over all slices);
// its four float64 partial sums go to part_out[0..3].
template <int P, int PAIRS, int MODE, int NB, bool OBJ, int EL = kE>
TOMO_DEV void rows_inv_body(unsigned char* smem, int blk, const cpx<float>* __restrict__ S2,
                            const float* __restrict__ xk, const float* __restrict__ xkm1,
                            const float* __restrict__ bvec, const float* __restrict__ gpv,
                            float* __restrict__ out, double* __restrict__ part_out, float mu,
                            float invL, const cpx<float>* __restrict__ tw, int N, int nz,
                            const PriorParams& pp) {
  using PL = fft::Plan<P, EL>;
  using LY = RowsInvLds<P, PAIRS, NB, EL>;
  constexpr int TPF = PL::TPF, E = PL::E, R0 = PL::radix(0), RL = PL::radix(PL::NS - 1);
  constexpr int NT = LY::NT, RB = LY::RB, H = LY::H;
  constexpr int REG = fft::row_region<P>();
  constexpr int CW = LY::CW, ZD = LY::ZD, YT = LY::YT;
  cpx<float>* fl = reinterpret_cast<cpx<float>*>(smem);
  float* ytile = reinterpret_cast<float*>(smem);
  float* tyt = reinterpret_cast<float*>(smem + (LY::OVER ? 0 : LY::A_BYTES));
  double* sred = reinterpret_cast<double*>(smem + LY::A_BYTES + LY::TY_BYTES);

  const int bps = (N + RB - 1) / RB;
  const int z = blk / bps;
  const int r0 = (blk - z * bps) * RB;
  const int t = threadIdx.x, pr = t / TPF, q = t - pr * TPF;
  const int r1 = r0 + 2 * pr;
  const bool active = r1 < N;

  // The point-wise epilogue (split-prior path) works on float4 groups: thread t owns the
  // groups t + u NT, u < 4, of the RB x N tile (RB N / 4 <= 4 NT since P >= 2N); its
  // operands are read after the transform (prefetching them before it costs registers,
  // hence occupancy, and was measured slower).
  constexpr bool PF = MODE != MODE_POWER && NB == 0;
  static_assert(H % 4 == 0, "float4 tile access");
  const int nq = N >> 2;
  const bool vec = PF && (N & 3) == 0 && RB * nq <= 4 * NT;

  // ---- C2R of rows r1, r1+1 packed as Z = X1 + i X2 over the full length P
  {
    const cpx<float>* s1 = S2 + ((idx_t)z * N + (active ? r1 : 0)) * H;
    const cpx<float>* s2 = s1 + H;
    cpx<float> v[E];
#pragma unroll
    for (int m = 0; m < E / R0; ++m)
#pragma unroll
      for (int r = 0; r < R0; ++r) {
        const int n = fft::reg_pos<P, TPF, R0>(q, m, r);
        cpx<float> zz = mk(0.f, 0.f);
        if (active) {
          if (n == 0) {
            const cpx<float> a = s1[0], b = s2[0];
            zz = mk(a.re, b.re);
          } else if (n == H) {
            const cpx<float> a = s1[0], b = s2[0];
            zz = mk(a.im, b.im);
          } else if (n < H) {
            const cpx<float> a = s1[n], b = s2[n];
            zz = mk(a.re - b.im, a.im + b.re);
          } else {
            const cpx<float> a = s1[P - n], b = s2[P - n];
            zz = mk(a.re + b.im, b.re - a.im);
          }
        }
        v[m * R0 + r] = zz;
      }
    fft::LdsRow<float> L{fl + pr * REG};
    fft::run_stages<PL, 0, +1>(v, q, tw, L);
#pragma unroll
    for (int m = 0; m < E / RL; ++m)
#pragma unroll
      for (int r = 0; r < RL; ++r) {
        const int n = fft::reg_pos<P, TPF, RL>(q, m, r);
        if (2 * r < RL && n < N) {  // positions >= P/2 (r >= RL/2) are cropped
          tyt[LY::ty(2 * pr, n)] = v[m * RL + r].re;
          tyt[LY::ty(2 * pr + 1, n)] = v[m * RL + r].im;
        }
      }
  }
  __syncthreads();

  double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
  if constexpr (PF) {
   if (vec) {
    // prior gradient precomputed by prior_kernel: point-wise epilogue on float4 groups
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = t + u * NT, ry = e / nq, row = r0 + ry;
      if (e < RB * nq && row < N) {
        const int col = 4 * (e - ry * nq);
        const idx_t o = ((idx_t)z * N + row) * N + col;
        // MODE_FISTA_Y: xkm1 holds y and gpv holds gp - b (b not read)
        const float4 xa4 = *reinterpret_cast<const float4*>(xk + o);
        const float4 gp4 = *reinterpret_cast<const float4*>(gpv + o);
        const float4 ty4 = *reinterpret_cast<const float4*>(tyt + LY::ty(ry, col));
        float bv[4] = {0.f, 0.f, 0.f, 0.f};
        if constexpr (MODE != MODE_FISTA_Y) {
          const float4 bv4 = *reinterpret_cast<const float4*>(bvec + o);
          bv[0] = bv4.x; bv[1] = bv4.y; bv[2] = bv4.z; bv[3] = bv4.w;
        }
        const float av[4] = {xa4.x, xa4.y, xa4.z, xa4.w};
        const float gv[4] = {gp4.x, gp4.y, gp4.z, gp4.w};
        const float tv[4] = {ty4.x, ty4.y, ty4.z, ty4.w};
        float km1[4] = {0.f, 0.f, 0.f, 0.f};
        if constexpr (MODE == MODE_FISTA || MODE == MODE_FISTA_Y) {
          const float4 b4 = *reinterpret_cast<const float4*>(xkm1 + o);
          km1[0] = b4.x; km1[1] = b4.y; km1[2] = b4.z; km1[3] = b4.w;
        }
        float res[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const float a = av[k];
          const float ys = (MODE == MODE_FISTA)   ? a + mu * (a - km1[k])
                           : (MODE == MODE_FISTA_Y) ? km1[k]
                                                    : a;
          const float g = (MODE == MODE_FISTA_Y) ? tv[k] + gv[k] : tv[k] - bv[k] + gv[k];
          if constexpr (MODE == MODE_FISTA || MODE == MODE_FISTA_Y) {
            const float xn = ys - g * invL;
            res[k] = xn;
            acc3 += (double)(ys - xn) * (double)(xn - a);
          } else {
            res[k] = g;
          }
          acc0 += (double)ys * (double)tv[k];
          if constexpr (MODE != MODE_FISTA_Y) acc1 += (double)ys * (double)bv[k];
        }
        *reinterpret_cast<float4*>(out + o) = make_float4(res[0], res[1], res[2], res[3]);
      }
    }
   } else {
    // prior gradient precomputed by prior_kernel: point-wise epilogue, no neighbour tile
    for (int e = t; e < RB * N; e += NT) {
      const int ry = e / N, col = e - ry * N, row = r0 + ry;
      if (row < N) {
        const idx_t o = ((idx_t)z * N + row) * N + col;
        const float a = xk[o];
        const float ys = (MODE == MODE_FISTA)   ? a + mu * (a - xkm1[o])
                         : (MODE == MODE_FISTA_Y) ? xkm1[o]
                                                  : a;
        const float ty = tyt[LY::ty(ry, col)];
        const float bs = (MODE == MODE_FISTA_Y) ? 0.f : bvec[o];
        const float g = ty - bs + gpv[o];
        if constexpr (MODE == MODE_FISTA || MODE == MODE_FISTA_Y) {
          const float xn = ys - g * invL;
          out[o] = xn;
          acc3 += (double)(ys - xn) * (double)(xn - a);
        } else {
          out[o] = g;
        }
        acc0 += (double)ys * (double)ty;
        acc1 += (double)ys * (double)bs;
      }
    }
   }
  } else if constexpr (MODE == MODE_POWER) {
    for (int e = t; e < RB * N; e += NT) {
      const int ry = e / N, col = e - ry * N, row = r0 + ry;
      if (row < N) {
        const float ty = tyt[LY::ty(ry, col)];
        out[((idx_t)z * N + row) * N + col] = ty;
        acc0 += (double)ty * (double)ty;
      }
    }
  } else {
    for (int c0 = 0; c0 < N; c0 += CW) {
      for (int e = t; e < YT; e += NT) {
        const int dzi = e / ((RB + 2) * (CW + 2));
        const int rem = e - dzi * (RB + 2) * (CW + 2);
        const int ry = rem / (CW + 2), cx = rem - ry * (CW + 2);
        const int zz = z + dzi - ZD / 2;
        const int row = r0 - 1 + ry, col = c0 - 1 + cx;
        float yv = 0.f;
        if (zz >= 0 && zz < nz && row >= 0 && row < N && col >= 0 && col < N) {
          const idx_t o = ((idx_t)zz * N + row) * N + col;
          const float a = xk[o];
          yv = (MODE == MODE_FISTA) ? a + mu * (a - xkm1[o]) : a;
        }
        ytile[e] = yv;
      }
      __syncthreads();
      for (int e = t; e < RB * CW; e += NT) {
        const int ry = e / CW, cx = e - ry * CW;
        const int row = r0 + ry, col = c0 + cx;
        if (row < N && col < N) {
          const int cidx = ((ZD / 2) * (RB + 2) + ry + 1) * (CW + 2) + cx + 1;
          const float ys = ytile[cidx];
          const bool vz[3] = {z > 0, true, z + 1 < nz};
          const bool vy[3] = {row > 0, true, row + 1 < N};
          const bool vx[3] = {col > 0, true, col + 1 < N};
          float gsum = 0.f, phi = 0.f;
#pragma unroll
          for (int dz = -1; dz <= 1; ++dz) {
            if (NB == 8 && dz != 0) continue;
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
              for (int dx = -1; dx <= 1; ++dx) {
                if (dz == 0 && dy == 0 && dx == 0) continue;
                // a neighbour outside the volume enters with difference 0, where rho and
                // rho' vanish exactly: the pair is omitted without a branch
                const bool valid = vz[dz + 1] && vy[dy + 1] && vx[dx + 1];
                const float yn = ytile[cidx + (dz * (RB + 2) + dy) * (CW + 2) + dx];
                const float wgt = pp.wts[(dz != 0) + (dy != 0) + (dx != 0)];
                float rp, rv = 0.f;
                qggmrf<OBJ>(valid ? ys - yn : 0.f, pp, rp, rv);
                gsum += wgt * rp;
                if constexpr (OBJ) {
                  // each unordered pair once: the lexicographically positive offset
                  const bool half = dz > 0 || (dz == 0 && (dy > 0 || (dy == 0 && dx > 0)));
                  if (half) phi += wgt * rv;
                }
              }
          }
          const idx_t o = ((idx_t)z * N + row) * N + col;
          const float ty = tyt[LY::ty(ry, col)];
          const float bs = bvec[o];
          const float g = ty - bs + pp.beta * gsum;
          if constexpr (MODE == MODE_FISTA) {
            const float xn = ys - g * invL;
            out[o] = xn;
            const float xo = xk[o];
            acc3 += (double)(ys - xn) * (double)(xn - xo);
          } else {
            out[o] = g;
          }
          acc0 += (double)ys * (double)ty;
          acc1 += (double)ys * (double)bs;
          if constexpr (OBJ) acc2 += (double)phi;
        }
      }
      __syncthreads();
    }
  }
  block_sum4<NT>(acc0, acc1, acc2, acc3, part_out, sred);
}

template <int P, int PAIRS, int MODE, int NB, bool OBJ>
__global__ void __launch_bounds__(PAIRS * (P / kE))
rows_inv_kernel(const cpx<float>* __restrict__ S2, const float* __restrict__ xk,
                const float* __restrict__ xkm1, const float* __restrict__ bvec,
                const float* __restrict__ gpv, float* __restrict__ out,
                double* __restrict__ partials, const double* __restrict__ scal,
                const cpx<float>* __restrict__ tw, int N, int nz, PriorParams pp) {
  __shared__ __align__(16) unsigned char smem[RowsInvLds<P, PAIRS, NB>::BYTES];
  const float mu = (MODE == MODE_FISTA) ? (float)scal[SC_MU] : 0.f;
  const float invL = (MODE == MODE_FISTA || MODE == MODE_FISTA_Y) ? (float)scal[SC_INVL] : 0.f;
  rows_inv_body<P, PAIRS, MODE, NB, OBJ>(smem, blockIdx.x, S2, xk, xkm1, bvec, gpv, out,
                                         partials + (idx_t)blockIdx.x * 4, mu, invL, tw, N, nz,
                                         pp);
}

// -------------------------------------------------------------------------------- finalize
// One block of FIN_NT threads: the partial sums are read with FIN_NT loads in flight (the
// kernel is bound by that latency), then summed in a fixed tree order.
constexpr int FIN_NT = 1024;
template <int MODE>
__global__ void __launch_bounds__(FIN_NT)
finalize_kernel(const double* __restrict__ partials, int nblocks,
                const double* __restrict__ prior_partials, int nprior, double* __restrict__ scal,
                double* __restrict__ hist, int32_t* __restrict__ rhist,
                double* __restrict__ obj_out) {
  __shared__ double sh[4][FIN_NT];
  const int t = threadIdx.x;
  double a[4] = {0, 0, 0, 0};
  for (int b = t; b < nblocks; b += FIN_NT) {
    const double4 pv = *reinterpret_cast<const double4*>(partials + (idx_t)b * 4);
    a[0] += pv.x;
    a[1] += pv.y;
    a[2] += pv.z;
    a[3] += pv.w;
  }
  // Phi from the separate prior kernel (slot 0 of its partials) lands in slot 2; its slot 1
  // holds <y, b> when the prior kernel wrote y and gp - b (zero otherwise)
  for (int b = t; b < nprior; b += FIN_NT) {
    a[2] += prior_partials[(idx_t)b * 4];
    a[1] += prior_partials[(idx_t)b * 4 + 1];
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) sh[i][t] = a[i];
  __syncthreads();
  for (int s = FIN_NT / 2; s > 0; s >>= 1) {
    if (t < s)
#pragma unroll
      for (int i = 0; i < 4; ++i) sh[i][t] += sh[i][t + s];
    __syncthreads();
  }
  if (t != 0) return;
  const double s0 = sh[0][0], s1 = sh[1][0], s2 = sh[2][0], s3 = sh[3][0];
  if constexpr (MODE == MODE_POWER) {
    const double wn = sqrt(s0);
    scal[SC_LAMBDA] = wn / scal[SC_VNORM];
    scal[SC_PSCALE] = wn > 0.0 ? 1.0 / wn : 0.0;
    scal[SC_VNORM] = 1.0;
    scal[SC_GSUM] = s0;
  } else if constexpr (MODE == MODE_GRAD) {
    const double obj = 0.5 * s0 - s1 + scal[SC_BETA] * s2;
    if (obj_out) obj_out[0] = obj;
    scal[SC_LASTOBJ] = obj;
  } else {
    const int k = (int)scal[SC_ITER];
    const double obj = 0.5 * s0 - s1 + 0.5 * scal[SC_GG] + scal[SC_BETA] * s2;
    if (hist) hist[k] = obj;
    scal[SC_LASTOBJ] = obj;
    const double tk = scal[SC_T];
    double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * tk * tk));
    const bool restart = scal[SC_RESTART_ON] != 0.0 && s3 > 0.0;
    double mu;
    if (restart) {
      tn = 1.0;
      mu = 0.0;
      scal[SC_NRESTART] += 1.0;
    } else {
      mu = (tk - 1.0) / tn;
    }
    if (rhist) rhist[k] = restart ? 1 : 0;
    const bool bad = !isfinite(s3) || !isfinite(s0) || !isfinite(s1) || (hist && !isfinite(obj));
    if (bad && scal[SC_NONFINITE] < 0.0) scal[SC_NONFINITE] = (double)k;
    scal[SC_T] = tn;
    scal[SC_MU] = mu;
    scal[SC_ITER] = (double)(k + 1);
  }
}

// ------------------------------------------------------------------- batched iteration
// One persistent launch advances every problem of a batch by one iteration.  Blocks take
// tiles from a queue ordered by phase: the pair-shared prior tiles of all problems (which also
// write y and gp - b), then pass R, pass C and pass R'.  A tile of phase h > 0 of problem j
// first waits until every phase h - 1 tile of j is finished.  Every tile waited on sits earlier
// in the queue and was taken by a block that is already running and never waits on a later
// tile, so the waits end; each is also bounded and raises ctl[2] instead of spinning forever.
// The block finishing the last pass-R' tile of a problem runs that problem's float64
// finalize.  The last block to leave resets the queue for the next launch.
//
// Each problem's transforms use EL = 8 or 16 elements per thread (its FFT radix schedule),
// chosen per FFT size by the batch autotuner; a tile of every phase is one 256-thread block.
constexpr int BT = kBatchThreads;

template <int P, int EL>
constexpr int bt_tpf() { return P / EL; }
template <int P, int EL>
constexpr int bt_pairs() { return BT / bt_tpf<P, EL>() < 1 ? 1 : BT / bt_tpf<P, EL>(); }
template <int P, int EL>
constexpr int bt_tc() { return bt_pairs<P, EL>(); }

template <int P, int EL>
constexpr int batch_lds_pe() {
  constexpr int a = rows_fwd_lds<P, bt_pairs<P, EL>()>();
  constexpr int b = cols_conv_lds<P, bt_tc<P, EL>()>();
  constexpr int c = RowsInvLds<P, bt_pairs<P, EL>(), 0, EL>::BYTES;
  constexpr int m = a > b ? a : b;
  return m > c ? m : c;
}
constexpr int cmax(int a, int b) { return a > b ? a : b; }
template <int P>
constexpr int batch_lds_p() { return cmax(batch_lds_pe<P, 8>(), batch_lds_pe<P, 16>()); }
constexpr int kBatchLds =
    cmax(cmax(cmax(batch_lds_p<256>(), batch_lds_p<512>()), cmax(batch_lds_p<1024>(), batch_lds_p<2048>())),
         cmax(cmax((int)sizeof(PriorLds<26, 16>), (int)sizeof(PriorLds<8, 16>)), 4 * BT * 8));
// with the in-plane prior evaluated inside pass R' (8-neighbour problems, no prior phase)
template <int P>
constexpr int batch_lds_fused_p() {
  return cmax(RowsInvLds<P, bt_pairs<P, 8>(), 8, 8>::BYTES, RowsInvLds<P, bt_pairs<P, 16>(), 8, 16>::BYTES);
}
constexpr int kBatchLdsFused =
    cmax(kBatchLds, cmax(cmax(batch_lds_fused_p<256>(), batch_lds_fused_p<512>()),
                         cmax(batch_lds_fused_p<1024>(), batch_lds_fused_p<2048>())));
static_assert(PriorShape<16>::NT == BT, "a batch prior tile is one block");

// Cross-XCD ordering of the tile counters.  The eight L2 caches are not coherent with one
// another for ordinary stores, so an agent-scope release writes this XCD's dirty L2 lines back
// and an agent-scope acquire invalidates its L2.  Polling therefore reads the counter with a
// relaxed agent-scope load (coherent, no cache maintenance) and takes the acquire once, after
// the wait ends; an acquire on every poll would keep invalidating the L2 under the tiles that
// other blocks of the XCD are transforming.
TOMO_DEV void bounded_wait(const int* ctr, int target, int* err) {
  if (threadIdx.x == 0) {
    int spins = 0;
    while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(2);
      if (++spins > (1 << 22)) {
        __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
}

// Each phase body is its own non-inlined function so that its registers are allocated on
// their own rather than across every variant the persistent kernel can dispatch to.
// A prior item is a strip of up to BP_SUB tiles of 16 x 16 voxels along a row band (and a
// chunk of PR_ZC slices), transformed one tile after the other by the same block: few queue
// items per problem however small its tiles are.
constexpr int BP_SUB = 16;

template <int NB, bool QUAD>
TOMO_DEV void batch_phase_prior_in(unsigned char* smem, int tile,
                                                            const BatchProb* pb, int ik, int ikm1) {
  using SH = PriorShape<16>;
  const int N = pb->N;
  const int ntx = (N + SH::TX - 1) / SH::TX, nty = (N + SH::TY - 1) / SH::TY;
  const int nst = (ntx + BP_SUB - 1) / BP_SUB;  // strips per row band
  const int strip = tile % nst, band = tile / nst;
  const int r0 = (band % nty) * SH::TY, z0 = (band / nty) * PR_ZC;
  const float mu = (float)pb->scal[SC_MU];
  auto& L = *reinterpret_cast<PriorLds<NB, 16>*>(smem);
  const int tx1 = min(ntx, (strip + 1) * BP_SUB);
  for (int tx = strip * BP_SUB; tx < tx1; ++tx) {
    const int c0 = tx * SH::TX;
    const bool interior = r0 >= 1 && c0 >= 1 && r0 + SH::TY + 1 <= N && c0 + SH::TX + 1 <= N;
    if (interior)
      prior_tile<NB, false, QUAD, false, true, 16>(L, pb->x[ik], pb->x[ikm1], pb->gp, pb->b, pb->y,
                                                   nullptr, N, pb->nz, c0, r0, z0, mu, true, pb->pp);
    else
      prior_tile<NB, false, QUAD, true, true, 16>(L, pb->x[ik], pb->x[ikm1], pb->gp, pb->b, pb->y,
                                                  nullptr, N, pb->nz, c0, r0, z0, mu, true, pb->pp);
    __syncthreads();  // the next tile rewrites the plane buffers
  }
}

// A queue item of passes R, C and R' is a run of pb->grp consecutive tiles (the last run of a
// problem may be shorter), transformed one after the other by the same block.
TOMO_DEV void item_tiles(int item, int grp, int ntiles, int* t0, int* t1) {
  *t0 = item * grp;
  *t1 = min(ntiles, *t0 + grp);
}

template <int P, int EL, bool ONE = false>
TOMO_DEV void batch_phase_r_in(unsigned char* smem, int item,
                                                        const BatchProb* pb, int ik, int ikm1) {
  int t0 = item, t1 = item + 1;  // ONE: the item is one tile (no loop to hoist across)
  if constexpr (!ONE) item_tiles(item, pb->grp, pb->nR, &t0, &t1);
  const float mu = (float)pb->scal[SC_MU];
  for (int tile = t0; tile < t1; ++tile) {
    if (tile > t0) __syncthreads();  // the previous tile's rows are read from LDS
    if (pb->fused)  // no prior phase: form y = x_k + mu (x_k - x_{k-1}) here
      rows_fwd_body<P, bt_pairs<P, EL>(), MODE_FISTA, EL>(smem, tile, pb->x[ik], pb->x[ikm1], mu, 1.f,
                                                          pb->S1, pb->tw, pb->N, pb->nz * (pb->N / 2));
    else
      rows_fwd_body<P, bt_pairs<P, EL>(), MODE_FISTA_Y, EL>(smem, tile, pb->y, pb->y, 0.f, 1.f, pb->S1,
                                                            pb->tw, pb->N, pb->nz * (pb->N / 2));
  }
}

template <int P, int EL, bool ONE = false>
TOMO_DEV void batch_phase_c_in(unsigned char* smem, int item,
                                                        const BatchProb* pb) {
  constexpr int TC = bt_tc<P, EL>();
  constexpr int ncol = (P / 2) / TC;
  int t0 = item, t1 = item + 1;  // ONE: the item is one tile (no loop to hoist across)
  if constexpr (!ONE) item_tiles(item, pb->grp, pb->nC, &t0, &t1);
  for (int tile = t0; tile < t1; ++tile) {
    if (tile > t0) __syncthreads();
    const int z = tile / ncol;
    cols_conv_body<P, TC, EL>(smem, tile - z * ncol, z, pb->S1, pb->S2, pb->fk, pb->fkn, pb->tw, pb->N);
  }
}

// pass R' of a step whose y and gp - b were written by the prior phase (x_{k-1} slot: y)
template <int P, int EL, bool ONE = false>
TOMO_DEV void batch_phase_rp_in(unsigned char* smem, int item,
                                                         const BatchProb* pb, int ik, int inext) {
  int t0 = item, t1 = item + 1;  // ONE: the item is one tile (no loop to hoist across)
  if constexpr (!ONE) item_tiles(item, pb->grp, pb->nRp, &t0, &t1);
  const float invL = (float)pb->scal[SC_INVL];
  for (int tile = t0; tile < t1; ++tile) {
    if (tile > t0) __syncthreads();
    rows_inv_body<P, bt_pairs<P, EL>(), MODE_FISTA_Y, 0, false, EL>(
        smem, tile, pb->S2, pb->x[ik], pb->y, nullptr, pb->gp, pb->x[inext],
        pb->partials + (idx_t)tile * 4, 0.f, invL, pb->tw, pb->N, pb->nz, pb->pp);
  }
}

// pass R' with the in-plane prior evaluated over a neighbour tile in its epilogue (each pair
// from both of its voxels): the 8-neighbour problems of a batch scheduled without prior phase
template <int P, int EL, bool ONE = false>
TOMO_DEV void batch_phase_rp_fused_in(unsigned char* smem, int item,
                                                               const BatchProb* pb, int ik, int ikm1,
                                                               int inext) {
  int t0 = item, t1 = item + 1;  // ONE: the item is one tile (no loop to hoist across)
  if constexpr (!ONE) item_tiles(item, pb->grp, pb->nRp, &t0, &t1);
  const float mu = (float)pb->scal[SC_MU];
  const float invL = (float)pb->scal[SC_INVL];
  for (int tile = t0; tile < t1; ++tile) {
    if (tile > t0) __syncthreads();
    rows_inv_body<P, bt_pairs<P, EL>(), MODE_FISTA, 8, false, EL>(
        smem, tile, pb->S2, pb->x[ik], pb->x[ikm1], pb->b, nullptr, pb->x[inext],
        pb->partials + (idx_t)tile * 4, mu, invL, pb->tw, pb->N, pb->nz, pb->pp);
  }
}

// Non-inlined entry points of the phase bodies for the persistent kernel, which may dispatch to
// every phase and size: each body's registers are then allocated on their own.  The
// per-phase kernels inline the bodies of their one phase instead.
template <int NB, bool QUAD>
__device__ __attribute__((noinline)) void batch_phase_prior(unsigned char* smem, int tile,
                                                            const BatchProb* pb, int ik, int ikm1) {
  batch_phase_prior_in<NB, QUAD>(smem, tile, pb, ik, ikm1);
}
template <int P, int EL>
__device__ __attribute__((noinline)) void batch_phase_r(unsigned char* smem, int item,
                                                        const BatchProb* pb, int ik, int ikm1) {
  batch_phase_r_in<P, EL>(smem, item, pb, ik, ikm1);
}
template <int P, int EL>
__device__ __attribute__((noinline)) void batch_phase_c(unsigned char* smem, int item,
                                                        const BatchProb* pb) {
  batch_phase_c_in<P, EL>(smem, item, pb);
}
template <int P, int EL>
__device__ __attribute__((noinline)) void batch_phase_rp(unsigned char* smem, int item,
                                                         const BatchProb* pb, int ik, int inext) {
  batch_phase_rp_in<P, EL>(smem, item, pb, ik, inext);
}
template <int P, int EL>
__device__ __attribute__((noinline)) void batch_phase_rp_fused(unsigned char* smem, int item,
                                                               const BatchProb* pb, int ik, int ikm1,
                                                               int inext) {
  batch_phase_rp_fused_in<P, EL>(smem, item, pb, ik, ikm1, inext);
}

// One item of phase PH (1 R, 2 C, 3 R') of a problem with transform size P and EL elements
// per thread, inlined; with one launch per phase an item is one tile (the work list is built
// with one tile per item), so no tile loop keeps loop-invariant twiddles live.
template <int PH, int P, int EL, bool FUSED>
TOMO_DEV void batch_tile_inline(unsigned char* smem, int item, const BatchProb* pb, int ik,
                                int ikm1, int inext) {
  if constexpr (PH == 1) batch_phase_r_in<P, EL, true>(smem, item, pb, ik, ikm1);
  else if constexpr (PH == 2) batch_phase_c_in<P, EL, true>(smem, item, pb);
  else if (FUSED && pb->fused) batch_phase_rp_fused_in<P, EL, true>(smem, item, pb, ik, ikm1, inext);
  else batch_phase_rp_in<P, EL, true>(smem, item, pb, ik, inext);
}

template <int P, int EL, bool FUSED>
TOMO_DEV void batch_tile_pe(unsigned char* smem, int phase, int item, const BatchProb* pb, int ik,
                            int ikm1, int inext) {
  if (phase == 1) batch_phase_r<P, EL>(smem, item, pb, ik, ikm1);
  else if (phase == 2) batch_phase_c<P, EL>(smem, item, pb);
  else if (FUSED && pb->fused) batch_phase_rp_fused<P, EL>(smem, item, pb, ik, ikm1, inext);
  else batch_phase_rp<P, EL>(smem, item, pb, ik, inext);
}

template <int P, bool FUSED>
TOMO_DEV void batch_tile(unsigned char* smem, int phase, int tile, const BatchProb* pb, int ik,
                         int ikm1, int inext) {
  if (pb->el == 8) batch_tile_pe<P, 8, FUSED>(smem, phase, tile, pb, ik, ikm1, inext);
  else batch_tile_pe<P, 16, FUSED>(smem, phase, tile, pb, ik, ikm1, inext);
}

// Float64 reduction of one problem's partial sums and its momentum / restart update (the same
// arithmetic as finalize_kernel in FISTA mode), run by one whole block.
TOMO_DEV void batch_finalize(const BatchProb& pb, double* sh /* [4][BT] */) {
  const int t = threadIdx.x;
  double a[4] = {0, 0, 0, 0};
  for (int b = t; b < pb.nRp; b += BT)
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] += pb.partials[(idx_t)b * 4 + i];
#pragma unroll
  for (int i = 0; i < 4; ++i) sh[i * BT + t] = a[i];
  __syncthreads();
  for (int s = BT / 2; s > 0; s >>= 1) {
    if (t < s)
#pragma unroll
      for (int i = 0; i < 4; ++i) sh[i * BT + t] += sh[i * BT + t + s];
    __syncthreads();
  }
  if (t == 0) {
    double* scal = pb.scal;
    const double s0 = sh[0], s1 = sh[BT], s3 = sh[3 * BT];
    const int k = (int)scal[SC_ITER];
    const double obj = 0.5 * s0 - s1 + 0.5 * scal[SC_GG];
    if (pb.hist) pb.hist[k] = obj;
    scal[SC_LASTOBJ] = obj;
    const double tk = scal[SC_T];
    double tn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * tk * tk));
    const bool restart = scal[SC_RESTART_ON] != 0.0 && s3 > 0.0;
    double mu;
    if (restart) {
      tn = 1.0;
      mu = 0.0;
      scal[SC_NRESTART] += 1.0;
    } else {
      mu = (tk - 1.0) / tn;
    }
    if (pb.rhist) pb.rhist[k] = restart ? 1 : 0;
    if ((!isfinite(s3) || !isfinite(s0) || !isfinite(s1)) && scal[SC_NONFINITE] < 0.0)
      scal[SC_NONFINITE] = (double)k;
    scal[SC_T] = tn;
    scal[SC_MU] = mu;
    scal[SC_ITER] = (double)(k + 1);
  }
  __syncthreads();
}

// At most 168 VGPRs (3 waves per SIMD): the non-inlined phase bodies keep a small call frame in
// scratch instead of raising the register count to 182 (2 waves); a tighter bound (4 waves)
// grows the frames and was measured slower.
// FUSED: the instantiation whose 8-neighbour problems may take the prior inside pass R'
// (more LDS per block).
template <bool FUSED>
__global__ void __launch_bounds__(BT, 3)
batch_iter_kernel(const BatchProb* __restrict__ probs, const int2* __restrict__ items,
                  int n_items, int* ctl, int* cnt, int nprob, int ik, int ikm1, int inext) {
  __shared__ __align__(16) unsigned char smem[FUSED ? kBatchLdsFused : kBatchLds];
  __shared__ int s_item, s_fin;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(&ctl[0], 1);
    __syncthreads();
    const int it = s_item;
    if (it >= n_items) break;
    const int2 d = items[it];
    const int j = d.x & 0xffffff, ph = d.x >> 24, tile = d.y;
    const BatchProb& pb = probs[j];
    if (ph > 0) {
      const int need = ph == 1 ? pb.nPr : (ph == 2 ? pb.iR : pb.iC);
      bounded_wait(&cnt[(ph - 1) * nprob + j], need, &ctl[2]);
    }
    if (ph == 0) {
      if (pb.neighbours == 26) {
        if (pb.pp.quadratic) batch_phase_prior<26, true>(smem, tile, &pb, ik, ikm1);
        else batch_phase_prior<26, false>(smem, tile, &pb, ik, ikm1);
      } else {
        if (pb.pp.quadratic) batch_phase_prior<8, true>(smem, tile, &pb, ik, ikm1);
        else batch_phase_prior<8, false>(smem, tile, &pb, ik, ikm1);
      }
    } else {
      switch (pb.P) {
        case 256: batch_tile<256, FUSED>(smem, ph, tile, &pb, ik, ikm1, inext); break;
        case 512: batch_tile<512, FUSED>(smem, ph, tile, &pb, ik, ikm1, inext); break;
        case 1024: batch_tile<1024, FUSED>(smem, ph, tile, &pb, ik, ikm1, inext); break;
        case 2048: batch_tile<2048, FUSED>(smem, ph, tile, &pb, ik, ikm1, inext); break;
        default: break;
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // publish this tile's results
      const int done = __hip_atomic_fetch_add(&cnt[ph * nprob + j], 1, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
      s_fin = (ph == 3 && done == pb.iRp - 1) ? 1 : 0;
      if (s_fin) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // see every partial sum
    }
    __syncthreads();
    if (s_fin) batch_finalize(pb, reinterpret_cast<double*>(smem));
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    __threadfence();
    const int left = atomicAdd(&ctl[1], 1);
    if (left == (int)gridDim.x - 1) {
      // every other block has left the loop: reset the queue for the next launch
      ctl[0] = 0;
      ctl[1] = 0;
      for (int i = 0; i < 4 * nprob; ++i) cnt[i] = 0;
      __threadfence();
    }
  }
}

// The same iteration as one launch per phase instead of one persistent launch: block b of
// phase PH takes item b of that phase's part of the work list (all problems of the batch),
// and the launch boundaries order the phases, so there are no tile waits, counters or
// fences.  The same tile bodies write the same partial sums; batch_finalize_kernel then
// runs each problem's float64 finalize (one block per problem).
// LDS of one phase: the largest body it may run (every batch size, 8 or 16 elements).
template <int PH, int P, int EL, bool FUSED>
constexpr int batch_phase_lds_pe() {
  if constexpr (PH == 1) return rows_fwd_lds<P, bt_pairs<P, EL>()>();
  else if constexpr (PH == 2) return cols_conv_lds<P, bt_tc<P, EL>()>();
  else if constexpr (FUSED) return cmax(RowsInvLds<P, bt_pairs<P, EL>(), 0, EL>::BYTES,
                                        RowsInvLds<P, bt_pairs<P, EL>(), 8, EL>::BYTES);
  else return RowsInvLds<P, bt_pairs<P, EL>(), 0, EL>::BYTES;
}
template <int PH, int P, bool FUSED>
constexpr int batch_phase_lds_p() {
  return cmax(batch_phase_lds_pe<PH, P, 8, FUSED>(), batch_phase_lds_pe<PH, P, 16, FUSED>());
}
template <int PH, int P, int EL, bool FUSED>
constexpr int batch_phase_lds() {
  if constexpr (PH == 0) return cmax((int)sizeof(PriorLds<26, 16>), (int)sizeof(PriorLds<8, 16>));
  else return batch_phase_lds_pe<PH, P, EL, FUSED>();
}

// One launch covers the items of one phase and one transform size P with EL elements per
// thread (the prior phase: every problem, P and EL unused), so that each kernel holds the
// body of one schedule only.
template <int PH, int P, int EL, bool FUSED>
__global__ void __launch_bounds__(BT)
batch_phase_kernel(const BatchProb* __restrict__ probs, const int2* __restrict__ items, int ik,
                   int ikm1, int inext) {
  __shared__ __align__(16) unsigned char smem[batch_phase_lds<PH, P, EL, FUSED>()];
  const int2 d = items[blockIdx.x];
  const int j = d.x & 0xffffff, tile = d.y;
  const BatchProb& pb = probs[j];
  if constexpr (PH == 0) {
    if (pb.neighbours == 26) {
      if (pb.pp.quadratic) batch_phase_prior_in<26, true>(smem, tile, &pb, ik, ikm1);
      else batch_phase_prior_in<26, false>(smem, tile, &pb, ik, ikm1);
    } else {
      if (pb.pp.quadratic) batch_phase_prior_in<8, true>(smem, tile, &pb, ik, ikm1);
      else batch_phase_prior_in<8, false>(smem, tile, &pb, ik, ikm1);
    }
  } else {
    batch_tile_inline<PH, P, EL, FUSED>(smem, tile, &pb, ik, ikm1, inext);
  }
}

__global__ void __launch_bounds__(BT) batch_finalize_kernel(const BatchProb* __restrict__ probs) {
  __shared__ double sh[4 * BT];
  batch_finalize(probs[blockIdx.x], sh);
}

__global__ void fill_int_kernel(int* x, idx_t n, int v) {
  const idx_t i = (idx_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

// ------------------------------------------------------------------- launch configuration
constexpr int fwd_pairs(int P) {
  const int tpf = P / kE;
  int pairs = 256 / tpf;
  if (pairs < 1) pairs = 1;
  if (pairs > 64) pairs = 64;
  return pairs;
}
constexpr int inv_pairs(int P) {
  const int tpf = P / kE;
  int pairs = 256 / tpf;
  if (pairs < 1) pairs = 1;
  if (pairs > 8) pairs = 8;
  return pairs;
}
constexpr int col_tc(int P) {
  int tc = 8192 / P;  // 64 KiB of LDS per block
  if (tc > 16) tc = 16;
  if (tc < 1) tc = 1;
  return tc;
}

// Tile variants of the three transform passes, chosen per plan level by the autotuner:
// variant 0 halves, 1 keeps, 2 doubles the default number of row pairs (passes R, R') or
// columns (pass C) per block, within 1024 threads and 128 KiB of LDS per block.  Transform
// sizes below 256 have the default only.  Each row or column is transformed by the same code
// whatever the grouping, so all variants give identical results.
constexpr int kLdsCap = 128 * 1024;
constexpr int vsel(int base, int v) { return v == 0 ? (base > 1 ? base / 2 : 1) : (v == 2 ? 2 * base : base); }
constexpr int fwd_pairs_v(int P, int v) {
  int x = P < 256 ? fwd_pairs(P) : vsel(fwd_pairs(P), v);
  while (x > 1 && (x * (P / kE) > 1024 || x * (P + P / 16) * 8 > kLdsCap)) x /= 2;
  return x;
}
constexpr int col_tc_v(int P, int v) {
  int x = P < 256 ? col_tc(P) : vsel(col_tc(P), v);
  while (x > 1 && (x * (P / kE) > 1024 || x * P * 8 > kLdsCap)) x /= 2;
  return x;
}
constexpr int inv_pairs_v(int P, int v) {
  int x = P < 256 ? inv_pairs(P) : vsel(inv_pairs(P), v);
  while (x > 1 && (x * (P / kE) > 1024 || x * (P + P / 16) * 8 + x * P * 4 + 1024 > kLdsCap)) x /= 2;
  return x;
}

template <int P, int V>
hipError_t rows_fwd_pv(int mode, const float* xk, const float* xkm1, const double* scal,
                       cpx<float>* S1, const cpx<float>* tw, int N, int nz, hipStream_t st,
                       const double* pprev, int nprev) {
  constexpr int PAIRS = fwd_pairs_v(P, V);
  constexpr int NT = PAIRS * fft::Plan<P, kE>::TPF;
  const int n_pairs = nz * (N / 2);
  const dim3 grid((n_pairs + PAIRS - 1) / PAIRS);
  if (mode == MODE_POWER)
    hipLaunchKernelGGL((rows_fwd_kernel<P, PAIRS, MODE_POWER>), grid, dim3(NT), 0, st, xk, xkm1,
                       scal, S1, tw, N, n_pairs, pprev, nprev);
  else if (mode == MODE_FISTA_Y)
    hipLaunchKernelGGL((rows_fwd_kernel<P, PAIRS, MODE_FISTA_Y>), grid, dim3(NT), 0, st, xk, xkm1,
                       scal, S1, tw, N, n_pairs, nullptr, 0);
  else
    hipLaunchKernelGGL((rows_fwd_kernel<P, PAIRS, MODE_FISTA>), grid, dim3(NT), 0, st, xk, xkm1,
                       scal, S1, tw, N, n_pairs, nullptr, 0);
  return hipGetLastError();
}

template <int P>
hipError_t rows_fwd_p(int v, int mode, const float* xk, const float* xkm1, const double* scal,
                      cpx<float>* S1, const cpx<float>* tw, int N, int nz, hipStream_t st,
                      const double* pprev, int nprev) {
  if (v == 0) return rows_fwd_pv<P, 0>(mode, xk, xkm1, scal, S1, tw, N, nz, st, pprev, nprev);
  if (v == 2) return rows_fwd_pv<P, 2>(mode, xk, xkm1, scal, S1, tw, N, nz, st, pprev, nprev);
  return rows_fwd_pv<P, 1>(mode, xk, xkm1, scal, S1, tw, N, nz, st, pprev, nprev);
}

template <int P, int V>
hipError_t cols_conv_pv(const cpx<float>* S1, cpx<float>* S2, const float* fk, const float* fkn,
                        const cpx<float>* tw, int N, int nz, hipStream_t st) {
  constexpr int TC = col_tc_v(P, V);
  constexpr int NT = TC * fft::Plan<P, kE>::TPF;
  const dim3 grid(((P / 2) / TC) * nz);
  hipLaunchKernelGGL((cols_conv_kernel<P, TC>), grid, dim3(NT), 0, st, S1, S2, fk, fkn, tw, N,
                     nz);
  return hipGetLastError();
}

template <int P>
hipError_t cols_conv_p(int v, const cpx<float>* S1, cpx<float>* S2, const float* fk,
                       const float* fkn, const cpx<float>* tw, int N, int nz, hipStream_t st) {
  if (v == 0) return cols_conv_pv<P, 0>(S1, S2, fk, fkn, tw, N, nz, st);
  if (v == 2) return cols_conv_pv<P, 2>(S1, S2, fk, fkn, tw, N, nz, st);
  return cols_conv_pv<P, 1>(S1, S2, fk, fkn, tw, N, nz, st);
}

template <int P, int MODE, int NB, bool OBJ, int V = 1>
hipError_t rows_inv_launch(const cpx<float>* S2, const float* xk, const float* xkm1,
                           const float* b, const float* gpv, float* out, double* partials,
                           const double* scal, const cpx<float>* tw, int N, int nz,
                           const PriorParams& pp, int* nblocks, hipStream_t st) {
  constexpr int PAIRS = inv_pairs_v(P, V);
  constexpr int NT = PAIRS * fft::Plan<P, kE>::TPF;
  constexpr int RB = 2 * PAIRS;
  const int nb = nz * ((N + RB - 1) / RB);
  *nblocks = nb;
  hipLaunchKernelGGL((rows_inv_kernel<P, PAIRS, MODE, NB, OBJ>), dim3(nb), dim3(NT), 0, st, S2,
                     xk, xkm1, b, gpv, out, partials, scal, tw, N, nz, pp);
  return hipGetLastError();
}

template <int P>
hipError_t rows_inv_p(int v, int mode, int nbh, bool obj, const cpx<float>* S2, const float* xk,
                      const float* xkm1, const float* b, const float* gpv, float* out,
                      double* partials, const double* scal, const cpx<float>* tw, int N, int nz,
                      const PriorParams& pp, int* nblocks, hipStream_t st) {
#define TOMO_INV(MODE, NB, OBJ)                                                                 \
  return rows_inv_launch<P, MODE, NB, OBJ>(S2, xk, xkm1, b, gpv, out, partials, scal, tw, N, nz, \
                                           pp, nblocks, st)
#define TOMO_INV_V(MODE, V)                                                                      \
  return rows_inv_launch<P, MODE, 0, false, V>(S2, xk, xkm1, b, gpv, out, partials, scal, tw, N, \
                                               nz, pp, nblocks, st)
  if (mode == MODE_POWER) TOMO_INV(MODE_POWER, 8, false);
  if (mode == MODE_FISTA_Y) {  // y and gp - b from the prior kernel
    if (!gpv || !xkm1) return hipErrorInvalidValue;
    if (v == 0) TOMO_INV_V(MODE_FISTA_Y, 0);
    if (v == 2) TOMO_INV_V(MODE_FISTA_Y, 2);
    TOMO_INV_V(MODE_FISTA_Y, 1);
  }
  if (gpv) {  // prior gradient precomputed: the tile variant applies
    if (mode == MODE_GRAD) {
      if (v == 0) TOMO_INV_V(MODE_GRAD, 0);
      if (v == 2) TOMO_INV_V(MODE_GRAD, 2);
      TOMO_INV_V(MODE_GRAD, 1);
    }
    if (v == 0) TOMO_INV_V(MODE_FISTA, 0);
    if (v == 2) TOMO_INV_V(MODE_FISTA, 2);
    TOMO_INV_V(MODE_FISTA, 1);
  }
#undef TOMO_INV_V
  if (mode == MODE_GRAD) {
    if (nbh == 26) { if (obj) TOMO_INV(MODE_GRAD, 26, true); TOMO_INV(MODE_GRAD, 26, false); }
    if (obj) TOMO_INV(MODE_GRAD, 8, true);
    TOMO_INV(MODE_GRAD, 8, false);
  }
  if (nbh == 26) { if (obj) TOMO_INV(MODE_FISTA, 26, true); TOMO_INV(MODE_FISTA, 26, false); }
  if (obj) TOMO_INV(MODE_FISTA, 8, true);
  TOMO_INV(MODE_FISTA, 8, false);
#undef TOMO_INV
}

}  // namespace

int rows_inv_rows_per_block(int P, int v) {
  switch (P) {
    case 32: return 2 * inv_pairs_v(32, v);
    case 64: return 2 * inv_pairs_v(64, v);
    case 128: return 2 * inv_pairs_v(128, v);
    case 256: return 2 * inv_pairs_v(256, v);
    case 512: return 2 * inv_pairs_v(512, v);
    case 1024: return 2 * inv_pairs_v(1024, v);
    case 2048: return 2 * inv_pairs_v(2048, v);
    case 4096: return 2 * inv_pairs_v(4096, v);
  }
  return 2;
}

void tile_shapes(int P, int v_fwd, int v_cc, int v_inv, int* fwd, int* cc, int* inv) {
  *fwd = *cc = *inv = 0;
  switch (P) {
#define SHAPES(PP)                                                                          \
    case PP:                                                                                \
      *fwd = fwd_pairs_v(PP, v_fwd); *cc = col_tc_v(PP, v_cc); *inv = inv_pairs_v(PP, v_inv); \
      break;
    SHAPES(32) SHAPES(64) SHAPES(128) SHAPES(256) SHAPES(512) SHAPES(1024) SHAPES(2048)
    SHAPES(4096)
#undef SHAPES
  }
}

int cols_tile_width(int P) { return col_tc(P); }

bool batch_supports(int P) { return P >= 256 && P <= 2048; }

void batch_tile_counts(int N, int P, int nz, int el, int* nPr, int* nR, int* nC, int* nRp) {
  const int tpf = P / el;
  const int pairs = BT / tpf < 1 ? 1 : BT / tpf;
  const int tc = pairs;
  using SH = PriorShape<16>;
  const int ntx = (N + SH::TX - 1) / SH::TX;
  *nPr = ((ntx + BP_SUB - 1) / BP_SUB) * ((N + SH::TY - 1) / SH::TY) * ((nz + PR_ZC - 1) / PR_ZC);
  *nR = (nz * (N / 2) + pairs - 1) / pairs;
  *nC = nz * ((P / 2) / tc);
  *nRp = nz * ((N + 2 * pairs - 1) / (2 * pairs));
}

int batch_blocks_per_cu(bool fused) {
  int nb = 0;
  const hipError_t e =
      fused ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_iter_kernel<true>, BT, 0)
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_iter_kernel<false>, BT, 0);
  if (e != hipSuccess || nb < 1) nb = 1;
  return nb;
}

hipError_t launch_batch_iteration(bool fused, const BatchProb* probs, const int2* items, int n_items,
                                  int* ctl, int* cnt, int nprob, int ik, int ikm1, int inext,
                                  int grid, hipStream_t st) {
  if (fused)
    hipLaunchKernelGGL(batch_iter_kernel<true>, dim3(grid), dim3(BT), 0, st, probs, items, n_items,
                       ctl, cnt, nprob, ik, ikm1, inext);
  else
    hipLaunchKernelGGL(batch_iter_kernel<false>, dim3(grid), dim3(BT), 0, st, probs, items, n_items,
                       ctl, cnt, nprob, ik, ikm1, inext);
  return hipGetLastError();
}

template <int PH, int P, int EL>
void batch_phase_launch(bool fused, const BatchProb* probs, const int2* items, int cnt, int ik,
                        int ikm1, int inext, hipStream_t st) {
  if (fused)
    hipLaunchKernelGGL((batch_phase_kernel<PH, P, EL, true>), dim3((unsigned)cnt), dim3(BT), 0,
                       st, probs, items, ik, ikm1, inext);
  else
    hipLaunchKernelGGL((batch_phase_kernel<PH, P, EL, false>), dim3((unsigned)cnt), dim3(BT), 0,
                       st, probs, items, ik, ikm1, inext);
}

hipError_t launch_batch_phases(bool fused, const BatchProb* probs, const int2* items,
                               const int4* segs, int nseg, int nprob, int ik, int ikm1, int inext,
                               hipStream_t st) {
  for (int k = 0; k < nseg; ++k) {
    // y: the transform size and the elements per thread (P | EL << 16)
    const int ph = segs[k].x, P = segs[k].y & 0xffff, el = segs[k].y >> 16;
    const int off = segs[k].z, cnt = segs[k].w;
    if (cnt <= 0) continue;
    const int2* it = items + off;
    if (ph == 0) {
      batch_phase_launch<0, 0, 0>(fused, probs, it, cnt, ik, ikm1, inext, st);
      continue;
    }
#define TOMO_PHPE(PHV, PV)                                                                      \
  if (el == 8) batch_phase_launch<PHV, PV, 8>(fused, probs, it, cnt, ik, ikm1, inext, st);      \
  else batch_phase_launch<PHV, PV, 16>(fused, probs, it, cnt, ik, ikm1, inext, st);
#define TOMO_PHP(PHV)                                       \
  switch (P) {                                              \
    case 256: { TOMO_PHPE(PHV, 256) } break;                \
    case 512: { TOMO_PHPE(PHV, 512) } break;                \
    case 1024: { TOMO_PHPE(PHV, 1024) } break;              \
    case 2048: { TOMO_PHPE(PHV, 2048) } break;              \
    default: return hipErrorInvalidValue;                   \
  }
    if (ph == 1) { TOMO_PHP(1) }
    else if (ph == 2) { TOMO_PHP(2) }
    else { TOMO_PHP(3) }
#undef TOMO_PHP
#undef TOMO_PHPE
  }
  hipLaunchKernelGGL(batch_finalize_kernel, dim3(nprob), dim3(BT), 0, st, probs);
  return hipGetLastError();
}

hipError_t launch_fill_int(int* x, idx_t n, int v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_int_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, n, v);
  return hipGetLastError();
}

#define TOMO_PSWITCH(CALL)          \
  switch (P) {                      \
    case 32: return CALL(32);       \
    case 64: return CALL(64);       \
    case 128: return CALL(128);     \
    case 256: return CALL(256);     \
    case 512: return CALL(512);     \
    case 1024: return CALL(1024);   \
    case 2048: return CALL(2048);   \
    case 4096: return CALL(4096);   \
  }                                 \
  return hipErrorInvalidValue;

hipError_t launch_rows_fwd(int P, int v, int mode, const float* xk, const float* xkm1,
                           const double* scal, cpx<float>* S1, const cpx<float>* tw, int N,
                           int nz, hipStream_t st, const double* pprev, int nprev) {
  if (pprev && (mode != MODE_POWER || nprev < 1)) return hipErrorInvalidValue;
#define CALL(PP) rows_fwd_p<PP>(v, mode, xk, xkm1, scal, S1, tw, N, nz, st, pprev, nprev)
  TOMO_PSWITCH(CALL)
#undef CALL
}

hipError_t launch_cols_conv(int P, int v, const cpx<float>* S1, cpx<float>* S2, const float* fk,
                            const float* fkn, const cpx<float>* tw, int N, int nz,
                            hipStream_t st) {
#define CALL(PP) cols_conv_p<PP>(v, S1, S2, fk, fkn, tw, N, nz, st)
  TOMO_PSWITCH(CALL)
#undef CALL
}

hipError_t launch_rows_inv(int P, int v, int mode, int neighbours, bool with_obj,
                           const cpx<float>* S2,
                           const float* xk, const float* xkm1, const float* b, const float* gpv,
                           float* out, double* partials, const double* scal,
                           const cpx<float>* tw, int N, int nz, const PriorParams& pp,
                           int* nblocks_out, hipStream_t st) {
#define CALL(PP)                                                                              \
  rows_inv_p<PP>(v, mode, neighbours, with_obj, S2, xk, xkm1, b, gpv, out, partials, scal, tw, N, \
                 nz, pp, nblocks_out, st)
  TOMO_PSWITCH(CALL)
#undef CALL
}

int prior_blocks(int N, int nz) {
  return ((N + PR_TX - 1) / PR_TX) * ((N + PR_TY - 1) / PR_TY) * ((nz + PR_ZC - 1) / PR_ZC);
}

template <int NB, bool OBJ, bool QUAD>
void prior_launch(dim3 grid, hipStream_t st, const float* xk, const float* xkm1,
                  const double* scal, float* gp, const float* b, float* yout, double* part,
                  int N, int nz, int fista, const PriorParams& pp) {
  if (yout)
    hipLaunchKernelGGL((prior_kernel<NB, OBJ, QUAD, true>), grid, dim3(PR_NT), 0, st, xk, xkm1,
                       scal, gp, b, yout, part, N, nz, fista, pp);
  else
    hipLaunchKernelGGL((prior_kernel<NB, OBJ, QUAD, false>), grid, dim3(PR_NT), 0, st, xk, xkm1,
                       scal, gp, b, yout, part, N, nz, fista, pp);
}

hipError_t launch_prior(int mode, int neighbours, bool with_obj, const float* xk,
                        const float* xkm1, const double* scal, float* gp, const float* b,
                        float* yout, double* partials, int N, int nz, const PriorParams& pp,
                        hipStream_t st) {
  if ((yout != nullptr) != (b != nullptr) || (yout && mode != MODE_FISTA))
    return hipErrorInvalidValue;
  const dim3 grid(prior_blocks(N, nz));
  const int fista = mode == MODE_FISTA ? 1 : 0;
  double* part = with_obj ? partials : nullptr;
  const bool quad = pp.quadratic != 0;
#define PRIOR_CALL(NB, OBJ, QUAD) \
  prior_launch<NB, OBJ, QUAD>(grid, st, xk, xkm1, scal, gp, b, yout, part, N, nz, fista, pp)
  if (neighbours == 26) {
    if (with_obj) { if (quad) PRIOR_CALL(26, true, true); else PRIOR_CALL(26, true, false); }
    else { if (quad) PRIOR_CALL(26, false, true); else PRIOR_CALL(26, false, false); }
  } else {
    if (with_obj) { if (quad) PRIOR_CALL(8, true, true); else PRIOR_CALL(8, true, false); }
    else { if (quad) PRIOR_CALL(8, false, true); else PRIOR_CALL(8, false, false); }
  }
#undef PRIOR_CALL
  return hipGetLastError();
}

hipError_t launch_finalize(int mode, const double* partials, int nblocks,
                           const double* prior_partials, int nprior, double* scal,
                           double* obj_hist, int32_t* restart_hist, double* obj_out,
                           hipStream_t st) {
  if (mode == MODE_POWER)
    hipLaunchKernelGGL((finalize_kernel<MODE_POWER>), dim3(1), dim3(FIN_NT), 0, st, partials,
                       nblocks, prior_partials, nprior, scal, obj_hist, restart_hist, obj_out);
  else if (mode == MODE_GRAD)
    hipLaunchKernelGGL((finalize_kernel<MODE_GRAD>), dim3(1), dim3(FIN_NT), 0, st, partials,
                       nblocks, prior_partials, nprior, scal, obj_hist, restart_hist, obj_out);
  else  // MODE_FISTA, MODE_FISTA_Y
    hipLaunchKernelGGL((finalize_kernel<MODE_FISTA>), dim3(1), dim3(FIN_NT), 0, st, partials,
                       nblocks, prior_partials, nprior, scal, obj_hist, restart_hist, obj_out);
  return hipGetLastError();
}

}  // namespace tomo
