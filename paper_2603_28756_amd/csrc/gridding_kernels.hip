// Back-projection R* g and point-spread-function precompute on gfx950.
//
// Sec. 2, Eq. 4: R* g = NUFFT1( F g ) — a 1D DFT along each projection's radial
// axis, then the adjoint non-uniform transform from the polar samples
// k_il = (l / n_det)(cos theta_i, sin theta_i) to the image grid.
// Sec. 2.1: K = NUFFT1(1) on the polar samples, needed on [-(N-1), N-1]^2, and
// its padded spectrum F K, computed once before iterating.
//
// NUFFT1 is evaluated by Kaiser-Bessel gridding: each sample is spread onto an
// oversampled M x M grid with the separable kernel
// phi(u) = I0(beta sqrt(1 - (2u/W)^2)), |u| < W/2, the grid is inverse-FFT'd,
// cropped, and divided by the kernel's Fourier transform
// phi^(xi) = W sinh(sqrt(beta^2 - (pi W xi)^2)) / sqrt(beta^2 - (pi W xi)^2).
//
// Spreading is a deterministic gather with no atomics: the samples of one angle
// lie on a line sorted by l, so each grid cell finds, per angle, the contiguous
// range of l whose footprints can reach it, and tests exact membership against
// the integer footprint origin stored per sample.  The per-sample 1D weights
// are tabulated once per geometry (float64).
#include "common.hpp"
#include "fft.hpp"
#include "kernels.hpp"

namespace tomo {
namespace {

// Hardware workgroup id -> logical block id such that each of the 8 XCDs (own L2 each) gets
// one contiguous range of logical blocks (a bijection on [0, total)).
TOMO_DEV int xcd_band_index(int hw, int total) {
  constexpr int X = 8;
  const int q = total / X, r = total % X;
  const int xcd = hw % X, local = hw / X;
  return xcd < r ? xcd * (q + 1) + local : r * (q + 1) + (xcd - r) * q + local;
}

// Modified Bessel function I0 from its power series sum_k ((x/2)^k / k!)^2 (float64).
__device__ double bessel_i0(double x) {
  const double q = 0.25 * x * x;
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 200; ++k) {
    term *= q / ((double)k * (double)k);
    sum += term;
    if (term < 1e-17 * sum) break;
  }
  return sum;
}

__device__ double kb_phi(double u, int W, double beta) {
  const double h = 0.5 * W;
  if (fabs(u) >= h) return 0.0;
  const double r = 2.0 * u / W;
  return bessel_i0(beta * sqrt(1.0 - r * r));
}

__device__ double kb_phihat(double xi, int W, double beta) {
  const double a = M_PI * W * xi;
  const double s2 = beta * beta - a * a;
  if (s2 > 1e-12) {
    const double s = sqrt(s2);
    return W * sinh(s) / s;
  }
  if (s2 < -1e-12) {
    const double s = sqrt(-s2);
    return W * sin(s) / s;
  }
  return (double)W;
}

// ------------------------------------------------------------------------------- tables
template <typename T>
__global__ void twiddle_kernel(cpx<T>* tw, int P) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= P) return;
  double s, c;
  sincospi(2.0 * (double)m / (double)P, &s, &c);
  tw[m] = mk((T)c, (T)(-s));
}

__global__ void fill_kernel(float* x, idx_t n, float v) {
  const idx_t i = (idx_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

__global__ void set_scalars_kernel(double* scal, int first, int count, const double* src,
                                   double v) {
  const int i = threadIdx.x;
  if (i < count) scal[first + i] = src ? src[i] : v;
}

// out = {lambda, L, 1 / L} with L = a lambda + c, lambda from the power iteration's scalars;
// the products and sums are rounded one at a time (no contraction), as on the host.
__global__ void lipschitz_kernel(const double* scal, double a, double c, double* out) {
  if (threadIdx.x != 0) return;
  const double lam = scal[SC_LAMBDA];
  const double L = __dadd_rn(__dmul_rn(a, lam), c);
  out[0] = lam;
  out[1] = L;
  out[2] = __ddiv_rn(1.0, L);
}

__global__ void angle_table_kernel(const double* ang, double* tab, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s, c;
  sincos(ang[i], &s, &c);
  tab[2 * i] = c;
  tab[2 * i + 1] = s;
}

// DFT table tab[m] = exp(-2 pi i m / nd) and per-frequency factor
// post[l] = (1/nd)(1/stride) exp(+2 pi i l c / nd) * (ramp ? pi |l| / (nd n_angles) : 1).
__global__ void radial_tables_kernel(cpx<float>* tab, cpx<float>* post, float* rampf, int nd,
                                     double c, int stride, int n_angles, int ramp) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m < nd) {
    double s, co;
    sincospi(2.0 * (double)m / (double)nd, &s, &co);
    tab[m] = mk((float)co, (float)(-s));
  }
  if (m < nd - 1) {
    const int l = m - (nd / 2 - 1);
    double s, co;
    sincospi(2.0 * (double)l * c / (double)nd, &s, &co);
    double f = 1.0 / ((double)nd * (double)stride);
    const double rf = M_PI * fabs((double)l) / ((double)nd * (double)n_angles);
    if (ramp) f *= rf;
    post[m] = mk((float)(co * f), (float)(s * f));
    if (rampf) rampf[m] = (float)rf;
  }
}

// G[row][l] = post[l] * sum_j g[row][j*stride] exp(-2 pi i l j / nd), rows = (slice, angle).
constexpr int RD_ROWS = 16, RD_JC = 256;
__global__ void __launch_bounds__(256)
radial_dft_kernel(const float* __restrict__ sino, int nd_full, int nd, int stride, int rows,
                  int n_angles, int nz, cpx<float>* __restrict__ ghat,
                  const cpx<float>* __restrict__ tab, const cpx<float>* __restrict__ post) {
  __shared__ float gt[RD_ROWS][RD_JC];
  const int t = threadIdx.x;
  const int nl = nd - 1;
  const int lidx = blockIdx.x * 256 + t;
  const int l = lidx - (nd / 2 - 1);
  const int lpos = ((l % nd) + nd) % nd;
  const int row0 = blockIdx.y * RD_ROWS;
  float ar[RD_ROWS], ai[RD_ROWS];
#pragma unroll
  for (int r = 0; r < RD_ROWS; ++r) ar[r] = ai[r] = 0.f;
  for (int j0 = 0; j0 < nd; j0 += RD_JC) {
    for (int e = t; e < RD_ROWS * RD_JC; e += 256) {
      const int rr = e / RD_JC, jj = e - rr * RD_JC;
      const int row = row0 + rr, j = j0 + jj;
      gt[rr][jj] = (row < rows && j < nd) ? sino[(idx_t)row * nd_full + (idx_t)j * stride] : 0.f;
    }
    __syncthreads();
    int idx = (int)(((long long)lpos * (long long)j0) % nd);
    const int jn = min(RD_JC, nd - j0);
    for (int jj = 0; jj < jn; ++jj) {
      const cpx<float> w = tab[idx];
      idx += lpos;
      if (idx >= nd) idx -= nd;
#pragma unroll
      for (int r = 0; r < RD_ROWS; ++r) {
        const float g = gt[r][jj];
        ar[r] += g * w.re;
        ai[r] += g * w.im;
      }
    }
    __syncthreads();
  }
  if (lidx < nl) {
    const cpx<float> f = post[lidx];
#pragma unroll
    for (int r = 0; r < RD_ROWS; ++r) {
      const int row = row0 + r;
      if (row < rows) {
        // slice-innermost layout: sample p = (angle, l), all slices of p contiguous
        const int z = row / n_angles, i = row - z * n_angles;
        ghat[((idx_t)i * nl + lidx) * nz + z] = cmul(mk(ar[r], ai[r]), f);
      }
    }
  }
}

// ------------------------------------------------------ radial DFT by chirp-z (Bluestein)
// The same G[row][l] as radial_dft_kernel in O(L log L) per row: with c_j = exp(-pi i j^2 / n)
// and b_m = exp(+pi i m^2 / n) (n = n_det of the level), 2 kj = k^2 + j^2 - (k - j)^2 gives
//   X[k] = sum_j x_j exp(-2 pi i k j / n) = c_k sum_j (x_j c_j) b_(k-j),
// a linear convolution evaluated as a length-L cyclic one (L >= 2n - 1, a power of two):
// forward FFT of x c (zero beyond n), times B = FFT(b wrapped to [0, L)), inverse FFT.
// Tables, float64-evaluated once per level (exponents reduced modulo 2n exactly):
//   chirp[j] = c_j,  fac[l_idx] = c_k post[l_idx] / L (k = l mod n),  bspec = B.
__global__ void czt_tables_kernel(cpx<float>* __restrict__ chirp, cpx<float>* __restrict__ fac,
                                  int nd, double c, int stride, int L) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  const long long twon = 2LL * nd;
  if (m < nd) {
    double s, co;
    sincospi(-(double)(((long long)m * m) % twon) / (double)nd, &s, &co);
    chirp[m] = mk((float)co, (float)s);
  }
  if (m < nd - 1) {
    const int l = m - (nd / 2 - 1);
    const int k = ((l % nd) + nd) % nd;
    double s1, c1, s2, c2;
    sincospi(-(double)(((long long)k * k) % twon) / (double)nd, &s1, &c1);
    sincospi(2.0 * (double)l * c / (double)nd, &s2, &c2);
    const double f = 1.0 / ((double)nd * (double)stride * (double)L);
    fac[m] = mk((float)((c1 * c2 - s1 * s2) * f), (float)((c1 * s2 + s1 * c2) * f));
  }
}

// bspec[k] = sum over m in [0, n) and L - m for m in [1, n) of b_m exp(-2 pi i m k / L)
// (float64, the phase m k reduced modulo L exactly).
__global__ void czt_bspec_kernel(cpx<float>* __restrict__ bspec, int nd, int L) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= L) return;
  const long long twon = 2LL * nd;
  double ar = 0.0, ai = 0.0;
  for (int m = 0; m < nd; ++m) {
    double sb, cb;
    sincospi((double)(((long long)m * m) % twon) / (double)nd, &sb, &cb);
    for (int side = 0; side < (m == 0 ? 1 : 2); ++side) {
      const long long pos = side == 0 ? m : L - m;
      double sw, cw;
      sincospi(-2.0 * (double)((pos * k) % L) / (double)L, &sw, &cw);
      ar += cb * cw - sb * sw;
      ai += cb * sw + sb * cw;
    }
  }
  bspec[k] = mk((float)ar, (float)ai);
}

// Block: R rows of one angle and consecutive slices (so that the slice-innermost output of a
// frequency is written R values at a time); one row = TPF = L/16 threads.  Rows are taken
// angle-major (row = angle * nz + slice) in XCD-contiguous block order.
template <int L>
constexpr int czt_rows() { return (L / 16) >= 256 ? 1 : 256 / (L / 16); }

template <int L>
__global__ void __launch_bounds__(czt_rows<L>() * (L / 16))
radial_czt_kernel(const float* __restrict__ sino, int nd_full, int nd, int stride, int n_angles,
                  int nz, cpx<float>* __restrict__ ghat, const cpx<float>* __restrict__ chirp,
                  const cpx<float>* __restrict__ bspec, const cpx<float>* __restrict__ fac,
                  const cpx<float>* __restrict__ tw) {
  using PL = fft::Plan<L, 16>;
  using IPL = fft::RevPlan<PL>;
  constexpr int TPF = PL::TPF, E = PL::E, R0 = PL::radix(0), RL = PL::radix(PL::NS - 1);
  constexpr int R = czt_rows<L>(), REG = fft::row_region<L>();
  static_assert(E == R0, "one first-stage butterfly per thread");
  __shared__ cpx<float> lds[R * REG];
  const int t = threadIdx.x, rr = t / TPF, q = t - rr * TPF;
  const int rows = nz * n_angles;
  const int nblk_ = (rows + R - 1) / R;
  const int blk = xcd_band_index(blockIdx.x, nblk_);
  const int row = blk * R + rr;  // angle-major
  const bool active = row < rows;
  const int ang = active ? row / nz : 0, z = active ? row - ang * nz : 0;
  const float* g = sino + ((idx_t)z * n_angles + ang) * nd_full;
  cpx<float> v[E];
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int j = q + r * TPF;  // positions >= L/2 >= n are the zero padding
    cpx<float> a = mk(0.f, 0.f);
    if (2 * r < E && active && j < nd) a = scale(chirp[j], g[(idx_t)j * stride]);
    v[r] = a;
  }
  fft::LdsRow<float> Ls{lds + rr * REG};
  fft::run_stages<PL, 0, -1, true>(v, q, tw, Ls);
#pragma unroll
  for (int m = 0; m < E / RL; ++m)
#pragma unroll
    for (int r = 0; r < RL; ++r) v[m * RL + r] = cmul(v[m * RL + r], bspec[fft::reg_pos<L, TPF, RL>(q, m, r)]);
  fft::run_stages<IPL, 0, +1>(v, q, tw, Ls);
  if (!active) return;
  const int nl = nd - 1, lmax = nd / 2 - 1;
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int k = q + r * TPF;  // y_k in the first-stage layout
    int lidx = -1;
    if (k <= lmax) lidx = k + lmax;
    else if (k < nd && k >= nd - lmax) lidx = k - nd + lmax;
    if (lidx >= 0 && k < nd)
      ghat[((idx_t)ang * nl + lidx) * nz + z] = cmul(v[r], fac[lidx]);
  }
}

// Per-sample footprint origin and 1D kernel weights on an M-grid (grid units).
template <typename T>
__global__ void point_table_kernel(const double* __restrict__ atab, int2* __restrict__ g0,
                                   T* __restrict__ wx, T* __restrict__ wy, int nd, int n_angles,
                                   int M, int W, double beta) {
  const int nl = nd - 1;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_angles * nl) return;
  const int i = p / nl, lidx = p - i * nl;
  const int l = lidx - (nd / 2 - 1);
  const double d = (double)M / (double)nd;
  const double kx = (double)l * d * atab[2 * i];
  const double ky = (double)l * d * atab[2 * i + 1];
  const int ox = (int)floor(kx - 0.5 * W) + 1;
  const int oy = (int)floor(ky - 0.5 * W) + 1;
  g0[p] = make_int2(ox, oy);
  for (int a = 0; a < W; ++a) {
    wx[(idx_t)p * W + a] = (T)kb_phi((double)(ox + a) - kx, W, beta);
    wy[(idx_t)p * W + a] = (T)kb_phi((double)(oy + a) - ky, W, beta);
  }
}

// Every sample p whose footprint covers grid cell (ix, iy), in a fixed order (wrap shift,
// angle, l): f(p, wx[p][ox] * wy[p][oy]).
template <typename T, class F>
TOMO_DEV void visit_cell(int ix, int iy, const double* __restrict__ atab,
                         const int2* __restrict__ g0, const T* __restrict__ wx,
                         const T* __restrict__ wy, int M, int nd, int n_angles, int W, F&& f) {
  const int half = M / 2;
  const int gx = ix < half ? ix : ix - M;
  const int gy = iy < half ? iy : iy - M;
  const int nl = nd - 1, lmax = nd / 2 - 1;
  const float step = (float)M / (float)nd;
  const float hw = 0.5f * (float)W + 1.5f;
  const float reach = (float)half + hw;
  for (int sx = -1; sx <= 1; ++sx) {
    const int gxp = gx + sx * M;
    if (fabsf((float)gxp) > reach) continue;
    for (int sy = -1; sy <= 1; ++sy) {
      const int gyp = gy + sy * M;
      if (fabsf((float)gyp) > reach) continue;
      for (int i = 0; i < n_angles; ++i) {
        const float cx = (float)atab[2 * i] * step, cy = (float)atab[2 * i + 1] * step;
        float lo = (float)(-lmax), hi = (float)lmax;
        if (fabsf(cx) > 1e-6f) {
          const float a = ((float)gxp - hw) / cx, b = ((float)gxp + hw) / cx;
          lo = fmaxf(lo, fminf(a, b));
          hi = fminf(hi, fmaxf(a, b));
        } else if (fabsf((float)gxp) > hw) {
          continue;
        }
        if (fabsf(cy) > 1e-6f) {
          const float a = ((float)gyp - hw) / cy, b = ((float)gyp + hw) / cy;
          lo = fmaxf(lo, fminf(a, b));
          hi = fminf(hi, fmaxf(a, b));
        } else if (fabsf((float)gyp) > hw) {
          continue;
        }
        const int l0 = (int)ceilf(lo), l1 = (int)floorf(hi);
        for (int l = l0; l <= l1; ++l) {
          const int p = i * nl + (l + lmax);
          const int2 o = g0[p];
          const int ox = gxp - o.x, oy = gyp - o.y;
          if ((unsigned)ox < (unsigned)W && (unsigned)oy < (unsigned)W)
            f(p, wx[(idx_t)p * W + ox] * wy[(idx_t)p * W + oy]);
        }
      }
    }
  }
}

// Cell-sorted contribution lists (CSR over grid cells): count, then fill at scanned offsets.
template <typename T>
__global__ void __launch_bounds__(256)
csr_count_kernel(int* __restrict__ cnt, const double* __restrict__ atab,
                 const int2* __restrict__ g0, const T* __restrict__ wx,
                 const T* __restrict__ wy, int M, int nd, int n_angles, int W) {
  const idx_t cell = (idx_t)blockIdx.x * 256 + threadIdx.x;
  if (cell >= (idx_t)M * M) return;
  const int iy = (int)(cell / M), ix = (int)(cell - (idx_t)iy * M);
  int c = 0;
  visit_cell<T>(ix, iy, atab, g0, wx, wy, M, nd, n_angles, W, [&](int, T) { ++c; });
  cnt[cell] = c;
}

// Weights only (float64), in the same visit order: the lists of the point-spread grid, whose
// samples all carry the same value.
__global__ void __launch_bounds__(256)
csr_fill_w64_kernel(const int* __restrict__ row_ptr, double* __restrict__ wts,
                    const double* __restrict__ atab, const int2* __restrict__ g0,
                    const double* __restrict__ wx, const double* __restrict__ wy, int M, int nd,
                    int n_angles, int W) {
  const idx_t cell = (idx_t)blockIdx.x * 256 + threadIdx.x;
  if (cell >= (idx_t)M * M) return;
  const int iy = (int)(cell / M), ix = (int)(cell - (idx_t)iy * M);
  int k = row_ptr[cell];
  visit_cell<double>(ix, iy, atab, g0, wx, wy, M, nd, n_angles, W, [&](int, double w) { wts[k++] = w; });
}

// Point-spread grid (Sec. 2.1, Eq. 8: the adjoint NUFFT of the all-ones function, every sample
// weighted 1 / n_det): grid[cell] = sum over the cell's list, in list order, of w c (the
// cell's samples angle by angle, then along each ray).
__global__ void __launch_bounds__(256)
psf_grid_kernel(const int* __restrict__ row_ptr, const double* __restrict__ wts,
                cpx<double>* __restrict__ grid, idx_t cells, double c) {
  const idx_t cell = (idx_t)blockIdx.x * 256 + threadIdx.x;
  if (cell >= cells) return;
  double a = 0.0;
  for (int k = row_ptr[cell], k1 = row_ptr[cell + 1]; k < k1; ++k) a += wts[k] * c;
  grid[cell] = mk(a, 0.0);
}

__global__ void __launch_bounds__(256)
csr_fill_kernel(const int* __restrict__ row_ptr, int* __restrict__ idx, float* __restrict__ wts,
                const double* __restrict__ atab, const int2* __restrict__ g0,
                const float* __restrict__ wx, const float* __restrict__ wy, int M, int nd,
                int n_angles, int W) {
  const idx_t cell = (idx_t)blockIdx.x * 256 + threadIdx.x;
  if (cell >= (idx_t)M * M) return;
  const int iy = (int)(cell / M), ix = (int)(cell - (idx_t)iy * M);
  int k = row_ptr[cell];
  visit_cell<float>(ix, iy, atab, g0, wx, wy, M, nd, n_angles, W, [&](int p, float w) {
    idx[k] = p;
    wts[k] = w;
    ++k;
  });
}

// Ramp-filtered list weights (Sec. 2.2, the FBP start): out[k] = wts[k] rampf[l] for the
// radial index l = idx[k] mod (n_det - 1) of the entry's sample.
__global__ void csr_ramp_kernel(const int* __restrict__ idx, const float* __restrict__ wts,
                                const float* __restrict__ rampf, idx_t nnz, int nl,
                                float* __restrict__ out) {
  const idx_t k = (idx_t)blockIdx.x * 256 + threadIdx.x;
  if (k < nnz) out[k] = wts[k] * rampf[idx[k] % nl];
}

// Exclusive scan of n ints (block-local scans of 4096 elements, then their sums).
constexpr int SCAN_PER_BLOCK = 4096;
__global__ void __launch_bounds__(1024)
scan_blocks_kernel(const int* __restrict__ in, int* __restrict__ out, int* __restrict__ sums,
                   idx_t n) {
  __shared__ int sh[1024];
  const idx_t base = (idx_t)blockIdx.x * SCAN_PER_BLOCK + (idx_t)threadIdx.x * 4;
  int v[4], tsum = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    v[j] = base + j < n ? in[base + j] : 0;
    tsum += v[j];
  }
  sh[threadIdx.x] = tsum;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int add = threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
    __syncthreads();
    sh[threadIdx.x] += add;
    __syncthreads();
  }
  int run = sh[threadIdx.x] - tsum;  // exclusive prefix of this thread
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (base + j < n) out[base + j] = run;
    run += v[j];
  }
  if (threadIdx.x == 1023) sums[blockIdx.x] = sh[1023];
}

__global__ void __launch_bounds__(1024)
scan_sums_kernel(int* __restrict__ sums, int nb, int* __restrict__ total_out) {
  __shared__ int sh[1024];
  const int per = (nb + 1023) / 1024;
  const int b0 = threadIdx.x * per;
  int tsum = 0;
  for (int j = 0; j < per; ++j)
    if (b0 + j < nb) tsum += sums[b0 + j];
  sh[threadIdx.x] = tsum;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int add = threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
    __syncthreads();
    sh[threadIdx.x] += add;
    __syncthreads();
  }
  int run = sh[threadIdx.x] - tsum;
  for (int j = 0; j < per; ++j)
    if (b0 + j < nb) {
      const int v = sums[b0 + j];
      sums[b0 + j] = run;
      run += v;
    }
  if (threadIdx.x == 1023) *total_out = sh[1023];
}

__global__ void scan_add_kernel(int* __restrict__ out, const int* __restrict__ sums, idx_t n) {
  const idx_t i = (idx_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) out[i] += sums[i / SCAN_PER_BLOCK];
}

// H[z][cell] = sum over the cell's list of w * c[p][z0 + z], z < nzb (w: the list's plain or
// ramp-weighted weights); samples hold all slices contiguously.
template <int ZB>
__global__ void __launch_bounds__(256)
gather_kernel(const cpx<float>* __restrict__ vals, cpx<float>* __restrict__ grid,
              const int* __restrict__ row_ptr, const int* __restrict__ idx,
              const float* __restrict__ wts, int M, int nz, int z0, int nzb) {
  const idx_t cell = (idx_t)blockIdx.x * 256 + threadIdx.x;
  if (cell >= (idx_t)M * M) return;
  float ar[ZB], ai[ZB];
#pragma unroll
  for (int z = 0; z < ZB; ++z) ar[z] = ai[z] = 0.f;
  const int k0 = row_ptr[cell], k1 = row_ptr[cell + 1];
  for (int k = k0; k < k1; ++k) {
    const int p = idx[k];
    const float w = wts[k];
    const cpx<float>* c = vals + (idx_t)p * nz + z0;
#pragma unroll
    for (int z = 0; z < ZB; ++z) {
      if (z < nzb) {
        const cpx<float> v = c[z];
        ar[z] += w * v.re;
        ai[z] += w * v.im;
      }
    }
  }
#pragma unroll
  for (int z = 0; z < ZB; ++z)
    if (z < nzb) grid[(idx_t)z * M * M + cell] = mk(ar[z], ai[z]);
}

// Same sums with lanes over slices: a wave walks the lists of 64/ZL cells at a time, each
// group of ZL lanes reading ZL x SPL consecutive slices of a sample (one contiguous line; SPL
// slices per lane in 8- or 16-byte loads); results are transposed through LDS so that each
// slice's row of 64 cells is written contiguously.  The walk is bound by the latency of its
// dependent loads (list bounds, then entries, then values), so more cells per wave step (two
// slices per lane) means fewer rounds for the same sums.  Every sum runs in list order.
// DUAL: one walk gives the sums with the list weights wts (grid) and with the second weights
// wts2 (grid2): R* g and the ramp-filtered back-projection.
template <int ZL, int SPL, bool DUAL>
__global__ void __launch_bounds__(256)
gather_z_kernel(const cpx<float>* __restrict__ vals, cpx<float>* __restrict__ grid,
                cpx<float>* __restrict__ grid2, const int* __restrict__ row_ptr,
                const int* __restrict__ idx, const float* __restrict__ wts,
                const float* __restrict__ wts2, int M, int nz, int z0, int nzb) {
  static_assert(SPL == 1 || SPL == 2 || SPL == 4, "slices per lane");
  constexpr int G = 64 / ZL;   // cells per wave step
  constexpr int CB = 64;       // cells per block
  constexpr int ZS = ZL * SPL; // slices per block row
  constexpr int NO = DUAL ? 2 : 1;
  __shared__ cpx<float> tile[NO][ZS][CB + 1];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane / ZL, zl = lane - g * ZL;
  const idx_t cells = (idx_t)M * M;
  const idx_t cell0 = (idx_t)blockIdx.x * CB;
  const int zi = blockIdx.y * ZS + zl * SPL;  // first slice of this lane
  for (int cs = wave * G + g; cs < CB; cs += 4 * G) {
    const idx_t cell = cell0 + cs;
    float ar[NO][SPL], ai[NO][SPL];
#pragma unroll
    for (int o = 0; o < NO; ++o)
#pragma unroll
      for (int s = 0; s < SPL; ++s) ar[o][s] = ai[o][s] = 0.f;
    if (cell < cells && zi < nzb) {
      const int k0 = row_ptr[cell], k1 = row_ptr[cell + 1];
      // eight entries per step: their indices and weights first, then eight independent
      // value loads in flight (cells near the origin have lists of ~n_angles * W entries)
      constexpr int U = 8;
      for (int k = k0; k < k1; k += U) {
        int pp[U];
        float w[NO][U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const bool in = k + u < k1;
          pp[u] = in ? idx[k + u] : 0;
          w[0][u] = in ? wts[k + u] : 0.f;
          if constexpr (DUAL) w[1][u] = in ? wts2[k + u] : 0.f;
        }
        constexpr int H = SPL == 1 ? 1 : SPL / 2;
        float4 v[U][H];
        cpx<float> v1[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          if constexpr (SPL == 1) {
            v1[u] = vals[(idx_t)pp[u] * nz + z0 + zi];
          } else {
            // slices zi .. zi + SPL - 1 of a sample: 16-byte loads (nz, z0 and zi are even)
#pragma unroll
            for (int h = 0; h < H; ++h)
              v[u][h] = *reinterpret_cast<const float4*>(vals + (idx_t)pp[u] * nz + z0 + zi + 2 * h);
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          if (k + u < k1) {
#pragma unroll
            for (int o = 0; o < NO; ++o) {
              const float wo = w[o][u];
              if constexpr (SPL == 1) {
                ar[o][0] += wo * v1[u].re;
                ai[o][0] += wo * v1[u].im;
              } else {
#pragma unroll
                for (int h = 0; h < H; ++h) {
                  ar[o][2 * h] += wo * v[u][h].x;
                  ai[o][2 * h] += wo * v[u][h].y;
                  ar[o][2 * h + 1] += wo * v[u][h].z;
                  ai[o][2 * h + 1] += wo * v[u][h].w;
                }
              }
            }
          }
        }
      }
    }
#pragma unroll
    for (int o = 0; o < NO; ++o)
#pragma unroll
      for (int s = 0; s < SPL; ++s) tile[o][zl * SPL + s][cs] = mk(ar[o][s], ai[o][s]);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < ZS * CB; e += 256) {
    const int z = e / CB, c = e - z * CB;
    const idx_t cell = cell0 + c;
    const int zo = blockIdx.y * ZS + z;
    if (cell < cells && zo < nzb) {
      grid[(idx_t)zo * cells + cell] = tile[0][z][c];
      if constexpr (DUAL) grid2[(idx_t)zo * cells + cell] = tile[NO - 1][z][c];
    }
  }
}

// ------------------------------------------------------------------- generic 2D C2C FFT
template <typename T>
constexpr int fftE() { return sizeof(T) == 8 ? 8 : 16; }

// keep > 0: only the outputs at positions [0, keep) and [P - keep, P) are stored (the columns
// that a following cropped column pass reads); keep = 0 stores every position.
template <typename T, int P, int ROWS, int DIR>
__global__ void __launch_bounds__(ROWS * (P / fftE<T>()))
fft_rows_kernel(cpx<T>* __restrict__ data, idx_t n_rows, const cpx<T>* __restrict__ tw,
                int keep = 0) {
  using PL = fft::Plan<P, fftE<T>()>;
  constexpr int TPF = PL::TPF, E = PL::E, R0 = PL::radix(0), RL = PL::radix(PL::NS - 1);
  constexpr int REG = fft::row_region<P>();
  __shared__ cpx<T> lds[ROWS * REG];
  const int t = threadIdx.x, rr = t / TPF, q = t - rr * TPF;
  const idx_t row = (idx_t)blockIdx.x * ROWS + rr;
  const bool active = row < n_rows;
  cpx<T>* d = data + (active ? row : 0) * P;
  cpx<T> v[E];
#pragma unroll
  for (int m = 0; m < E / R0; ++m)
#pragma unroll
    for (int r = 0; r < R0; ++r)
      v[m * R0 + r] = active ? d[fft::reg_pos<P, TPF, R0>(q, m, r)] : mk((T)0, (T)0);
  fft::LdsRow<T> L{lds + rr * REG};
  fft::run_stages<PL, 0, DIR>(v, q, tw, L);
  if (active)
#pragma unroll
    for (int m = 0; m < E / RL; ++m)
#pragma unroll
      for (int r = 0; r < RL; ++r) {
        const int pos = fft::reg_pos<P, TPF, RL>(q, m, r);
        if (keep == 0 || pos < keep || pos >= P - keep) d[pos] = v[m * RL + r];
      }
}

template <typename T, int P, int TC, int DIR>
__global__ void __launch_bounds__(TC * (P / fftE<T>()))
fft_cols_kernel(cpx<T>* __restrict__ data, const cpx<T>* __restrict__ tw) {
  using PL = fft::Plan<P, fftE<T>()>;
  constexpr int TPF = PL::TPF, E = PL::E, R0 = PL::radix(0), RL = PL::radix(PL::NS - 1);
  __shared__ cpx<T> lds[P * TC];
  const int t = threadIdx.x, c = t % TC, q = t / TC;
  cpx<T>* d = data + (idx_t)blockIdx.y * P * P + (idx_t)blockIdx.x * TC + c;
  cpx<T> v[E];
#pragma unroll
  for (int m = 0; m < E / R0; ++m)
#pragma unroll
    for (int r = 0; r < R0; ++r) v[m * R0 + r] = d[(idx_t)fft::reg_pos<P, TPF, R0>(q, m, r) * P];
  fft::LdsCols<T, TC> L{lds, c};
  fft::run_stages<PL, 0, DIR>(v, q, tw, L);
#pragma unroll
  for (int m = 0; m < E / RL; ++m)
#pragma unroll
    for (int r = 0; r < RL; ++r) d[(idx_t)fft::reg_pos<P, TPF, RL>(q, m, r) * P] = v[m * RL + r];
}

// Inverse-direction column transforms of the N columns that survive the crop of a
// back-projection grid, with the crop and deapodisation as the epilogue:
//   out[z][my][mx] = Re H[z][(my - N/2) mod P][(mx - N/2) mod P] inv[my] inv[mx],
// H the 2D transform of the rows already transformed by fft_rows_kernel (keep = N/2).
// Block (bx, z) takes kept columns mx = bx TC .. bx TC + TC - 1 (those >= N idle).
template <int P, int TC>
__global__ void __launch_bounds__(TC * (P / fftE<float>()))
fft_cols_crop_kernel(const cpx<float>* __restrict__ data, const cpx<float>* __restrict__ tw,
                     float* __restrict__ out, const float* __restrict__ inv, int N) {
  using PL = fft::Plan<P, fftE<float>()>;
  constexpr int TPF = PL::TPF, E = PL::E, R0 = PL::radix(0), RL = PL::radix(PL::NS - 1);
  __shared__ cpx<float> lds[P * TC];
  const int t = threadIdx.x, c = t % TC, q = t / TC;
  const int mx = blockIdx.x * TC + c;
  const bool active = mx < N;
  const int gx = (mx - N / 2 + P) % P;
  const cpx<float>* d = data + (idx_t)blockIdx.y * P * P + (active ? gx : 0);
  cpx<float> v[E];
#pragma unroll
  for (int m = 0; m < E / R0; ++m)
#pragma unroll
    for (int r = 0; r < R0; ++r)
      v[m * R0 + r] = active ? d[(idx_t)fft::reg_pos<P, TPF, R0>(q, m, r) * P] : mk(0.f, 0.f);
  fft::LdsCols<float, TC> L{lds, c};
  fft::run_stages<PL, 0, +1>(v, q, tw, L);
  if (!active) return;
  float* o = out + (idx_t)blockIdx.y * N * N + mx;
  const float sx = inv[mx];
#pragma unroll
  for (int m = 0; m < E / RL; ++m)
#pragma unroll
    for (int r = 0; r < RL; ++r) {
      const int my = (fft::reg_pos<P, TPF, RL>(q, m, r) + N / 2) % P;
      if (my < N) o[(idx_t)my * N] = v[m * RL + r].re * inv[my] * sx;
    }
}

template <typename T>
constexpr int rows_per_block(int P) {
  const int tpf = P / fftE<T>();
  int r = 256 / tpf;
  return r < 1 ? 1 : r;
}
template <typename T>
constexpr int cols_per_block(int P) {
  int tc = (65536 / (int)sizeof(cpx<T>)) / P;
  if (tc > 16) tc = 16;
  return tc < 1 ? 1 : tc;
}

template <typename T, int P>
hipError_t fft2d_p(cpx<T>* data, int batch, int dir, const cpx<T>* tw, hipStream_t st) {
  constexpr int ROWS = rows_per_block<T>(P);
  constexpr int TC = cols_per_block<T>(P);
  constexpr int TPF = fft::Plan<P, fftE<T>()>::TPF;
  const idx_t n_rows = (idx_t)batch * P;
  const dim3 gr((unsigned)((n_rows + ROWS - 1) / ROWS));
  const dim3 gc(P / TC, batch);
  if (dir < 0) {
    hipLaunchKernelGGL((fft_rows_kernel<T, P, ROWS, -1>), gr, dim3(ROWS * TPF), 0, st, data,
                       n_rows, tw);
    hipLaunchKernelGGL((fft_cols_kernel<T, P, TC, -1>), gc, dim3(TC * TPF), 0, st, data, tw);
  } else {
    hipLaunchKernelGGL((fft_rows_kernel<T, P, ROWS, +1>), gr, dim3(ROWS * TPF), 0, st, data,
                       n_rows, tw);
    hipLaunchKernelGGL((fft_cols_kernel<T, P, TC, +1>), gc, dim3(TC * TPF), 0, st, data, tw);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------- crop / deapodise
// out[z][my][mx] = Re H[z][(my - N/2) mod M][(mx - N/2) mod M] / (phi^(x/M) phi^(y/M))
// inv[m] = 1 / phi^((m - N/2) / M), m = 0..N-1 (float64 evaluation, float32 result).
__global__ void deapod_table_kernel(float* __restrict__ inv, int N, int M, int W, double beta) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m < N) inv[m] = (float)(1.0 / kb_phihat((double)(m - N / 2) / M, W, beta));
}

__global__ void crop_deapod_kernel(const cpx<float>* __restrict__ grid, float* __restrict__ out,
                                   const float* __restrict__ inv, int N, int M, int nzb) {
  const idx_t i = (idx_t)blockIdx.x * blockDim.x + threadIdx.x;
  const idx_t tot = (idx_t)nzb * N * N;
  if (i >= tot) return;
  const int z = (int)(i / ((idx_t)N * N));
  const int rem = (int)(i - (idx_t)z * N * N);
  const int my = rem / N, mx = rem - my * N;
  const int gx = (mx - N / 2 + M) % M, gy = (my - N / 2 + M) % M;
  out[i] = grid[(idx_t)z * M * M + (idx_t)gy * M + gx].re * inv[my] * inv[mx];
}

// Embedded PSF: emb[v][u] = K(dy, dx) for |dx|, |dy| <= N-1 (dy = v or v - P, dx likewise),
// zero elsewhere; K(d) = Re Kgrid[d mod M] / (phi^(dx/M) phi^(dy/M)).
__global__ void psf_embed_kernel(const cpx<double>* __restrict__ grid,
                                 cpx<double>* __restrict__ emb, int N, int P, int M, int W,
                                 double beta) {
  const idx_t i = (idx_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (idx_t)P * P) return;
  const int v = (int)(i / P), u = (int)(i - (idx_t)v * P);
  const int dy = v < P / 2 ? v : v - P;
  const int dx = u < P / 2 ? u : u - P;
  double k = 0.0;
  if (abs(dx) <= N - 1 && abs(dy) <= N - 1) {
    const int gx = (dx + M) % M, gy = (dy + M) % M;
    const double d = kb_phihat((double)dx / M, W, beta) * kb_phihat((double)dy / M, W, beta);
    k = grid[(idx_t)gy * M + gx].re / d;
  }
  emb[i] = mk(k, 0.0);
}

// fk[fk_index(v, u)] = Re S[v][u] / P^2 for u < P/2; fkn[v] = Re S[v][P/2] / P^2.
__global__ void fk_store_kernel(const cpx<double>* __restrict__ spec, float* __restrict__ fk,
                                float* __restrict__ fkn, int P) {
  const idx_t i = (idx_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int H = P / 2;
  if (i >= (idx_t)P * (H + 1)) return;
  const int v = (int)(i / (H + 1)), u = (int)(i - (idx_t)v * (H + 1));
  const double inv = 1.0 / ((double)P * (double)P);
  const double val = spec[(idx_t)v * P + u].re * inv;
  if (u < H) fk[fk_index(v, u, P)] = (float)val;
  else fkn[v] = (float)val;
}

__global__ void fk_export_kernel(const float* __restrict__ fk, const float* __restrict__ fkn,
                                 float* __restrict__ out, int P) {
  const idx_t i = (idx_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int H = P / 2;
  if (i >= (idx_t)P * (H + 1)) return;
  const int v = (int)(i / (H + 1)), u = (int)(i - (idx_t)v * (H + 1));
  const float s = (float)P * (float)P;
  out[i] = (u < H ? fk[fk_index(v, u, P)] : fkn[v]) * s;
}

// sum of (scale * g[row][j*stride])^2 over rows x n_out samples; two-stage deterministic.
__global__ void __launch_bounds__(256)
sumsq_kernel(const float* __restrict__ g, idx_t rows, int n_out, int stride, int n_full,
             double scale2, double* __restrict__ partials) {
  __shared__ double sh[256];
  const idx_t tot = rows * n_out;
  double a = 0.0;
  for (idx_t i = (idx_t)blockIdx.x * 256 + threadIdx.x; i < tot; i += (idx_t)gridDim.x * 256) {
    const idx_t r = i / n_out;
    const int j = (int)(i - r * n_out);
    const double v = g[r * n_full + (idx_t)j * stride];
    a += v * v;
  }
  sh[threadIdx.x] = a;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = sh[0] * scale2;
}

__global__ void __launch_bounds__(256) sum_partials_kernel(const double* __restrict__ partials,
                                                           int n, double* __restrict__ out) {
  __shared__ double sh[256];
  double a = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) a += partials[i];
  sh[threadIdx.x] = a;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

// ----------------------------------------------------------------- Lanczos-3 prolongation
// Normalised taps sinc(x) sinc(x/3) / sum, at offsets m - i/2 for odd fine index i.
__device__ float lanczos3(double x) {
  if (x == 0.0) return 1.0f;
  if (fabs(x) >= 3.0) return 0.0f;
  const double a = sinpi(x) / (M_PI * x);
  const double b = sinpi(x / 3.0) / (M_PI * x / 3.0);
  return (float)(a * b);
}

__global__ void lanczos_prolong_kernel(const float* __restrict__ in, float* __restrict__ out,
                                       int n, int nz) {
  const int n2 = 2 * n;
  const idx_t i = (idx_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (idx_t)nz * n2 * n2) return;
  const int z = (int)(i / ((idx_t)n2 * n2));
  const int rem = (int)(i - (idx_t)z * n2 * n2);
  const int fy = rem / n2, fx = rem - fy * n2;
  // 1D taps: even fine index copies the coarse sample; odd uses offsets m0-2..m0+3
  float wyv[6], wxv[6];
  int y0, x0, ny, nxx;
  double norm = 0.0;
  for (int a = -2; a <= 3; ++a) norm += (double)lanczos3(0.5 - (double)a);
  if (fy & 1) {
    y0 = fy / 2 - 2; ny = 6;
    for (int a = 0; a < 6; ++a) wyv[a] = (float)((double)lanczos3(0.5 - (double)(a - 2)) / norm);
  } else {
    y0 = fy / 2; ny = 1; wyv[0] = 1.0f;
  }
  if (fx & 1) {
    x0 = fx / 2 - 2; nxx = 6;
    for (int a = 0; a < 6; ++a) wxv[a] = (float)((double)lanczos3(0.5 - (double)(a - 2)) / norm);
  } else {
    x0 = fx / 2; nxx = 1; wxv[0] = 1.0f;
  }
  const float* src = in + (idx_t)z * n * n;
  float acc = 0.f;
  for (int a = 0; a < ny; ++a) {
    const int yy = y0 + a;
    if (yy < 0 || yy >= n) continue;
    float rowacc = 0.f;
    for (int b = 0; b < nxx; ++b) {
      const int xx = x0 + b;
      if (xx < 0 || xx >= n) continue;
      rowacc += wxv[b] * src[(idx_t)yy * n + xx];
    }
    acc += wyv[a] * rowacc;
  }
  out[i] = acc;
}

inline unsigned nblk(idx_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

// =================================================================================== API
hipError_t launch_twiddles_f32(cpx<float>* tw, int P, hipStream_t st) {
  hipLaunchKernelGGL((twiddle_kernel<float>), dim3(nblk(P, 256)), dim3(256), 0, st, tw, P);
  return hipGetLastError();
}
hipError_t launch_twiddles_f64(cpx<double>* tw, int P, hipStream_t st) {
  hipLaunchKernelGGL((twiddle_kernel<double>), dim3(nblk(P, 256)), dim3(256), 0, st, tw, P);
  return hipGetLastError();
}
hipError_t launch_fill(float* x, idx_t n, float v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_kernel, dim3(nblk(n, 256)), dim3(256), 0, st, x, n, v);
  return hipGetLastError();
}
hipError_t launch_set_scalars(double* scal, int first, int count, const double* src, double v,
                              hipStream_t st) {
  hipLaunchKernelGGL(set_scalars_kernel, dim3(1), dim3(64), 0, st, scal, first, count, src, v);
  return hipGetLastError();
}
hipError_t launch_lipschitz(const double* scal, double a, double c, double* out, hipStream_t st) {
  hipLaunchKernelGGL(lipschitz_kernel, dim3(1), dim3(64), 0, st, scal, a, c, out);
  return hipGetLastError();
}
hipError_t launch_angle_table(const double* angles_dev, double* tab, int n, hipStream_t st) {
  hipLaunchKernelGGL(angle_table_kernel, dim3(nblk(n, 256)), dim3(256), 0, st, angles_dev, tab, n);
  return hipGetLastError();
}
hipError_t launch_radial_tables(cpx<float>* dft_tab, cpx<float>* post, float* rampf,
                                const GridGeom& gg, int ramp, hipStream_t st) {
  hipLaunchKernelGGL(radial_tables_kernel, dim3(nblk(gg.n_det, 256)), dim3(256), 0, st, dft_tab,
                     post, rampf, gg.n_det, gg.c, gg.stride, gg.n_angles, ramp);
  return hipGetLastError();
}
hipError_t launch_radial_dft(const float* sino, int n_det_full, cpx<float>* ghat,
                             const cpx<float>* dft_tab, const cpx<float>* post,
                             const GridGeom& gg, int nz, hipStream_t st) {
  const int rows = nz * gg.n_angles;
  const dim3 grid(nblk(gg.n_det - 1, 256), nblk(rows, RD_ROWS));
  hipLaunchKernelGGL(radial_dft_kernel, grid, dim3(256), 0, st, sino, n_det_full, gg.n_det,
                     gg.stride, rows, gg.n_angles, nz, ghat, dft_tab, post);
  return hipGetLastError();
}
int czt_length(int nd) {
  int L = 256;
  while (L < 2 * nd - 1) L <<= 1;
  return L;
}
hipError_t launch_czt_tables(cpx<float>* chirp, cpx<float>* fac, cpx<float>* bspec,
                             const GridGeom& gg, hipStream_t st) {
  const int L = czt_length(gg.n_det);
  hipLaunchKernelGGL(czt_tables_kernel, dim3(nblk(gg.n_det, 256)), dim3(256), 0, st, chirp, fac,
                     gg.n_det, gg.c, gg.stride, L);
  hipLaunchKernelGGL(czt_bspec_kernel, dim3(nblk(L, 128)), dim3(128), 0, st, bspec, gg.n_det, L);
  return hipGetLastError();
}
hipError_t launch_radial_czt(const float* sino, int n_det_full, cpx<float>* ghat,
                             const cpx<float>* chirp, const cpx<float>* bspec,
                             const cpx<float>* fac, const cpx<float>* tw, const GridGeom& gg,
                             int nz, hipStream_t st) {
  const int L = czt_length(gg.n_det);
  const int rows = nz * gg.n_angles;
#define TOMO_CZT(LL)                                                                              \
  case LL: {                                                                                      \
    constexpr int R = czt_rows<LL>();                                                             \
    hipLaunchKernelGGL((radial_czt_kernel<LL>), dim3((unsigned)((rows + R - 1) / R)),               \
                       dim3(R * (LL / 16)), 0, st, sino, n_det_full, gg.n_det, gg.stride,         \
                       gg.n_angles, nz, ghat, chirp, bspec, fac, tw);                              \
    return hipGetLastError();                                                                     \
  }
  switch (L) {
    TOMO_CZT(256) TOMO_CZT(512) TOMO_CZT(1024) TOMO_CZT(2048) TOMO_CZT(4096) TOMO_CZT(8192)
  }
#undef TOMO_CZT
  return hipErrorInvalidValue;
}
hipError_t launch_csr_build(const double* atab, const int2* g0, const float* wx, const float* wy,
                            const GridGeom& gg, int* cnt, int* row_ptr, int* idx, float* wts,
                            int* scan_sums, hipStream_t st) {
  const idx_t cells = (idx_t)gg.M * gg.M;
  const unsigned nb = nblk(cells, 256);
  hipLaunchKernelGGL(csr_count_kernel<float>, dim3(nb), dim3(256), 0, st, cnt, atab, g0, wx, wy,
                     gg.M, gg.n_det, gg.n_angles, gg.W);
  const int nsb = (int)((cells + SCAN_PER_BLOCK - 1) / SCAN_PER_BLOCK);
  hipLaunchKernelGGL(scan_blocks_kernel, dim3(nsb), dim3(1024), 0, st, cnt, row_ptr, scan_sums,
                     cells);
  hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(1024), 0, st, scan_sums, nsb,
                     row_ptr + cells);
  hipLaunchKernelGGL(scan_add_kernel, dim3(nb), dim3(256), 0, st, row_ptr, scan_sums, cells);
  hipLaunchKernelGGL(csr_fill_kernel, dim3(nb), dim3(256), 0, st, row_ptr, idx, wts, atab, g0,
                     wx, wy, gg.M, gg.n_det, gg.n_angles, gg.W);
  return hipGetLastError();
}
hipError_t launch_psf_lists(const double* atab, const int2* g0, const double* wx,
                            const double* wy, const GridGeom& gg, int* cnt, int* row_ptr,
                            double* wts, int* scan_sums, hipStream_t st) {
  const idx_t cells = (idx_t)gg.M * gg.M;
  const unsigned nb = nblk(cells, 256);
  hipLaunchKernelGGL(csr_count_kernel<double>, dim3(nb), dim3(256), 0, st, cnt, atab, g0, wx, wy,
                     gg.M, gg.n_det, gg.n_angles, gg.W);
  const int nsb = (int)((cells + SCAN_PER_BLOCK - 1) / SCAN_PER_BLOCK);
  hipLaunchKernelGGL(scan_blocks_kernel, dim3(nsb), dim3(1024), 0, st, cnt, row_ptr, scan_sums,
                     cells);
  hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(1024), 0, st, scan_sums, nsb,
                     row_ptr + cells);
  hipLaunchKernelGGL(scan_add_kernel, dim3(nb), dim3(256), 0, st, row_ptr, scan_sums, cells);
  hipLaunchKernelGGL(csr_fill_w64_kernel, dim3(nb), dim3(256), 0, st, row_ptr, wts, atab, g0, wx,
                     wy, gg.M, gg.n_det, gg.n_angles, gg.W);
  return hipGetLastError();
}
hipError_t launch_csr_ramp(const int* idx, const float* wts, const float* rampf, idx_t nnz,
                           const GridGeom& gg, float* out, hipStream_t st) {
  hipLaunchKernelGGL(csr_ramp_kernel, dim3(nblk(nnz, 256)), dim3(256), 0, st, idx, wts, rampf, nnz,
                     gg.n_det - 1, out);
  return hipGetLastError();
}
hipError_t launch_psf_grid(const int* row_ptr, const double* wts, cpx<double>* grid,
                           const GridGeom& gg, hipStream_t st) {
  const idx_t cells = (idx_t)gg.M * gg.M;
  hipLaunchKernelGGL(psf_grid_kernel, dim3(nblk(cells, 256)), dim3(256), 0, st, row_ptr, wts, grid,
                     cells, 1.0 / (double)gg.n_det);
  return hipGetLastError();
}
hipError_t launch_gather(const cpx<float>* ghat, cpx<float>* grid, const int* row_ptr,
                         const int* idx, const float* wts, const GridGeom& gg, int nz, int z0,
                         int nzb, hipStream_t st) {
  const idx_t cells = (idx_t)gg.M * gg.M;
  if (nzb >= 3) {
    // two slices per lane where every 16-byte value load is aligned: nz, z0 and nzb even
    const bool two = nzb >= 8 && (nz % 2) == 0 && (z0 % 2) == 0 && (nzb % 2) == 0;
    const int zs = nzb > 32 ? 64 : nzb > 16 ? 32 : nzb > 4 ? 16 : 4;  // slices per block row
    const dim3 blocks(nblk(cells, 64), (nzb + zs - 1) / zs);
#define TOMO_GZ(ZLV, SPLV)                                                                        \
  hipLaunchKernelGGL((gather_z_kernel<ZLV, SPLV, false>), blocks, dim3(256), 0, st, ghat, grid,   \
                     nullptr, row_ptr, idx, wts, nullptr, gg.M, nz, z0, nzb)
    if (two) {
      if (zs == 64) TOMO_GZ(32, 2);
      else if (zs == 32) TOMO_GZ(16, 2);
      else TOMO_GZ(8, 2);
    } else {
      if (zs == 64) TOMO_GZ(64, 1);
      else if (zs == 32) TOMO_GZ(32, 1);
      else if (zs == 16) TOMO_GZ(16, 1);
      else TOMO_GZ(4, 1);
    }
#undef TOMO_GZ
    return hipGetLastError();
  }
  const dim3 blocks(nblk(cells, 256));
  if (nzb <= 1)
    hipLaunchKernelGGL((gather_kernel<1>), blocks, dim3(256), 0, st, ghat, grid, row_ptr, idx, wts,
                       gg.M, nz, z0, nzb);
  else if (nzb <= 4)
    hipLaunchKernelGGL((gather_kernel<4>), blocks, dim3(256), 0, st, ghat, grid, row_ptr, idx, wts,
                       gg.M, nz, z0, nzb);
  else if (nzb <= 16)
    hipLaunchKernelGGL((gather_kernel<16>), blocks, dim3(256), 0, st, ghat, grid, row_ptr, idx,
                       wts, gg.M, nz, z0, nzb);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}
hipError_t launch_gather_dual(const cpx<float>* ghat, cpx<float>* grid, cpx<float>* grid_ramp,
                              const int* row_ptr, const int* idx, const float* wts,
                              const float* wts_ramp, const GridGeom& gg, int nz, int z0, int nzb,
                              hipStream_t st) {
  const idx_t cells = (idx_t)gg.M * gg.M;
  if (nzb < 1 || nzb > 64) return hipErrorInvalidValue;
  const bool two = nzb >= 8 && (nz % 2) == 0 && (z0 % 2) == 0 && (nzb % 2) == 0;
  const int zs = nzb > 32 ? 64 : nzb > 16 ? 32 : nzb > 4 ? 16 : 4;
  const dim3 blocks(nblk(cells, 64), (nzb + zs - 1) / zs);
#define TOMO_GZ(ZLV, SPLV)                                                                        \
  hipLaunchKernelGGL((gather_z_kernel<ZLV, SPLV, true>), blocks, dim3(256), 0, st, ghat, grid,    \
                     grid_ramp, row_ptr, idx, wts, wts_ramp, gg.M, nz, z0, nzb)
  if (two) {
    if (zs == 64) TOMO_GZ(32, 2);
    else if (zs == 32) TOMO_GZ(16, 2);
    else TOMO_GZ(8, 2);
  } else {
    if (zs == 64) TOMO_GZ(64, 1);
    else if (zs == 32) TOMO_GZ(32, 1);
    else if (zs == 16) TOMO_GZ(16, 1);
    else TOMO_GZ(4, 1);
  }
#undef TOMO_GZ
  return hipGetLastError();
}
hipError_t launch_deapod_table(float* inv, const GridGeom& gg, hipStream_t st) {
  hipLaunchKernelGGL(deapod_table_kernel, dim3(nblk(gg.n, 256)), dim3(256), 0, st, inv, gg.n,
                     gg.M, gg.W, gg.beta);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_point_table(const double* atab, int2* g0, T* wx, T* wy, const GridGeom& gg,
                              hipStream_t st) {
  const int np = gg.n_angles * (gg.n_det - 1);
  hipLaunchKernelGGL((point_table_kernel<T>), dim3(nblk(np, 128)), dim3(128), 0, st, atab, g0,
                     wx, wy, gg.n_det, gg.n_angles, gg.M, gg.W, gg.beta);
  return hipGetLastError();
}
template hipError_t launch_point_table<float>(const double*, int2*, float*, float*,
                                              const GridGeom&, hipStream_t);
template hipError_t launch_point_table<double>(const double*, int2*, double*, double*,
                                               const GridGeom&, hipStream_t);

#define TOMO_MSWITCH(T, CALL)         \
  switch (M) {                        \
    case 32: return CALL(T, 32);      \
    case 64: return CALL(T, 64);      \
    case 128: return CALL(T, 128);    \
    case 256: return CALL(T, 256);    \
    case 512: return CALL(T, 512);    \
    case 1024: return CALL(T, 1024);  \
    case 2048: return CALL(T, 2048);  \
    case 4096: return CALL(T, 4096);  \
    case 8192: return CALL(T, 8192);  \
  }                                   \
  return hipErrorInvalidValue;

hipError_t launch_fft2d_f32(cpx<float>* data, int M, int batch, int dir, const cpx<float>* tw,
                            hipStream_t st) {
#define CALL(T, PP) fft2d_p<T, PP>(data, batch, dir, tw, st)
  TOMO_MSWITCH(float, CALL)
#undef CALL
}
template <int P>
hipError_t fft2d_crop_p(cpx<float>* data, int batch, const cpx<float>* tw, float* out,
                        const float* inv, int N, hipStream_t st) {
  constexpr int ROWS = rows_per_block<float>(P);
  constexpr int TC = cols_per_block<float>(P);
  constexpr int TPF = fft::Plan<P, fftE<float>()>::TPF;
  const idx_t n_rows = (idx_t)batch * P;
  const dim3 gr((unsigned)((n_rows + ROWS - 1) / ROWS));
  const dim3 gc((unsigned)((N + TC - 1) / TC), batch);
  hipLaunchKernelGGL((fft_rows_kernel<float, P, ROWS, +1>), gr, dim3(ROWS * TPF), 0, st, data,
                     n_rows, tw, N / 2);
  hipLaunchKernelGGL((fft_cols_crop_kernel<P, TC>), gc, dim3(TC * TPF), 0, st, data, tw, out, inv,
                     N);
  return hipGetLastError();
}
hipError_t launch_fft2d_crop_f32(cpx<float>* data, int M, int batch, const cpx<float>* tw,
                                 float* out, const float* inv, int N, hipStream_t st) {
  if (N < 2 || N > M || (N & 1)) return hipErrorInvalidValue;
#define CALL(T, PP) fft2d_crop_p<PP>(data, batch, tw, out, inv, N, st)
  TOMO_MSWITCH(float, CALL)
#undef CALL
}
hipError_t launch_fft2d_f64(cpx<double>* data, int M, int batch, int dir,
                            const cpx<double>* tw, hipStream_t st) {
#define CALL(T, PP) fft2d_p<T, PP>(data, batch, dir, tw, st)
  TOMO_MSWITCH(double, CALL)
#undef CALL
}

hipError_t launch_crop_deapod(const cpx<float>* grid, float* out, const float* inv,
                              const GridGeom& gg, int nzb, hipStream_t st) {
  const idx_t tot = (idx_t)nzb * gg.n * gg.n;
  hipLaunchKernelGGL(crop_deapod_kernel, dim3(nblk(tot, 256)), dim3(256), 0, st, grid, out, inv,
                     gg.n, gg.M, nzb);
  return hipGetLastError();
}
hipError_t launch_psf_embed(const cpx<double>* grid, cpx<double>* emb, const GridGeom& gg, int N,
                            int P, hipStream_t st) {
  hipLaunchKernelGGL(psf_embed_kernel, dim3(nblk((idx_t)P * P, 256)), dim3(256), 0, st, grid, emb,
                     N, P, gg.M, gg.W, gg.beta);
  return hipGetLastError();
}
hipError_t launch_fk_store(const cpx<double>* spec, float* fk, float* fkn, int P,
                           hipStream_t st) {
  hipLaunchKernelGGL(fk_store_kernel, dim3(nblk((idx_t)P * (P / 2 + 1), 256)), dim3(256), 0, st,
                     spec, fk, fkn, P);
  return hipGetLastError();
}
hipError_t launch_fk_export(const float* fk, const float* fkn, float* out, int P,
                            hipStream_t st) {
  hipLaunchKernelGGL(fk_export_kernel, dim3(nblk((idx_t)P * (P / 2 + 1), 256)), dim3(256), 0, st,
                     fk, fkn, out, P);
  return hipGetLastError();
}
hipError_t launch_sumsq_strided(const float* g, idx_t rows, int n_out, int stride, double scale,
                                double* partials, double* out, hipStream_t st) {
  // rows of the full detector width n_out*stride; 512 blocks of partial sums
  const int nb = 512;
  hipLaunchKernelGGL(sumsq_kernel, dim3(nb), dim3(256), 0, st, g, rows, n_out, stride,
                     n_out * stride, scale * scale, partials);
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(256), 0, st, partials, nb, out);
  return hipGetLastError();
}
hipError_t launch_lanczos_prolong(const float* in, float* out, int n, int nz, hipStream_t st) {
  const idx_t tot = (idx_t)nz * 4 * n * n;
  hipLaunchKernelGGL(lanczos_prolong_kernel, dim3(nblk(tot, 256)), dim3(256), 0, st, in, out, n,
                     nz);
  return hipGetLastError();
}

}  // namespace tomo
