// The direct (non-Toeplitz) operator R on gfx950: the forward projection of Sec. 2, Eq. 3,
// R f = F^-1 NUFFT2 f, evaluated as the exact transpose of the gridding back-projection of
// gridding_kernels.hip (Eq. 4), so that R and R* form an adjoint pair up to float32 rounding:
//
//   u[(m - N/2) mod M] = f[m] / (phi^(x_m / M) phi^(y_m / M))   (deapodise and embed)
//   U = sum_n u[n] exp(-2 pi i g.n / M)                          (M x M forward FFT)
//   F(k_p) = sum_{cells g of p's footprint} phi(g_x - k_px M) phi(g_y - k_py M) U[g mod M]
//   (R f)[i, j] = Re (1/n_det) sum_l F(k_il) exp(+2 pi i l (j - c) / n_det)
//
// The direct gradient R*(R f - g) takes both non-uniform transforms on every call, which is
// what the Toeplitz form of Sec. 2.1 replaces by one padded-FFT product.
#include "kernels.hpp"

namespace tomo {
namespace {

// grid[z][cell] for slices z0 .. z0 + nzb - 1: the deapodised image embedded at offset -N/2
// (mod M), zero elsewhere; every cell is written.
__global__ void embed_deapod_kernel(const float* __restrict__ f, cpx<float>* __restrict__ grid,
                                    const float* __restrict__ inv, int N, int M, int z0, int nzb) {
  const idx_t i = (idx_t)blockIdx.x * blockDim.x + threadIdx.x;
  const idx_t cells = (idx_t)M * M;
  if (i >= (idx_t)nzb * cells) return;
  const int zz = (int)(i / cells);
  const int rem = (int)(i - (idx_t)zz * cells);
  const int gy = rem / M, gx = rem - gy * M;
  const int my = (gy + N / 2) % M, mx = (gx + N / 2) % M;
  float v = 0.f;
  if (my < N && mx < N) v = f[((idx_t)(z0 + zz) * N + my) * N + mx] * inv[my] * inv[mx];
  grid[i] = mk(v, 0.f);
}

// fhat[z][p] = sum over the W x W footprint of sample p of wx wy U[z][cell] (the transpose of
// the gather of gridding_kernels.hip), for slices z0 .. z0 + nzb - 1 of the grid chunk.
__global__ void __launch_bounds__(256)
interp_kernel(const cpx<float>* __restrict__ grid, const int2* __restrict__ g0,
              const float* __restrict__ wx, const float* __restrict__ wy,
              cpx<float>* __restrict__ fhat, int npts, int M, int W, int z0, int nzb) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int zz = blockIdx.y;
  if (p >= npts || zz >= nzb) return;
  const int2 o = g0[p];
  const cpx<float>* gz = grid + (idx_t)zz * M * M;
  float ar = 0.f, ai = 0.f;
  for (int b = 0; b < W; ++b) {
    const int gy = ((o.y + b) % M + M) % M;
    const float wb = wy[(idx_t)p * W + b];
    const cpx<float>* row = gz + (idx_t)gy * M;
    float rr = 0.f, ri = 0.f;
    for (int a = 0; a < W; ++a) {
      const int gx = ((o.x + a) % M + M) % M;
      const float wa = wx[(idx_t)p * W + a];
      const cpx<float> v = row[gx];
      rr += wa * v.re;
      ri += wa * v.im;
    }
    ar += wb * rr;
    ai += wb * ri;
  }
  fhat[(idx_t)(z0 + zz) * npts + p] = mk(ar, ai);
}

// out[row][j] = Re sum_l conj(post[l]) fhat[row][l] exp(+2 pi i l j / nd) (minus sino[row][j]
// when given), rows = (slice, angle); with sino, part[block] = sum of out^2 over the block's
// outputs (float64, fixed order).  tab[m] = exp(-2 pi i m / nd), post[l] = (1/nd) exp(+2 pi i
// l c / nd): the transpose of the radial DFT of the back-projection.
constexpr int RI_ROWS = 16, RI_LC = 256;
__global__ void __launch_bounds__(256)
radial_idft_kernel(const cpx<float>* __restrict__ fhat, const float* __restrict__ sino,
                   float* __restrict__ out, double* __restrict__ part, int nd, int rows,
                   const cpx<float>* __restrict__ tab, const cpx<float>* __restrict__ post) {
  __shared__ cpx<float> ft[RI_ROWS][RI_LC];
  __shared__ double sred[256];
  const int t = threadIdx.x;
  const int nl = nd - 1, lmax = nd / 2 - 1;
  const int j = blockIdx.x * 256 + t;
  const int row0 = blockIdx.y * RI_ROWS;
  float acc[RI_ROWS];
#pragma unroll
  for (int r = 0; r < RI_ROWS; ++r) acc[r] = 0.f;
  for (int l0 = 0; l0 < nl; l0 += RI_LC) {
    for (int e = t; e < RI_ROWS * RI_LC; e += 256) {
      const int rr = e / RI_LC, ll = e - rr * RI_LC;
      const int row = row0 + rr, lidx = l0 + ll;
      cpx<float> v = mk(0.f, 0.f);
      if (row < rows && lidx < nl) v = cmul(fhat[(idx_t)row * nl + lidx], conj(post[lidx]));
      ft[rr][ll] = v;
    }
    __syncthreads();
    const int ln = min(RI_LC, nl - l0);
    // exp(+2 pi i l j / nd) = conj(tab[(l j) mod nd]), l = l0 - lmax + ll
    const int jp = j < nd ? j : 0;
    int idx = (int)((((long long)(l0 - lmax) * jp) % nd + nd) % nd);
    for (int ll = 0; ll < ln; ++ll) {
      const cpx<float> w = tab[idx];
      idx += jp;
      if (idx >= nd) idx -= nd;
#pragma unroll
      for (int r = 0; r < RI_ROWS; ++r) {
        const cpx<float> v = ft[r][ll];
        acc[r] += v.re * w.re + v.im * w.im;  // Re(v conj(w))
      }
    }
    __syncthreads();
  }
  double sq = 0.0;
  if (j < nd) {
#pragma unroll
    for (int r = 0; r < RI_ROWS; ++r) {
      const int row = row0 + r;
      if (row < rows) {
        const idx_t o = (idx_t)row * nd + j;
        float v = acc[r];
        if (sino) {
          v -= sino[o];
          sq += (double)v * (double)v;
        }
        out[o] = v;
      }
    }
  }
  if (!part) return;
  sred[t] = sq;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) sred[t] += sred[t + s];
    __syncthreads();
  }
  if (t == 0) part[(idx_t)blockIdx.y * gridDim.x + blockIdx.x] = sred[0];
}

__global__ void add_kernel(float* __restrict__ a, const float* __restrict__ b, idx_t n) {
  const idx_t i = (idx_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] += b[i];
}

// out = 1/2 sum rpart + beta sum of slot 0 of the prior partials (fixed order, one block)
__global__ void __launch_bounds__(256)
direct_objective_kernel(const double* __restrict__ rpart, int nr, const double* __restrict__ ppart,
                        int np, double beta, double* __restrict__ out) {
  __shared__ double sa[256], sb[256];
  const int t = threadIdx.x;
  double a = 0.0, b = 0.0;
  for (int k = t; k < nr; k += 256) a += rpart[k];
  for (int k = t; k < np; k += 256) b += ppart[(idx_t)k * 4];
  sa[t] = a;
  sb[t] = b;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) {
      sa[t] += sa[t + s];
      sb[t] += sb[t + s];
    }
    __syncthreads();
  }
  if (t == 0) out[0] = 0.5 * sa[0] + beta * sb[0];
}

unsigned nblk(idx_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

hipError_t launch_embed_deapod(const float* f, cpx<float>* grid, const float* inv, int N, int M,
                               int z0, int nzb, hipStream_t st) {
  const idx_t n = (idx_t)nzb * M * M;
  hipLaunchKernelGGL(embed_deapod_kernel, dim3(nblk(n, 256)), dim3(256), 0, st, f, grid, inv, N, M,
                     z0, nzb);
  return hipGetLastError();
}

hipError_t launch_interp(const cpx<float>* grid, const int2* g0, const float* wx, const float* wy,
                         cpx<float>* fhat, int npts, int M, int W, int z0, int nzb, hipStream_t st) {
  hipLaunchKernelGGL(interp_kernel, dim3(nblk(npts, 256), nzb), dim3(256), 0, st, grid, g0, wx, wy,
                     fhat, npts, M, W, z0, nzb);
  return hipGetLastError();
}

int radial_idft_blocks(int nd, int rows) {
  return (int)nblk(nd, 256) * (int)nblk(rows, RI_ROWS);
}

hipError_t launch_radial_idft(const cpx<float>* fhat, const float* sino, float* out, double* part,
                              int nd, int rows, const cpx<float>* tab, const cpx<float>* post,
                              hipStream_t st) {
  hipLaunchKernelGGL(radial_idft_kernel, dim3(nblk(nd, 256), nblk(rows, RI_ROWS)), dim3(256), 0, st,
                     fhat, sino, out, part, nd, rows, tab, post);
  return hipGetLastError();
}

hipError_t launch_add(float* a, const float* b, idx_t n, hipStream_t st) {
  hipLaunchKernelGGL(add_kernel, dim3(nblk(n, 256)), dim3(256), 0, st, a, b, n);
  return hipGetLastError();
}

hipError_t launch_direct_objective(const double* rpart, int nr, const double* ppart, int np,
                                   double beta, double* out, hipStream_t st) {
  hipLaunchKernelGGL(direct_objective_kernel, dim3(1), dim3(256), 0, st, rpart, nr, ppart, np, beta,
                     out);
  return hipGetLastError();
}

}  // namespace tomo
