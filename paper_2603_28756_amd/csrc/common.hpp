// Shared device-side helpers for libtomo (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#define TOMO_DEV __device__ __forceinline__

template <typename T>
struct alignas(2 * sizeof(T)) cpx {
  T re, im;
};

template <typename T> TOMO_DEV cpx<T> mk(T r, T i) { cpx<T> c; c.re = r; c.im = i; return c; }
template <typename T> TOMO_DEV cpx<T> operator+(cpx<T> a, cpx<T> b) { return mk(a.re + b.re, a.im + b.im); }
template <typename T> TOMO_DEV cpx<T> operator-(cpx<T> a, cpx<T> b) { return mk(a.re - b.re, a.im - b.im); }
template <typename T> TOMO_DEV cpx<T> cmul(cpx<T> a, cpx<T> b) {
  return mk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename T> TOMO_DEV cpx<T> conj(cpx<T> a) { return mk(a.re, -a.im); }
template <typename T> TOMO_DEV cpx<T> scale(cpx<T> a, T s) { return mk(a.re * s, a.im * s); }

// Row-major element counts can exceed 2^31 for the largest grids.
typedef int64_t idx_t;

// Layout of F K / P^2 ([P] rows v, P/2 columns u; the Nyquist column is stored apart):
// columns in groups of 4, each group row-major [P][4], so that the columns of a pass-C
// column tile are contiguous along the rows that pass walks.
TOMO_DEV idx_t fk_index(int v, int u, int P) {
  return ((idx_t)(u >> 2) * P + v) * 4 + (u & 3);
}

// Parameters of the qGGMRF potential passed by value to kernels.
struct PriorParams {
  float beta;        // prior weight
  float p;           // exponent p
  float qmp;         // q - p
  float q_over_p;    // q / p
  float inv_Tsigma;  // 1 / (T sigma)
  float c_grad;      // (T sigma)^(p-q) / sigma^p  (rho' prefactor for q = 2 form)
  float c_val;       // (T sigma)^p / (p sigma^p)  (rho prefactor)
  float qm1;         // q - 1
  float lw0;         // (q - p) log2(1 / (T sigma))
  float qop_m1;      // q / p - 1
  float c_val2;      // c_val / (T sigma)^2  (rho = c_val2 d^2 / (1 + w))
  float wts[4];      // neighbour weights: [0] unused, [1] axis, [2] face diagonal, [3] body diagonal
  int neighbours;    // 8 or 26
  int quadratic;     // 1 when p == q (w == 1)
};
