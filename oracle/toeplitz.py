"""Point-spread function, padded spectrum and Toeplitz normal operator (oracle, FP64).

Sec. 2.1, Eqs. (7)-(9): R*R f equals the convolution of f with a point-spread
function K obtained by applying the adjoint non-uniform transform to the
all-ones function on the polar samples; K is needed on a grid of at least 2N-1
points per axis, f is zero-padded, and the product is evaluated by FFTs and
restricted to N x N:

    R*R f = Res_{NxN} F^-1( F K  .  F Pad f ).

With the operator pair of ``oracle.radon`` (the 1/n_det of the radial inverse
transform included), K(d) = (1/n_det) sum_{i,l} cos(2 pi k_il . d) for integer
offsets d in [-(N-1), N-1]^2; K is real and even.

Reading (padding, Sec. 2.1): the paper asks for at least 2N-1 points; any FFT
size P >= 2N-1 gives the same cropped product because no cropped output ever
reaches an offset beyond N-1.  K is placed in the P x P circulant at offsets
|d| <= N-1 and the rest of the circulant is zero.
"""
from __future__ import annotations

import numpy as np

from .geometry import Geometry, radial_freqs


def psf(geom: Geometry) -> np.ndarray:
    """K(d) for d in [-(N-1), N-1]^2, array [2N-1, 2N-1] indexed [dy + N-1, dx + N-1]."""
    n = geom.n
    d = np.arange(-(n - 1), n, dtype=np.float64)
    w = radial_freqs(geom.n_det)
    k = np.zeros((2 * n - 1, 2 * n - 1), dtype=np.float64)
    for th in geom.theta:
        ex = np.exp(2j * np.pi * np.outer(w * np.cos(th), d))   # [n_l, dx]
        ey = np.exp(2j * np.pi * np.outer(w * np.sin(th), d))   # [n_l, dy]
        k += (ey.T @ ex).real
    return k / geom.n_det


def embed(k: np.ndarray, n: int, p: int) -> np.ndarray:
    """Place K(d), |d_x|,|d_y| <= N-1, at index d mod P of a P x P array; zero elsewhere."""
    if p < 2 * n - 1:
        raise ValueError("padded size must be at least 2N-1")
    kc = np.zeros((p, p), dtype=np.float64)
    idx = np.arange(-(n - 1), n) % p
    kc[np.ix_(idx, idx)] = k
    return kc


def spectrum(kc: np.ndarray) -> np.ndarray:
    """F K: 2D DFT of the embedded kernel (real because K is real and even)."""
    return np.fft.fft2(kc).real


def psf_spectrum(geom: Geometry, p: int) -> np.ndarray:
    """F K for padded size P (the quantity precomputed once before iterating, Sec. 2.1)."""
    return spectrum(embed(psf(geom), geom.n, p))


def apply(f: np.ndarray, fk: np.ndarray, n: int) -> np.ndarray:
    """Res_{NxN} F^-1(F K . F Pad f) for f [N, N] or [n_z, N, N] (Sec. 2.1, Eq. 9)."""
    f = np.asarray(f, dtype=np.float64)
    p = fk.shape[0]
    if f.ndim == 3:
        return np.stack([apply(s, fk, n) for s in f])
    fp = np.zeros((p, p), dtype=np.float64)
    fp[:n, :n] = f
    return np.fft.ifft2(fk * np.fft.fft2(fp))[:n, :n].real


def data_term(f: np.ndarray, tf: np.ndarray, b: np.ndarray, gg: float) -> float:
    """e = 1/2 f^T (K*f) - f^T R*g + 1/2 g^T g (Sec. 2.1, Eq. 10)."""
    return 0.5 * float(np.vdot(f, tf)) - float(np.vdot(f, b)) + 0.5 * gg


def data_gradient(tf: np.ndarray, b: np.ndarray) -> np.ndarray:
    """grad e = K*f - R*g (Sec. 2.1, Eq. 11)."""
    return tf - b
