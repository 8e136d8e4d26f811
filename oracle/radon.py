"""Exact non-uniform-DFT Radon transform and its adjoint (oracle, FP64).

Sec. 2, Eq. (3): R f = F^-1 NUFFT2 f — sample the 2D Fourier transform of the
image on the polar grid, then inverse-transform each projection along its
radial axis.  Eq. (4): R* g = NUFFT1 F g — transform each projection along its
radial axis, then take the adjoint non-uniform transform back to the image.

The oracle evaluates both non-uniform transforms exactly (direct sums, written as
one matrix product per angle), so it carries no gridding approximation:

    f^(k)      = sum_m f_m exp(-2 pi i k . x_m)                       (image -> polar)
    (A f)[i,j] = (1/n_det) sum_l exp(+2 pi i l (j - c)/n_det) f^(k_il)   (polar -> projection)
    G[i,l]     = (1/n_det) sum_j g[i,j] exp(-2 pi i l (j - c)/n_det)      (projection -> polar)
    (A^T g)_m  = Re sum_{i,l} G[i,l] exp(+2 pi i k_il . x_m)             (polar -> image)

A maps real images to real sinograms (the radial sample set is symmetric), and
A^T as written is its exact transpose.
"""
from __future__ import annotations

import numpy as np

from .geometry import Geometry, pixel_coords, polar_points, radial_indices, radial_freqs


def _angle_factors(geom: Geometry, i: int, sign: float):
    """exp(sign 2 pi i omega_l cos(theta) x) and the same for y, each [n_l, N]."""
    w = radial_freqs(geom.n_det)
    x = pixel_coords(geom.n)
    th = geom.theta[i]
    ex = np.exp(sign * 2j * np.pi * np.outer(w * np.cos(th), x))
    ey = np.exp(sign * 2j * np.pi * np.outer(w * np.sin(th), x))
    return ex, ey


def image_to_polar(f: np.ndarray, geom: Geometry) -> np.ndarray:
    """f^(k_il) for one slice f[N, N]; returns complex [n_angles, n_det-1]."""
    f = np.asarray(f, dtype=np.float64)
    out = np.empty((geom.n_angles, geom.n_det - 1), dtype=np.complex128)
    for i in range(geom.n_angles):
        ex, ey = _angle_factors(geom, i, -1.0)
        # sum_{y,x} ey[l,y] f[y,x] ex[l,x]
        out[i] = np.sum((ey @ f) * ex, axis=1)
    return out


def _radial_phase(geom: Geometry, sign: float) -> np.ndarray:
    """exp(sign 2 pi i l (j - c)/n_det) as [n_l, n_det]."""
    l = radial_indices(geom.n_det).astype(np.float64)
    t = np.arange(geom.n_det, dtype=np.float64) - geom.c
    return np.exp(sign * 2j * np.pi * np.outer(l, t) / geom.n_det)


def polar_to_projection(fh: np.ndarray, geom: Geometry) -> np.ndarray:
    """1D inverse radial transform of each angle: [n_angles, n_det-1] -> real [n_angles, n_det]."""
    e = _radial_phase(geom, +1.0)
    return (fh @ e).real / geom.n_det


def forward(f: np.ndarray, geom: Geometry) -> np.ndarray:
    """A f.  f is [N, N] or [n_z, N, N]; returns [n_angles, n_det] or [n_z, n_angles, n_det]."""
    f = np.asarray(f, dtype=np.float64)
    if f.ndim == 3:
        return np.stack([forward(s, geom) for s in f])
    return polar_to_projection(image_to_polar(f, geom), geom)


def sino_spectrum(g: np.ndarray, geom: Geometry) -> np.ndarray:
    """G[i,l] = (1/n_det) sum_j g[i,j] exp(-2 pi i l (j - c)/n_det) for one slice [n_angles, n_det]."""
    e = _radial_phase(geom, -1.0)
    return (np.asarray(g, dtype=np.float64) @ e.T) / geom.n_det


def polar_to_image(gh: np.ndarray, geom: Geometry) -> np.ndarray:
    """Re sum_{i,l} G[i,l] exp(+2 pi i k_il . x_m) for one slice; returns [N, N]."""
    out = np.zeros((geom.n, geom.n), dtype=np.float64)
    for i in range(geom.n_angles):
        ex, ey = _angle_factors(geom, i, +1.0)
        # sum_l ey[l,y] gh[l] ex[l,x]
        out += (ey.T @ (gh[i][:, None] * ex)).real
    return out


def adjoint(g: np.ndarray, geom: Geometry) -> np.ndarray:
    """A^T g.  g is [n_angles, n_det] or [n_z, n_angles, n_det]."""
    g = np.asarray(g, dtype=np.float64)
    if g.ndim == 3:
        return np.stack([adjoint(s, geom) for s in g])
    return polar_to_image(sino_spectrum(g, geom), geom)


def polar_to_pixels(gh: np.ndarray, geom: Geometry, ys, xs) -> np.ndarray:
    """The same sum as ``polar_to_image`` evaluated only at pixels (ys[m], xs[m])."""
    k = polar_points(geom)
    c = pixel_coords(geom.n)
    out = np.empty(len(ys), dtype=np.float64)
    for m, (iy, ix) in enumerate(zip(ys, xs)):
        phase = 2.0 * np.pi * (k[..., 0] * c[ix] + k[..., 1] * c[iy])
        out[m] = float(np.sum((gh * np.exp(1j * phase)).real))
    return out
