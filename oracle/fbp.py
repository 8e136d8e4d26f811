"""Ramp-filtered back-projection initial estimate (oracle, FP64).

Sec. 2.2, Eqs. (12)-(14): each projection is convolved with the ramp filter,
whose Fourier response is |omega|, and the filtered projections are
back-projected, f0 = R* g~.

Readings:
* the ramp is applied in the radial Fourier domain that the back-projector
  already uses (Eq. 4), i.e. G[i,l] is multiplied by |omega_l| = |l|/n_det before
  the adjoint polar-to-image sum; no extra zero padding is needed because the
  multiplication is exact on the radial samples;
* the parallel-beam inversion formula carries the angular quadrature weight
  pi / n_angles, which the paper's Eq. (14) omits; it is included so that f0
  has the scale of f.
"""
from __future__ import annotations

import numpy as np

from .geometry import Geometry, radial_freqs
from .radon import polar_to_image, sino_spectrum


def fbp(g: np.ndarray, geom: Geometry) -> np.ndarray:
    """f0 = (pi/n_angles) Re sum_{i,l} |omega_l| G[i,l] exp(2 pi i k_il . x)."""
    g = np.asarray(g, dtype=np.float64)
    if g.ndim == 3:
        return np.stack([fbp(s, geom) for s in g])
    ramp = np.abs(radial_freqs(geom.n_det))
    gh = sino_spectrum(g, geom) * ramp[None, :]
    return (np.pi / geom.n_angles) * polar_to_image(gh, geom)
