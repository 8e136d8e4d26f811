"""Parallel-beam geometry and the polar Fourier sample set (oracle, FP64).

Sec. 2, Eqs. (1)-(2): the projection at angle theta integrates f along the line
x cos(theta) + y sin(theta) = t, and its 1D Fourier transform is the radial
slice of the 2D transform of f along (cos(theta), sin(theta)).

Units are pixels; a detector bin is one pixel wide.  Pixel (m_y, m_x) of an
N x N image has centre (m_x - N/2, m_y - N/2); detector bin j sits at
t_j = j - c with c the rotation-centre bin (default n_det/2).

Reading (radial sample set, Sec. 2, Eq. 3): the radial frequencies are
omega_l = l / n_det for l = -(n_det/2 - 1) ... n_det/2 - 1.  The unpaired
Nyquist bin l = -n_det/2 of the length-n_det FFT grid is dropped, which makes the
forward operator exactly real and its normal operator exactly Toeplitz.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np


@dataclasses.dataclass(frozen=True)
class Geometry:
    """One reconstruction grid and its projection geometry."""

    n: int                      # image width N (N x N pixels per slice)
    angles: tuple               # projection angles in radians
    n_det: int                  # detector bins per projection (even)
    center: Optional[float] = None  # rotation-centre bin; None -> n_det / 2

    def __post_init__(self):
        if self.n_det % 2:
            raise ValueError("n_det must be even")
        object.__setattr__(self, "angles", tuple(float(a) for a in self.angles))

    @property
    def c(self) -> float:
        return self.n_det / 2.0 if self.center is None else float(self.center)

    @property
    def n_angles(self) -> int:
        return len(self.angles)

    @property
    def theta(self) -> np.ndarray:
        return np.asarray(self.angles, dtype=np.float64)


def pixel_coords(n: int) -> np.ndarray:
    """Centred pixel coordinates m - N/2, m = 0..N-1."""
    return np.arange(n, dtype=np.float64) - n / 2.0


def detector_coords(geom: Geometry) -> np.ndarray:
    """t_j = j - c, j = 0..n_det-1."""
    return np.arange(geom.n_det, dtype=np.float64) - geom.c


def radial_indices(n_det: int) -> np.ndarray:
    """l = -(n_det/2 - 1) .. n_det/2 - 1 (Nyquist bin dropped; see module docstring)."""
    h = n_det // 2
    return np.arange(-(h - 1), h, dtype=np.int64)


def radial_freqs(n_det: int) -> np.ndarray:
    """omega_l = l / n_det in cycles per pixel."""
    return radial_indices(n_det).astype(np.float64) / n_det


def polar_points(geom: Geometry) -> np.ndarray:
    """k_{i,l} = omega_l (cos theta_i, sin theta_i); array [n_angles, n_det-1, 2]."""
    w = radial_freqs(geom.n_det)
    th = geom.theta
    return np.stack([np.cos(th)[:, None] * w[None, :], np.sin(th)[:, None] * w[None, :]], axis=-1)
