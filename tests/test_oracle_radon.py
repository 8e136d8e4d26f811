"""Pins of the oracle's exact Radon pair against closed forms (CPU only).

* A smooth off-centre Gaussian has an analytic Radon transform; the exact
  non-uniform-DFT forward operator must reproduce it to rounding (this fixes the
  centring, the orientation, the sign of the exponent and the scale).
* A uniform disk has chord-length projections 2 sqrt(r^2 - t^2); pixelisation
  limits the agreement to a few percent, so the tolerance is loose.
* <A f, g> = <f, A^T g> for random f, g (the adjoint is the exact transpose).
"""
import numpy as np
import pytest

import synth
from oracle import geometry as G
from oracle import radon


@pytest.mark.parametrize("n,n_angles,n_det,x0,y0,s,center", [
    (64, 45, 92, 5.3, -7.1, 2.5, None),
    (48, 30, 70, -5.0, 3.25, 2.5, None),
    (64, 17, 96, 2.0, 8.0, 3.0, 47.25),     # rotation centre off the middle bin
])
def test_gaussian_blob_matches_analytic_radon(n, n_angles, n_det, x0, y0, s, center):
    geom = G.Geometry(n, synth.uniform_angles(n_angles), n_det, center)
    f = synth.gaussian_blob(n, x0, y0, s)
    g = radon.forward(f, geom)
    ga = synth.gaussian_blob_sinogram(n_det, geom.theta, x0, y0, s, center)
    assert np.linalg.norm(g - ga) / np.linalg.norm(ga) < 1e-12


def test_nonuniform_angles_blob():
    rng = np.random.default_rng(11)
    ang = np.sort(rng.uniform(0.0, np.pi, 23))
    geom = G.Geometry(48, ang, 58)
    f = synth.gaussian_blob(48, -3.0, 4.0, 2.5)
    g = radon.forward(f, geom)
    ga = synth.gaussian_blob_sinogram(58, ang, -3.0, 4.0, 2.5)
    assert np.linalg.norm(g - ga) / np.linalg.norm(ga) < 1e-12


def test_disk_chord_length():
    n, r = 64, 20.0
    geom = G.Geometry(n, synth.uniform_angles(36), 92)
    c = np.arange(n) - n / 2.0
    disk = ((c[None, :] ** 2 + c[:, None] ** 2) <= r * r).astype(np.float64)
    g = radon.forward(disk, geom)
    t = np.arange(92) - 46.0
    chord = 2.0 * np.sqrt(np.maximum(r * r - t * t, 0.0))
    err = np.linalg.norm(g - chord[None, :]) / np.linalg.norm(np.broadcast_to(chord, g.shape))
    assert err < 5e-2


def test_forward_is_real():
    geom = G.Geometry(24, synth.uniform_angles(11), 36)
    f = np.random.default_rng(3).standard_normal((24, 24))
    fh = radon.image_to_polar(f, geom)
    e = radon._radial_phase(geom, +1.0)
    full = fh @ e / geom.n_det
    assert np.max(np.abs(full.imag)) < 1e-12 * np.max(np.abs(full.real))


@pytest.mark.parametrize("n,n_angles,n_det,center", [(32, 20, 46, None), (24, 9, 40, 19.5)])
def test_adjoint_identity(n, n_angles, n_det, center):
    rng = np.random.default_rng(n)
    geom = G.Geometry(n, synth.uniform_angles(n_angles), n_det, center)
    f = rng.standard_normal((n, n))
    g = rng.standard_normal((n_angles, n_det))
    lhs = float(np.vdot(radon.forward(f, geom), g))
    rhs = float(np.vdot(f, radon.adjoint(g, geom)))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)


def test_volume_is_slicewise():
    geom = G.Geometry(16, synth.uniform_angles(7), 24)
    rng = np.random.default_rng(5)
    vol = rng.standard_normal((3, 16, 16))
    g = radon.forward(vol, geom)
    for z in range(3):
        assert np.allclose(g[z], radon.forward(vol[z], geom), rtol=0, atol=1e-12)


def test_polar_to_pixels_matches_full_image():
    geom = G.Geometry(20, synth.uniform_angles(9), 30, 14.5)
    rng = np.random.default_rng(8)
    g = rng.standard_normal((9, 30))
    gh = radon.sino_spectrum(g, geom)
    full = radon.polar_to_image(gh, geom)
    ys, xs = rng.integers(0, 20, 7), rng.integers(0, 20, 7)
    assert np.allclose(radon.polar_to_pixels(gh, geom, ys, xs), full[ys, xs], rtol=0, atol=1e-12)
