"""Pins of the oracle's PSF, padded spectrum and Toeplitz product (CPU only).

* T f = A^T (A f) computed directly with the exact operator pair, for several
  grids, padded sizes P >= 2N-1 (power of two or not), angle sets and centres.
* K(d) equals an independent closed form: summing the radial samples of one
  angle in closed form gives a Dirichlet kernel,
      sum_{l=-L..L} cos(l phi) = sin((L + 1/2) phi) / sin(phi / 2),
  with L = n_det/2 - 1 and phi = 2 pi (cos(theta) d_x + sin(theta) d_y) / n_det.
* K(0) = n_angles (n_det - 1) / n_det exactly; K is even; F K is real.
* The data term e of Eq. (10) equals 1/2 ||A f - g||^2 and its gradient A^T(Af - g).
"""
import math

import numpy as np
import pytest

import synth
from oracle import geometry as G
from oracle import radon, toeplitz


def _dirichlet_psf(geom):
    n = geom.n
    d = np.arange(-(n - 1), n, dtype=np.float64)
    dx = d[None, :]
    dy = d[:, None]
    big_l = geom.n_det // 2 - 1
    k = np.zeros((2 * n - 1, 2 * n - 1))
    for th in geom.theta:
        phi = 2.0 * math.pi * (math.cos(th) * dx + math.sin(th) * dy) / geom.n_det
        den = np.sin(phi / 2.0)
        small = np.abs(den) < 1e-9
        num = np.sin((big_l + 0.5) * phi)
        val = np.where(small, 0.0, num / np.where(small, 1.0, den))
        # limit at phi = 0 (mod 2 pi): 2L+1 times +-1
        lim = (2 * big_l + 1) * np.cos((big_l + 0.5) * phi) / np.cos(phi / 2.0)
        k += np.where(small, lim, val)
    return k / geom.n_det


@pytest.mark.parametrize("n,p,n_angles,n_det,center", [
    (16, 32, 17, 24, None),
    (16, 40, 17, 24, None),       # non power-of-two padding
    (16, 31, 9, 22, None),        # the minimum 2N-1
    (24, 64, 13, 34, 16.5),       # off-centre rotation axis
    (20, 64, 31, 28, None),
])
def test_toeplitz_equals_direct_normal_operator(n, p, n_angles, n_det, center):
    rng = np.random.default_rng(n * 7 + p)
    geom = G.Geometry(n, synth.uniform_angles(n_angles), n_det, center)
    f = rng.standard_normal((n, n))
    direct = radon.adjoint(radon.forward(f, geom), geom)
    fk = toeplitz.psf_spectrum(geom, p)
    tf = toeplitz.apply(f, fk, n)
    assert np.linalg.norm(direct - tf) / np.linalg.norm(direct) < 1e-12


def test_toeplitz_random_angles():
    rng = np.random.default_rng(21)
    ang = rng.uniform(0.0, np.pi, 12)
    geom = G.Geometry(18, ang, 26)
    f = rng.standard_normal((18, 18))
    direct = radon.adjoint(radon.forward(f, geom), geom)
    tf = toeplitz.apply(f, toeplitz.psf_spectrum(geom, 64), 18)
    assert np.linalg.norm(direct - tf) / np.linalg.norm(direct) < 1e-12


@pytest.mark.parametrize("n,n_angles,n_det", [(32, 45, 46), (24, 30, 36)])
def test_psf_closed_form(n, n_angles, n_det):
    geom = G.Geometry(n, synth.uniform_angles(n_angles), n_det)
    k = toeplitz.psf(geom)
    kd = _dirichlet_psf(geom)
    assert np.max(np.abs(k - kd)) < 1e-11 * np.max(np.abs(kd))
    assert k[n - 1, n - 1] == pytest.approx(n_angles * (n_det - 1) / n_det, rel=1e-14)
    assert np.allclose(k, k[::-1, ::-1], rtol=0, atol=1e-12)


def test_spectrum_is_real():
    geom = G.Geometry(20, np.random.default_rng(1).uniform(0, np.pi, 9), 30)
    kc = toeplitz.embed(toeplitz.psf(geom), 20, 40)
    full = np.fft.fft2(kc)
    assert np.max(np.abs(full.imag)) < 1e-10 * np.max(np.abs(full.real))


def test_data_term_and_gradient_identities():
    rng = np.random.default_rng(4)
    n = 20
    geom = G.Geometry(n, synth.uniform_angles(15), 30)
    f = rng.standard_normal((n, n))
    g = rng.standard_normal((15, 30))
    fk = toeplitz.psf_spectrum(geom, 64)
    tf = toeplitz.apply(f, fk, n)
    b = radon.adjoint(g, geom)
    e = toeplitz.data_term(f, tf, b, float(np.vdot(g, g)))
    r = radon.forward(f, geom) - g
    assert e == pytest.approx(0.5 * float(np.vdot(r, r)), rel=1e-12)
    grad = toeplitz.data_gradient(tf, b)
    assert np.allclose(grad, radon.adjoint(r, geom), rtol=0, atol=1e-10 * np.max(np.abs(grad)))


def test_embed_rejects_small_padding():
    with pytest.raises(ValueError):
        toeplitz.embed(np.zeros((31, 31)), 16, 30)
