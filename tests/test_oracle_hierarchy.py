"""Pins of the oracle's coarse-to-fine pieces (CPU only).

* L(n) = delta_n at integers, so even fine samples copy the coarse samples.
* The normalised prolongation reproduces constants exactly away from the edge
  and a low-frequency cosine to 1e-3.
* Subsampling: the analytic projections of a blob on the fine detector, kept
  every s-th bin and divided by s, equal the analytic projections of the same
  blob expressed in coarse pixel units on the coarse detector (centre c/s).
* The coarse operator applied to the coarse-sampled blob matches that subsampled
  sinogram (same centring on both levels).
* A one-level hierarchy is plain FISTA.
"""
import numpy as np
import pytest

import synth
from oracle import geometry as G
from oracle import hierarchy, radon, solver
from oracle import prior as qg


def test_lanczos_interpolates_integers():
    x = np.arange(-4, 5, dtype=np.float64)
    assert np.allclose(hierarchy.lanczos(x), (x == 0).astype(float), atol=1e-15)
    # symmetric and supported on |x| < 3
    xs = np.linspace(-3.5, 3.5, 71)
    assert np.allclose(hierarchy.lanczos(xs), hierarchy.lanczos(-xs))
    assert np.all(hierarchy.lanczos(np.array([3.0, 3.2, -3.01])) == 0.0)
    # centre taps positive (the garbled printed kernel gives negative ones)
    assert hierarchy.lanczos(np.array([0.5]))[0] > 0.6


def test_prolong_copies_even_samples_and_reproduces_smooth_signals():
    n = 32
    rng = np.random.default_rng(0)
    f = rng.standard_normal((n, n))
    up = hierarchy.prolong(f)
    assert np.allclose(up[::2, ::2], f, rtol=0, atol=1e-14)
    ones = hierarchy.prolong(np.ones((n, n)))
    assert np.allclose(ones[6:-6, 6:-6], 1.0, rtol=0, atol=1e-14)
    m = np.arange(n)
    coarse = np.cos(2 * np.pi * 1.5 * m / n)
    fine = hierarchy.prolong(np.outer(np.ones(n), coarse))
    i = np.arange(2 * n)
    exact = np.cos(2 * np.pi * 1.5 * (i / 2.0) / n)
    assert np.max(np.abs(fine[10, 8:-8] - exact[8:-8])) < 1e-3


def test_subsampled_sinogram_is_coarse_sinogram():
    n_det, s = 96, 2
    ang = synth.uniform_angles(20)
    fine = synth.gaussian_blob_sinogram(n_det, ang, 6.0, -4.0, 3.0)
    sub = hierarchy.subsample_sinogram(fine, s)
    coarse = synth.gaussian_blob_sinogram(n_det // s, ang, 6.0 / s, -4.0 / s, 3.0 / s, center=n_det / 2 / s)
    assert np.allclose(sub, coarse, rtol=0, atol=1e-13)


def test_level_operator_centring():
    geom = G.Geometry(128, synth.uniform_angles(24), 184)
    lg = hierarchy.level_geometry(geom, 2)
    assert (lg.n, lg.n_det, lg.c) == (64, 92, 46.0)
    blob = synth.gaussian_blob(64, 3.0, -2.5, 3.0)
    g_coarse = radon.forward(blob, lg)
    fine = synth.gaussian_blob_sinogram(184, geom.theta, 6.0, -5.0, 6.0)
    assert np.linalg.norm(g_coarse - hierarchy.subsample_sinogram(fine, 2)) / np.linalg.norm(g_coarse) < 1e-12


def test_single_level_is_fista():
    prob_in = synth.make_problem(24, 1, 12, 34, 0.01, 7, 4)
    geom = G.Geometry(24, prob_in["angles"], 34)
    pr = qg.QGGMRF(neighbours=8)
    h = hierarchy.reconstruct(geom, prob_in["sino"], pr, 0.01, [5], init="zero")
    prob = solver.build(geom, prob_in["sino"], pr, 0.01)
    f = solver.fista(prob, np.zeros((1, 24, 24)), 5)
    assert np.allclose(h.x, f.x, rtol=0, atol=1e-14)


def test_two_level_runs_and_improves():
    prob_in = synth.make_problem(32, 1, 24, 44, 0.0, 8, 5)
    geom = G.Geometry(32, prob_in["angles"], 44)
    pr = qg.QGGMRF(neighbours=8)
    h = hierarchy.reconstruct(geom, prob_in["sino"], pr, 0.001, [10, 10], init="fbp")
    assert h.x.shape == (1, 32, 32)
    hist = h.levels[1].history
    assert hist[-1] < hist[0]
    with pytest.raises(ValueError):
        hierarchy.level_geometry(G.Geometry(30, synth.uniform_angles(3), 42), 4)
