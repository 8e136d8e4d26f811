"""Pins of the oracle's FBP, step size and FISTA (CPU only).

* FBP of a smooth Gaussian recovers the Gaussian within a few percent, and
  converges to it as the detector widens (fixes the ramp and the pi/n_angles
  quadrature weight).
* The power-iteration lambda never exceeds, and lies within 1% of, the largest
  eigenvalue of the dense normal matrix A^T A.
* With beta = 0, FISTA converges to the least-squares minimiser from a dense
  solve, and before any restart obeys F(x_k) - F* <= 2 L ||x0 - x*||^2 / (k+1)^2.
* The objective equals 1/2 ||A y - g||^2 + beta Phi(y) computed directly.
* The restart test fires under momentum overshoot and then restarts from x_{k+1}.
* FISTA reaches the dense-solve minimiser of a quadratic-prior problem.
"""
import numpy as np
import pytest

import synth
from oracle import fbp, radon, solver, toeplitz
from oracle import geometry as G
from oracle import prior as qg


def test_fbp_recovers_gaussian():
    # The ramp acts circularly on the n_det radial samples, which shifts the
    # baseline by a term that falls like 1/n_det^2; widening the detector makes
    # FBP converge to the blob, which pins both the ramp and the pi/n_angles weight.
    n = 64
    ft = synth.gaussian_blob(n, 5.3, -7.1, 2.5)
    errs = {}
    for n_angles, n_det in ((45, 92), (90, 92), (90, 184), (90, 368)):
        geom = G.Geometry(n, synth.uniform_angles(n_angles), n_det)
        g = synth.gaussian_blob_sinogram(n_det, geom.theta, 5.3, -7.1, 2.5)
        f0 = fbp.fbp(g, geom)
        errs[(n_angles, n_det)] = np.linalg.norm(f0 - ft) / np.linalg.norm(ft)
    assert errs[(45, 92)] < 0.05
    assert errs[(90, 184)] < 0.3 * errs[(90, 92)]
    assert errs[(90, 368)] < 0.003
    assert f0.max() == pytest.approx(1.0, rel=0.01)


def _dense_problem(n=12, n_angles=10, n_det=18, seed=0):
    rng = np.random.default_rng(seed)
    geom = G.Geometry(n, synth.uniform_angles(n_angles), n_det)
    a = np.stack([radon.forward(e.reshape(n, n), geom).ravel() for e in np.eye(n * n)], axis=1)
    g = rng.standard_normal((n_angles, n_det))
    return geom, a, g


def test_power_iteration_lambda():
    geom, a, _ = _dense_problem()
    lam_max = np.linalg.eigvalsh(a.T @ a)[-1]
    fk = toeplitz.psf_spectrum(geom, 32)
    lam = solver.power_lambda(fk, geom.n, 30)
    assert lam <= lam_max * (1 + 1e-12)
    assert lam >= 0.99 * lam_max


def test_fista_converges_to_least_squares():
    geom, a, g = _dense_problem()
    pr = qg.QGGMRF(neighbours=8)
    prob = solver.build(geom, g, pr, beta=0.0)
    xstar = np.linalg.lstsq(a, g.ravel(), rcond=None)[0].reshape(1, geom.n, geom.n)
    fstar = solver.objective(xstar, prob)
    x0 = np.zeros((1, geom.n, geom.n))
    res = solver.fista(prob, x0, 60, restart=False)
    lam_max = np.linalg.eigvalsh(a.T @ a)[-1]
    L = res.L
    assert L >= lam_max
    # FISTA rate bound on the iterates x_k (objective at x_k evaluated directly)
    x = x0.copy()
    y = x0.copy()
    t = 1.0
    r0 = float(np.vdot(x0 - xstar, x0 - xstar))
    for k in range(60):
        xn = y - solver.gradient(y, prob) / L
        tn = (1 + np.sqrt(1 + 4 * t * t)) / 2
        y = xn + ((t - 1) / tn) * (xn - x)
        x, t = xn, tn
        assert solver.objective(x, prob) - fstar <= 2 * L * r0 / (k + 2) ** 2 + 1e-9
    assert np.allclose(x, res.x, rtol=0, atol=1e-12)


def test_fista_converges_to_dense_quadratic_minimiser():
    # p = q = 2 makes the prior quadratic, beta Phi = beta/(4 sigma^2) sum_pairs b (x_s - x_r)^2,
    # so the minimiser solves (A^T A + beta/(2 sigma^2) Lap) x = A^T g with a dense solve.
    geom, a, g = _dense_problem(n=10, n_angles=8, n_det=16, seed=2)
    n = geom.n
    sigma, beta = 0.3, 0.5
    pr = qg.QGGMRF(p=2.0, q=2.0, sigma=sigma, T=1.0, neighbours=8)
    w = qg.weights(8)
    lap = np.zeros((n * n, n * n))
    for y in range(n):
        for x in range(n):
            for (_, dy, dx), b in w.items():
                yy, xx = y + dy, x + dx
                if 0 <= yy < n and 0 <= xx < n:
                    lap[y * n + x, y * n + x] += b
                    lap[y * n + x, yy * n + xx] -= b
    h = a.T @ a + beta / (2 * sigma ** 2) * lap
    xstar = np.linalg.solve(h, a.T @ g.ravel()).reshape(1, n, n)
    prob = solver.build(geom, g, pr, beta=beta)
    res = solver.fista(prob, np.zeros((1, n, n)), 1500, restart=True)
    assert np.linalg.norm(res.x - xstar) / np.linalg.norm(xstar) < 1e-8


def test_objective_matches_direct():
    geom, _, g = _dense_problem(seed=3)
    pr = qg.QGGMRF(p=1.2, q=2.0, sigma=0.1, T=1.0, neighbours=8)
    prob = solver.build(geom, g, pr, beta=0.05)
    y = np.random.default_rng(1).standard_normal((1, geom.n, geom.n))
    r = radon.forward(y[0], geom) - g
    direct = 0.5 * float(np.vdot(r, r)) + 0.05 * qg.value(y, pr)
    assert solver.objective(y, prob) == pytest.approx(direct, rel=1e-12)


def test_restart_rule():
    # In a strongly convex problem momentum overshoots and the gradient-mapping
    # test fires; after a restart the next extrapolation point is x_{k+1} itself.
    geom, _, g = _dense_problem(n=10, n_angles=8, n_det=16, seed=2)
    pr = qg.QGGMRF(p=2.0, q=2.0, sigma=0.3, T=1.0, neighbours=8)
    prob = solver.build(geom, g, pr, beta=0.5)
    x0 = np.zeros((1, 10, 10))
    res = solver.fista(prob, x0, 100)
    assert len(res.restarts) >= 2 and 0 not in res.restarts
    no = solver.fista(prob, x0, 100, restart=False)
    assert no.restarts == []
    assert res.history[-1] <= no.history[-1]
    k = res.restarts[0]
    before = solver.fista(prob, x0, k + 1)
    after = solver.fista(prob, x0, k + 2)
    # F(y_{k+1}) with y_{k+1} = x_{k+1}
    assert after.history[-1] == pytest.approx(solver.objective(before.x, prob), rel=1e-14)
    assert res.history[:k + 2] == after.history


def test_pad_size():
    assert solver.pad_size(128) == 256
    assert solver.pad_size(192) == 512
    assert solver.pad_size(100) == 256
