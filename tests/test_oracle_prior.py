"""Pins of the oracle's qGGMRF prior (CPU only).

* Central finite differences of Phi reproduce dPhi/df (8 and 26 neighbours,
  interior and boundary voxels).
* p = q = 2 reduces rho to D^2 / (4 sigma^2), so grad Phi is the weighted graph
  Laplacian / (2 sigma^2), checked against a plain loop stencil.
* Brute force over every unordered voxel pair of a tiny volume.
* rho at D = T sigma has w = 1; small-D asymptote D^2 / (p T^(2-p) sigma^2); the
  curvature never exceeds rho''(0) (which sets the step size).
* Weights: 8 or 26 offsets, proportional to 1/distance, summing to one.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import prior as qg


@pytest.mark.parametrize("nb,shape", [(26, (3, 6, 7)), (8, (1, 9, 8)), (26, (2, 5, 5)), (8, (3, 5, 6))])
def test_gradient_matches_finite_differences(nb, shape):
    pr = qg.QGGMRF(p=1.2, q=2.0, sigma=0.1, T=1.0, neighbours=nb)
    rng = np.random.default_rng(sum(shape) + nb)
    x = 0.2 * rng.standard_normal(shape)
    g = qg.gradient(x, pr)
    h = 1e-6
    for idx in [(0, 0, 0), tuple(s // 2 for s in shape), tuple(s - 1 for s in shape), (0, shape[1] - 1, 1)]:
        e = np.zeros_like(x)
        e[idx] = h
        fd = (qg.value(x + e, pr) - qg.value(x - e, pr)) / (2 * h)
        assert fd == pytest.approx(g[idx], rel=1e-6, abs=1e-7)


def test_quadratic_case_is_weighted_laplacian():
    sigma = 0.3
    pr = qg.QGGMRF(p=2.0, q=2.0, sigma=sigma, T=1.0, neighbours=26)
    rng = np.random.default_rng(9)
    x = rng.standard_normal((3, 5, 4))
    w = qg.weights(26)
    lap = np.zeros_like(x)
    nz, ny, nx = x.shape
    for z, y, xx in itertools.product(range(nz), range(ny), range(nx)):
        for (dz, dy, dx), b in w.items():
            zz, yy, xq = z + dz, y + dy, xx + dx
            if 0 <= zz < nz and 0 <= yy < ny and 0 <= xq < nx:
                lap[z, y, xx] += b * (x[z, y, xx] - x[zz, yy, xq])
    assert np.allclose(qg.gradient(x, pr), lap / (2 * sigma ** 2), rtol=1e-12, atol=1e-12)
    assert qg.rho(np.array([0.7]), pr)[0] == pytest.approx(0.49 / (4 * sigma ** 2), rel=1e-14)


def test_value_brute_force_pairs():
    pr = qg.QGGMRF(p=1.3, q=2.0, sigma=0.2, T=0.8, neighbours=26)
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 3, 3))
    vox = list(itertools.product(range(2), range(3), range(3)))
    w = qg.weights(26)
    total = 0.0
    for i, s in enumerate(vox):
        for r in vox[i + 1:]:
            o = tuple(rr - ss for rr, ss in zip(r, s))
            if max(abs(c) for c in o) == 1:
                total += w[o] * qg.rho(np.array([x[s] - x[r]]), pr)[0]
    assert qg.value(x, pr) == pytest.approx(total, rel=1e-13)


def test_rho_special_values():
    pr = qg.QGGMRF(p=1.2, q=2.0, sigma=0.1, T=2.0, neighbours=8)
    d = pr.T * pr.sigma
    assert qg.rho(np.array([d]), pr)[0] == pytest.approx(d ** pr.p / (pr.p * pr.sigma ** pr.p) / 2, rel=1e-14)
    small = 1e-9
    assert qg.rho(np.array([small]), pr)[0] == pytest.approx(
        small ** 2 / (pr.p * pr.T ** (2 - pr.p) * pr.sigma ** 2), rel=1e-5)
    assert qg.rho_prime(np.array([0.0]), pr)[0] == 0.0
    # odd derivative
    assert qg.rho_prime(np.array([-0.3]), pr)[0] == pytest.approx(-qg.rho_prime(np.array([0.3]), pr)[0])


@pytest.mark.parametrize("p,T,sigma", [(1.2, 1.0, 0.1), (1.0, 1.0, 0.5), (1.5, 0.5, 2.0), (1.99, 1.0, 1.0)])
def test_curvature_bounded_by_value_at_zero(p, T, sigma):
    pr = qg.QGGMRF(p=p, q=2.0, sigma=sigma, T=T, neighbours=8)
    d = np.linspace(1e-4, 20 * sigma * T, 20001)
    h = 1e-6 * sigma
    second = (qg.rho_prime(d + h, pr) - qg.rho_prime(d - h, pr)) / (2 * h)
    assert np.max(second) <= qg.rho_second_at_zero(pr) * (1 + 1e-6)


def test_weights():
    for nb, count in ((8, 8), (26, 26)):
        w = qg.weights(nb)
        assert len(w) == count
        assert sum(w.values()) == pytest.approx(1.0, rel=1e-15)
        base = w[(0, 0, 1)]
        for o, v in w.items():
            assert v == pytest.approx(base / math.sqrt(sum(c * c for c in o)), rel=1e-14)
    assert len(qg.half_offsets(26)) == 13 and len(qg.half_offsets(8)) == 4


def test_invalid_parameters():
    with pytest.raises(ValueError):
        qg.QGGMRF(p=2.2)
    with pytest.raises(ValueError):
        qg.QGGMRF(p=1.5, q=1.2)
    with pytest.raises(ValueError):
        qg.QGGMRF(neighbours=6)


@pytest.mark.parametrize("nb", [8, 26])
def test_gradient_at_matches_full_gradient(nb):
    pr = qg.QGGMRF(neighbours=nb)
    rng = np.random.default_rng(nb)
    x = 0.2 * rng.standard_normal((3, 7, 6))
    full = qg.gradient(x, pr)
    vox = [(0, 0, 0), (1, 3, 2), (2, 6, 5), (0, 6, 0), (2, 0, 5)]
    got = qg.gradient_at(x, pr, vox)
    assert np.allclose(got, [full[v] for v in vox], rtol=1e-13, atol=1e-13)
