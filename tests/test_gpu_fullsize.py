"""Parity at the full size and launch configuration that bench.py times.

The 64 x 512^2 volume workload (180 angles x 724 bins, Kaiser-Bessel width 6,
oversampling 2, P = 1024, 26 neighbours) is too large for the oracle to
reconstruct in a test, so each operator is checked where the oracle can
compute exact values:
* F K and the step constant L in full (oracle PSF by direct sums, ~10-30 s);
* T x and the whole gradient in full over all 64 slices (oracle padded-FFT product with the
  oracle's F K, itself pinned to A^T A applied directly, and the oracle prior gradient);
* R* g and FBP at sampled pixels of several slices (exact sums per pixel);
* T x at sampled pixels of one slice (oracle A then A^T per pixel);
* the full gradient at sampled voxels (T x, b and the prior one voxel at a time).
Tolerance: relative L2 <= 1e-5 over the sampled values (gradient normalised by
||T x|| + ||b|| + beta ||grad Phi|| over the samples).
"""
import numpy as np
import pytest
import torch

import synth
from oracle import fbp as ofbp  # noqa: F401  (documents the definition the samples follow)
from oracle import radon, solver, toeplitz
from oracle import geometry as G
from oracle import prior as qg

from gpu_util import dev, rel_l2, to_dev, to_np

pytestmark = pytest.mark.gpu

WL = synth.WORKLOADS["volume_64x512"]


@pytest.fixture(scope="module")
def setup():
    from paper_2603_28756_amd import tomo
    pr = synth.make_problem(WL.n, WL.n_slices, WL.n_angles, WL.n_det, WL.noise, WL.seed, WL.n_objects)
    sino32 = pr["sino"].astype(np.float32)
    plan = tomo.Plan(WL.n, WL.n_slices, WL.n_angles, WL.n_det, angles=list(pr["angles"]),
                     kb_width=WL.kb_width, kb_oversamp=WL.kb_oversamp, beta=WL.beta, p=WL.p,
                     q=WL.q, sigma=WL.sigma, T=WL.T, neighbours=WL.neighbours)
    plan.precompute_psf()
    geom = G.Geometry(WL.n, pr["angles"], WL.n_det)
    return {"plan": plan, "geom": geom, "sino": sino32.astype(np.float64),
            "sino_dev": torch.from_numpy(sino32).to(dev()), "phantom": pr["phantom"]}


def _sample_pixels(rng, n, count):
    ys = rng.integers(0, n, count)
    xs = rng.integers(0, n, count)
    ys[:4] = [0, n - 1, 0, n // 2]
    xs[:4] = [0, n - 1, n - 1, n // 2]
    return ys, xs


@pytest.fixture(scope="module")
def oracle_fk(setup):
    _, _, P = setup["plan"].level_dims(0)
    return toeplitz.psf_spectrum(setup["geom"], P)


def test_fullsize_psf_spectrum_and_step(setup, oracle_fk):
    plan = setup["plan"]
    fk_gpu, L_gpu, lam_gpu = plan.psf_info()
    _, _, P = plan.level_dims(0)
    fk = oracle_fk
    assert rel_l2(to_np(fk_gpu), fk[:, : P // 2 + 1]) < 1e-5
    lam = solver.power_lambda(fk, WL.n, 30)
    assert abs(lam_gpu - lam) / lam < 1e-5


@pytest.mark.parametrize("ramp", [False, True])
def test_fullsize_backprojection_sampled(setup, ramp):
    plan, geom, sino = setup["plan"], setup["geom"], setup["sino"]
    out = torch.empty((WL.n_slices, WL.n, WL.n), dtype=torch.float32, device=dev())
    plan.backproject(setup["sino_dev"], out, ramp=ramp)
    got = to_np(out)
    rng = np.random.default_rng(5 + ramp)
    gpu_vals, ref_vals = [], []
    ramp_w = np.abs(G.radial_freqs(WL.n_det)) if ramp else None
    for z in (0, 17, 40, 63):
        gh = radon.sino_spectrum(sino[z], geom)
        if ramp:
            gh = gh * ramp_w[None, :] * (np.pi / WL.n_angles)
        ys, xs = _sample_pixels(rng, WL.n, 24)
        ref_vals.append(radon.polar_to_pixels(gh, geom, ys, xs))
        gpu_vals.append(got[z, ys, xs])
    assert rel_l2(np.concatenate(gpu_vals), np.concatenate(ref_vals)) < 1e-5


def test_fullsize_normal_operator_and_gradient_sampled(setup):
    plan, geom = setup["plan"], setup["geom"]
    rng = np.random.default_rng(11)
    x = (setup["phantom"] + 0.05 * rng.standard_normal(setup["phantom"].shape)).astype(np.float32)
    b = (0.5 * rng.standard_normal(x.shape)).astype(np.float32)
    xd, bd = to_dev(x), to_dev(b)
    tx = torch.empty_like(xd)
    grad = torch.empty_like(xd)
    plan.apply_normal(xd, tx)
    plan.gradient(xd, bd, grad)
    tx_np, grad_np = to_np(tx), to_np(grad)
    x64, b64 = x.astype(np.float64), b.astype(np.float64)
    pr = qg.QGGMRF(p=WL.p, q=WL.q, sigma=WL.sigma, T=WL.T, neighbours=WL.neighbours)
    zs = (31, 0)
    t_gpu, t_ref, g_gpu, g_ref, parts = [], [], [], [], [0.0, 0.0, 0.0]
    for z in zs:
        gh = radon.sino_spectrum(radon.forward(x64[z], geom), geom)
        ys, xs = _sample_pixels(rng, WL.n, 20)
        tref = radon.polar_to_pixels(gh, geom, ys, xs)
        t_ref.append(tref)
        t_gpu.append(tx_np[z, ys, xs])
        vox = [(z, int(y), int(xx)) for y, xx in zip(ys, xs)]
        gphi = qg.gradient_at(x64, pr, vox)
        g_ref.append(tref - b64[z, ys, xs] + WL.beta * gphi)
        g_gpu.append(grad_np[z, ys, xs])
        parts[0] += float(np.sum(tref ** 2))
        parts[1] += float(np.sum(b64[z, ys, xs] ** 2))
        parts[2] += float(np.sum(gphi ** 2))
    assert rel_l2(np.concatenate(t_gpu), np.concatenate(t_ref)) < 1e-5
    norm = np.sqrt(parts[0]) + np.sqrt(parts[1]) + WL.beta * np.sqrt(parts[2])
    err = np.linalg.norm(np.concatenate(g_gpu) - np.concatenate(g_ref))
    assert err / norm < 1e-5


def test_fullsize_normal_operator_and_gradient_full_arrays(setup, oracle_fk):
    """T x and grad = T x - b + beta grad Phi(x) over the whole 64 x 512^2 volume."""
    plan = setup["plan"]
    rng = np.random.default_rng(23)
    x = (setup["phantom"] + 0.05 * rng.standard_normal(setup["phantom"].shape)).astype(np.float32)
    b = (0.5 * rng.standard_normal(x.shape)).astype(np.float32)
    xd, bd = to_dev(x), to_dev(b)
    tx = torch.empty_like(xd)
    grad = torch.empty_like(xd)
    plan.apply_normal(xd, tx)
    plan.gradient(xd, bd, grad)
    tx_np, grad_np = to_np(tx), to_np(grad)
    del tx, grad, xd, bd
    x64, b64 = x.astype(np.float64), b.astype(np.float64)
    tref = toeplitz.apply(x64, oracle_fk, WL.n)
    assert rel_l2(tx_np, tref) < 1e-5
    pr = qg.QGGMRF(p=WL.p, q=WL.q, sigma=WL.sigma, T=WL.T, neighbours=WL.neighbours)
    gphi = qg.gradient(x64, pr)
    gref = tref - b64 + WL.beta * gphi
    norm = np.linalg.norm(tref) + np.linalg.norm(b64) + WL.beta * np.linalg.norm(gphi)
    assert np.linalg.norm(grad_np - gref) / norm < 1e-5
