"""Shared helpers of the GPU parity tests: seeded inputs, plan construction, metrics.

Inputs come from ``synth``; expected values come from ``oracle`` only.  The
float32 values handed to the GPU are cast back to float64 for the oracle so both
sides see identical inputs.
"""
import numpy as np
import torch

import synth
from oracle import geometry as G
from oracle import prior as qg


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def dev():
    return torch.device("cuda", 0)


def to_dev(a) -> torch.Tensor:
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device=dev())


def to_np(t: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def problem(n, nz, n_angles, n_det, noise=0.01, seed=0, n_objects=6, center=None):
    """Seeded phantom and sinogram; returns (sino float32 as float64, angles, center)."""
    pr = synth.make_problem(n, nz, n_angles, n_det, noise, seed, n_objects, center)
    sino32 = pr["sino"].astype(np.float32)
    return sino32.astype(np.float64), pr["angles"], pr["center"], pr["phantom"]


def oracle_geom(n, angles, n_det, center=None):
    return G.Geometry(n, angles, n_det, center)


def make_plan(n, nz, angles, n_det, center=None, neighbours=26, beta=0.01, p=1.2, sigma=0.1,
              T=1.0, kb_width=8, n_levels=1, pad=0, graphs=True, fused_prior=False,
              concurrent_prior=False):
    from paper_2603_28756_amd import tomo
    return tomo.Plan(n, nz, len(angles), n_det, angles=list(angles), center=center, pad=pad,
                     n_levels=n_levels, kb_width=kb_width, beta=beta, p=p, sigma=sigma, T=T,
                     neighbours=neighbours, graphs=graphs, fused_prior=fused_prior,
                     concurrent_prior=concurrent_prior)


def oracle_prior(neighbours=26, p=1.2, sigma=0.1, T=1.0):
    return qg.QGGMRF(p=p, q=2.0, sigma=sigma, T=T, neighbours=neighbours)


def objective_err(got, ref, sino) -> float:
    """Largest objective difference relative to F(0) = <g, g>/2.  The Toeplitz-form objective
    (Eq. 10) is a difference of terms of size ~<g, g>, so float32 operators leave an absolute
    error of order 1e-7 <g, g> however small F itself becomes near the optimum."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    f0 = 0.5 * float(np.vdot(sino, sino))
    return float(np.max(np.abs(got - ref)) / f0)
