"""MBIR objective, its gradient, the step size and FISTA with restart (oracle, FP64).

Sec. 2, Eq. (5): minimise F(f) = 1/2 ||R f - g||^2 + beta Phi(f).
Sec. 2.1, Eqs. (10)-(11): the data term and its gradient in Toeplitz form,
    e = 1/2 <f, K*f> - <f, R*g> + 1/2 <g, g>,   grad e = K*f - R*g.
Sec. 2, Eq. (6): gradient step with 1/L, L the Lipschitz constant of grad F.
Sec. 2 (end): accelerated gradient method with restart.

Readings:
* Eq. (6) prints "- lambda grad Phi"; differentiating Eq. (5) gives "+", which is
  used: grad F = K*f - R*g + beta grad Phi.
* L is not given in the paper.  L = 1.01 * lambda_pow + 2 beta rho''(0), where
  lambda_pow = ||T v|| / ||v|| after 30 power iterations of the Toeplitz operator
  T from the all-ones image, and 2 rho''(0) bounds the prior Hessian (the
  normalised weighted graph Laplacian has eigenvalues at most 2).
* The momentum and restart rule are not printed.  Standard FISTA momentum with
  the gradient-mapping restart test is used: with t_0 = 1 and y_0 = x_0,
      x_{k+1} = y_k - grad F(y_k) / L
      t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2
      if <y_k - x_{k+1}, x_{k+1} - x_k> > 0:  t_{k+1} = 1, y_{k+1} = x_{k+1}   (restart)
      else: y_{k+1} = x_{k+1} + ((t_k - 1)/t_{k+1}) (x_{k+1} - x_k)
  A dot product of exactly zero does not restart.  No positivity constraint.
* The recorded objective history holds F(y_k), the objective at the point
  where the gradient of iteration k is evaluated.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

from . import prior as qg
from . import radon, toeplitz
from .geometry import Geometry


@dataclasses.dataclass
class Problem:
    geom: Geometry
    fk: np.ndarray          # P x P real PSF spectrum
    b: np.ndarray           # R* g, [n_z, N, N]
    gg: float               # <g, g>
    prior: qg.QGGMRF
    beta: float


def pad_size(n: int) -> int:
    """Smallest power of two >= 2N (any P >= 2N-1 gives the same product)."""
    p = 1
    while p < 2 * n:
        p *= 2
    return p


def build(geom: Geometry, sino: np.ndarray, prior: qg.QGGMRF, beta: float,
          pad: Optional[int] = None) -> Problem:
    """Precompute F K and R* g once before iterating (Sec. 2.1)."""
    sino = np.asarray(sino, dtype=np.float64)
    if sino.ndim == 2:
        sino = sino[None]
    p = pad_size(geom.n) if pad is None else pad
    fk = toeplitz.psf_spectrum(geom, p)
    b = radon.adjoint(sino, geom)
    return Problem(geom, fk, b, float(np.vdot(sino, sino)), prior, beta)


def objective(y: np.ndarray, prob: Problem, ty: Optional[np.ndarray] = None) -> float:
    if ty is None:
        ty = toeplitz.apply(y, prob.fk, prob.geom.n)
    return toeplitz.data_term(y, ty, prob.b, prob.gg) + prob.beta * qg.value(y, prob.prior)


def gradient(y: np.ndarray, prob: Problem, ty: Optional[np.ndarray] = None) -> np.ndarray:
    if ty is None:
        ty = toeplitz.apply(y, prob.fk, prob.geom.n)
    return toeplitz.data_gradient(ty, prob.b) + prob.beta * qg.gradient(y, prob.prior)


def power_lambda(fk: np.ndarray, n: int, iters: int = 30) -> float:
    """||T v_k|| / ||v_k|| at the last of ``iters`` normalised power iterations from ones."""
    v = np.ones((n, n), dtype=np.float64)
    lam = 0.0
    for _ in range(iters):
        w = toeplitz.apply(v, fk, n)
        lam = float(np.linalg.norm(w) / np.linalg.norm(v))
        v = w / np.linalg.norm(w)
    return lam


def lipschitz(prob: Problem, iters: int = 30) -> float:
    lam = power_lambda(prob.fk, prob.geom.n, iters)
    curv = qg.rho_second_at_zero(prob.prior) if prob.beta != 0.0 else 0.0
    return 1.01 * lam + 2.0 * prob.beta * curv


@dataclasses.dataclass
class FistaResult:
    x: np.ndarray
    history: list          # F(y_k), k = 0..iters-1
    restarts: list         # iterations k at which the restart test fired
    L: float


def fista(prob: Problem, x0: np.ndarray, iters: int, L: Optional[float] = None,
          restart: bool = True) -> FistaResult:
    if L is None:
        L = lipschitz(prob)
    x = np.array(x0, dtype=np.float64, copy=True)
    if x.ndim == 2:
        x = x[None]
    y = x.copy()
    t = 1.0
    hist = []
    restarts = []
    for k in range(iters):
        ty = toeplitz.apply(y, prob.fk, prob.geom.n)
        hist.append(objective(y, prob, ty))
        x_new = y - gradient(y, prob, ty) / L
        t_new = (1.0 + math.sqrt(1.0 + 4.0 * t * t)) / 2.0
        dot = float(np.vdot(y - x_new, x_new - x))
        if restart and dot > 0.0:
            t_new = 1.0
            y = x_new
            restarts.append(k)
        else:
            y = x_new + ((t - 1.0) / t_new) * (x_new - x)
        x = x_new
        t = t_new
    return FistaResult(x, hist, restarts, L)
