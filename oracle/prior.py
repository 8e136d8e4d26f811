"""qGGMRF edge-preserving prior over an 8- or 26-neighbourhood (oracle, FP64).

Sec. 2, Eq. (5) names an edge-preserving qGGMRF prior Phi, couples the whole 3D
volume through it (Sec. 2, after Eq. 6; Sec. 2.4: 26 nearest neighbours) and
defers its form to the MBIR literature it cites (Venkatakrishnan et al. 2013;
Mohan et al. 2014).  Reading taken from those references, with 1 <= p < q <= 2
(or p = q = 2):

    rho(D)  = |D|^p / (p sigma^p) * w / (1 + w),   w = (|D| / (T sigma))^(q - p)
    rho'(D) = sign(D) |D|^(p-1) / sigma^p * w (q/p + w) / (1 + w)^2
    Phi(f)  = sum over unordered neighbour pairs {s, r} of b_{s-r} rho(f_s - f_r)
    dPhi/df_s = sum_{r in N(s)} b_{s-r} rho'(f_s - f_r)

Weights b are proportional to 1/distance (1, 1/sqrt 2, 1/sqrt 3) and normalised
to sum to one over the chosen neighbourhood (8 in-plane neighbours for a single
slice, 26 for a volume).  Pairs that leave the volume are omitted.  The
notation Phi(|grad f|) of Eq. (5) is read as this pairwise-difference form.

Arrays are [n_z, N, N] (z, y, x).
"""
from __future__ import annotations

import dataclasses
import itertools
import math

import numpy as np


@dataclasses.dataclass(frozen=True)
class QGGMRF:
    p: float = 1.2
    q: float = 2.0
    sigma: float = 0.1
    T: float = 1.0
    neighbours: int = 26

    def __post_init__(self):
        if not (1.0 <= self.p <= self.q <= 2.0):
            raise ValueError("need 1 <= p <= q <= 2")
        if self.neighbours not in (8, 26):
            raise ValueError("neighbours must be 8 or 26")


def offsets(neighbours: int) -> list:
    """All neighbour offsets (dz, dy, dx): 8 in-plane or 26 in 3D."""
    out = []
    for dz, dy, dx in itertools.product((-1, 0, 1), repeat=3):
        if (dz, dy, dx) == (0, 0, 0):
            continue
        if neighbours == 8 and dz != 0:
            continue
        out.append((dz, dy, dx))
    return out


def weights(neighbours: int) -> dict:
    """b_o proportional to 1/|o|, normalised to sum to 1 over the neighbourhood."""
    offs = offsets(neighbours)
    raw = {o: 1.0 / math.sqrt(o[0] ** 2 + o[1] ** 2 + o[2] ** 2) for o in offs}
    s = sum(raw.values())
    return {o: v / s for o, v in raw.items()}


def half_offsets(neighbours: int) -> list:
    """One offset of each +-pair (the lexicographically positive one): unordered pairs."""
    return [o for o in offsets(neighbours) if o > (0, 0, 0)]


def rho(d: np.ndarray, pr: QGGMRF) -> np.ndarray:
    a = np.abs(d)
    w = (a / (pr.T * pr.sigma)) ** (pr.q - pr.p)
    return a ** pr.p / (pr.p * pr.sigma ** pr.p) * w / (1.0 + w)


def rho_prime(d: np.ndarray, pr: QGGMRF) -> np.ndarray:
    a = np.abs(d)
    w = (a / (pr.T * pr.sigma)) ** (pr.q - pr.p)
    with np.errstate(divide="ignore", invalid="ignore"):
        val = np.sign(d) * a ** (pr.p - 1.0) / pr.sigma ** pr.p * w * (pr.q / pr.p + w) / (1.0 + w) ** 2
    return np.where(a == 0.0, 0.0, val)


def rho_second_at_zero(pr: QGGMRF) -> float:
    """rho''(0): 2/(p T^(2-p) sigma^2) for p < q = 2; 1/(2 sigma^2) for p = q = 2."""
    if pr.q != 2.0:
        raise ValueError("rho''(0) is finite only for q = 2")
    if pr.p == pr.q:
        return 1.0 / (2.0 * pr.sigma ** 2)
    return 2.0 / (pr.p * pr.T ** (2.0 - pr.p) * pr.sigma ** 2)


def _pair_views(f: np.ndarray, o: tuple):
    """(f_s, f_{s+o}) over every s whose neighbour s+o lies inside the volume."""
    src = []
    dst = []
    for ax, d in enumerate(o):
        n = f.shape[ax]
        if d >= 0:
            src.append(slice(0, n - d))
            dst.append(slice(d, n))
        else:
            src.append(slice(-d, n))
            dst.append(slice(0, n + d))
    return tuple(src), tuple(dst)


def value(f: np.ndarray, pr: QGGMRF) -> float:
    """Phi(f): sum over unordered in-volume pairs of b rho(f_s - f_r)."""
    f = np.asarray(f, dtype=np.float64)
    w = weights(pr.neighbours)
    total = 0.0
    for o in half_offsets(pr.neighbours):
        s, r = _pair_views(f, o)
        total += w[o] * float(np.sum(rho(f[s] - f[r], pr)))
    return total


def gradient(f: np.ndarray, pr: QGGMRF) -> np.ndarray:
    """dPhi/df_s = sum over in-volume neighbours r of b rho'(f_s - f_r)."""
    f = np.asarray(f, dtype=np.float64)
    w = weights(pr.neighbours)
    g = np.zeros_like(f)
    for o in offsets(pr.neighbours):
        s, r = _pair_views(f, o)
        g[s] += w[o] * rho_prime(f[s] - f[r], pr)
    return g


def gradient_at(f: np.ndarray, pr: QGGMRF, voxels) -> np.ndarray:
    """dPhi/df_s at the listed voxels (z, y, x), summing over in-volume neighbours."""
    f = np.asarray(f, dtype=np.float64)
    w = weights(pr.neighbours)
    nz, ny, nx = f.shape
    out = np.zeros(len(voxels), dtype=np.float64)
    for m, (z, y, x) in enumerate(voxels):
        acc = 0.0
        for (dz, dy, dx), b in w.items():
            zz, yy, xx = z + dz, y + dy, x + dx
            if 0 <= zz < nz and 0 <= yy < ny and 0 <= xx < nx:
                acc += b * float(rho_prime(np.array([f[z, y, x] - f[zz, yy, xx]]), pr)[0])
        out[m] = acc
    return out
