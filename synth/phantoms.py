"""Seeded phantoms and their analytic parallel-beam projections.

Conventions (pixel units, bin width equal to pixel width):

* image array ``f[m_y, m_x]`` of width ``N``; pixel centre ``(x, y) = (m_x - N/2, m_y - N/2)``;
* detector bin ``j`` sits at ``t_j = j - c`` with rotation centre ``c = n_det/2``;
* a projection at angle ``theta`` integrates along ``x cos(theta) + y sin(theta) = t``;
* angles are uniform, ``theta_i = i * pi / n_angles``.

Phantom parameters use normalised coordinates ``u = x / (N/2)``.  Ellipse
projections use the textbook chord-length formula for an ellipse (Kak & Slaney,
Principles of Computerized Tomographic Imaging, ch. 3): for an ellipse with
semi-axes ``a, b`` rotated by ``phi`` and density ``mu``, the line integral at
signed distance ``tau`` from its centre is ``2 mu a b sqrt(s^2 - tau^2) / s^2``
for ``|tau| < s``, where ``s^2 = a^2 cos^2(theta - phi) + b^2 sin^2(theta - phi)``.
These are inputs only: the reconstruction method itself never evaluates them.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence

import numpy as np

__all__ = [
    "Workload", "WORKLOADS", "detector_bins_for", "uniform_angles", "ellipse_params",
    "ellipsoid_params", "rasterize_ellipses", "ellipse_sinogram", "ellipsoid_volume",
    "ellipsoid_sinogram", "gaussian_blob", "gaussian_blob_sinogram", "add_noise",
    "make_problem", "textured_slice", "textured_batch", "uneven_problems",
]


def rng_for(seed: int) -> np.random.Generator:
    """PCG64 generator seeded through a SeedSequence."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))


def detector_bins_for(n: int) -> int:
    """Detector bins covering the image diagonal: round(N*sqrt(2)), bumped to even."""
    nd = int(round(n * math.sqrt(2.0)))
    return nd + (nd & 1)


def uniform_angles(n_angles: int) -> np.ndarray:
    """theta_i = i*pi/n_angles, i = 0..n_angles-1 (radians, float64)."""
    return np.arange(n_angles, dtype=np.float64) * (np.pi / n_angles)


# ----------------------------------------------------------------------------- 2D ellipses
def ellipse_params(rng: np.random.Generator, count: int) -> np.ndarray:
    """Random ellipses, one row each: (cx, cy, a, b, phi, mu), normalised units.

    Draw order per ellipse: centre U[-0.7,0.7]^2, semi-axes U[0.05,0.4]^2,
    angle U[0,pi), intensity U[0,1].
    """
    out = np.empty((count, 6), dtype=np.float64)
    for k in range(count):
        cx, cy = rng.uniform(-0.7, 0.7, size=2)
        a, b = rng.uniform(0.05, 0.4, size=2)
        phi = rng.uniform(0.0, np.pi)
        mu = rng.uniform(0.0, 1.0)
        out[k] = (cx, cy, a, b, phi, mu)
    return out


def _to_pixels(params: np.ndarray, n: int) -> np.ndarray:
    p = np.array(params, dtype=np.float64, copy=True).reshape(-1, 6)
    half = n / 2.0
    p[:, 0:4] *= half
    return p


def rasterize_ellipses(params: np.ndarray, n: int) -> np.ndarray:
    """Sum of ellipse indicator functions point-sampled at pixel centres ([N, N], float64)."""
    p = _to_pixels(params, n)
    c = np.arange(n, dtype=np.float64) - n / 2.0
    x = c[None, :]
    y = c[:, None]
    img = np.zeros((n, n), dtype=np.float64)
    for cx, cy, a, b, phi, mu in p:
        dx = x - cx
        dy = y - cy
        u = dx * np.cos(phi) + dy * np.sin(phi)
        v = -dx * np.sin(phi) + dy * np.cos(phi)
        img += mu * ((u / a) ** 2 + (v / b) ** 2 <= 1.0)
    return img


def ellipse_sinogram(params: np.ndarray, n: int, angles: np.ndarray, n_det: int,
                     center: Optional[float] = None) -> np.ndarray:
    """Exact line integrals of the ellipse sum at detector bin centres ([n_angles, n_det])."""
    p = _to_pixels(params, n)
    c = n_det / 2.0 if center is None else float(center)
    t = np.arange(n_det, dtype=np.float64) - c
    th = np.asarray(angles, dtype=np.float64)[:, None]
    g = np.zeros((th.shape[0], n_det), dtype=np.float64)
    for cx, cy, a, b, phi, mu in p:
        s2 = (a * np.cos(th - phi)) ** 2 + (b * np.sin(th - phi)) ** 2
        tau = t[None, :] - (cx * np.cos(th) + cy * np.sin(th))
        inside = tau * tau < s2
        chord = np.where(inside, np.sqrt(np.maximum(s2 - tau * tau, 0.0)), 0.0)
        g += 2.0 * mu * a * b * chord / s2
    return g


# ----------------------------------------------------------------------------- 3D ellipsoids
def ellipsoid_params(rng: np.random.Generator, count: int) -> np.ndarray:
    """Random ellipsoids rotated about z: (cx, cy, cz, a, b, c, phi, mu), normalised units.

    Draw order per ellipsoid: centre U[-0.7,0.7]^3, semi-axes U[0.05,0.4]^3,
    in-plane angle U[0,pi), intensity U[0,1].
    """
    out = np.empty((count, 8), dtype=np.float64)
    for k in range(count):
        cx, cy, cz = rng.uniform(-0.7, 0.7, size=3)
        a, b, c = rng.uniform(0.05, 0.4, size=3)
        phi = rng.uniform(0.0, np.pi)
        mu = rng.uniform(0.0, 1.0)
        out[k] = (cx, cy, cz, a, b, c, phi, mu)
    return out


def _slice_ellipses(params: np.ndarray, n_slices: int, z: int) -> np.ndarray:
    """Cross-section of each ellipsoid with slice z (normalised z over the slice count)."""
    zn = (z + 0.5 - n_slices / 2.0) / (n_slices / 2.0)
    rows = []
    for cx, cy, cz, a, b, c, phi, mu in np.asarray(params).reshape(-1, 8):
        r = (zn - cz) / c
        if abs(r) < 1.0:
            s = math.sqrt(1.0 - r * r)
            rows.append((cx, cy, a * s, b * s, phi, mu))
    return np.array(rows, dtype=np.float64).reshape(-1, 6)


def ellipsoid_volume(params: np.ndarray, n: int, n_slices: int) -> np.ndarray:
    vol = np.zeros((n_slices, n, n), dtype=np.float64)
    for z in range(n_slices):
        vol[z] = rasterize_ellipses(_slice_ellipses(params, n_slices, z), n)
    return vol


def ellipsoid_sinogram(params: np.ndarray, n: int, n_slices: int, angles: np.ndarray,
                       n_det: int, center: Optional[float] = None) -> np.ndarray:
    g = np.zeros((n_slices, len(angles), n_det), dtype=np.float64)
    for z in range(n_slices):
        g[z] = ellipse_sinogram(_slice_ellipses(params, n_slices, z), n, angles, n_det, center)
    return g


# ----------------------------------------------------------------------------- smooth blob
def gaussian_blob(n: int, x0: float, y0: float, s: float) -> np.ndarray:
    """exp(-|x - x0|^2 / (2 s^2)) sampled at pixel centres (pixel units, centred coords)."""
    c = np.arange(n, dtype=np.float64) - n / 2.0
    return np.exp(-((c[None, :] - x0) ** 2 + (c[:, None] - y0) ** 2) / (2.0 * s * s))


def gaussian_blob_sinogram(n_det: int, angles: np.ndarray, x0: float, y0: float, s: float,
                           center: Optional[float] = None) -> np.ndarray:
    """Line integrals of the continuous blob: sqrt(2 pi) s exp(-(t - x0.theta)^2 / (2 s^2))."""
    c = n_det / 2.0 if center is None else float(center)
    t = np.arange(n_det, dtype=np.float64) - c
    th = np.asarray(angles, dtype=np.float64)[:, None]
    tc = x0 * np.cos(th) + y0 * np.sin(th)
    return math.sqrt(2.0 * math.pi) * s * np.exp(-((t[None, :] - tc) ** 2) / (2.0 * s * s))


# ----------------------------------------------------------------------------- texture
def blob_params(rng: np.random.Generator, count: int, n: int) -> np.ndarray:
    """Texture blobs, one row each: (x0, y0, s, amplitude) in pixel units.

    Draw order per blob: centre uniform in the disc of radius 0.75 N/2, width U[1.5, 6]
    pixels, amplitude U[0.03, 0.12] with a random sign.
    """
    out = np.empty((count, 4), dtype=np.float64)
    for k in range(count):
        r = 0.75 * (n / 2.0) * math.sqrt(rng.uniform(0.0, 1.0))
        ang = rng.uniform(0.0, 2.0 * math.pi)
        s = rng.uniform(1.5, 6.0)
        amp = rng.uniform(0.03, 0.12) * (1.0 if rng.uniform() < 0.5 else -1.0)
        out[k] = (r * math.cos(ang), r * math.sin(ang), s, amp)
    return out


def textured_slice(n: int, n_angles: int, n_det: int, noise: float, seed: int,
                   n_ellipses: int = 10, n_blobs: int = 48, raster: bool = True) -> dict:
    """One slice: random ellipses plus a texture of small Gaussian blobs, its analytic
    sinogram (chord lengths plus blob line integrals, no inverse crime) and noise."""
    rng = rng_for(seed)
    angles = uniform_angles(n_angles)
    prm = ellipse_params(rng, n_ellipses)
    blobs = blob_params(rng, n_blobs, n)
    img = rasterize_ellipses(prm, n) if raster else None
    g = ellipse_sinogram(prm, n, angles, n_det)
    c = n / 2.0
    cx = np.arange(n, dtype=np.float64) - c
    t = np.arange(n_det, dtype=np.float64) - n_det / 2.0
    th = angles[None, :, None]
    x0, y0, sb, amp = (blobs[:, k][:, None, None] for k in range(4))
    tc = x0 * np.cos(th) + y0 * np.sin(th)
    g = g + np.sum(amp * math.sqrt(2.0 * math.pi) * sb * np.exp(-((t[None, None, :] - tc) ** 2) / (2.0 * sb * sb)),
                   axis=0)
    for bx, by, bs, ba in (blobs if raster else ()):
        img += ba * np.exp(-((cx[None, :] - bx) ** 2 + (cx[:, None] - by) ** 2) / (2.0 * bs * bs))
    return {"phantom": img, "sino": add_noise(g, rng, noise), "angles": angles}


def _textured_sino(args):
    n, na, nd, noise, seed = args
    return textured_slice(n, na, nd, noise, seed, raster=False)["sino"].astype(np.float32)


def textured_batch(count: int, n: int, n_angles: int, n_det: int, noise: float, seed0: int,
                   workers: int = 1) -> np.ndarray:
    """Sinograms [count, n_angles, n_det] (float32) of slices seeded seed0, seed0+1, ..."""
    jobs = [(n, n_angles, n_det, noise, seed0 + k) for k in range(count)]
    # worker processes are forked, which is only safe before the parent touches a GPU;
    # afterwards (or when asked for one worker) the slices are made in this process
    import sys
    torch_mod = sys.modules.get("torch")
    gpu_up = torch_mod is not None and torch_mod.cuda.is_initialized()
    if workers <= 1 or gpu_up:
        return np.stack([_textured_sino(j) for j in jobs])
    import concurrent.futures as cf
    import multiprocessing as mp
    with cf.ProcessPoolExecutor(max_workers=min(workers, 8), mp_context=mp.get_context("fork")) as ex:
        return np.stack(list(ex.map(_textured_sino, jobs, chunksize=8)))


# ----------------------------------------------------------------------------- uneven batch
def uneven_problems(count: int, seed: int, sizes=(128, 192, 256, 384, 512, 768, 1024),
                    angle_range=(30, 360), noise_range=(0.01, 0.05), n_objects: int = 10) -> list:
    """Independent single-slice problems of uneven size: per problem, draw N uniformly from
    `sizes`, the angle count uniformly from the integers in angle_range and the noise
    fraction uniformly from noise_range; 10 random ellipses; n_det = round(N sqrt 2), even.
    Returns dicts with n, n_angles, n_det, noise, angles and the float32 sinogram
    [1, n_angles, n_det]."""
    rng = rng_for(seed)
    out = []
    for _ in range(count):
        n = int(sizes[rng.integers(0, len(sizes))])
        na = int(rng.integers(angle_range[0], angle_range[1] + 1))
        noise = float(rng.uniform(*noise_range))
        nd = detector_bins_for(n)
        angles = uniform_angles(na)
        prm = ellipse_params(rng, n_objects)
        g = add_noise(ellipse_sinogram(prm, n, angles, nd), rng, noise)
        out.append({"n": n, "n_angles": na, "n_det": nd, "noise": noise, "angles": angles,
                    "sino": g[None].astype(np.float32)})
    return out


# ----------------------------------------------------------------------------- noise
def add_noise(g: np.ndarray, rng: np.random.Generator, frac: float) -> np.ndarray:
    """g + sigma_n * N(0,1), sigma_n = frac * max(g) over the whole array."""
    if frac <= 0.0:
        return np.array(g, dtype=np.float64, copy=True)
    sigma = frac * float(np.max(g))
    return g + sigma * rng.standard_normal(g.shape)


# ----------------------------------------------------------------------------- workloads
@dataclasses.dataclass(frozen=True)
class Workload:
    """A named synthetic reconstruction problem (sizes, seed, solver settings)."""

    name: str
    n: int
    n_slices: int
    n_angles: int
    n_det: int
    noise: float
    seed: int
    n_objects: int
    iterations: Sequence[int]
    neighbours: int
    levels: int = 1
    kb_width: int = 6
    kb_oversamp: float = 2.0
    p: float = 1.2
    q: float = 2.0
    beta: float = 0.01
    sigma: float = 0.1
    T: float = 1.0
    description: str = ""

    @property
    def voxels(self) -> int:
        return self.n * self.n * self.n_slices


WORKLOADS = {
    "single_slice_128": Workload(
        "single_slice_128", n=128, n_slices=1, n_angles=90, n_det=182, noise=0.01, seed=1,
        n_objects=10, iterations=(20,), neighbours=8,
        description="1 slice 128^2, 10 ellipses, 90 angles x 182 bins, 1% noise, FBP init, "
                    "qGGMRF p=1.2 q=2 beta=0.01, 20 iterations"),
    "volume_64x512": Workload(
        "volume_64x512", n=512, n_slices=64, n_angles=180, n_det=724, noise=0.01, seed=2,
        n_objects=20, iterations=(100,), neighbours=26,
        description="64 slices of 512^2, 20 ellipsoids, 180 angles x 724 bins, 1% noise, "
                    "PSF spectrum 1024^2, KB width 6 oversampling 2, 100 iterations, "
                    "26-neighbour qGGMRF"),
    "learned_init_512": Workload(
        "learned_init_512", n=512, n_slices=64, n_angles=60, n_det=724, noise=0.01, seed=100000,
        n_objects=10, iterations=(400,), neighbours=8,
        description="learned start: 2000 training and 64 held-out 512^2 slices (10 ellipses + "
                    "48 Gaussian texture blobs), 60 angles x 724 bins, 1% noise, 8-neighbour "
                    "qGGMRF p=1.2 beta=0.01; time to 1e-4 relative objective gap, U-Net start "
                    "against FBP start"),
    "hier_32x2048": Workload(
        "hier_32x2048", n=2048, n_slices=32, n_angles=91, n_det=2896, noise=0.02, seed=3,
        n_objects=20, iterations=(40, 20, 10), neighbours=26, levels=3,
        description="32 slices of 2048^2, 91 angles x 2896 bins, 2% noise, 3-level "
                    "hierarchy 512->1024->2048 with Lanczos-3 prolongation"),
}


def make_problem(n: int, n_slices: int, n_angles: int, n_det: int, noise: float, seed: int,
                 n_objects: int, center: Optional[float] = None) -> dict:
    """Phantom, clean and noisy sinogram for one seeded problem (float64 arrays).

    A single slice uses 2D ellipses; several slices use z-rotated ellipsoids.
    """
    rng = rng_for(seed)
    angles = uniform_angles(n_angles)
    if n_slices == 1:
        prm = ellipse_params(rng, n_objects)
        phantom = rasterize_ellipses(prm, n)[None]
        clean = ellipse_sinogram(prm, n, angles, n_det, center)[None]
    else:
        prm = ellipsoid_params(rng, n_objects)
        phantom = ellipsoid_volume(prm, n, n_slices)
        clean = ellipsoid_sinogram(prm, n, n_slices, angles, n_det, center)
    sino = add_noise(clean, rng, noise)
    return {
        "phantom": phantom,
        "clean": clean,
        "sino": sino,
        "angles": angles,
        "center": n_det / 2.0 if center is None else float(center),
        "params": prm,
    }
