"""Write the stored oracle results that the full-geometry GPU parity tests compare against.

Every stored value here is computed by ``oracle/`` (FP64) from inputs drawn by ``synth``;
nothing comes from the GPU path.  The oracle runs are too long to repeat inside a test
(minutes of CPU per case), so their results are kept as compressed float32/float64 arrays:

* ``volume_512_slab.npz`` — an 18-slice contiguous slab (slices 23..40) of the 64 x 512^2
  volume workload (20 ellipsoids, seed 2, 180 angles x 724 bins, 1% noise): FBP start,
  100 accelerated iterations with restart, 26-neighbour qGGMRF (p 1.2, q 2, beta 0.01,
  sigma 0.1, T 1); the final iterate, F(y_k) per iteration, the restart iterations, L.
* ``batch_sizes.npz`` — for every image width N >= 192 of the uneven batch (256 problems,
  seed 4), the first problem of that width: FBP start, 20 iterations, 8-neighbour qGGMRF.
* ``hier_2048_subvolume.npz`` — a 4-slice contiguous sub-volume (slices 14..17) of the
  32 x 2048^2 hierarchy workload (20 ellipsoids, seed 3, 91 angles x 2896 bins, 2% noise):
  three levels 512 -> 1024 -> 2048 with 10, 5 and 3 iterations, 26-neighbour qGGMRF; the
  central 512 x 512 crop of every final slice (the whole result is 64 MB), the objective
  history, the restart iterations and the step constants.

Usage (repository root): python tests/golden/make_golden.py [slab|batch|hier|all]
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import fbp as ofbp  # noqa: E402
from oracle import geometry as G  # noqa: E402
from oracle import hierarchy  # noqa: E402
from oracle import prior as qg  # noqa: E402
from oracle import solver  # noqa: E402

SLAB = dict(n=512, n_slices=64, n_angles=180, n_det=724, noise=0.01, seed=2, n_objects=20,
            z0=23, nz=18, iters=100)
BATCH = dict(count=256, seed=4, iters=20, min_n=192)
HIER = dict(n=2048, n_slices=32, n_angles=91, n_det=2896, noise=0.02, seed=3, n_objects=20,
            z0=14, nz=4, iters=(10, 5, 3), crop=512)


def slab_inputs():
    """float32 sinogram of the slab (as float64) and its angles; shared with the GPU test."""
    c = SLAB
    pr = synth.make_problem(c["n"], c["n_slices"], c["n_angles"], c["n_det"], c["noise"],
                            c["seed"], c["n_objects"])
    sino = pr["sino"][c["z0"]:c["z0"] + c["nz"]].astype(np.float32).astype(np.float64)
    return sino, pr["angles"]


def batch_picks(probs):
    """Index of the first problem of every width >= min_n, in increasing width."""
    firsts = {}
    for j, p in enumerate(probs):
        if p["n"] >= BATCH["min_n"]:
            firsts.setdefault(p["n"], j)
    return [firsts[n] for n in sorted(firsts)]


def _fista(geom, sino, neighbours, iters):
    prob = solver.build(geom, sino, qg.QGGMRF(neighbours=neighbours), 0.01)
    return solver.fista(prob, ofbp.fbp(sino, geom), iters)


def make_slab():
    t0 = time.time()
    sino, angles = slab_inputs()
    geom = G.Geometry(SLAB["n"], angles, SLAB["n_det"])
    ref = _fista(geom, sino, 26, SLAB["iters"])
    np.savez_compressed(os.path.join(HERE, "volume_512_slab.npz"), x=ref.x.astype(np.float32),
                        history=np.array(ref.history), restarts=np.array(ref.restarts, dtype=np.int64),
                        L=ref.L, sino_sum=float(np.sum(sino)))
    print(f"slab: {time.time() - t0:.0f} s, restarts {ref.restarts}, L {ref.L:.6g}")


def make_batch():
    t0 = time.time()
    probs = synth.uneven_problems(BATCH["count"], seed=BATCH["seed"])
    out = {}
    for j in batch_picks(probs):
        p = probs[j]
        sino = p["sino"].astype(np.float64)
        geom = G.Geometry(p["n"], p["angles"], p["n_det"])
        ref = _fista(geom, sino, 8, BATCH["iters"])
        out[f"x_{j}"] = ref.x.astype(np.float32)
        out[f"history_{j}"] = np.array(ref.history)
        out[f"restarts_{j}"] = np.array(ref.restarts, dtype=np.int64)
        out[f"L_{j}"] = ref.L
        out[f"sino_sum_{j}"] = float(np.sum(sino))
        print(f"batch problem {j}: N {p['n']}, {p['n_angles']} angles, {time.time() - t0:.0f} s",
              flush=True)
    np.savez_compressed(os.path.join(HERE, "batch_sizes.npz"), **out)


def hier_inputs():
    """float32 sinogram of the sub-volume (as float64) and its angles; shared with the GPU test."""
    c = HIER
    pr = synth.make_problem(c["n"], c["n_slices"], c["n_angles"], c["n_det"], c["noise"],
                            c["seed"], c["n_objects"])
    sino = pr["sino"][c["z0"]:c["z0"] + c["nz"]].astype(np.float32).astype(np.float64)
    return sino, pr["angles"]


def hier_crop(x):
    """Central crop x [..., c0:c0+crop, c0:c0+crop] of the finest level."""
    c0 = (HIER["n"] - HIER["crop"]) // 2
    return x[..., c0:c0 + HIER["crop"], c0:c0 + HIER["crop"]]


def make_hier():
    t0 = time.time()
    sino, angles = hier_inputs()
    geom = G.Geometry(HIER["n"], angles, HIER["n_det"])
    res = hierarchy.reconstruct(geom, sino, qg.QGGMRF(neighbours=26), 0.01, list(HIER["iters"]),
                                init="fbp")
    hist = [v for lv in res.levels for v in lv.history]
    rst, off = [], 0
    for lv, it in zip(res.levels, HIER["iters"]):
        rst += [off + k for k in lv.restarts]
        off += it
    np.savez_compressed(os.path.join(HERE, "hier_2048_subvolume.npz"),
                        x_crop=hier_crop(res.x).astype(np.float32), history=np.array(hist),
                        restarts=np.array(rst, dtype=np.int64),
                        L=np.array([lv.L for lv in res.levels]), sino_sum=float(np.sum(sino)),
                        x_norm=float(np.linalg.norm(res.x)))
    print(f"hier: {time.time() - t0:.0f} s, restarts {rst}")


if __name__ == "__main__":
    what = sys.argv[1] if len(sys.argv) > 1 else "all"
    if what in ("slab", "all"):
        make_slab()
    if what in ("batch", "all"):
        make_batch()
    if what in ("hier", "all"):
        make_hier()
