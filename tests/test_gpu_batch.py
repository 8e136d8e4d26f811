"""Batched iteration of independent problems of uneven size (one persistent launch per
iteration over the pass tiles of every problem) against the same problems run one plan at a
time, and a small subset against the FP64 oracle.

The batched kernel groups rows and columns into tiles differently from the per-plan kernels,
which changes only the order of the float64 partial sums, so batched and per-plan results
agree to ~1e-7 (not bit for bit); parity with the oracle is <= 1e-4 after 20 iterations.
"""
import numpy as np
import pytest
import torch

from oracle import fbp as ofbp
from oracle import solver

from gpu_util import dev, make_plan, oracle_geom, oracle_prior, problem, rel_l2, to_dev, to_np

pytestmark = pytest.mark.gpu

PROBLEMS = [  # n, n_angles, seed   (P = 256, 512, 512, 1024, 256)
    (128, 40, 1), (192, 60, 2), (256, 33, 3), (384, 90, 4), (160, 120, 5),
]


def _setup():
    items = []
    for n, na, seed in PROBLEMS:
        nd = int(round(n * np.sqrt(2)))
        nd += nd & 1
        sino, ang, center, _ = problem(n, 1, na, nd, seed=seed, n_objects=6)
        items.append((n, na, nd, sino, ang))
    return items


def test_batch_matches_single_plans_and_oracle():
    from paper_2603_28756_amd import tomo
    iters = 20
    items = _setup()
    plans = [make_plan(n, 1, ang, nd, neighbours=8) for n, na, nd, sino, ang in items]
    batch = tomo.Batch(plans)
    sinos = [to_dev(it[3]) for it in items]
    xs = [torch.empty((1, it[0], it[0]), dtype=torch.float32, device=dev()) for it in items]
    stats = batch.reconstruct(sinos, xs, iters)
    assert stats["wait_timeouts"] == 0 and stats["n_nonfinite"] == 0
    got = [to_np(x) for x in xs]
    # repeat: the queue and counters reset themselves between launches and calls
    stats2 = batch.reconstruct(sinos, xs, iters)
    assert stats2["wait_timeouts"] == 0
    for g, x in zip(got, xs):
        assert rel_l2(to_np(x), g) < 1e-6
    for (n, na, nd, sino, ang), g in zip(items, got):
        single = make_plan(n, 1, ang, nd, neighbours=8)
        xx = torch.empty((1, n, n), dtype=torch.float32, device=dev())
        single.reconstruct(to_dev(sino), xx, [iters], init=tomo.INIT_FBP)
        assert rel_l2(g, to_np(xx)) < 1e-6
    for k in (0, 4):
        n, na, nd, sino, ang = items[k]
        geom = oracle_geom(n, ang, nd)
        prob = solver.build(geom, sino, oracle_prior(8), 0.01)
        ref = solver.fista(prob, ofbp.fbp(sino, geom), iters)
        assert rel_l2(got[k], ref.x) < 1e-4


def test_batch_rejects_unsupported_sizes():
    from paper_2603_28756_amd import tomo
    sino, ang, center, _ = problem(64, 1, 20, 92, seed=1)
    small = make_plan(64, 1, ang, 92, neighbours=8)   # P = 128
    with pytest.raises(tomo.TomoError):
        tomo.Batch([small])
