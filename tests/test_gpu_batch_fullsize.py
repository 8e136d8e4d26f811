"""The uneven batch at its real size: 256 independent single-slice problems with N drawn
from {128, 192, 256, 384, 512, 768, 1024}, 30..360 angles and 1..5% noise, advanced by one
persistent launch per iteration.  Every problem must stay finite with no tile wait timing
out; one problem of every size is compared with its own single plan (<= 1e-6, only the
float64 partial-sum order differs) and with the FP64 oracle (<= 1e-4): the smallest width
computed in the test, every width >= 192 against the stored oracle runs of
tests/golden/batch_sizes.npz (written by tests/golden/make_golden.py from oracle/ only).
"""
import os

import numpy as np
import pytest
import torch

import synth
from oracle import fbp as ofbp
from oracle import solver

from gpu_util import dev, oracle_geom, oracle_prior, rel_l2, to_np

pytestmark = pytest.mark.gpu


def _plan(p):
    from paper_2603_28756_amd import tomo
    return tomo.Plan(p["n"], 1, p["n_angles"], p["n_det"], angles=list(p["angles"]), kb_width=8,
                     neighbours=8, beta=0.01)


def test_uneven_batch_of_256():
    from paper_2603_28756_amd import tomo
    iters = 20
    probs = synth.uneven_problems(256, seed=4)
    plans = [_plan(p) for p in probs]
    batch = tomo.Batch(plans)
    sinos = [torch.from_numpy(p["sino"]).to(dev()) for p in probs]
    xs = [torch.empty((1, p["n"], p["n"]), dtype=torch.float32, device=dev()) for p in probs]
    st = batch.reconstruct(sinos, xs, iters)
    assert st["wait_timeouts"] == 0 and st["n_nonfinite"] == 0
    assert all(torch.isfinite(x).all().item() for x in xs)
    firsts = {}
    for j, p in enumerate(probs):
        firsts.setdefault(p["n"], j)
    for n, j in sorted(firsts.items()):
        single = _plan(probs[j])
        xx = torch.empty_like(xs[j])
        single.reconstruct(sinos[j], xx, [iters], init=tomo.INIT_FBP)
        assert rel_l2(to_np(xs[j]), to_np(xx)) < 1e-6, n
    j = min((k for k, p in enumerate(probs) if p["n"] == 128), key=lambda k: probs[k]["n_angles"])
    p = probs[j]
    sino = p["sino"].astype(np.float64)
    geom = oracle_geom(p["n"], p["angles"], p["n_det"])
    prob = solver.build(geom, sino, oracle_prior(8), 0.01)
    ref = solver.fista(prob, ofbp.fbp(sino, geom), iters)
    assert rel_l2(to_np(xs[j]), ref.x) < 1e-4
    gold = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "batch_sizes.npz"))
    checked = []
    for n, j in sorted(firsts.items()):
        if n < 192:
            continue
        s_ref = float(gold[f"sino_sum_{j}"])
        assert abs(float(np.sum(probs[j]["sino"].astype(np.float64))) - s_ref) <= 1e-9 * abs(s_ref)
        err = rel_l2(to_np(xs[j]), gold[f"x_{j}"])
        print(f"batch problem {j}: N {n}, {probs[j]['n_angles']} angles: rel-L2 vs oracle {err:.3e}",
              flush=True)
        assert err < 1e-4, (n, err)
        checked.append(n)
    assert checked == [192, 256, 384, 512, 768, 1024]
