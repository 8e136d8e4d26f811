"""What the trained network gains over the method without it (GPU, end to end).

512 training slices (ellipses + Gaussian texture, 128^2, 60 angles, 1% noise) are
reconstructed by the method itself (300 iterations from FBP) to make the targets; the
U-Net (3 levels, 32 base channels) is trained by its own GPU kernels; on 32 held-out
slices the learned start (TOMO_INIT_LEARNED, with its per-slice FBP fallback) must lower the
relative objective gap at the start and the number of iterations to a gap of 1e-4 compared
with the FBP start, keeping the network's start on nearly every slice.
"""
import numpy as np
import pytest
import torch

import synth

from gpu_util import dev

pytestmark = pytest.mark.gpu


def test_learned_start_beats_fbp_start():
    from paper_2603_28756_amd import learned, tomo
    n, na = 128, 60
    nd = synth.detector_bins_for(n)
    train_s = synth.textured_batch(512, n, na, nd, 0.01, 1000)
    test_s = synth.textured_batch(32, n, na, nd, 0.01, 900000)
    pr = learned.Problem(n, na, nd, synth.uniform_angles(na))
    fbp, tgt = learned.fbp_and_targets(pr, train_s, 300, dev())
    scale = float(torch.sqrt(torch.mean(fbp * fbp)).item())
    net = tomo.UNet(n, n, levels=3, base=32, max_batch=16)
    net.set_params(learned.init_params(3, 32, 1, dev()))
    losses = learned.train(net, fbp, tgt, scale, epochs=20, batch=16, lr=1e-3, seed=1)
    assert np.all(np.isfinite(losses))
    assert losses[-10:].mean() < 0.6 * losses[:10].mean()
    learned.record_domain(net, pr)
    res = learned.compare_starts(pr, test_s, net, scale, dev(), long_iters=1500)
    assert res["F_star_tail_change"] < 1e-3
    # the objective test inside tomo_reconstruct keeps the network's start on (nearly) every slice
    assert res["learned_slices"] >= 30
    assert res["gap_at_start"]["unet"] < 0.1 * res["gap_at_start"]["fbp"]
    assert res["iterations"]["fbp"] is not None and res["iterations"]["unet"] is not None
    assert res["iterations"]["unet"] < res["iterations"]["fbp"]
