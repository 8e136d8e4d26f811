"""The weight gradient without caller scratch against the entry point that takes scratch.

Both run the same kernels with the same fixed-order split sums, so the results must be
bit-identical; each is also held to the float64 oracle (relative L2 <= 1e-5, float32 sums of
exact bfloat16 products).  Two calls in a row, the second smaller (fewer splits, and the
per-tap kernel for a width that is not a multiple of 32), show that what the first call left
in the shared static scratch does not leak into the second.
"""
import numpy as np
import pytest
import torch

from oracle import unet as U

from gpu_util import dev

pytestmark = pytest.mark.gpu


def _bf(a) -> torch.Tensor:
    return torch.as_tensor(np.asarray(a, dtype=np.float32)).to(torch.bfloat16).to(dev())


def _np(t: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    return t.detach().float().cpu().numpy().astype(np.float64)


def _case(B, H, W, cin, cout, seed):
    rng = np.random.default_rng(seed)
    return _bf(rng.standard_normal((B, H, W, cout))), _bf(rng.standard_normal((B, H, W, cin)))


def test_wgrad_noalloc_matches_scratch_entry_point_twice():
    from paper_2603_28756_amd import tomo
    cases = [(2, 128, 128, 64, 64, 21), (1, 9, 40, 32, 96, 22)]
    for B, H, W, cin, cout, seed in cases:
        print(f"wgrad noalloc: B {B} H {H} W {W} cin {cin} cout {cout}", flush=True)
        dz, x = _case(B, H, W, cin, cout, seed)
        dw_ref, db_ref = tomo.nn_conv3x3_wgrad(dz, x, cin, cout)
        dw, db = tomo.nn_conv3x3_wgrad_noalloc(dz, x, cin, cout)
        assert torch.equal(dw, dw_ref) and torch.equal(db, db_ref)
        rw, rb = U.conv3x3_wgrad(_np(dz), _np(x))
        assert np.linalg.norm(_np(dw) - rw) / np.linalg.norm(rw) < 1e-5
        assert np.linalg.norm(_np(db) - rb) / np.linalg.norm(rb) < 1e-5


def test_wgrad_noalloc_rejects_oversized_split_sums():
    from paper_2603_28756_amd import tomo
    # 1024 x 1024 channels: one split of 1024 x (9 x 1024 + 1) floats, beyond the static array
    dz = torch.zeros((1, 1, 8, 1024), dtype=torch.bfloat16, device=dev())
    x = torch.zeros((1, 1, 8, 1024), dtype=torch.bfloat16, device=dev())
    with pytest.raises(tomo.TomoError) as ei:
        tomo.nn_conv3x3_wgrad_noalloc(dz, x, 1024, 1024)
    assert ei.value.status == tomo.TOMO_ERR_WORKSPACE_TOO_SMALL
