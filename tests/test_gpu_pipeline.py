"""Streaming a volume through a smaller plan (include/tomo_pipeline.h; Sec. 2.4's three-thread
host/device pipeline).  With the 8-neighbour prior and no restart test the slices of a volume
iterate independently, so the streamed volume must equal the whole-volume reconstruction bit
for bit for every window layout and queue depth.  With the restart test, or with the
26-neighbour prior (slices coupled; `halo` context slices per window), each window is its own
solve: the difference to the whole-volume solve is reported and bounded, and for the
26-neighbour prior it shrinks as the halo grows.
"""
import numpy as np
import pytest
import torch

from gpu_util import dev, make_plan, problem, rel_l2, to_dev, to_np

pytestmark = pytest.mark.gpu

N, NA, ND = 96, 40, 136


def _volume(n_total, seed):
    sino, ang, c, _ = problem(N, n_total, NA, ND, seed=seed, n_objects=6)
    return np.ascontiguousarray(sino, dtype=np.float32), ang


def _whole(sino, ang, neighbours, iters, restart):
    from paper_2603_28756_amd import tomo
    nz = sino.shape[0]
    plan = make_plan(N, nz, ang, ND, neighbours=neighbours)
    x = torch.empty((nz, N, N), dtype=torch.float32, device=dev())
    plan.reconstruct(to_dev(sino), x, [iters], init=tomo.INIT_FBP, restart=restart)
    return to_np(x).astype(np.float32)


@pytest.mark.parametrize("nz,depth", [(4, 2), (3, 1), (5, 3)])
def test_streamed_8_neighbour_volume_equals_whole_volume(nz, depth):
    from paper_2603_28756_amd import tomo
    n_total, iters = 11, 15
    sino, ang = _volume(n_total, seed=31)
    ref = _whole(sino, ang, 8, iters, restart=False)
    plan = make_plan(N, nz, ang, ND, neighbours=8)
    pipe = tomo.Pipeline(plan, n_total, halo=0, depth=depth)
    x = np.full((n_total, N, N), np.nan, dtype=np.float32)
    st = pipe.run(sino, x, [iters], init=tomo.INIT_FBP, restart=False)
    assert st["n_windows"] == -(-n_total // nz) and st["nonfinite_window"] == -1
    assert np.array_equal(x, ref)
    # a second run through the same pipeline (slots and staging reused)
    x2 = np.zeros_like(x)
    pipe.run(sino, x2, [iters], init=tomo.INIT_FBP, restart=False, stats=False)
    assert np.array_equal(x2, ref)


def test_streamed_with_restart_is_close_to_whole_volume():
    from paper_2603_28756_amd import tomo
    n_total, iters = 9, 20
    sino, ang = _volume(n_total, seed=32)
    ref = _whole(sino, ang, 8, iters, restart=True)
    plan = make_plan(N, 3, ang, ND, neighbours=8)
    pipe = tomo.Pipeline(plan, n_total, halo=0, depth=2)
    x = np.empty((n_total, N, N), dtype=np.float32)
    st = pipe.run(sino, x, [iters], init=tomo.INIT_FBP, restart=True)
    err = rel_l2(x, ref)
    print(f"\n[pipeline] 8 neighbours, per-window restarts ({st['n_restarts']}): rel-L2 {err:.2e}")
    assert err < 1e-2


def test_streamed_26_neighbour_volume_approaches_whole_volume_with_halo():
    from paper_2603_28756_amd import tomo
    n_total, iters = 12, 20
    sino, ang = _volume(n_total, seed=33)
    ref = _whole(sino, ang, 26, iters, restart=False)
    errs = {}
    for halo, nz in ((0, 4), (1, 6), (2, 8)):
        plan = make_plan(N, nz, ang, ND, neighbours=26)
        pipe = tomo.Pipeline(plan, n_total, halo=halo, depth=2)
        x = np.empty((n_total, N, N), dtype=np.float32)
        pipe.run(sino, x, [iters], init=tomo.INIT_FBP, restart=False)
        errs[halo] = rel_l2(x, ref)
    print(f"\n[pipeline] 26 neighbours, rel-L2 to the whole volume by halo: "
          + ", ".join(f"{h}: {e:.2e}" for h, e in errs.items()))
    assert errs[2] < errs[0] and errs[1] < errs[0] and errs[2] < 1e-2


def test_pipeline_reports_nonfinite_window_and_argument_errors():
    from paper_2603_28756_amd import tomo
    n_total = 8
    sino, ang = _volume(n_total, seed=34)
    sino[5, 3, 7] = np.nan   # window 1 of 2 (4 slices each)
    plan = make_plan(N, 4, ang, ND, neighbours=8)
    pipe = tomo.Pipeline(plan, n_total, halo=0, depth=2)
    x = np.zeros((n_total, N, N), dtype=np.float32)
    with pytest.raises(tomo.TomoError) as e:
        pipe.run(sino, x, [5], init=tomo.INIT_FBP)
    assert e.value.status == tomo.TOMO_ERR_NONFINITE and "window 1" in str(e.value)
    with pytest.raises(tomo.TomoError) as e:
        pipe.run(sino, x, [5], init=tomo.INIT_USER)
    assert e.value.status == tomo.TOMO_ERR_INVALID_ARG
    with pytest.raises(tomo.TomoError) as e:
        tomo.Pipeline(plan, 3, halo=0)     # volume smaller than one window
    assert e.value.status == tomo.TOMO_ERR_INVALID_ARG
    with pytest.raises(tomo.TomoError) as e:
        tomo.Pipeline(plan, 8, halo=2)     # no interior slice left
    assert e.value.status == tomo.TOMO_ERR_INVALID_ARG
