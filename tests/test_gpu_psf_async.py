"""The PSF precompute (spectrum F K and step constant L, Sec. 2.1) runs on a stream of the plan's
own beside the back-projections of the following reconstruction.  Its result must not depend
on that overlap: a reconstruction enqueued right behind the precompute equals one started after
the host waited for it, bit for bit, over repeated precompute + reconstruct steps (the spectrum
is rewritten while the previous step's graphs may still be queued)."""
import numpy as np
import pytest
import torch

from gpu_util import dev, make_plan, problem, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,nz,levels", [(128, 4, 1), (256, 3, 2)])
def test_overlapped_precompute_is_bit_identical(n, nz, levels):
    from paper_2603_28756_amd import tomo
    nd = int(round(n * np.sqrt(2)))
    nd += (-nd) % (2 ** levels)  # even bins on every level
    sino, ang, c, _ = problem(n, nz, 60, nd, seed=21)
    g = to_dev(sino)
    iters = [5] * (levels - 1) + [12]
    plan = make_plan(n, nz, ang, nd, n_levels=levels)
    x = torch.empty((nz, n, n), dtype=torch.float32, device=dev())
    # host waits for the precompute before the reconstruction is enqueued
    plan.precompute_psf()
    _, L_ref, lam_ref = plan.psf_info(with_spectrum=False)
    st = plan.reconstruct(g, x, iters, init=tomo.INIT_FBP)
    ref = to_np(x)
    assert st["L"][levels - 1] == L_ref and st["lambda_pow"][levels - 1] == lam_ref
    # enqueued back to back, several steps in a row, no host wait in between
    outs = []
    for _ in range(3):
        plan.precompute_psf()
        plan.reconstruct(g, x, iters, init=tomo.INIT_FBP, stats=False)
        outs.append(x.clone())
    torch.cuda.synchronize()
    for o in outs:
        assert np.array_equal(to_np(o), ref)
    # the constants read on the host after an overlapped step are the same
    _, L2, lam2 = plan.psf_info(with_spectrum=False)
    assert L2 == L_ref and lam2 == lam_ref


def test_gradient_and_normal_wait_for_the_precompute():
    from paper_2603_28756_amd import tomo  # noqa: F401
    n, nz = 128, 2
    nd = 182
    sino, ang, c, phantom = problem(n, nz, 45, nd, seed=22)
    plan = make_plan(n, nz, ang, nd)
    xd = to_dev(phantom.astype(np.float32))
    out1 = torch.empty_like(xd)
    out2 = torch.empty_like(xd)
    plan.precompute_psf()
    plan.apply_normal(xd, out1)          # enqueued right behind the precompute
    plan.precompute_psf()
    plan.psf_info(with_spectrum=False)   # host waits
    plan.apply_normal(xd, out2)
    torch.cuda.synchronize()
    assert np.array_equal(to_np(out1), to_np(out2))


def test_replayed_precompute_matches_direct_launches_and_follows_tile_changes():
    """The precompute of a level is captured once into a graph and replayed; launched one by
    one (kernel timing on), captured, replayed, and captured again after the tile variants
    change, it gives the same spectrum, lambda and L bit for bit."""
    from paper_2603_28756_amd import tomo
    n, nz, nd = 128, 2, 182
    _, ang, _, _ = problem(n, nz, 45, nd, seed=23)
    plan = make_plan(n, nz, ang, nd)
    plan.timing_enable(range(tomo.T_COUNT))  # direct launches
    plan.precompute_psf()
    fk0, L0, lam0 = plan.psf_info()
    plan.timing_enable([])
    runs = []
    for _ in range(2):  # captured, then replayed
        plan.precompute_psf()
        runs.append(plan.psf_info())
    sched = plan.tiles()
    sched[0].update({"rows_fwd": 0, "cols_conv": 2, "rows_inv": 0})
    plan.tiles(sched)
    plan.precompute_psf()  # captured again with the new tiles
    runs.append(plan.psf_info())
    for fk, L, lam in runs:
        assert np.array_equal(to_np(fk), to_np(fk0))
        assert L == L0 and lam == lam0
