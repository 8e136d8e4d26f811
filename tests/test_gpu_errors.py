"""Failure handling through the C ABI on the GPU: non-finite data and starts are reported as
TOMO_ERR_NONFINITE (with the iteration), and call-order and workspace errors come back as their
status codes.  NaN and Inf are ordinary floating-point values to the kernels (no trap), so
these runs end normally; the library detects them in its float64 reductions.
"""
import ctypes

import numpy as np
import pytest
import torch

from gpu_util import dev, make_plan, problem, to_dev

pytestmark = pytest.mark.gpu


def _small():
    return problem(32, 2, 20, 46, seed=3)


@pytest.mark.parametrize("where", ["sinogram_nan", "sinogram_inf", "start_nan"])
def test_nonfinite_input_is_reported(where):
    from paper_2603_28756_amd import tomo
    sino, ang, c, _ = _small()
    sino = sino.copy()
    x = torch.zeros((2, 32, 32), dtype=torch.float32, device=dev())
    init = tomo.INIT_FBP
    if where == "sinogram_nan":
        sino[1, 5, 20] = np.nan
    elif where == "sinogram_inf":
        sino[0, 3, 10] = np.inf
    else:
        x[1, 7, 9] = float("nan")
        init = tomo.INIT_USER
    plan = make_plan(32, 2, ang, 46)
    with pytest.raises(tomo.TomoError) as ei:
        plan.reconstruct(to_dev(sino), x, [9], init=init)
    assert ei.value.status == tomo.TOMO_ERR_NONFINITE
    assert "iteration 0" in str(ei.value)
    # the same call without stats_host does not synchronise and reports nothing
    assert plan.reconstruct(to_dev(sino), x, [9], init=init, stats=False) is None


def test_finite_run_reports_no_nonfinite_iteration():
    from paper_2603_28756_amd import tomo
    sino, ang, c, _ = _small()
    plan = make_plan(32, 2, ang, 46)
    x = torch.empty((2, 32, 32), dtype=torch.float32, device=dev())
    st = plan.reconstruct(to_dev(sino), x, [9], init=tomo.INIT_FBP)
    assert st["nonfinite_iter"] == -1


def _raw_plan(lib, n=32, nz=2, na=20, nd=46):
    from paper_2603_28756_amd import tomo
    g = tomo.Geometry()
    g.n, g.n_slices, g.n_angles, g.n_det = n, nz, na, nd
    g.center = float("nan")
    g.kb_width, g.kb_oversamp, g.beta, g.p, g.q, g.sigma, g.T = 8, 2.0, 0.01, 1.2, 2.0, 0.1, 1.0
    g.neighbours = 26
    h = ctypes.c_void_p()
    st = lib.tomo_plan_create(ctypes.byref(g), None, ctypes.byref(h))
    assert st == tomo.TOMO_OK
    return h


def test_call_order_and_workspace_errors():
    from paper_2603_28756_amd import tomo
    lib = tomo.load_library()
    h = _raw_plan(lib)
    try:
        # no workspace attached yet
        assert lib.tomo_precompute_psf(h) == tomo.TOMO_ERR_NO_WORKSPACE
        x = torch.zeros((2, 32, 32), dtype=torch.float32, device=dev())
        out = torch.zeros_like(x)
        assert lib.tomo_apply_normal(h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr())) == \
            tomo.TOMO_ERR_NO_WORKSPACE
        need = ctypes.c_size_t()
        assert lib.tomo_plan_workspace_size(h, ctypes.byref(need)) == tomo.TOMO_OK
        buf = torch.empty(need.value + 512, dtype=torch.uint8, device=dev())
        base = buf.data_ptr() + (-buf.data_ptr()) % 256
        # too small, then misaligned, then correct
        assert lib.tomo_plan_set_workspace(h, ctypes.c_void_p(base), need.value - 256) == \
            tomo.TOMO_ERR_WORKSPACE_TOO_SMALL
        assert lib.tomo_plan_set_workspace(h, ctypes.c_void_p(base + 64), need.value) == \
            tomo.TOMO_ERR_INVALID_ARG
        assert lib.tomo_plan_set_workspace(h, ctypes.c_void_p(base), need.value) == tomo.TOMO_OK
        # the PSF spectrum is needed before the Toeplitz product
        assert lib.tomo_apply_normal(h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr())) == \
            tomo.TOMO_ERR_NOT_READY
        assert "PSF" in lib.tomo_last_error(h).decode()
        # misaligned device arrays are rejected
        assert lib.tomo_apply_normal(h, ctypes.c_void_p(x.data_ptr() + 4), ctypes.c_void_p(out.data_ptr())) == \
            tomo.TOMO_ERR_INVALID_ARG
        assert lib.tomo_precompute_psf(h) == tomo.TOMO_OK
        assert lib.tomo_apply_normal(h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr())) == \
            tomo.TOMO_OK
        # re-attaching a workspace invalidates the precomputed spectrum
        assert lib.tomo_plan_set_workspace(h, ctypes.c_void_p(base), need.value) == tomo.TOMO_OK
        assert lib.tomo_apply_normal(h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr())) == \
            tomo.TOMO_ERR_NOT_READY
        torch.cuda.synchronize()
    finally:
        lib.tomo_plan_destroy(h)


def test_batch_and_network_workspace_errors():
    from paper_2603_28756_amd import tomo
    lib = tomo.load_library()
    net = ctypes.c_void_p()
    assert lib.tomo_unet_create(2, 32, 1, 32, 32, None, ctypes.byref(net)) == tomo.TOMO_OK
    try:
        theta = torch.zeros(16, dtype=torch.float32, device=dev())
        assert lib.tomo_unet_set_params(net, ctypes.c_void_p(theta.data_ptr())) == tomo.TOMO_ERR_NO_WORKSPACE
        need = ctypes.c_size_t()
        assert lib.tomo_unet_workspace_size(net, ctypes.byref(need)) == tomo.TOMO_OK
        buf = torch.empty(need.value + 256, dtype=torch.uint8, device=dev())
        base = buf.data_ptr() + (-buf.data_ptr()) % 256
        assert lib.tomo_unet_set_workspace(net, ctypes.c_void_p(base), need.value - 1) == \
            tomo.TOMO_ERR_WORKSPACE_TOO_SMALL
        assert lib.tomo_unet_set_workspace(net, ctypes.c_void_p(base), need.value) == tomo.TOMO_OK
        img = torch.zeros((1, 32, 32), dtype=torch.float32, device=dev())
        assert lib.tomo_unet_forward(net, ctypes.c_void_p(img.data_ptr()), ctypes.c_void_p(img.data_ptr()), 1,
                                     ctypes.c_float(1.0)) == tomo.TOMO_ERR_NOT_READY
    finally:
        lib.tomo_unet_destroy(net)
    sino, ang, c, _ = problem(128, 1, 20, 182, seed=2)
    plan = make_plan(128, 1, ang, 182, neighbours=8)
    b = ctypes.c_void_p()
    arr = (ctypes.c_void_p * 1)(plan._h.value)
    assert lib.tomo_batch_create(arr, 1, None, ctypes.byref(b)) == tomo.TOMO_OK
    try:
        xs = (ctypes.c_void_p * 1)(0)
        assert lib.tomo_batch_reconstruct(b, xs, xs, 3, 1, None) == tomo.TOMO_ERR_NO_WORKSPACE
        need = ctypes.c_size_t()
        assert lib.tomo_batch_workspace_size(b, ctypes.byref(need)) == tomo.TOMO_OK
        buf = torch.empty(need.value + 256, dtype=torch.uint8, device=dev())
        base = buf.data_ptr() + (-buf.data_ptr()) % 256
        assert lib.tomo_batch_set_workspace(b, ctypes.c_void_p(base), need.value - 256) == \
            tomo.TOMO_ERR_WORKSPACE_TOO_SMALL
    finally:
        lib.tomo_batch_destroy(b)
