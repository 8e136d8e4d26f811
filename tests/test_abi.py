"""C-ABI checks that need no GPU: the library loads, exports every symbol that
include/tomo.h declares, and its host-side validation rejects bad geometry with
TOMO_ERR_INVALID_ARG before any device call.  On a host without a GPU a valid
geometry is reported as TOMO_ERR_NO_DEVICE.
"""
import ctypes
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in sorted(os.listdir(os.path.join(ROOT, "include")))
           if f.endswith(".h")]


def _lib():
    from paper_2603_28756_amd import tomo
    if not os.path.exists(tomo.LIB_PATH):
        pytest.skip("libtomo.so not built (run __graft_entry__.build())")
    return tomo, tomo.load_library()


def _declared():
    text = "".join(open(h).read() for h in HEADERS)
    return sorted(set(re.findall(r"^(?:tomo_status|const char\*)\s+(tomo_\w+)\s*\(", text, re.M)))


def test_header_declares_entry_points():
    names = _declared()
    for required in ("tomo_plan_create", "tomo_precompute_psf", "tomo_gradient", "tomo_reconstruct",
                     "tomo_backproject", "tomo_plan_destroy", "tomo_autotune", "tomo_unet_create",
                     "tomo_unet_train_step", "tomo_unet_forward", "tomo_nn_conv3x3"):
        assert required in names


def test_library_exports_every_declared_symbol():
    tomo, lib = _lib()
    for name in _declared():
        assert hasattr(lib, name), name
        assert name in tomo.EXPORTS, f"binding lacks {name}"


def test_status_strings():
    _, lib = _lib()
    for s in range(10):
        assert lib.tomo_status_string(s).decode()
    assert lib.tomo_status_string(99).decode() == "unknown status"


def _geom(tomo, **kw):
    g = tomo.Geometry()
    g.n, g.n_slices, g.n_angles, g.n_det = 64, 2, 30, 92
    g.center = math.nan
    g.pad, g.n_levels, g.kb_width = 0, 1, 6
    g.kb_oversamp, g.kb_beta = 2.0, 0.0
    g.beta, g.p, g.q, g.sigma, g.T = 0.01, 1.2, 2.0, 0.1, 1.0
    g.neighbours, g.flags = 26, 0
    for k, v in kw.items():
        setattr(g, k, v)
    return g


@pytest.mark.parametrize("bad", [
    dict(n=15), dict(n=17), dict(n=4096), dict(n_slices=0), dict(n_angles=0), dict(n_det=91),
    dict(n_det=2), dict(pad=100), dict(pad=64), dict(n_levels=7), dict(n_levels=3, n=40),
    dict(n_levels=2, n_det=90), dict(kb_width=1), dict(kb_width=17), dict(kb_oversamp=1.0),
    dict(beta=-1.0), dict(p=0.9), dict(p=2.5), dict(q=1.5), dict(sigma=0.0), dict(T=-1.0),
    dict(neighbours=6), dict(flags=8), dict(center=math.inf),
])
def test_invalid_geometry_rejected_on_host(bad):
    tomo, lib = _lib()
    g = _geom(tomo, **bad)
    h = ctypes.c_void_p(123)
    st = lib.tomo_plan_create(ctypes.byref(g), None, ctypes.byref(h))
    assert st == 1, (bad, lib.tomo_last_error(None).decode())
    assert h.value is None
    assert lib.tomo_last_error(None).decode()


def test_null_arguments():
    tomo, lib = _lib()
    g = _geom(tomo)
    assert lib.tomo_plan_create(None, None, ctypes.byref(ctypes.c_void_p())) == 1
    assert lib.tomo_plan_create(ctypes.byref(g), None, None) == 1
    assert lib.tomo_plan_destroy(None) == 0
    assert lib.tomo_precompute_psf(None) == 1
    assert lib.tomo_lanczos_prolong(None, None, 8, 1, None) == 1


def test_valid_geometry_without_gpu_reports_no_device():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    tomo, lib = _lib()
    g = _geom(tomo)
    h = ctypes.c_void_p()
    assert lib.tomo_plan_create(ctypes.byref(g), None, ctypes.byref(h)) == 2


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2603_28756_amd import tomo
    monkeypatch.setattr(tomo, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(tomo, "_lib", None)
    with pytest.raises(ImportError):
        tomo.load_library()


@pytest.mark.parametrize("args", [
    (0, 32, 1, 64, 64), (7, 32, 1, 64, 64), (4, 16, 1, 64, 64), (4, 48, 1, 64, 64), (4, 32, 0, 64, 64),
    (4, 32, 1, 60, 64), (4, 32, 1, 64, 4), (6, 64, 1, 64, 64), (1, 288, 1, 64, 64),
    (1, 32, 1, 32768, 8),
])
def test_unet_create_rejects_bad_shapes(args):
    _, lib = _lib()
    h = ctypes.c_void_p(123)
    assert lib.tomo_unet_create(*args, None, ctypes.byref(h)) == 1
    assert h.value is None
    assert lib.tomo_unet_last_error(None).decode()


def test_unet_create_without_gpu_reports_no_device():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    _, lib = _lib()
    h = ctypes.c_void_p()
    assert lib.tomo_unet_create(4, 32, 2, 64, 64, None, ctypes.byref(h)) == 2


def test_nn_entry_points_validate_on_host():
    _, lib = _lib()
    p = ctypes.c_void_p(256)
    # cin not a multiple of 32, NULL arrays, misaligned pointers: rejected before any launch
    assert lib.tomo_nn_conv3x3(p, 48, p, None, p, 32, None, 0, 48, 32, 1, 4, 4, 0, None) == 1
    assert lib.tomo_nn_conv3x3(None, 32, p, None, p, 32, None, 0, 32, 32, 1, 4, 4, 0, None) == 1
    assert lib.tomo_nn_conv3x3(ctypes.c_void_p(258), 32, p, None, p, 32, None, 0, 32, 32, 1, 4, 4, 0, None) == 1
    assert lib.tomo_nn_conv3x3(p, 32, p, None, p, 32, None, 0, 32, 32, 1, 4, 4, 1, None) == 1  # ReLU needs bias
    assert lib.tomo_nn_conv3x3(p, 32, p, None, p, 36, None, 0, 32, 32, 1, 4, 4, 0, None) == 1  # ld % 8
    assert lib.tomo_nn_conv3x3(p, 32, p, None, p, 32, None, 0, 32, 32, 1, 32768, 4, 0, None) == 1  # H
    n = ctypes.c_size_t()
    assert lib.tomo_nn_wgrad_scratch(32, 64, 1000, ctypes.byref(n)) == 0 and n.value > 0
    assert lib.tomo_nn_wgrad_scratch(30, 64, 1000, ctypes.byref(n)) == 1
