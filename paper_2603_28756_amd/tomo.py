"""ctypes binding of libtomo (the C ABI declared in include/tomo.h).

Argument marshalling only: every numerical step runs in the library's HIP
kernels.  PyTorch supplies device memory (tensors, the workspace) and the HIP
stream.  If the shared library has not been built, importing the binding's
functions raises; there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libtomo.so")

TOMO_OK = 0
(TOMO_ERR_INVALID_ARG, TOMO_ERR_NO_DEVICE, TOMO_ERR_UNSUPPORTED_ARCH, TOMO_ERR_NO_WORKSPACE,
 TOMO_ERR_WORKSPACE_TOO_SMALL, TOMO_ERR_NOT_READY, TOMO_ERR_HIP, TOMO_ERR_NONFINITE,
 TOMO_ERR_INTERNAL) = range(1, 10)
STATUS_NAMES = {
    0: "OK", 1: "INVALID_ARG", 2: "NO_DEVICE", 3: "UNSUPPORTED_ARCH", 4: "NO_WORKSPACE",
    5: "WORKSPACE_TOO_SMALL", 6: "NOT_READY", 7: "HIP", 8: "NONFINITE", 9: "INTERNAL",
}
INIT_FBP, INIT_ZERO, INIT_USER, INIT_LEARNED = 0, 1, 2, 3
LEARNED_NOT_REQUESTED, LEARNED_TESTED, LEARNED_OUT_OF_DOMAIN = 0, 1, 2
T_ROWS_FWD, T_COLS_CONV, T_ROWS_INV, T_FINALIZE, T_BACKPROJECT, T_PSF, T_PRIOR, T_COUNT = range(8)
FLAG_NO_GRAPH = 1
FLAG_FUSED_PRIOR = 2
FLAG_CONCURRENT_PRIOR = 4


class TomoError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"tomo status {STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class Geometry(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32), ("n_slices", ctypes.c_int32), ("n_angles", ctypes.c_int32),
        ("n_det", ctypes.c_int32), ("angles", ctypes.POINTER(ctypes.c_double)),
        ("center", ctypes.c_double), ("pad", ctypes.c_int32), ("n_levels", ctypes.c_int32),
        ("kb_width", ctypes.c_int32), ("kb_oversamp", ctypes.c_double), ("kb_beta", ctypes.c_double),
        ("beta", ctypes.c_double), ("p", ctypes.c_double), ("q", ctypes.c_double),
        ("sigma", ctypes.c_double), ("T", ctypes.c_double), ("neighbours", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
    ]


class ReconOpts(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.POINTER(ctypes.c_int32)), ("init", ctypes.c_int32),
        ("restart", ctypes.c_int32), ("L_override", ctypes.c_double),
        ("objective_dev", ctypes.c_void_p), ("restart_dev", ctypes.c_void_p),
        ("unet", ctypes.c_void_p), ("unet_scale", ctypes.c_float), ("init_choice_dev", ctypes.c_void_p),
    ]


class ReconStats(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_double * 6), ("lambda_pow", ctypes.c_double * 6),
        ("n_restarts", ctypes.c_int32), ("nonfinite_iter", ctypes.c_int32),
        ("learned_state", ctypes.c_int32), ("learned_slices", ctypes.c_int32),
    ]


class UnetDomain(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32), ("n_det", ctypes.c_int32), ("n_angles_min", ctypes.c_int32),
        ("n_angles_max", ctypes.c_int32), ("center", ctypes.c_double), ("beta", ctypes.c_double),
        ("p", ctypes.c_double), ("sigma", ctypes.c_double), ("T", ctypes.c_double),
        ("neighbours", ctypes.c_int32),
    ]


class PipelineStats(ctypes.Structure):
    _fields_ = [
        ("n_windows", ctypes.c_int32), ("nonfinite_window", ctypes.c_int32),
        ("n_restarts", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("wall_ms", ctypes.c_double), ("upload_ms", ctypes.c_double),
        ("compute_ms", ctypes.c_double), ("download_ms", ctypes.c_double),
    ]


class BatchStats(ctypes.Structure):
    _fields_ = [("n_nonfinite", ctypes.c_int32), ("n_restarts", ctypes.c_int32),
                ("wait_timeouts", ctypes.c_int32)]


BATCH_MAX_SIZES = 8


class BatchSchedule(ctypes.Structure):
    _fields_ = [("n_sizes", ctypes.c_int32), ("pad", ctypes.c_int32 * BATCH_MAX_SIZES),
                ("elems", ctypes.c_int32 * BATCH_MAX_SIZES), ("group", ctypes.c_int32 * BATCH_MAX_SIZES),
                ("fused_prior", ctypes.c_int32),
                ("iter_ms", ctypes.c_float), ("base_ms", ctypes.c_float),
                ("phase_launches", ctypes.c_int32)]

    def as_dict(self) -> dict:
        k = self.n_sizes
        return {"sizes": {int(self.pad[i]): int(self.elems[i]) for i in range(k)},
                "group": {int(self.pad[i]): int(self.group[i]) for i in range(k)},
                "fused_prior": bool(self.fused_prior),
                "phase_launches": bool(self.phase_launches),
                "iter_ms": float(self.iter_ms), "base_ms": float(self.base_ms)}


class Tiles(ctypes.Structure):
    _fields_ = [("rows_fwd", ctypes.c_int32), ("cols_conv", ctypes.c_int32), ("rows_inv", ctypes.c_int32),
                ("fwd_pairs", ctypes.c_int32), ("col_tile", ctypes.c_int32), ("inv_pairs", ctypes.c_int32),
                ("ms", (ctypes.c_float * 3) * 3), ("chunks", ctypes.c_int32),
                ("ms_chunks", ctypes.c_float * 3)]

    def as_dict(self) -> dict:
        return {"rows_fwd": self.rows_fwd, "cols_conv": self.cols_conv, "rows_inv": self.rows_inv,
                "fwd_pairs": self.fwd_pairs, "col_tile": self.col_tile, "inv_pairs": self.inv_pairs,
                "chunks": self.chunks, "ms_chunks": [float(v) for v in self.ms_chunks],
                "ms": [[float(self.ms[i][j]) for j in range(3)] for i in range(3)]}


EXPORTS = {
    "tomo_plan_create": ([ctypes.POINTER(Geometry), ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
    "tomo_plan_workspace_size": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "tomo_plan_set_workspace": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t], ctypes.c_int),
    "tomo_precompute_psf": ([ctypes.c_void_p], ctypes.c_int),
    "tomo_backproject": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int], ctypes.c_int),
    "tomo_apply_normal": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "tomo_gradient": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "tomo_forward_project": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "tomo_gradient_direct": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
                             ctypes.c_int),
    "tomo_reconstruct": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ReconOpts),
                          ctypes.POINTER(ReconStats)], ctypes.c_int),
    "tomo_psf_info": ([ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                       ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "tomo_level_dims": ([ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                         ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "tomo_lanczos_prolong": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p],
                             ctypes.c_int),
    "tomo_timing_enable": ([ctypes.c_void_p, ctypes.c_uint32], ctypes.c_int),
    "tomo_timing_read": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)],
                         ctypes.c_int),
    "tomo_autotune": ([ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(Tiles)], ctypes.c_int),
    "tomo_tiles": ([ctypes.c_void_p, ctypes.POINTER(Tiles), ctypes.POINTER(Tiles)], ctypes.c_int),
    "tomo_plan_destroy": ([ctypes.c_void_p], ctypes.c_int),
    "tomo_batch_create": ([ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32, ctypes.c_void_p,
                           ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
    "tomo_batch_workspace_size": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "tomo_batch_set_workspace": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t], ctypes.c_int),
    "tomo_batch_reconstruct": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
                                ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(BatchStats)], ctypes.c_int),
    "tomo_batch_autotune": ([ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(BatchSchedule)], ctypes.c_int),
    "tomo_batch_schedule": ([ctypes.c_void_p, ctypes.POINTER(BatchSchedule), ctypes.POINTER(BatchSchedule)],
                            ctypes.c_int),
    "tomo_batch_destroy": ([ctypes.c_void_p], ctypes.c_int),
    "tomo_plan_geometry": ([ctypes.c_void_p, ctypes.POINTER(Geometry), ctypes.POINTER(ctypes.c_void_p),
                            ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "tomo_pipeline_window": ([ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                              ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                              ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "tomo_pipeline_create": ([ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                              ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
    "tomo_pipeline_workspace_size": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "tomo_pipeline_set_workspace": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t], ctypes.c_int),
    "tomo_pipeline_run": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ReconOpts),
                           ctypes.POINTER(PipelineStats)], ctypes.c_int),
    "tomo_pipeline_last_error": ([ctypes.c_void_p], ctypes.c_char_p),
    "tomo_pipeline_destroy": ([ctypes.c_void_p], ctypes.c_int),
    "tomo_unet_create": ([ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                          ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
    "tomo_unet_workspace_size": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "tomo_unet_set_workspace": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t], ctypes.c_int),
    "tomo_unet_num_params": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "tomo_unet_set_params": ([ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "tomo_unet_get_params": ([ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "tomo_unet_forward": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_float],
                          ctypes.c_int),
    "tomo_unet_loss_grad": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_float,
                             ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "tomo_unet_train_step": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_float,
                              ctypes.c_float, ctypes.c_void_p], ctypes.c_int),
    "tomo_unet_set_domain": ([ctypes.c_void_p, ctypes.POINTER(UnetDomain)], ctypes.c_int),
    "tomo_unet_destroy": ([ctypes.c_void_p], ctypes.c_int),
    "tomo_unet_last_error": ([ctypes.c_void_p], ctypes.c_char_p),
    "tomo_nn_conv3x3": ([ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                         ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                         ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p],
                        ctypes.c_int),
    "tomo_nn_wgrad_scratch": ([ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)],
                              ctypes.c_int),
    "tomo_nn_conv3x3_wgrad": ([ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                               ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                               ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p], ctypes.c_int),
    "tomo_nn_conv3x3_wgrad_noalloc": ([ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p],
                                      ctypes.c_int),
    "tomo_status_string": ([ctypes.c_int], ctypes.c_char_p),
    "tomo_last_error": ([ctypes.c_void_p], ctypes.c_char_p),
}

_lib = None


def load_library() -> ctypes.CDLL:
    """Load libtomo.so from the package's lib/ directory; raise if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2603_28756_amd.build` "
            "(there is no non-HIP implementation)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (argt, rest) in EXPORTS.items():
        fn = getattr(lib, name)
        fn.argtypes = argt
        fn.restype = rest
    _lib = lib
    return lib


def _check(status: int, plan=None):
    if status != TOMO_OK:
        lib = load_library()
        msg = lib.tomo_last_error(plan).decode()
        raise TomoError(status, msg)


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def _stream_ptr(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Plan:
    """One geometry/prior configuration bound to a device stream and a workspace tensor."""

    def __init__(self, n: int, n_slices: int, n_angles: int, n_det: int,
                 angles: Optional[Sequence[float]] = None, center: Optional[float] = None,
                 pad: int = 0, n_levels: int = 1, kb_width: int = 6, kb_oversamp: float = 2.0,
                 kb_beta: float = 0.0, beta: float = 0.01, p: float = 1.2, q: float = 2.0,
                 sigma: float = 0.1, T: float = 1.0, neighbours: int = 26, stream=None,
                 device: Optional[torch.device] = None, graphs: bool = True,
                 fused_prior: bool = False, concurrent_prior: bool = False):
        lib = load_library()
        self._lib = lib
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else device
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._angles = None
        g = Geometry()
        g.n, g.n_slices, g.n_angles, g.n_det = n, n_slices, n_angles, n_det
        if angles is not None:
            self._angles = (ctypes.c_double * n_angles)(*[float(a) for a in angles])
            g.angles = ctypes.cast(self._angles, ctypes.POINTER(ctypes.c_double))
        g.center = math.nan if center is None else float(center)
        g.pad, g.n_levels, g.kb_width = pad, n_levels, kb_width
        g.kb_oversamp, g.kb_beta = kb_oversamp, kb_beta
        g.beta, g.p, g.q, g.sigma, g.T = beta, p, q, sigma, T
        g.neighbours = neighbours
        g.flags = (0 if graphs else FLAG_NO_GRAPH) | (FLAG_FUSED_PRIOR if fused_prior else 0) | (
            FLAG_CONCURRENT_PRIOR if concurrent_prior else 0)
        self.geometry = g
        self.n, self.n_slices, self.n_angles, self.n_det = n, n_slices, n_angles, n_det
        self.n_levels = n_levels
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib.tomo_plan_create(ctypes.byref(g), _stream_ptr(self.stream), ctypes.byref(h)))
        self._h = h
        sz = ctypes.c_size_t()
        _check(lib.tomo_plan_workspace_size(self._h, ctypes.byref(sz)), self._h)
        self.workspace_bytes = sz.value
        # 256-byte aligned caller-owned workspace
        self._ws = torch.empty(sz.value + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        off = (-base) % 256
        _check(lib.tomo_plan_set_workspace(self._h, ctypes.c_void_p(base + off), sz.value), self._h)

    # ------------------------------------------------------------------ lifecycle
    def close(self):
        if getattr(self, "_h", None):
            self._lib.tomo_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ calls
    def precompute_psf(self):
        _check(self._lib.tomo_precompute_psf(self._h), self._h)

    def backproject(self, sino: torch.Tensor, out: torch.Tensor, ramp: bool = False):
        _check(self._lib.tomo_backproject(self._h, _ptr(sino), _ptr(out), int(ramp)), self._h)

    def apply_normal(self, x: torch.Tensor, out: torch.Tensor):
        _check(self._lib.tomo_apply_normal(self._h, _ptr(x), _ptr(out)), self._h)

    def gradient(self, x: torch.Tensor, b: torch.Tensor, grad: torch.Tensor,
                 obj: Optional[torch.Tensor] = None):
        _check(self._lib.tomo_gradient(self._h, _ptr(x), _ptr(b), _ptr(grad), _ptr(obj)), self._h)

    def forward_project(self, x: torch.Tensor, out: torch.Tensor):
        _check(self._lib.tomo_forward_project(self._h, _ptr(x), _ptr(out)), self._h)

    def gradient_direct(self, x: torch.Tensor, sino: torch.Tensor, grad: torch.Tensor,
                        obj: Optional[torch.Tensor] = None):
        _check(self._lib.tomo_gradient_direct(self._h, _ptr(x), _ptr(sino), _ptr(grad), _ptr(obj)),
               self._h)

    def reconstruct(self, sino: torch.Tensor, x: torch.Tensor, iters: Sequence[int],
                    init: int = INIT_FBP, restart: bool = True, L_override: float = 0.0,
                    objective: Optional[torch.Tensor] = None,
                    restarts: Optional[torch.Tensor] = None, stats: bool = True,
                    unet: Optional["UNet"] = None, unet_scale: float = 0.0,
                    init_choice: Optional[torch.Tensor] = None):
        it = (ctypes.c_int32 * len(iters))(*[int(i) for i in iters])
        o = ReconOpts()
        o.iters = ctypes.cast(it, ctypes.POINTER(ctypes.c_int32))
        o.init, o.restart, o.L_override = init, int(restart), float(L_override)
        o.objective_dev = _ptr(objective)
        o.restart_dev = _ptr(restarts)
        o.unet = unet._h.value if unet is not None else None
        o.unet_scale = float(unet_scale)
        o.init_choice_dev = _ptr(init_choice)
        st = ReconStats() if stats else None
        status = self._lib.tomo_reconstruct(self._h, _ptr(sino), _ptr(x), ctypes.byref(o),
                                            ctypes.byref(st) if st is not None else None)
        _check(status, self._h)
        if st is None:
            return None
        return {"L": list(st.L)[: self.n_levels], "lambda_pow": list(st.lambda_pow)[: self.n_levels],
                "n_restarts": st.n_restarts, "nonfinite_iter": st.nonfinite_iter,
                "learned_state": st.learned_state, "learned_slices": st.learned_slices}

    def psf_info(self, level: int = -1, with_spectrum: bool = True):
        level = self.n_levels - 1 if level < 0 else level
        n, nd, pad = self.level_dims(level)
        fk = torch.empty((pad, pad // 2 + 1), dtype=torch.float32, device=self.device) if with_spectrum else None
        L = ctypes.c_double()
        lam = ctypes.c_double()
        _check(self._lib.tomo_psf_info(self._h, level, _ptr(fk), ctypes.byref(L), ctypes.byref(lam)), self._h)
        return fk, L.value, lam.value

    def timing_enable(self, classes: Sequence[int]):
        mask = 0
        for c in classes:
            mask |= 1 << int(c)
        _check(self._lib.tomo_timing_enable(self._h, mask), self._h)

    def timing_read(self):
        ms = (ctypes.c_double * T_COUNT)()
        cnt = (ctypes.c_int64 * T_COUNT)()
        _check(self._lib.tomo_timing_read(self._h, ms, cnt), self._h)
        return list(ms), list(cnt)

    def autotune(self, reps: int = 5) -> list:
        """Time the tile variants of the three passes per level and keep the fastest."""
        out = (Tiles * self.n_levels)()
        _check(self._lib.tomo_autotune(self._h, reps, out), self._h)
        return [t.as_dict() for t in out]

    def tiles(self, set_to: Optional[Sequence[dict]] = None) -> list:
        """Set (list of {rows_fwd, cols_conv, rows_inv[, chunks]} per level) and return the schedule."""
        arg = None
        if set_to is not None:
            arg = (Tiles * self.n_levels)()
            for i, d in enumerate(set_to):
                arg[i].rows_fwd, arg[i].cols_conv, arg[i].rows_inv = (
                    int(d["rows_fwd"]), int(d["cols_conv"]), int(d["rows_inv"]))
                arg[i].chunks = int(d.get("chunks", 1))
        out = (Tiles * self.n_levels)()
        _check(self._lib.tomo_tiles(self._h, arg, out), self._h)
        return [t.as_dict() for t in out]

    def level_dims(self, level: int):
        n, nd, pad = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(self._lib.tomo_level_dims(self._h, level, ctypes.byref(n), ctypes.byref(nd), ctypes.byref(pad)),
               self._h)
        return n.value, nd.value, pad.value


def lanczos_prolong(x: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """2x Lanczos-3 prolongation of each slice of x [n_z, n, n] (HIP kernel)."""
    lib = load_library()
    nz, n, n2 = x.shape
    assert n == n2
    if out is None:
        out = torch.empty((nz, 2 * n, 2 * n), dtype=torch.float32, device=x.device)
    _check(lib.tomo_lanczos_prolong(_ptr(x), _ptr(out), n, nz, _stream_ptr(stream)))
    return out


def pipeline_window(n_total: int, n_slices: int, halo: int, k: int):
    """(first, keep0, keep1, n_windows) of window k (host arithmetic of include/tomo_pipeline.h)."""
    lib = load_library()
    f, a, b, w = (ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32())
    st = lib.tomo_pipeline_window(int(n_total), int(n_slices), int(halo), int(k), ctypes.byref(f),
                                  ctypes.byref(a), ctypes.byref(b), ctypes.byref(w))
    if st != TOMO_OK:
        raise TomoError(st, lib.tomo_pipeline_last_error(None).decode())
    return f.value, a.value, b.value, w.value


class Pipeline:
    """A volume of n_total slices in host memory streamed through `plan` (window = the plan's
    n_slices, `halo` context slices per side, `depth` windows in flight): include/tomo_pipeline.h.
    The device workspace of the window slots is a torch tensor owned by this object."""

    def __init__(self, plan: "Plan", n_total: int, halo: int = 0, depth: int = 2):
        lib = load_library()
        self._lib = lib
        self.plan = plan
        self.n_total, self.halo, self.depth = int(n_total), int(halo), int(depth)
        h = ctypes.c_void_p()
        with torch.cuda.device(plan.device):
            st = lib.tomo_pipeline_create(plan._h, self.n_total, self.halo, self.depth, ctypes.byref(h))
        if st != TOMO_OK:
            raise TomoError(st, lib.tomo_pipeline_last_error(None).decode())
        self._h = h
        sz = ctypes.c_size_t()
        self._pcheck(lib.tomo_pipeline_workspace_size(self._h, ctypes.byref(sz)))
        self._ws = torch.empty(sz.value + 256, dtype=torch.uint8, device=plan.device)
        base = self._ws.data_ptr()
        self._pcheck(lib.tomo_pipeline_set_workspace(self._h, ctypes.c_void_p(base + (-base) % 256), sz.value))

    def _pcheck(self, status: int):
        if status != TOMO_OK:
            raise TomoError(status, self._lib.tomo_pipeline_last_error(self._h).decode())

    def run(self, sino: "np.ndarray", x: "np.ndarray", iters: Sequence[int], init: int = INIT_FBP,
            restart: bool = True, L_override: float = 0.0, stats: bool = True,
            unet: Optional["UNet"] = None, unet_scale: float = 0.0):
        """sino [n_total][n_angles][n_det] and x [n_total][N][N]: C-contiguous float32 host arrays."""
        import numpy as np
        for a in (sino, x):
            if not (isinstance(a, np.ndarray) and a.dtype == np.float32 and a.flags["C_CONTIGUOUS"]):
                raise TypeError("expected C-contiguous float32 numpy arrays")
        g = self.plan
        if sino.shape != (self.n_total, g.n_angles, g.n_det) or x.shape != (self.n_total, g.n, g.n):
            raise ValueError("array shapes do not match the pipeline's volume")
        if not x.flags["WRITEABLE"]:
            raise ValueError("x must be writeable")
        it = (ctypes.c_int32 * len(iters))(*[int(i) for i in iters])
        o = ReconOpts()
        o.iters = ctypes.cast(it, ctypes.POINTER(ctypes.c_int32))
        o.init, o.restart, o.L_override = init, int(restart), float(L_override)
        o.unet = unet._h.value if unet is not None else None
        o.unet_scale = float(unet_scale)
        st = PipelineStats() if stats else None
        torch.cuda.current_stream(g.device).synchronize()  # device work queued before the call
        self._pcheck(self._lib.tomo_pipeline_run(self._h, ctypes.c_void_p(sino.ctypes.data),
                                                 ctypes.c_void_p(x.ctypes.data), ctypes.byref(o),
                                                 ctypes.byref(st) if st is not None else None))
        if st is None:
            return None
        return {k: getattr(st, k) for k, _ in PipelineStats._fields_ if k != "reserved"}

    def close(self):
        if getattr(self, "_h", None):
            self._lib.tomo_pipeline_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Independent single-level plans advanced together, one persistent launch per iteration."""

    def __init__(self, plans: Sequence[Plan], stream=None):
        lib = load_library()
        self._lib = lib
        self.plans = list(plans)
        self.device = self.plans[0].device
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        arr = (ctypes.c_void_p * len(self.plans))(*[p._h.value for p in self.plans])
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib.tomo_batch_create(arr, len(self.plans), _stream_ptr(self.stream), ctypes.byref(h)))
        self._h = h
        sz = ctypes.c_size_t()
        _check(lib.tomo_batch_workspace_size(self._h, ctypes.byref(sz)))
        self._ws = torch.empty(sz.value + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        _check(lib.tomo_batch_set_workspace(self._h, ctypes.c_void_p(base + (-base) % 256), sz.value))

    def reconstruct(self, sinos: Sequence[torch.Tensor], xs: Sequence[torch.Tensor], iters: int,
                    restart: bool = True):
        n = len(self.plans)
        sp = (ctypes.c_void_p * n)(*[t.data_ptr() for t in sinos])
        xp = (ctypes.c_void_p * n)(*[t.data_ptr() for t in xs])
        for t in list(sinos) + list(xs):
            _ptr(t)
        st = BatchStats()
        _check(self._lib.tomo_batch_reconstruct(self._h, sp, xp, int(iters), int(restart), ctypes.byref(st)))
        return {"n_nonfinite": st.n_nonfinite, "n_restarts": st.n_restarts,
                "wait_timeouts": st.wait_timeouts}

    def autotune(self, reps: int = 5) -> dict:
        out = BatchSchedule()
        _check(self._lib.tomo_batch_autotune(self._h, int(reps), ctypes.byref(out)))
        return out.as_dict()

    def schedule(self, set_to: Optional[dict] = None, fused_prior: bool = False,
                 group: Optional[dict] = None, phase_launches: bool = False) -> dict:
        """Read (and with set_to = {pad: elems} first set, with the prior scheme, the tiles per
        item {pad: group}, default 8, and the launch scheme) the schedule."""
        st = None
        if set_to is not None:
            st = BatchSchedule()
            st.fused_prior = int(fused_prior)
            st.phase_launches = int(phase_launches)
            st.n_sizes = len(set_to)
            for i, (p, e) in enumerate(sorted(set_to.items())):
                st.pad[i], st.elems[i] = int(p), int(e)
                st.group[i] = int((group or {}).get(p, 8))
        out = BatchSchedule()
        _check(self._lib.tomo_batch_schedule(self._h, ctypes.byref(st) if st is not None else None,
                                             ctypes.byref(out)))
        return out.as_dict()

    def close(self):
        if getattr(self, "_h", None):
            self._lib.tomo_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------------------- learned start
def _unet_check(status: int, h):
    if status != TOMO_OK:
        lib = load_library()
        raise TomoError(status, lib.tomo_unet_last_error(h).decode())


def _bf16_ptr(t: torch.Tensor) -> int:
    if t.dtype != torch.bfloat16 or t.device.type != "cuda":
        raise TypeError("expected a bfloat16 device tensor")
    return t.data_ptr()


class UNet:
    """U-Net learned start (include/tomo_nn.h): parameters, forward, loss/gradient, Adam."""

    def __init__(self, height: int, width: int, levels: int = 4, base: int = 32, max_batch: int = 1,
                 device=None, stream=None):
        self._lib = load_library()
        self.device = torch.device(device) if device is not None else torch.device("cuda", 0)
        self.height, self.width, self.levels, self.base, self.max_batch = height, width, levels, base, max_batch
        st = stream if stream is not None else torch.cuda.current_stream(self.device).cuda_stream
        h = ctypes.c_void_p()
        _unet_check(self._lib.tomo_unet_create(levels, base, max_batch, height, width, ctypes.c_void_p(st),
                                               ctypes.byref(h)), None)
        self._h = h
        nbytes = ctypes.c_size_t()
        _unet_check(self._lib.tomo_unet_workspace_size(h, ctypes.byref(nbytes)), h)
        self._ws = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        _unet_check(self._lib.tomo_unet_set_workspace(h, ctypes.c_void_p(self._ws.data_ptr()), nbytes.value), h)
        n = ctypes.c_int64()
        _unet_check(self._lib.tomo_unet_num_params(h, ctypes.byref(n)), h)
        self.n_params = n.value
        self._loss = torch.zeros(1, dtype=torch.float64, device=self.device)

    def __del__(self):
        if getattr(self, "_h", None) is not None and self._lib is not None:
            self._lib.tomo_unet_destroy(self._h)
            self._h = None

    def set_domain(self, n: int, n_det: int, n_angles_min: int, n_angles_max: int, beta: float,
                   p: float = 1.2, sigma: float = 0.1, T: float = 1.0, neighbours: int = 8,
                   center: Optional[float] = None):
        """Record the training domain (tomo_unet_domain_t) the learned start is used in."""
        d = UnetDomain(int(n), int(n_det), int(n_angles_min), int(n_angles_max),
                       float("nan") if center is None else float(center), float(beta), float(p),
                       float(sigma), float(T), int(neighbours))
        _unet_check(self._lib.tomo_unet_set_domain(self._h, ctypes.byref(d)), self._h)

    def clear_domain(self):
        _unet_check(self._lib.tomo_unet_set_domain(self._h, None), self._h)

    def set_params(self, theta: torch.Tensor):
        t = theta.to(device=self.device, dtype=torch.float32).contiguous()
        if t.numel() != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters, got {t.numel()}")
        _unet_check(self._lib.tomo_unet_set_params(self._h, ctypes.c_void_p(t.data_ptr())), self._h)
        torch.cuda.synchronize(self.device)

    def params(self) -> torch.Tensor:
        out = torch.empty(self.n_params, dtype=torch.float32, device=self.device)
        _unet_check(self._lib.tomo_unet_get_params(self._h, ctypes.c_void_p(out.data_ptr())), self._h)
        return out

    def _img(self, t: torch.Tensor) -> torch.Tensor:
        if t.dtype != torch.float32 or t.device.type != "cuda" or not t.is_contiguous():
            raise TypeError("images must be contiguous float32 device tensors")
        if tuple(t.shape[-2:]) != (self.height, self.width):
            raise ValueError("image size differs from the network's")
        return t

    def forward(self, fbp: torch.Tensor, scale: float, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        fbp = self._img(fbp)
        b = fbp.numel() // (self.height * self.width)
        out = torch.empty_like(fbp) if out is None else self._img(out)
        _unet_check(self._lib.tomo_unet_forward(self._h, ctypes.c_void_p(fbp.data_ptr()),
                                                ctypes.c_void_p(out.data_ptr()), b, float(scale)), self._h)
        return out

    def loss_grad(self, fbp: torch.Tensor, target: torch.Tensor, scale: float):
        fbp, target = self._img(fbp), self._img(target)
        b = fbp.numel() // (self.height * self.width)
        g = torch.empty(self.n_params, dtype=torch.float32, device=self.device)
        _unet_check(self._lib.tomo_unet_loss_grad(self._h, ctypes.c_void_p(fbp.data_ptr()),
                                                  ctypes.c_void_p(target.data_ptr()), b, float(scale),
                                                  ctypes.c_void_p(g.data_ptr()),
                                                  ctypes.c_void_p(self._loss.data_ptr())), self._h)
        return float(self._loss.item()), g

    def train_step(self, fbp: torch.Tensor, target: torch.Tensor, scale: float, lr: float,
                   loss_out: Optional[torch.Tensor] = None):
        """One Adam step; the batch loss (before the step) goes to loss_out[0] (float64) if given."""
        fbp, target = self._img(fbp), self._img(target)
        b = fbp.numel() // (self.height * self.width)
        lp = loss_out.data_ptr() if loss_out is not None else self._loss.data_ptr()
        _unet_check(self._lib.tomo_unet_train_step(self._h, ctypes.c_void_p(fbp.data_ptr()),
                                                   ctypes.c_void_p(target.data_ptr()), b, float(scale),
                                                   float(lr), ctypes.c_void_p(lp)), self._h)


def nn_conv3x3(x: torch.Tensor, w: torch.Tensor, bias: Optional[torch.Tensor], cin: int, cout: int,
               relu: bool = False, mask: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None,
               x_ld: Optional[int] = None, out_ld: Optional[int] = None, mask_ld: Optional[int] = None,
               stream=None) -> torch.Tensor:
    """3x3 convolution of NHWC bfloat16 x ([B, H, W, ld], channels 0..cin-1) by w [cout, 3, 3, cin] (bf16)."""
    lib = load_library()
    B, H, W = x.shape[0], x.shape[1], x.shape[2]
    ldx = x_ld if x_ld is not None else x.shape[3]
    if out is None:
        out = torch.empty((B, H, W, cout), dtype=torch.bfloat16, device=x.device)
    ldy = out_ld if out_ld is not None else out.shape[3]
    ldm = (mask_ld if mask_ld is not None else mask.shape[3]) if mask is not None else 0
    st = stream if stream is not None else torch.cuda.current_stream(x.device).cuda_stream
    status = lib.tomo_nn_conv3x3(ctypes.c_void_p(_bf16_ptr(x)), ldx, ctypes.c_void_p(_bf16_ptr(w)),
                                 _ptr(bias), ctypes.c_void_p(_bf16_ptr(out)), ldy,
                                 ctypes.c_void_p(_bf16_ptr(mask)) if mask is not None else None, ldm,
                                 cin, cout, B, H, W, int(relu), ctypes.c_void_p(st))
    _unet_check(status, None)
    return out


def nn_conv3x3_wgrad(dz: torch.Tensor, x: torch.Tensor, cin: int, cout: int, dz_ld: Optional[int] = None,
                     x_ld: Optional[int] = None, stream=None):
    """(dw [cout, 3, 3, cin], db [cout]) float32 for NHWC bfloat16 dz and x."""
    lib = load_library()
    B, H, W = x.shape[0], x.shape[1], x.shape[2]
    ldz = dz_ld if dz_ld is not None else dz.shape[3]
    ldx = x_ld if x_ld is not None else x.shape[3]
    n = ctypes.c_size_t()
    _unet_check(lib.tomo_nn_wgrad_scratch(cin, cout, B * H * W, ctypes.byref(n)), None)
    scratch = torch.empty(max(n.value, 1), dtype=torch.float32, device=x.device)
    dw = torch.empty((cout, 3, 3, cin), dtype=torch.float32, device=x.device)
    db = torch.empty(cout, dtype=torch.float32, device=x.device)
    st = stream if stream is not None else torch.cuda.current_stream(x.device).cuda_stream
    _unet_check(lib.tomo_nn_conv3x3_wgrad(ctypes.c_void_p(_bf16_ptr(dz)), ldz, ctypes.c_void_p(_bf16_ptr(x)), ldx,
                                          ctypes.c_void_p(dw.data_ptr()), ctypes.c_void_p(db.data_ptr()), cin, cout,
                                          B, H, W, ctypes.c_void_p(scratch.data_ptr()), n.value,
                                          ctypes.c_void_p(st)), None)
    return dw, db


def nn_conv3x3_wgrad_noalloc(dz: torch.Tensor, x: torch.Tensor, cin: int, cout: int,
                             dz_ld: Optional[int] = None, x_ld: Optional[int] = None, stream=None,
                             dw: Optional[torch.Tensor] = None, db: Optional[torch.Tensor] = None):
    """Like nn_conv3x3_wgrad, with the split sums in the library's static device scratch."""
    lib = load_library()
    B, H, W = x.shape[0], x.shape[1], x.shape[2]
    ldz = dz_ld if dz_ld is not None else dz.shape[3]
    ldx = x_ld if x_ld is not None else x.shape[3]
    if dw is None:
        dw = torch.empty((cout, 3, 3, cin), dtype=torch.float32, device=x.device)
    if db is None:
        db = torch.empty(cout, dtype=torch.float32, device=x.device)
    st = stream if stream is not None else torch.cuda.current_stream(x.device).cuda_stream
    _unet_check(lib.tomo_nn_conv3x3_wgrad_noalloc(ctypes.c_void_p(_bf16_ptr(dz)), ldz,
                                                  ctypes.c_void_p(_bf16_ptr(x)), ldx,
                                                  ctypes.c_void_p(dw.data_ptr()), ctypes.c_void_p(db.data_ptr()),
                                                  cin, cout, B, H, W, ctypes.c_void_p(st)), None)
    return dw, db
