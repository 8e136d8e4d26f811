"""The paper's two ablations on one GPU, through libtomo only (this module sequences calls).

* Start (Sec. 3.2): the constant start against the ramp-filtered back-projection start of
  Sec. 2.2 (and, on data where a trained network is at hand, the learned start), on the
  finest grid alone: iterations and time until the objective reaches a relative gap.
* Hierarchy (Sec. 3.3): the single-resolution solve against the coarse-to-fine solve of
  Sec. 2.3 (levels N/4, N/2, N with fixed coarse iteration counts): iterations on the finest
  level and total time until the finest objective reaches the same gap.

Gap measures, with F* the lowest objective seen in any run of the comparison:
  r_k = (F(y_k) - F*) / (F(0) - F*) <= tol  with F(0) = 1/2 <g, g>  (init-independent), and
  the tighter (F(y_k) - F*) / |F*| <= rel_tol.
F* is reported with the change of the best run over its last quarter, so that the reader
can see how far F* is converged.
"""
from __future__ import annotations

from typing import Optional, Sequence

import numpy as np
import torch

from . import tomo


def first_below(hist: np.ndarray, f0: float, fstar: float, tol: float) -> Optional[int]:
    """First k with (F_k - F*)/(f0 - F*) <= tol, or None."""
    r = (np.asarray(hist, dtype=np.float64) - fstar) / (f0 - fstar)
    hit = np.nonzero(r <= tol)[0]
    return int(hit[0]) if hit.size else None


def _timed(fn, device) -> float:
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    fn()
    e1.record()
    torch.cuda.synchronize(device)
    return e0.elapsed_time(e1)


def run_history(plan: "tomo.Plan", sino: torch.Tensor, iters: Sequence[int], init: int,
                **kw) -> np.ndarray:
    x = torch.empty((plan.n_slices, plan.n, plan.n), dtype=torch.float32, device=sino.device)
    h = torch.zeros(sum(iters), dtype=torch.float64, device=sino.device)
    plan.reconstruct(sino, x, list(iters), init=init, objective=h, stats=False, **kw)
    return h.cpu().numpy()


def call_ms(plan: "tomo.Plan", sino: torch.Tensor, iters: Sequence[int], init: int, reps: int = 3,
            **kw) -> float:
    """Median wall time of a whole tomo_reconstruct call (start, precomputed PSF reused); long
    calls are timed once after the warm-up."""
    if sum(iters) > 200:
        reps = 1
    x = torch.empty((plan.n_slices, plan.n, plan.n), dtype=torch.float32, device=sino.device)
    fn = lambda: plan.reconstruct(sino, x, list(iters), init=init, stats=False, **kw)  # noqa: E731
    fn()
    return float(np.median([_timed(fn, sino.device) for _ in range(reps)]))


def compare_starts(plan: "tomo.Plan", sino: torch.Tensor, long_iters: int, tol: float = 1e-4,
                   rel_tol: float = 1e-3, learned: Optional[dict] = None) -> dict:
    """Constant (zero) vs FBP (vs learned) start on a single-level plan."""
    starts = {"constant": (tomo.INIT_ZERO, {}), "fbp": (tomo.INIT_FBP, {})}
    if learned is not None:
        starts["learned"] = (tomo.INIT_LEARNED, learned)
    hist = {k: run_history(plan, sino, [long_iters], init, **kw) for k, (init, kw) in starts.items()}
    f0 = 0.5 * float(torch.sum(sino.double() ** 2).item())
    best = min(hist, key=lambda k: hist[k].min())
    fstar = float(hist[best].min())
    tail = abs(hist[best][-1] - hist[best][-(long_iters // 4)]) / abs(fstar)
    it_ms = (call_ms(plan, sino, [long_iters], tomo.INIT_FBP, 1) - call_ms(plan, sino, [0], tomo.INIT_FBP)) / long_iters
    out = {"F0": f0, "F_star": fstar, "F_star_from": best, "F_star_change_last_quarter": tail,
           "tol": tol, "rel_tol": rel_tol, "iteration_ms": it_ms, "starts": {}}
    for k, (init, kw) in starts.items():
        h = hist[k]
        k_gap = first_below(h, f0, fstar, tol)
        k_rel = first_below(h, fstar + abs(fstar), fstar, rel_tol)
        start_ms = call_ms(plan, sino, [0], init, **kw)
        out["starts"][k] = {
            "gap_at_start": (h[0] - fstar) / (f0 - fstar),
            "iterations_to_gap": k_gap, "iterations_to_rel_fstar": k_rel,
            "start_ms": start_ms,
            "ms_to_gap": None if k_gap is None else start_ms + k_gap * it_ms,
            "ms_to_rel_fstar": None if k_rel is None else start_ms + k_rel * it_ms,
        }
    return out


def compare_hierarchy(single: "tomo.Plan", hier: "tomo.Plan", sino: torch.Tensor,
                      coarse_iters: Sequence[int], long_iters: int, tol: float = 1e-4,
                      rel_tol: float = 1e-3) -> dict:
    """Single-resolution solve against the coarse-to-fine solve (FBP start on the coarsest
    grid), measured on the finest objective."""
    h1 = run_history(single, sino, [long_iters], tomo.INIT_FBP)
    hh_all = run_history(hier, sino, list(coarse_iters) + [long_iters], tomo.INIT_FBP)
    hh = hh_all[sum(coarse_iters):]  # the finest level's objective
    f0 = 0.5 * float(torch.sum(sino.double() ** 2).item())
    fstar = float(min(h1.min(), hh.min()))
    best = h1 if h1.min() <= hh.min() else hh
    tail = abs(best[-1] - best[-(long_iters // 4)]) / abs(fstar)
    res = {"F0": f0, "F_star": fstar, "F_star_change_last_quarter": tail, "tol": tol, "rel_tol": rel_tol,
           "coarse_iterations": list(coarse_iters), "levels": [hier.level_dims(l)[0] for l in range(hier.n_levels)]}
    for name, plan, h, pre in (("single", single, h1, []), ("hierarchy", hier, hh, list(coarse_iters))):
        out = {}
        for key, f0_, tl in (("gap", f0, tol), ("rel_fstar", fstar + abs(fstar), rel_tol)):
            k = first_below(h, f0_, fstar, tl)
            out[f"finest_iterations_to_{key}"] = k
            out[f"ms_to_{key}"] = None if k is None else call_ms(plan, sino, pre + [k], tomo.INIT_FBP)
        out["gap_at_finest_start"] = (h[0] - fstar) / (f0 - fstar)
        res[name] = out
    for key in ("gap", "rel_fstar"):
        a, b = res["single"][f"ms_to_{key}"], res["hierarchy"][f"ms_to_{key}"]
        res[f"speedup_to_{key}"] = (a / b) if a and b else None
    return res
