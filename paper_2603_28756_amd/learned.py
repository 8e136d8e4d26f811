"""Learned start for the accelerated iteration, end to end on the GPU through libtomo.

The paper starts the iteration from a ramp-filtered back-projection (Sec. 2.2) and counts
a better start as iterations saved (Sec. 3.2).  Here a U-Net (include/tomo_nn.h) is
trained to map the FBP image to the method's own converged reconstruction, and the two
starts are compared by the time to reach a relative objective gap
    r_k = (F(y_k) - F*) / (F(0) - F*) <= tol,
F* being the lowest objective seen in long runs from both starts and F(0) = 1/2 <g, g>
(and, tighter, (F(y_k) - F*) / |F*| <= tol).  The learned start runs inside
tomo_reconstruct (TOMO_INIT_LEARNED), which keeps the FBP start on every slice where the
network's start has the larger objective, or everywhere outside the network's training domain.

This module only sequences library calls (reconstruction plans, U-Net training steps);
every arithmetic step runs in the HIP kernels.
"""
from __future__ import annotations

import dataclasses
import time
from typing import Optional, Sequence

import numpy as np
import torch

from . import tomo


@dataclasses.dataclass
class Problem:
    n: int
    n_angles: int
    n_det: int
    angles: Sequence[float]
    beta: float = 0.01
    p: float = 1.2
    kb_width: int = 6
    neighbours: int = 8


def layer_shapes(levels: int, base: int) -> list:
    """(cin, cout) of every 3x3 conv in the order of the parameter vector (tomo_nn.h)."""
    ch = [base << l for l in range(levels)]
    out = []
    for l in range(levels):
        out += [(1 if l == 0 else ch[l - 1], ch[l]), (ch[l], ch[l])]
    for l in range(levels - 2, -1, -1):
        out += [(ch[l + 1] + ch[l], ch[l]), (ch[l], ch[l])]
    return out


def init_params(levels: int, base: int, seed: int, device) -> torch.Tensor:
    """He-normal weights (std sqrt(2 / fan_in)), zero biases, head weights 0.1 sqrt(1/C):
    a flat float32 vector in the layout of tomo_nn.h."""
    gen = torch.Generator(device="cpu").manual_seed(seed)
    parts = []
    for cin, cout in layer_shapes(levels, base):
        parts.append(torch.randn(cout * 9 * cin, generator=gen, dtype=torch.float64) * (2.0 / (9 * cin)) ** 0.5)
        parts.append(torch.zeros(cout, dtype=torch.float64))
    parts.append(0.1 * torch.randn(base, generator=gen, dtype=torch.float64) * (1.0 / base) ** 0.5)
    parts.append(torch.zeros(1, dtype=torch.float64))
    return torch.cat(parts).to(device=device, dtype=torch.float32)


def make_plan(pr: Problem, nz: int, device) -> "tomo.Plan":
    plan = tomo.Plan(pr.n, nz, pr.n_angles, pr.n_det, angles=list(pr.angles), kb_width=pr.kb_width,
                     beta=pr.beta, p=pr.p, neighbours=pr.neighbours, device=device)
    plan.precompute_psf()
    return plan


def fbp_and_targets(pr: Problem, sinos: np.ndarray, iters: int, device, batch: int = 64):
    """FBP images and reconstructions after `iters` iterations (FBP start), [k, n, n] float32.

    Slices are processed `batch` at a time in one plan; with the in-plane (8-neighbour)
    prior the slices of a batch are independent problems.
    """
    k = sinos.shape[0]
    bsz = min(batch, k)
    plan = make_plan(pr, bsz, device)
    fbp = torch.empty((k, pr.n, pr.n), dtype=torch.float32, device=device)
    tgt = torch.empty_like(fbp)
    x = torch.empty((bsz, pr.n, pr.n), dtype=torch.float32, device=device)
    g = torch.zeros((bsz, pr.n_angles, pr.n_det), dtype=torch.float32, device=device)
    for i in range(0, k, bsz):
        m = min(bsz, k - i)
        g.zero_()
        g[:m].copy_(torch.from_numpy(sinos[i:i + m]))
        plan.backproject(g, x, ramp=True)
        fbp[i:i + m].copy_(x[:m])
        plan.reconstruct(g, x, [iters], init=tomo.INIT_FBP, stats=False)
        tgt[i:i + m].copy_(x[:m])
    torch.cuda.synchronize(device)
    return fbp, tgt


def train(net: "tomo.UNet", fbp: torch.Tensor, target: torch.Tensor, scale: float, epochs: int,
          batch: int, lr: float, seed: int = 0, final_lr_frac: float = 0.1) -> np.ndarray:
    """Adam over shuffled mini-batches; the learning rate decays geometrically to
    final_lr_frac * lr.  Returns the per-step batch losses."""
    n = fbp.shape[0]
    rng = np.random.default_rng(seed)
    steps_per_epoch = n // batch
    total = max(1, epochs * steps_per_epoch)
    losses = torch.zeros(total, dtype=torch.float64, device=fbp.device)
    step = 0
    for _ in range(epochs):
        perm = torch.as_tensor(rng.permutation(n), device=fbp.device)
        for i in range(steps_per_epoch):
            idx = perm[i * batch:(i + 1) * batch]
            f = fbp.index_select(0, idx).contiguous()
            t = target.index_select(0, idx).contiguous()
            lr_t = lr * final_lr_frac ** (step / total)
            net.train_step(f, t, scale, lr_t, loss_out=losses[step:step + 1])
            step += 1
    return losses.cpu().numpy()


def infer(net: "tomo.UNet", fbp: torch.Tensor, scale: float, batch: int) -> torch.Tensor:
    out = torch.empty_like(fbp)
    for i in range(0, fbp.shape[0], batch):
        m = min(batch, fbp.shape[0] - i)
        net.forward(fbp[i:i + m].contiguous(), scale, out=out[i:i + m])
    return out


def iterations_to_gap(hist: np.ndarray, f0: float, fstar: float, tol: float) -> Optional[int]:
    """First k with (F(y_k) - F*)/(F(0) - F*) <= tol (k = 0 is the start), or None."""
    r = (np.asarray(hist, dtype=np.float64) - fstar) / (f0 - fstar)
    hit = np.nonzero(r <= tol)[0]
    return int(hit[0]) if hit.size else None


def record_domain(net: "tomo.UNet", pr: Problem, n_angles_min: Optional[int] = None,
                  n_angles_max: Optional[int] = None):
    """Record the training domain of a network trained on problems like `pr` (tomo_nn.h)."""
    net.set_domain(pr.n, pr.n_det, n_angles_min or pr.n_angles, n_angles_max or pr.n_angles, pr.beta,
                   p=pr.p, neighbours=pr.neighbours)


def compare_starts(pr: Problem, sinos: np.ndarray, net: "tomo.UNet", scale: float, device,
                   long_iters: int = 2000, tol: float = 1e-4, reps: int = 5) -> dict:
    """Time to the relative gap `tol` from the FBP start and from the learned start
    (tomo_reconstruct with TOMO_INIT_LEARNED: network inference, the per-slice objective test
    and the FBP fallback all inside the call) on the held-out slices `sinos`, solved together
    as one batch of independent slices.  The network's training domain must be recorded."""
    k = sinos.shape[0]
    plan = make_plan(pr, k, device)
    g = torch.from_numpy(np.ascontiguousarray(sinos)).to(device)
    x = torch.empty((k, pr.n, pr.n), dtype=torch.float32, device=device)
    hist0 = torch.zeros(1, dtype=torch.float64, device=device)
    plan.reconstruct(g, x, [1], init=tomo.INIT_ZERO, objective=hist0, stats=False)
    f0 = float(hist0.item())
    learned_kw = {"unet": net, "unet_scale": scale}
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def init_ms(init, **kw):
        """Median time of a zero-iteration call: R* g plus the start (FBP, or FBP, network,
        objective test and choice)."""
        plan.reconstruct(g, x, [0], init=init, stats=False, **kw)  # warm-up
        ts = []
        for _ in range(reps):
            ev0.record()
            plan.reconstruct(g, x, [0], init=init, stats=False, **kw)
            ev1.record()
            torch.cuda.synchronize(device)
            ts.append(ev0.elapsed_time(ev1))
        return float(np.median(ts))

    fbp_ms = init_ms(tomo.INIT_FBP)
    learned_ms = init_ms(tomo.INIT_LEARNED, **learned_kw)

    def run(init, **kw):
        h = torch.zeros(long_iters, dtype=torch.float64, device=device)
        st = plan.reconstruct(g, x, [long_iters], init=init, objective=h, **kw)
        return h.cpu().numpy(), st

    h_fbp, _ = run(tomo.INIT_FBP)
    h_net, st_net = run(tomo.INIT_LEARNED, **learned_kw)
    h_zero, _ = run(tomo.INIT_ZERO)
    fstar = float(min(h_fbp.min(), h_net.min(), h_zero.min()))
    tail = abs(h_fbp[-1] - h_fbp[-long_iters // 4]) / abs(fstar)
    k_fbp = iterations_to_gap(h_fbp, f0, fstar, tol)
    k_net = iterations_to_gap(h_net, f0, fstar, tol)
    # the same in the tighter measure (F - F*) / |F*|
    k_fbp_abs = iterations_to_gap(h_fbp, fstar + abs(fstar), fstar, tol)
    k_net_abs = iterations_to_gap(h_net, fstar + abs(fstar), fstar, tol)

    # per-iteration time of this batch (graph replay), from two run lengths
    def timed(iters):
        ev0.record()
        plan.reconstruct(g, x, [iters], init=tomo.INIT_FBP, stats=False)
        ev1.record()
        torch.cuda.synchronize(device)
        return ev0.elapsed_time(ev1)
    timed(50)
    it_ms = (timed(450) - timed(50)) / 400.0

    def total(init, kk):
        return init + (kk if kk is not None else np.nan) * it_ms
    t_fbp, t_net = total(fbp_ms, k_fbp), total(learned_ms, k_net)
    k_zero = iterations_to_gap(h_zero, f0, fstar, tol)
    zero_ms = init_ms(tomo.INIT_ZERO)
    return {
        "slices": k, "tol": tol, "F0": f0, "F_star": fstar, "F_star_tail_change": tail,
        "gap_at_start": {"fbp": (h_fbp[0] - fstar) / (f0 - fstar), "unet": (h_net[0] - fstar) / (f0 - fstar),
                         "constant": (h_zero[0] - fstar) / (f0 - fstar)},
        "iterations": {"fbp": k_fbp, "unet": k_net, "constant": k_zero},
        "iterations_rel_fstar": {"fbp": k_fbp_abs, "unet": k_net_abs,
                                 "constant": iterations_to_gap(h_zero, fstar + abs(fstar), fstar, tol)},
        "learned_slices": st_net["learned_slices"], "learned_state": st_net["learned_state"],
        "fallback_to_fbp": st_net["learned_slices"] < k,
        "ms": {"fbp_start": fbp_ms, "learned_start": learned_ms, "constant_start": zero_ms,
               "total_constant": total(zero_ms, k_zero), "iteration": it_ms,
               "total_fbp": t_fbp, "total_unet": t_net,
               "total_fbp_rel_fstar": total(fbp_ms, k_fbp_abs),
               "total_unet_rel_fstar": total(learned_ms, k_net_abs)},
        "speedup": t_fbp / t_net if t_net and np.isfinite(t_net) else None,
    }
