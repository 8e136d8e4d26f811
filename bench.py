#!/usr/bin/env python3
"""Throughput of the Toeplitz MBIR path on one MI355X, as one JSON line.

A step is one whole reconstruction of the 64 x 512^2 volume workload (180
angles x 724 bins, 1% noise, Kaiser-Bessel width 6 and oversampling 2, PSF
spectrum 1024^2, 100 accelerated-gradient iterations with the 26-neighbour
qGGMRF prior): the float64 PSF-spectrum and step-constant precompute, the
back-projection R* g, the FBP start and the 100 iterations.  Inputs are resident
in device memory before the timed region starts.

value = N^2 * n_slices * iterations / (seconds per step)   [gradient voxel-updates/s]

roofline: the kernel class with the largest share of the step is timed live with
HIP events on the plan's stream over a second pass of the same steps (events turn
off graph replay, so they are kept out of the timed region); its algorithmic bytes per
launch over the mean launch time are compared with the 8 TB/s HBM peak (the path is
memory-bound by design).  Alongside, the ALU view of the two arithmetic-heavy kernels:
pass C's FFT flops (5 P log2 P per transform) against the non-packed FP32 vector peak,
256 CUs x 64 lanes x 2 x 2.4 GHz = 78.6 TFLOP/s, and the prior's algorithmic VALU
lane-operations (transcendentals weighted 2, their measured issue cost on gfx950) against
256 CUs x 64 lanes x 2.4 GHz = 39.3 T lane-ops/s.
iteration_hbm: measured HBM bytes per iteration (rocprofv3 FETCH_SIZE + WRITE_SIZE summary,
when it matches the current kernel sources) over the wall time of the graph-replayed
iteration loop, against 8 TB/s; and the same for the compulsory 20.5 B/voxel and the
three-pass 56 B/voxel model.  Precompute and iteration loop are also timed separately
(median of 5).
--hbm-rates: only the HBM rates plain streaming kernels reach on this part (a sum, a fill and
an elementwise copy of 512 MiB), the practical ceiling beside the 8 TB/s the rooflines use.
cpu_baseline: the FP64 oracle's own iteration (Toeplitz product by numpy FFTs, prior,
update) on a 4-slice slab of the same volume, run in one process per host core (the box's
CPU share) at once; plus the oracle's direct A^T(A x) against its Toeplitz product at
N = 128 and 256 (the CPU analogue of the paper's direct-vs-Toeplitz comparison).  Both run
in a child process that does not touch the GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12   # lane-operations per second, packed FP32 unused
FP32_PEAK_TFLOPS = 2 * VALU_PEAK_TOPS        # fused multiply-add = 2 flops, non-packed
CLASS_NAMES = ["rows_fwd", "cols_conv", "rows_inv", "finalize", "backproject", "psf", "prior"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_volume_64x512.txt")


# sources that determine the iteration kernels and their launch configuration
HOT_SOURCES = ("common.hpp", "fft.hpp", "kernels.hpp", "tomo_api.cpp", "toeplitz_kernels.hip")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2603_28756_amd", "csrc")
    for name in HOT_SOURCES:
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def read_traffic(cls: str, key: str = "bytes_per_launch"):
    """HBM bytes of kernel class `cls` from the counter summary, or None.

    The summary holds a `source_hash` line and `kernel <class> ... bytes_per_launch <B>
    ... bytes_per_iteration <B>` lines (passes R, C, R' launch once per slice chunk); it is
    ignored when the kernel sources changed after the counters were taken.
    """
    if not os.path.exists(TRAFFIC_FILE):
        return None
    src, found = None, {}
    with open(TRAFFIC_FILE) as f:
        for line in f:
            tok = line.split()
            if len(tok) >= 2 and tok[0] == "source_hash":
                src = tok[1]
            elif len(tok) >= 2 and tok[0] == "kernel" and key in tok:
                found[tok[1]] = float(tok[tok.index(key) + 1])
    if src != kernel_source_hash():
        return None
    return found.get(cls)


def iteration_traffic():
    """Measured HBM bytes of one iteration (passes R, C, R', prior, finalize) from the counter
    summary, or None when it does not match the current kernel sources."""
    vals = [read_traffic(c, "bytes_per_iteration")
            for c in ("rows_fwd", "cols_conv", "rows_inv", "prior", "finalize")]
    return None if any(v is None for v in vals) else float(sum(vals))


def prior_lane_ops(n: int, nz: int, neighbours: int) -> float:
    """Algorithmic VALU lane-operations of one prior launch.

    Per neighbour pair (each evaluated once): the difference, fma, 1 + w, fma and two
    multiplies (6 full-rate operations) and log2, exp2, reciprocal (3 transcendentals,
    each issuing in twice the cycles of a full-rate operation on gfx950: weight 2) = 12;
    each pair value enters both of its voxels with one fused multiply-add = 2.
    26 neighbours: 13 pairs per voxel -> 182 per voxel; 8 neighbours: 4 pairs -> 56.
    """
    pairs = 13 if neighbours == 26 else 4
    return float(n) * n * nz * pairs * (12 + 2)


def cols_conv_flops(n: int, nz: int, P: int) -> float:
    """Algorithmic flops of one pass-C launch: per slice H = P/2 complex columns, each a
    forward and an inverse complex FFT of length P (5 P log2 P flops each, the standard
    count) and a real scaling by F K (2 flops per element)."""
    import math
    return float(nz) * (P // 2) * (2 * 5 * P * math.log2(P) + 2 * P)


def algorithmic_bytes(cls: str, n: int, nz: int, P: int, fused_prior: bool = False,
                      concurrent_prior: bool = False) -> float:
    """Bytes each kernel class must move per launch (compulsory reads + writes).

    In sequence (the default) the prior kernel of a FISTA step also writes y and
    gp - b, which passes R and R' then read in place of x_{k-1}, b and gp; with the
    fused prior or the prior on its own stream the passes read x_k, x_{k-1}, b (and gp).
    """
    H = P // 2
    spec = 8.0 * nz * n * H          # one half spectrum S1 or S2 (complex64)
    vol = 4.0 * nz * n * n           # one float32 volume
    fk = 4.0 * P * (H + 1)           # PSF spectrum (float32)
    yg = not fused_prior and not concurrent_prior
    if cls == "rows_fwd":            # read y (or x_k, x_{k-1}); write S1
        return (1 if yg else 2) * vol + spec
    if cls == "cols_conv":           # read S1 and F K; write S2
        return 2 * spec + fk
    if cls == "rows_inv":            # read S2, x_k, y, gp - b (or S2, x_k, x_{k-1}, b[, gp]); write x_{k+1}
        return spec + (4 if yg else (4 if fused_prior else 5)) * vol
    if cls == "prior":               # read x_k, x_{k-1}[, b]; write gp[ - b, y]
        return (5 if yg else 3) * vol
    return float("nan")


_POOL_PROB = None   # the oracle problem each forked worker iterates on


def _oracle_worker(arg):
    iters, L = arg
    from oracle import solver
    x0 = _POOL_PROB.b * 0.0
    t0 = time.perf_counter()
    solver.fista(_POOL_PROB, x0, iters, L=L)
    return time.perf_counter() - t0


def cpu_share() -> int:
    """Host cores this process may use, at most 16 (one GPU's share of the box)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(wl, prob_np, iters: int = 5, slices: int = 4) -> dict:
    """Oracle FISTA on a contiguous slab of `slices` slices, `iters` iterations, in one forked
    process per core (each on its own copy of the slab); aggregate voxel-updates/s."""
    import multiprocessing as mp
    import numpy as np
    from oracle import geometry as G
    from oracle import prior as qg
    from oracle import radon, solver, toeplitz
    global _POOL_PROB
    geom = G.Geometry(wl.n, prob_np["angles"], wl.n_det)
    z0 = wl.n_slices // 2 - slices // 2
    sino = prob_np["sino32"][z0:z0 + slices].astype(np.float64)
    pr = qg.QGGMRF(p=wl.p, q=wl.q, sigma=wl.sigma, T=wl.T, neighbours=wl.neighbours)
    P = solver.pad_size(wl.n)
    t0 = time.perf_counter()
    fk = toeplitz.psf_spectrum(geom, P)
    b = radon.adjoint(sino, geom)
    t_pre = time.perf_counter() - t0
    _POOL_PROB = solver.Problem(geom, fk, b, float(np.vdot(sino, sino)), pr, wl.beta)
    L = solver.lipschitz(_POOL_PROB)
    workers = cpu_share()
    with mp.get_context("fork").Pool(workers) as pool:
        t0 = time.perf_counter()
        times = pool.map(_oracle_worker, [(iters, L)] * workers, chunksize=1)
        wall = time.perf_counter() - t0
    vox = workers * slices * wl.n * wl.n * iters
    return {"value": vox / wall, "unit": "voxel-updates/s", "cores": workers, "kind": "oracle",
            "sample": (f"{workers} processes at once, each {iters} FISTA iterations of the float64 oracle "
                       f"(numpy FFT Toeplitz product, {wl.neighbours}-neighbour prior, update) on a copy of "
                       f"slices {z0}..{z0 + slices - 1} of the {wl.n_slices} x {wl.n}^2 volume; wall "
                       f"{wall:.1f} s, per process {min(times):.1f}-{max(times):.1f} s; the oracle's PSF "
                       f"spectrum and R* g of the slab ({t_pre:.1f} s) and its step constant are not in "
                       f"the rate"),
            "single_process_value": slices * wl.n * wl.n * iters / min(times),
            "host_cpus": os.cpu_count()}


def cpu_direct_vs_toeplitz() -> dict:
    """The oracle's direct A^T(A x) (exact non-uniform DFTs as dense products) against its
    padded-FFT Toeplitz product on one slice, N = 128 (90 angles) and 256 (180 angles)."""
    import numpy as np
    import synth
    from oracle import geometry as G
    from oracle import radon, solver, toeplitz
    out = []
    for n, na in ((128, 90), (256, 180)):
        nd = synth.detector_bins_for(n)
        geom = G.Geometry(n, synth.uniform_angles(na), nd)
        x = np.random.default_rng(n).standard_normal((n, n))
        fk = toeplitz.psf_spectrum(geom, solver.pad_size(n))
        t0 = time.perf_counter()
        direct = radon.adjoint(radon.forward(x, geom), geom)
        t_dir = time.perf_counter() - t0
        reps = 5
        t0 = time.perf_counter()
        for _ in range(reps):
            toep = toeplitz.apply(x, fk, n)
        t_toe = (time.perf_counter() - t0) / reps
        out.append({"n": n, "n_angles": na, "n_det": nd, "direct_ms": 1e3 * t_dir,
                    "toeplitz_ms": 1e3 * t_toe, "speedup": t_dir / t_toe,
                    "rel_diff": float(np.linalg.norm(direct - toep) / np.linalg.norm(direct))})
    return {"kind": "oracle", "precision": "f64", "cases": out}


def run_cpu_only(args) -> int:
    """Host-only measurements (no GPU is touched): one JSON line."""
    import numpy as np
    import synth
    wl = synth.WORKLOADS[args.workload]
    pr = synth.make_problem(wl.n, wl.n_slices, wl.n_angles, wl.n_det, wl.noise, wl.seed, wl.n_objects)
    prob_np = {"angles": pr["angles"], "sino32": pr["sino"].astype(np.float32)}
    print(json.dumps({"cpu_baseline": cpu_baseline(wl, prob_np),
                      "cpu_direct_vs_toeplitz": cpu_direct_vs_toeplitz()}))
    return 0


def cpu_measurements(workload: str) -> dict:
    """run_cpu_only in a child process started before or after the GPU work of this one."""
    import subprocess
    res = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-only", "--workload", workload],
                         capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"cpu measurements failed:\n{res.stderr[-2000:]}")
    return json.loads(res.stdout.strip().splitlines()[-1])


def run_batch(args) -> int:
    """256 independent uneven single-slice problems advanced together (the autotuned batch
    schedule: one persistent launch, or one launch per phase and size, per iteration,
    graph-captured) against the same problems run one plan at a time.  The
    per-iteration time comes from two run lengths (3 and 33 iterations), so it excludes the
    per-problem FBP start and precompute.  One JSON line."""
    import numpy as np
    import synth
    import torch
    from paper_2603_28756_amd import tomo
    probs = synth.uneven_problems(256, seed=4)
    dev = torch.device("cuda", 0)
    plans = [tomo.Plan(p["n"], 1, p["n_angles"], p["n_det"], angles=list(p["angles"]), kb_width=6,
                       neighbours=8, beta=0.01, device=dev) for p in probs]
    batch = tomo.Batch(plans)
    sinos = [torch.from_numpy(p["sino"]).to(dev) for p in probs]
    t0 = time.perf_counter()
    schedule = batch.autotune(reps=5)   # per-size radix choice, once per batch
    tune_s = time.perf_counter() - t0
    print(f"batch schedule: {schedule} ({tune_s:.2f} s)", file=sys.stderr, flush=True)
    xs = [torch.empty((1, p["n"], p["n"]), dtype=torch.float32, device=dev) for p in probs]
    vox = float(sum(p["n"] ** 2 for p in probs))
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn):
        ev0.record()
        fn()
        ev1.record()
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1)

    batch.reconstruct(sinos, xs, 3)
    t3 = min(timed(lambda: batch.reconstruct(sinos, xs, 3)) for _ in range(2))
    t33 = min(timed(lambda: batch.reconstruct(sinos, xs, 33)) for _ in range(2))
    it_batch = (t33 - t3) / 30.0
    print(f"batch: {it_batch:.3f} ms per iteration", file=sys.stderr, flush=True)
    it_seq = 0.0
    for p, plan, g, x in zip(probs, plans, sinos, xs):
        plan.reconstruct(g, x, [3], init=tomo.INIT_FBP, stats=False)
        a = timed(lambda: plan.reconstruct(g, x, [3], init=tomo.INIT_FBP, stats=False))
        b = timed(lambda: plan.reconstruct(g, x, [33], init=tomo.INIT_FBP, stats=False))
        it_seq += (b - a) / 30.0
    print(f"one plan at a time: {it_seq:.3f} ms per iteration", file=sys.stderr, flush=True)
    sizes = sorted({p["n"] for p in probs})
    out = {
        "metric": "batched gradient voxel-updates/s (256 uneven problems)",
        "value": vox / (it_batch * 1e-3), "unit": "voxel-updates/s", "n_gpus": 1, "steps": 30, "warmup": 1,
        "ms_per_step": it_batch, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batch_256_uneven", "problems": len(probs), "sizes": sizes,
                   "count_per_size": {str(n): sum(1 for p in probs if p["n"] == n) for n in sizes},
                   "angles": [min(p["n_angles"] for p in probs), max(p["n_angles"] for p in probs)],
                   "noise": [0.01, 0.05], "neighbours": 8, "kb_width": 6,
                   "voxels_per_iteration": vox,
                   "schedule": {"elements_per_thread_by_fft_size": schedule["sizes"],
                                "tiles_per_item_by_fft_size": schedule["group"],
                                "prior": ("inside pass R' (8 neighbours, each pair from both voxels)"
                                          if schedule["fused_prior"] else "pair-shared prior phase"),
                                "autotune_iter_ms": schedule["iter_ms"],
                                "starting_schedule_iter_ms": schedule["base_ms"], "autotune_s": tune_s,
                                "launch": ("one launch per phase and transform size (prior; R, C, R' of "
                                           "every problem), one tile per block, and a per-problem "
                                           "finalize launch, graph-captured"
                                           if schedule.get("phase_launches") else
                                           "one persistent launch per iteration (prior, R, C, R' items "
                                           "of all problems from one queue), graph-captured")}},
        "one_plan_at_a_time": {"ms_per_iteration": it_seq, "voxel_updates_per_s": vox / (it_seq * 1e-3)},
        "batching_speedup": it_seq / it_batch,
    }
    print(json.dumps(out))
    return 0


def run_learned(args) -> int:
    """Time to a 1e-4 relative objective gap from the U-Net start against the FBP start.

    2000 training and 64 held-out 512^2 slices (ellipses + Gaussian texture, 60 angles,
    1% noise); training targets are the method's own reconstructions (300 iterations from
    FBP); the U-Net (--unet-levels levels, default 2, 32 base channels) is trained on the GPU; both starts are run
    on the held-out slices (solved together) and timed.  One JSON line.
    """
    import numpy as np
    import synth
    wl = synth.WORKLOADS["learned_init_512"]
    n_train = args.train_slices
    t0 = time.perf_counter()
    # sinograms are made before the GPU is touched (forked workers)
    train_s = synth.textured_batch(n_train, wl.n, wl.n_angles, wl.n_det, wl.noise, wl.seed, workers=8)
    test_s = synth.textured_batch(wl.n_slices, wl.n, wl.n_angles, wl.n_det, wl.noise, wl.seed + 10 ** 6,
                                  workers=8)
    data_s = time.perf_counter() - t0
    print(f"sinograms: {data_s:.1f} s", file=sys.stderr, flush=True)
    import torch
    from paper_2603_28756_amd import learned, tomo
    dev = torch.device("cuda", 0)
    pr = learned.Problem(wl.n, wl.n_angles, wl.n_det, synth.uniform_angles(wl.n_angles), beta=wl.beta,
                         p=wl.p, kb_width=wl.kb_width, neighbours=wl.neighbours)
    t0 = time.perf_counter()
    fbp, tgt = learned.fbp_and_targets(pr, train_s, args.target_iters, dev)
    target_s = time.perf_counter() - t0
    print(f"targets: {target_s:.1f} s", file=sys.stderr, flush=True)
    scale = float(torch.sqrt(torch.mean(fbp * fbp)).item())
    levels = args.unet_levels
    net = tomo.UNet(wl.n, wl.n, levels=levels, base=32, max_batch=max(args.batch, args.infer_batch))
    net.set_params(learned.init_params(levels, 32, 7, dev))
    t0 = time.perf_counter()
    losses = learned.train(net, fbp, tgt, scale, args.epochs, args.batch, args.lr, seed=7)
    torch.cuda.synchronize()
    train_s_time = time.perf_counter() - t0
    print(f"training: {train_s_time:.1f} s, loss {np.mean(losses[:20]):.3e} -> {np.mean(losses[-20:]):.3e}",
          file=sys.stderr, flush=True)
    del fbp, tgt
    learned.record_domain(net, pr)
    res = learned.compare_starts(pr, test_s, net, scale, dev, long_iters=2000)
    # 3x3 convolutions dominate: 2 x 9 cin cout flops per pixel at each level's resolution
    shapes = learned.layer_shapes(levels, 32)
    lvl = [l for l in range(levels) for _ in (0, 1)] + [l for l in range(levels - 2, -1, -1) for _ in (0, 1)]
    fwd_flop = sum(18.0 * ci * co * (wl.n >> l) ** 2 for (ci, co), l in zip(shapes, lvl))
    step_flop = 3 * fwd_flop * args.batch  # forward + backward of one batch
    out = {
        "metric": "time to 1e-4 relative objective gap, U-Net start (FBP start alongside)",
        "value": res["ms"]["total_unet"], "unit": "ms", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": res["ms"]["total_unet"], "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16 network, f32 reconstruction", "data": "synthetic",
        "config": {"workload": wl.name, "n": wl.n, "n_angles": wl.n_angles, "n_det": wl.n_det,
                   "noise": wl.noise, "train_slices": n_train, "test_slices": wl.n_slices,
                   "target_iterations": args.target_iters,
                   "unet": {"levels": levels, "base": 32, "forward_gflop_per_slice": fwd_flop / 1e9},
                   "epochs": args.epochs, "batch": args.batch, "infer_batch": args.infer_batch,
                   "lr": args.lr, "neighbours": wl.neighbours},
        "result": res,
        "training": {"seconds": train_s_time, "steps": int(len(losses)),
                     "ms_per_step": 1e3 * train_s_time / max(1, len(losses)),
                     "approx_tflops": step_flop / (train_s_time / max(1, len(losses))) / 1e12,
                     "loss_first": float(np.mean(losses[:20])), "loss_last": float(np.mean(losses[-20:]))},
        "prep_seconds": {"sinograms": data_s, "targets": target_s},
    }
    print(json.dumps(out))
    return 0


def run_direct(args) -> int:
    """Toeplitz gradient (passes R, C, R', prior, finalize; PSF precomputed once) against the
    direct gradient R*(R x - g) + beta grad Phi (both non-uniform transforms every call) over
    image widths: median launch-to-finish time of each on the same inputs, and their relative
    difference.  One JSON line."""
    import numpy as np
    import synth
    import torch
    from paper_2603_28756_amd import tomo
    dev = torch.device("cuda", 0)
    nz, na, reps = 8, 180, 10
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def med_ms(fn):
        fn()
        ts = []
        for _ in range(reps):
            ev0.record()
            fn()
            ev1.record()
            torch.cuda.synchronize()
            ts.append(ev0.elapsed_time(ev1))
        return float(np.median(ts))

    cases = []
    for n in (128, 256, 512, 1024, 2048):
        nd = synth.detector_bins_for(n)
        pr = synth.make_problem(n, nz, na, nd, 0.01, 40 + n, 20)
        sino = torch.from_numpy(pr["sino"].astype(np.float32)).to(dev)
        rng = np.random.default_rng(n)
        x = torch.from_numpy((pr["phantom"] + 0.05 * rng.standard_normal(pr["phantom"].shape))
                             .astype(np.float32)).to(dev)
        plan = tomo.Plan(n, nz, na, nd, angles=list(pr["angles"]), kb_width=6, neighbours=26, device=dev)
        plan.precompute_psf()
        b = torch.empty_like(x)
        plan.backproject(sino, b, ramp=False)
        g_t, g_d, tx = torch.empty_like(x), torch.empty_like(x), torch.empty_like(x)
        o_t = torch.zeros(1, dtype=torch.float64, device=dev)
        o_d = torch.zeros(1, dtype=torch.float64, device=dev)
        t_toe = med_ms(lambda: plan.gradient(x, b, g_t, o_t))
        t_dir = med_ms(lambda: plan.gradient_direct(x, sino, g_d, o_d))
        plan.apply_normal(x, tx)
        torch.cuda.synchronize()
        gt, gd = g_t.double(), g_d.double()
        d_terms = float(torch.linalg.norm(gd - gt) / (torch.linalg.norm(tx.double()) + torch.linalg.norm(b.double())))
        d_grad = float(torch.linalg.norm(gd - gt) / torch.linalg.norm(gt))
        half_gg = 0.5 * float(torch.sum(sino.double() ** 2))
        d_loss = abs(float(o_d.item()) - float(o_t.item()) - half_gg) / half_gg
        cases.append({"n": n, "n_det": nd, "toeplitz_ms": t_toe, "direct_ms": t_dir,
                      "speedup": t_dir / t_toe, "grad_rel_diff_of_terms": d_terms,
                      "grad_rel_diff": d_grad, "loss_rel_diff_of_F0": d_loss})
        print(f"N {n}: Toeplitz {t_toe:.3f} ms, direct {t_dir:.3f} ms, gradient difference {d_terms:.2e} "
              f"of the terms ({d_grad:.2e} of the gradient), loss {d_loss:.2e}", file=sys.stderr, flush=True)
        del plan, x, b, g_t, g_d, tx, sino
        torch.cuda.empty_cache()
    big = cases[-1]
    out = {
        "metric": "gradient time, Toeplitz vs direct (two non-uniform transforms)",
        "value": big["direct_ms"] / big["toeplitz_ms"], "unit": "x (direct / Toeplitz time at 2048^2)",
        "n_gpus": 1, "steps": reps, "warmup": 1, "ms_per_step": big["toeplitz_ms"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "direct_vs_toeplitz", "slices": nz, "n_angles": na, "kb_width": 6,
                   "oversampling": 2, "neighbours": 26, "widths": [c["n"] for c in cases],
                   "toeplitz": "PSF spectrum precomputed once, not timed; one gradient = passes R, C, R', "
                               "prior, float64 objective",
                   "direct": "forward projection (deapodise, grid FFT, KB interpolation, radial inverse DFT), "
                             "residual, back-projection (radial DFT, KB gridding, grid IFFT, crop), prior, "
                             "float64 objective"},
        "cases": cases,
    }
    print(json.dumps(out))
    return 0


def run_ablation(args) -> int:
    """The paper's start and hierarchy ablations on the 32 x 2048^2 workload (91 angles x 2896
    bins, 2% noise, 26-neighbour prior): constant vs FBP start on the finest grid alone, and the
    single-resolution solve vs the 3-level hierarchy (512 -> 1024 -> 2048, 40 and 20 coarse
    iterations), to the same relative objective gap.  One JSON line."""
    import numpy as np
    import synth
    import torch
    from paper_2603_28756_amd import ablation, tomo
    wl = synth.WORKLOADS["hier_32x2048"]
    dev = torch.device("cuda", 0)
    pr = synth.make_problem(wl.n, wl.n_slices, wl.n_angles, wl.n_det, wl.noise, wl.seed, wl.n_objects)
    sino = torch.from_numpy(pr["sino"].astype(np.float32)).to(dev)
    kw = dict(angles=list(pr["angles"]), kb_width=wl.kb_width, beta=wl.beta, p=wl.p, sigma=wl.sigma,
              T=wl.T, neighbours=wl.neighbours, device=dev)
    single = tomo.Plan(wl.n, wl.n_slices, wl.n_angles, wl.n_det, n_levels=1, **kw)
    single.precompute_psf()
    t0 = time.perf_counter()
    starts = ablation.compare_starts(single, sino, args.iters or 3000)
    print(f"starts: {time.perf_counter() - t0:.1f} s {starts['starts']}", file=sys.stderr, flush=True)
    hier = tomo.Plan(wl.n, wl.n_slices, wl.n_angles, wl.n_det, n_levels=3, **kw)
    hier.precompute_psf()
    t0 = time.perf_counter()
    hierarchy = ablation.compare_hierarchy(single, hier, sino, [40, 20], args.iters or 3000)
    print(f"hierarchy: {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    out = {
        "metric": "time to 1e-4 objective gap: hierarchy vs single resolution (and constant vs FBP start)",
        "value": hierarchy["speedup_to_gap"], "unit": "x (single-resolution time / hierarchy time)",
        "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": hierarchy["hierarchy"]["ms_to_gap"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "ablation_32x2048", "n": wl.n, "n_slices": wl.n_slices,
                   "n_angles": wl.n_angles, "n_det": wl.n_det, "noise": wl.noise, "kb_width": wl.kb_width,
                   "neighbours": wl.neighbours, "long_iterations": args.iters or 3000},
        "starts": starts, "hierarchy": hierarchy,
    }
    print(json.dumps(out))
    return 0


def run_stream(args) -> int:
    """A volume kept in host memory and streamed through a smaller plan (the three-thread
    upload / compute / download pipeline of Sec. 2.4): 256 slices of 512^2 (180 angles x 724
    bins, 26-neighbour prior, 100 iterations) through a 64-slice plan with 2 context slices per
    side (5 windows).  Queue depth 1 runs the windows one after the other; depth 2 and 3 overlap
    a window's transfers with its neighbours' solves.  One JSON line; value = voxel-updates/s of
    the streamed volume at depth 2 (host-to-host)."""
    import numpy as np
    import synth
    import torch
    from paper_2603_28756_amd import tomo
    wl = synth.WORKLOADS["volume_64x512"]
    n_total, win, halo = 256, 64, 2
    iters = [args.iters or wl.iterations[0]]
    dev = torch.device("cuda", 0)
    pr = synth.make_problem(wl.n, n_total, wl.n_angles, wl.n_det, wl.noise, wl.seed, wl.n_objects)
    sino = np.ascontiguousarray(pr["sino"], dtype=np.float32)
    plan = tomo.Plan(wl.n, win, wl.n_angles, wl.n_det, angles=list(pr["angles"]), kb_width=wl.kb_width,
                     kb_oversamp=wl.kb_oversamp, beta=wl.beta, p=wl.p, q=wl.q, sigma=wl.sigma, T=wl.T,
                     neighbours=wl.neighbours, device=dev)
    tiles = plan.autotune(reps=5)
    x = np.empty((n_total, wl.n, wl.n), dtype=np.float32)
    runs = {}
    for depth in (1, 2, 3):
        pipe = tomo.Pipeline(plan, n_total, halo=halo, depth=depth)
        pipe.run(sino, x, iters, init=tomo.INIT_FBP, stats=False)   # warm-up (PSF, graphs)
        best = None
        for _ in range(3):
            t0 = time.perf_counter()
            pipe.run(sino, x, iters, init=tomo.INIT_FBP, stats=False)
            wall = (time.perf_counter() - t0) * 1e3
            best = wall if best is None else min(best, wall)
        st = pipe.run(sino, x, iters, init=tomo.INIT_FBP, stats=True)
        runs[depth] = {"wall_ms": best, "checked_run": st}
        print(f"depth {depth}: {best:.1f} ms", file=sys.stderr, flush=True)
        pipe.close()
    # the same windows solved from device-resident data (no transfers), one after the other
    sd = torch.from_numpy(sino[:win]).to(dev)
    xd = torch.empty((win, wl.n, wl.n), dtype=torch.float32, device=dev)
    plan.reconstruct(sd, xd, iters, init=tomo.INIT_FBP, stats=False)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(3):
        plan.reconstruct(sd, xd, iters, init=tomo.INIT_FBP, stats=False)
    e1.record()
    torch.cuda.synchronize()
    win_ms = e0.elapsed_time(e1) / 3
    n_win = tomo.pipeline_window(n_total, win, halo, 0)[3]
    vox = float(wl.n * wl.n * n_total * sum(iters))
    out = {
        "metric": "streamed gradient voxel-updates/s (volume in host memory)",
        "value": vox / (runs[2]["wall_ms"] * 1e-3), "unit": "voxel-updates/s", "n_gpus": 1,
        "steps": 3, "warmup": 1, "ms_per_step": runs[2]["wall_ms"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "stream_256x512", "n": wl.n, "n_total": n_total, "window": win, "halo": halo,
                   "windows": n_win, "n_angles": wl.n_angles, "n_det": wl.n_det, "iterations": iters,
                   "neighbours": wl.neighbours, "kb_width": wl.kb_width,
                   "tiles": [{k: t[k] for k in ("fwd_pairs", "col_tile", "inv_pairs", "chunks")} for t in tiles]},
        "depth_wall_ms": {str(d): r["wall_ms"] for d, r in runs.items()},
        "checked_runs": {str(d): r["checked_run"] for d, r in runs.items()},
        "device_resident_window_ms": win_ms,
        "device_resident_windows_ms": win_ms * n_win,
        "overlap_gain_depth2_vs_depth1": runs[1]["wall_ms"] / runs[2]["wall_ms"],
        "streaming_overhead_vs_device_resident": runs[2]["wall_ms"] / (win_ms * n_win),
    }
    print(json.dumps(out))
    return 0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="volume_64x512")
    ap.add_argument("--iters", type=int, default=0, help="override the workload's iteration count")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--fused-prior", action="store_true",
                    help="evaluate the prior in the inverse-row epilogue (comparison variant)")
    ap.add_argument("--concurrent-prior", action="store_true",
                    help="launch the prior kernel on its own stream beside the row/column passes")
    ap.add_argument("--train-slices", type=int, default=2000, help="learned start: training slices")
    ap.add_argument("--target-iters", type=int, default=300, help="learned start: target iterations")
    ap.add_argument("--epochs", type=int, default=10, help="learned start: training epochs")
    ap.add_argument("--batch", type=int, default=8, help="learned start: mini-batch")
    ap.add_argument("--lr", type=float, default=1e-3, help="learned start: Adam learning rate")
    ap.add_argument("--unet-levels", type=int, default=2, help="learned start: U-Net levels")
    ap.add_argument("--infer-batch", type=int, default=8, help="learned start: slices per inference call")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default tile schedule instead of the autotuned one")
    ap.add_argument("--tiles", default="",
                    help="finest level's schedule as rows_fwd,cols_conv,rows_inv,chunks (no autotune); "
                         "counter runs use it to repeat the schedule a timed run chose")
    ap.add_argument("--copy-calib", action="store_true",
                    help="only run a plain copy kernel of known size (counter calibration)")
    ap.add_argument("--hbm-rates", action="store_true",
                    help="only time plain streaming kernels (read, write, copy of 512 MiB) for "
                         "the HBM rates this part reaches outside the path")
    ap.add_argument("--cpu-only", action="store_true",
                    help="only the host measurements (oracle baseline, direct vs Toeplitz); no GPU")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(this build runs the one-GPU share of a slice-axis sharding)", file=sys.stderr)
        return 2

    if args.cpu_only:
        return run_cpu_only(args)
    if args.workload == "learned_init_512":
        return run_learned(args)
    if args.workload == "batch_256":
        return run_batch(args)
    if args.workload == "direct_vs_toeplitz":
        return run_direct(args)
    if args.workload == "stream_256x512":
        return run_stream(args)
    if args.workload == "ablation_32x2048":
        return run_ablation(args)

    import numpy as np
    import torch
    dev = torch.device("cuda", 0)

    if args.copy_calib:
        n = 256 * 1024 * 1024 // 4   # 256 MiB read + 256 MiB written per copy
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(5):
            torch.mul(a, 1.0, out=b)   # one elementwise kernel: reads a, writes b
        torch.cuda.synchronize()
        print(json.dumps({"copy_calib_bytes_read": 4 * n, "copy_calib_bytes_written": 4 * n}))
        return 0

    if args.hbm_rates:
        return run_hbm_rates(torch, dev)

    import synth
    from paper_2603_28756_amd import tomo

    wl = synth.WORKLOADS[args.workload]
    iters = list(wl.iterations) if not args.iters else [args.iters] * wl.levels
    pr = synth.make_problem(wl.n, wl.n_slices, wl.n_angles, wl.n_det, wl.noise, wl.seed, wl.n_objects)
    sino32 = pr["sino"].astype(np.float32)
    sino = torch.from_numpy(sino32).to(dev)
    plan = tomo.Plan(wl.n, wl.n_slices, wl.n_angles, wl.n_det, angles=list(pr["angles"]),
                     n_levels=wl.levels, kb_width=wl.kb_width, kb_oversamp=wl.kb_oversamp,
                     beta=wl.beta, p=wl.p, q=wl.q, sigma=wl.sigma, T=wl.T,
                     neighbours=wl.neighbours, device=dev, fused_prior=args.fused_prior,
                     concurrent_prior=args.concurrent_prior)
    x = torch.empty((wl.n_slices, wl.n, wl.n), dtype=torch.float32, device=dev)
    _, _, P = plan.level_dims(wl.levels - 1)

    def step():
        plan.precompute_psf()
        plan.reconstruct(sino, x, iters, init=tomo.INIT_FBP, stats=False)

    # plan-time tile choice (once per geometry, outside the timed steps)
    tiles, tune_s = None, 0.0
    if args.tiles:
        f, c, i, k = (int(v) for v in args.tiles.split(","))
        sched = plan.tiles()
        sched[-1].update({"rows_fwd": f, "cols_conv": c, "rows_inv": i, "chunks": k})
        tiles = plan.tiles(sched)
    elif not args.no_autotune:
        t0 = time.perf_counter()
        tiles = plan.autotune(reps=5)
        tune_s = time.perf_counter() - t0
    for _ in range(args.warmup):
        step()
    # one step with every class timed: the breakdown, and which class dominates
    plan.timing_enable(range(tomo.T_COUNT))
    step()
    ms_all, cnt_all = plan.timing_read()
    breakdown = {CLASS_NAMES[i]: {"total_ms": ms_all[i], "launches": cnt_all[i],
                                  "mean_ms": ms_all[i] / cnt_all[i] if cnt_all[i] else None}
                 for i in range(tomo.T_COUNT)}
    iter_classes = [tomo.T_ROWS_FWD, tomo.T_COLS_CONV, tomo.T_ROWS_INV, tomo.T_PRIOR]
    hot = max(iter_classes, key=lambda i: ms_all[i])

    # timed region, run as a caller would: no per-kernel events, so the iteration loop
    # replays its captured graphs
    plan.timing_enable([])
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    ms_per_step = e0.elapsed_time(e1) / args.steps

    # roofline pass: the same steps again with HIP events around every launch of the
    # dominant kernel class on the plan's stream (event recording disables graph replay,
    # which changes launch gaps, not kernel durations)
    plan.timing_enable([hot])
    for _ in range(args.steps):
        step()
    ms_hot, cnt_hot = plan.timing_read()
    plan.timing_enable([])
    mean_hot_ms = ms_hot[hot] / max(cnt_hot[hot], 1)

    # phases timed on their own (median of 5): the float64 precompute, R* g and FBP, and the
    # iteration loop as the wall time of a full call minus a zero-iteration call (graph replay)
    def ev_ms(fn, reps=5):
        ts = []
        for _ in range(reps):
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))
    tmp = torch.empty_like(x)
    phases = {
        # the precompute runs on the plan's PSF stream; reading F K back orders the plan's
        # stream after it (and L on the host waits for it)
        "psf_spectrum_and_step_ms": ev_ms(lambda: (plan.precompute_psf(), plan.psf_info())),
        "backprojection_ms": ev_ms(lambda: plan.backproject(sino, tmp, ramp=False)),
        "fbp_ms": ev_ms(lambda: plan.backproject(sino, tmp, ramp=True)),
        "call_without_iterations_ms": ev_ms(
            lambda: plan.reconstruct(sino, x, [0] * wl.levels, init=tomo.INIT_FBP, stats=False)),
        "call_with_iterations_ms": ev_ms(
            lambda: plan.reconstruct(sino, x, iters, init=tomo.INIT_FBP, stats=False)),
    }
    del tmp
    loop_ms = phases["call_with_iterations_ms"] - phases["call_without_iterations_ms"]
    phases["iteration_loop_ms"] = loop_ms
    phases["iteration_wall_ms"] = loop_ms / sum(iters)

    total_iters = sum(iters)
    vox = wl.n * wl.n * wl.n_slices * total_iters
    value = vox / (ms_per_step * 1e-3)
    iter_ms = sum(breakdown[CLASS_NAMES[i]]["total_ms"]
                  for i in iter_classes + [tomo.T_FINALIZE]) / total_iters
    name = CLASS_NAMES[hot]
    alg = algorithmic_bytes(name, wl.n, wl.n_slices, P, args.fused_prior, args.concurrent_prior)
    traffic = read_traffic(name)
    achieved = alg / (mean_hot_ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "kernel": name, "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "algorithmic_bytes_per_launch": alg}
    if name == "prior":
        ops = prior_lane_ops(wl.n, wl.n_slices, wl.neighbours)
        a_ops = ops / (mean_hot_ms * 1e-3) / 1e12
        roof["alu"] = {"achieved": a_ops, "peak": VALU_PEAK_TOPS,
                       "unit": "T lane-ops/s (VALU, FP32 non-packed)", "frac": a_ops / VALU_PEAK_TOPS,
                       "algorithmic_lane_ops_per_launch": ops}
    elif name == "cols_conv":
        flops = cols_conv_flops(wl.n, wl.n_slices, P)
        a_fl = flops / (mean_hot_ms * 1e-3) / 1e12
        roof["alu"] = {"achieved": a_fl, "peak": FP32_PEAK_TFLOPS,
                       "unit": "TFLOP/s (FP32 vector, non-packed; FFT flops 5 P log2 P)",
                       "frac": a_fl / FP32_PEAK_TFLOPS, "algorithmic_flops_per_launch": flops}
    roof.update({"mean_launch_ms": mean_hot_ms, "launches_timed": cnt_hot[hot]})
    # whole iteration against HBM: measured bytes (counter summary) and the byte models
    vox1 = float(wl.n * wl.n * wl.n_slices)
    it_s = phases["iteration_wall_ms"] * 1e-3
    meas = iteration_traffic()
    iteration_hbm = {
        "wall_ms": phases["iteration_wall_ms"],
        "measured_bytes": meas,
        "measured_frac": (meas / it_s / 1e9 / HBM_PEAK_GBS) if meas else None,
        "design_bytes": sum(algorithmic_bytes(c, wl.n, wl.n_slices, P, args.fused_prior,
                                              args.concurrent_prior)
                            for c in ("rows_fwd", "cols_conv", "rows_inv", "prior")),
        "model_56B_frac": 56.0 * vox1 / it_s / 1e9 / HBM_PEAK_GBS,
        "compulsory_20_5B_frac": 20.5 * vox1 / it_s / 1e9 / HBM_PEAK_GBS,
        "voxel_updates_per_s": vox1 / it_s,
    }
    iteration_hbm["design_frac"] = iteration_hbm["design_bytes"] / it_s / 1e9 / HBM_PEAK_GBS
    out = {
        "metric": "gradient voxel-updates/s",
        "value": value,
        "unit": "voxel-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": wl.name, "n": wl.n, "n_slices": wl.n_slices, "n_angles": wl.n_angles,
            "n_det": wl.n_det, "iterations": iters, "pad": P, "kb_width": wl.kb_width,
            "kb_oversamp": wl.kb_oversamp, "neighbours": wl.neighbours, "noise": wl.noise,
            "step": "PSF spectrum + step constant precompute, R*g, FBP start, iterations",
            "tiles": ([{k: t[k] for k in ("fwd_pairs", "col_tile", "inv_pairs", "chunks")} for t in tiles]
                      if tiles else "default"),
            "prior": ("fused epilogue" if args.fused_prior else
                      "pair-shared kernel, " + ("own stream beside the row/column passes"
                                                if args.concurrent_prior else "in sequence")),
        },
        "roofline": roof,
        "iteration_hbm": iteration_hbm,
        "phases_ms_median5": phases,
        "iteration_kernel_ms": iter_ms,
        "breakdown_one_step": breakdown,
        "autotune": {"seconds": tune_s, "levels": tiles} if tiles else None,
        "kernel_source_hash": kernel_source_hash(),
    }
    if not args.no_cpu_baseline:
        cpu = cpu_measurements(args.workload)
        out["cpu_baseline"] = cpu["cpu_baseline"]
        out["cpu_direct_vs_toeplitz"] = cpu["cpu_direct_vs_toeplitz"]
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out))
    return 0


def run_hbm_rates(torch, dev) -> int:
    """HBM rates of plain streaming kernels on 512 MiB buffers (twice the 256 MB Infinity Cache):
    a sum (read only), a fill (write only) and an elementwise copy (256 MiB each way), timed
    with events, best and median of 10 launches after 2 warm-ups.  They give the rates a
    kernel with no arithmetic reaches, beside the 8 TB/s of the data sheet."""
    nbytes = 512 * 1024 * 1024
    a = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    half = nbytes // 8
    acc = torch.empty((), dtype=torch.float32, device=dev)
    cases = {
        "read": (lambda: torch.sum(a, dim=0, out=acc), nbytes),
        "write": (lambda: b.fill_(1.0), nbytes),
        "copy": (lambda: torch.mul(a[:half], 1.0, out=b[:half]), nbytes),
    }
    out = {"metric": "streaming HBM rate", "unit": "GB/s", "buffer_bytes": nbytes}
    for name, (fn, moved) in cases.items():
        ts = []
        for i in range(12):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            if i >= 2:
                ts.append(e0.elapsed_time(e1) * 1e-3)
        ts.sort()
        out[name] = {"best_gbs": moved / ts[0] / 1e9, "median_gbs": moved / ts[len(ts) // 2] / 1e9,
                     "bytes": moved, "frac_of_8tbs": moved / ts[0] / 1e9 / HBM_PEAK_GBS}
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
