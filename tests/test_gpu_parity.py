"""GPU vs oracle parity of every operator on the hot path (through the C ABI).

Tolerances: relative L2 <= 1e-5 per operator application and <= 1e-4 for
reconstructions after a fixed iteration count.  The precompute uses a
Kaiser-Bessel width of 8 (gridding error ~1e-7); the full gradient is
normalised by ||T x|| + ||b|| + beta ||grad Phi||, not by ||grad F||, which
vanishes near the optimum.  Sizes cover several tiles, ragged tails (N not a
power of two, row blocks not dividing N), 8 and 26 neighbours, off-centre
rotation axes and single slices.
"""
import numpy as np
import pytest
import torch

import synth

from oracle import fbp as ofbp
from oracle import hierarchy, radon, solver, toeplitz
from oracle import prior as qg

from gpu_util import (make_plan, objective_err, oracle_geom, oracle_prior, problem, rel_l2, to_dev, to_np,
                      dev)

pytestmark = pytest.mark.gpu

CASES = [
    # n, nz, n_angles, n_det, center
    (32, 2, 20, 46, None),
    (64, 3, 45, 92, None),
    (100, 2, 30, 142, 70.5),    # ragged: P = 256, rows not a multiple of the block
    (128, 1, 90, 182, None),    # the single-slice 128^2 workload shape
]


@pytest.mark.parametrize("n,nz,na,nd,c", CASES)
def test_psf_spectrum_and_step(n, nz, na, nd, c):
    sino, ang, center, _ = problem(n, nz, na, nd, seed=n, center=c)
    plan = make_plan(n, nz, ang, nd, center=center)
    plan.precompute_psf()
    fk_gpu, L_gpu, lam_gpu = plan.psf_info()
    geom = oracle_geom(n, ang, nd, center)
    _, _, P = plan.level_dims(0)
    fk = toeplitz.psf_spectrum(geom, P)
    assert rel_l2(to_np(fk_gpu), fk[:, : P // 2 + 1]) < 1e-5
    lam = solver.power_lambda(fk, n, 30)
    assert abs(lam_gpu - lam) / lam < 1e-5
    L = 1.01 * lam + 2 * 0.01 * qg.rho_second_at_zero(oracle_prior())
    assert abs(L_gpu - L) / L < 1e-5


@pytest.mark.parametrize("n,nz,na,nd,c", CASES)
def test_apply_normal(n, nz, na, nd, c):
    sino, ang, center, _ = problem(n, nz, na, nd, seed=n + 1, center=c)
    plan = make_plan(n, nz, ang, nd, center=center)
    plan.precompute_psf()
    rng = np.random.default_rng(n)
    x = rng.standard_normal((nz, n, n)).astype(np.float32).astype(np.float64)
    out = torch.empty((nz, n, n), dtype=torch.float32, device=dev())
    plan.apply_normal(to_dev(x), out)
    _, _, P = plan.level_dims(0)
    ref = toeplitz.apply(x, toeplitz.psf_spectrum(oracle_geom(n, ang, nd, center), P), n)
    assert rel_l2(to_np(out), ref) < 1e-5


@pytest.mark.parametrize("n,nz,na,nd,c", CASES)
def test_backproject_and_fbp(n, nz, na, nd, c):
    sino, ang, center, _ = problem(n, nz, na, nd, seed=n + 2, center=c)
    plan = make_plan(n, nz, ang, nd, center=center)
    g = to_dev(sino)
    out = torch.empty((nz, n, n), dtype=torch.float32, device=dev())
    geom = oracle_geom(n, ang, nd, center)
    plan.backproject(g, out, ramp=False)
    assert rel_l2(to_np(out), radon.adjoint(sino, geom)) < 1e-5
    plan.backproject(g, out, ramp=True)
    assert rel_l2(to_np(out), ofbp.fbp(sino, geom)) < 1e-5


@pytest.mark.parametrize("fused", [False, True])
@pytest.mark.parametrize("nb", [8, 26])
@pytest.mark.parametrize("n,nz,na,nd,c", CASES[:3] + [(48, 37, 20, 68, None)])
def test_gradient_and_objective(n, nz, na, nd, c, nb, fused):
    # nz = 37 spans three z-chunks of the prior kernel with a ragged last chunk
    sino, ang, center, phantom = problem(n, nz, na, nd, seed=n + 3, center=c)
    plan = make_plan(n, nz, ang, nd, center=center, neighbours=nb, fused_prior=fused)
    plan.precompute_psf()
    geom = oracle_geom(n, ang, nd, center)
    _, _, P = plan.level_dims(0)
    fk = toeplitz.psf_spectrum(geom, P)
    b = radon.adjoint(sino, geom)
    rng = np.random.default_rng(7)
    x = (phantom + 0.05 * rng.standard_normal(phantom.shape)).astype(np.float32).astype(np.float64)
    b32 = b.astype(np.float32).astype(np.float64)
    grad = torch.empty((nz, n, n), dtype=torch.float32, device=dev())
    obj = torch.zeros(1, dtype=torch.float64, device=dev())
    plan.gradient(to_dev(x), to_dev(b32), grad, obj)
    pr = oracle_prior(nb)
    tx = toeplitz.apply(x, fk, n)
    gphi = qg.gradient(x, pr)
    ref = tx - b32 + 0.01 * gphi
    norm = np.linalg.norm(tx) + np.linalg.norm(b32) + 0.01 * np.linalg.norm(gphi)
    assert np.linalg.norm(to_np(grad) - ref) / norm < 1e-5
    obj_ref = 0.5 * float(np.vdot(x, tx)) - float(np.vdot(x, b32)) + 0.01 * qg.value(x, pr)
    scale = 0.5 * abs(float(np.vdot(x, tx))) + abs(float(np.vdot(x, b32))) + 0.01 * qg.value(x, pr)
    assert abs(float(to_np(obj)[0]) - obj_ref) / scale < 1e-5


@pytest.mark.parametrize("fused", [False, True])
@pytest.mark.parametrize("p", [1.2, 2.0])
@pytest.mark.parametrize("nb", [8, 26])
@pytest.mark.parametrize("n,nz", [(16, 1), (48, 37), (80, 18)])
def test_prior_dominated_gradient(n, nz, nb, p, fused):
    # beta = 1e3 makes beta grad Phi the bulk of the gradient, so this checks the prior kernel
    # (interior tiles, edge tiles, ragged z-chunks; p < q and the quadratic p = q = 2) to 1e-5.
    na, nd = 24, synth.detector_bins_for(n)
    sino, ang, center, phantom = problem(n, nz, na, nd, seed=n + nz)
    beta = 1e3
    plan = make_plan(n, nz, ang, nd, neighbours=nb, beta=beta, p=p, fused_prior=fused)
    plan.precompute_psf()
    geom = oracle_geom(n, ang, nd, center)
    _, _, P = plan.level_dims(0)
    fk = toeplitz.psf_spectrum(geom, P)
    rng = np.random.default_rng(n * nz)
    x = (phantom + 0.1 * rng.standard_normal(phantom.shape)).astype(np.float32).astype(np.float64)
    b = np.zeros_like(x)
    grad = torch.empty((nz, n, n), dtype=torch.float32, device=dev())
    obj = torch.zeros(1, dtype=torch.float64, device=dev())
    plan.gradient(to_dev(x), to_dev(b), grad, obj)
    pr = oracle_prior(nb, p=p)
    tx = toeplitz.apply(x, fk, n)
    gphi = qg.gradient(x, pr)
    ref = tx + beta * gphi
    norm = np.linalg.norm(tx) + beta * np.linalg.norm(gphi)
    assert beta * np.linalg.norm(gphi) > 10 * np.linalg.norm(tx)
    assert np.linalg.norm(to_np(grad) - ref) / norm < 1e-5
    obj_ref = 0.5 * float(np.vdot(x, tx)) + beta * qg.value(x, pr)
    assert abs(float(to_np(obj)[0]) - obj_ref) / abs(obj_ref) < 1e-5


def _oracle_fista(sino, ang, nd, center, n, nb, iters, init, restart=True, L=None, beta=0.01):
    geom = oracle_geom(n, ang, nd, center)
    prob = solver.build(geom, sino, oracle_prior(nb), beta)
    x0 = ofbp.fbp(sino, geom) if init == "fbp" else np.zeros_like(prob.b)
    return solver.fista(prob, x0, iters, L=L, restart=restart)


@pytest.mark.parametrize("fused", [False, True])
@pytest.mark.parametrize("n,nz,na,nd,nb,iters", [(64, 3, 45, 92, 26, 20), (128, 1, 90, 182, 8, 20),
                                                 (100, 2, 30, 142, 26, 12)])
def test_reconstruct_parity(n, nz, na, nd, nb, iters, fused):
    from paper_2603_28756_amd import tomo
    sino, ang, center, _ = problem(n, nz, na, nd, seed=n + 4)
    plan = make_plan(n, nz, ang, nd, neighbours=nb, fused_prior=fused)
    x = torch.empty((nz, n, n), dtype=torch.float32, device=dev())
    hist = torch.zeros(iters, dtype=torch.float64, device=dev())
    rs = torch.zeros(iters, dtype=torch.int32, device=dev())
    stats = plan.reconstruct(to_dev(sino), x, [iters], init=tomo.INIT_FBP, objective=hist,
                             restarts=rs)
    ref = _oracle_fista(sino, ang, nd, center, n, nb, iters, "fbp")
    assert rel_l2(to_np(x), ref.x) < 1e-4
    assert abs(stats["L"][0] - ref.L) / ref.L < 1e-5
    # The Toeplitz-form objective (Eq. 10) is a difference of terms of size ~<g, g>, each
    # known to ~1e-6 relative in float32, so its error is measured against <g, g>.
    h = to_np(hist)
    assert np.max(np.abs(h - np.array(ref.history))) / float(np.vdot(sino, sino)) < 1e-5
    assert [int(k) for k in np.nonzero(to_np(rs))[0]] == ref.restarts
    assert stats["nonfinite_iter"] == -1


def test_reconstruct_restart_log():
    # A strong prior makes the problem strongly convex; momentum then overshoots and the
    # gradient-mapping test fires (at iteration 26 here, with |cos| of the tested vectors
    # >= 0.02 around the decision, far above float32 noise).  Both sides must restart at
    # the same iterations.
    from paper_2603_28756_amd import tomo
    n, nz, na, nd = 64, 2, 40, 92
    sino, ang, center, _ = problem(n, nz, na, nd, seed=9)
    plan = make_plan(n, nz, ang, nd, neighbours=26, beta=50.0)
    iters = 32
    x = torch.empty((nz, n, n), dtype=torch.float32, device=dev())
    rs = torch.zeros(iters, dtype=torch.int32, device=dev())
    stats = plan.reconstruct(to_dev(sino), x, [iters], init=tomo.INIT_ZERO, restarts=rs)
    ref = _oracle_fista(sino, ang, nd, center, n, 26, iters, "zero", beta=50.0)
    assert len(ref.restarts) > 0
    assert [int(k) for k in np.nonzero(to_np(rs))[0]] == ref.restarts
    assert stats["n_restarts"] == len(ref.restarts)
    assert rel_l2(to_np(x), ref.x) < 1e-4


def test_hierarchy_parity():
    from paper_2603_28756_amd import tomo
    n, nz, na, nd = 128, 2, 36, 184
    sino, ang, center, _ = problem(n, nz, na, nd, seed=12)
    plan = make_plan(n, nz, ang, nd, neighbours=26, n_levels=2)
    x = torch.empty((nz, n, n), dtype=torch.float32, device=dev())
    iters = [10, 6]
    plan.reconstruct(to_dev(sino), x, iters, init=tomo.INIT_FBP)
    ref = hierarchy.reconstruct(oracle_geom(n, ang, nd), sino, oracle_prior(26), 0.01, iters,
                                init="fbp")
    assert rel_l2(to_np(x), ref.x) < 1e-4


def test_three_level_hierarchy_parity():
    """Three levels (64 -> 128 -> 256, projections subsampled by 4 and 2 on the coarse levels)
    with the 26-neighbour prior, against the oracle's level loop."""
    from paper_2603_28756_amd import tomo
    n, nz, na, nd = 256, 3, 40, 368
    sino, ang, center, _ = problem(n, nz, na, nd, seed=14)
    plan = make_plan(n, nz, ang, nd, neighbours=26, n_levels=3)
    assert [plan.level_dims(l)[:2] for l in range(3)] == [(64, 92), (128, 184), (256, 368)]
    x = torch.empty((nz, n, n), dtype=torch.float32, device=dev())
    iters = [10, 6, 4]
    hist = torch.zeros(sum(iters), dtype=torch.float64, device=dev())
    rs = torch.zeros(sum(iters), dtype=torch.int32, device=dev())
    plan.reconstruct(to_dev(sino), x, iters, init=tomo.INIT_FBP, objective=hist, restarts=rs)
    ref = hierarchy.reconstruct(oracle_geom(n, ang, nd), sino, oracle_prior(26), 0.01, iters,
                                init="fbp")
    ref_hist = [v for lv in ref.levels for v in lv.history]
    ref_rst, off = [], 0
    for lv, it in zip(ref.levels, iters):
        ref_rst += [off + k for k in lv.restarts]
        off += it
    assert [int(k) for k in np.nonzero(to_np(rs))[0]] == ref_rst
    # the objective is a difference of terms of size <g, g> (Eq. 10): graded against F(0)
    assert objective_err(to_np(hist), ref_hist, sino) < 1e-5
    assert rel_l2(to_np(x), ref.x) < 1e-4


def test_lanczos_prolong_parity():
    from paper_2603_28756_amd import tomo
    rng = np.random.default_rng(3)
    f = rng.standard_normal((3, 40, 40)).astype(np.float32).astype(np.float64)
    out = tomo.lanczos_prolong(to_dev(f))
    assert rel_l2(to_np(out), hierarchy.prolong(f)) < 1e-6


def test_not_ready_before_psf():
    from paper_2603_28756_amd import tomo
    sino, ang, center, _ = problem(32, 1, 10, 46, seed=1)
    plan = make_plan(32, 1, ang, 46)
    x = torch.zeros((1, 32, 32), dtype=torch.float32, device=dev())
    with pytest.raises(tomo.TomoError) as e:
        plan.gradient(x, x.clone(), torch.empty_like(x))
    assert e.value.status == 6


def test_graph_replay_matches_direct_launches():
    # The iteration loop replays captured 3-iteration graphs; every replay must equal the
    # directly launched iterations bit for bit, also after unrelated eager work between calls,
    # with the prior kernel on its own stream or in sequence.  In sequence the prior kernel
    # also writes y and gp - b for passes R and R' (a different rounding order of the same
    # sums), so the two settings agree to rounding, not bit for bit.
    from paper_2603_28756_amd import tomo
    n, nz, na, nd, iters = 64, 2, 30, 92, 20
    sino, ang, center, _ = problem(n, nz, na, nd, seed=21)
    g = to_dev(sino)
    outs = {False: [], True: []}
    # (graphs, concurrent prior): the prior kernel in sequence or on its own stream
    for graphs, conc in ((False, False), (False, True), (True, True), (True, False)):
        plan = make_plan(n, nz, ang, nd, neighbours=26, graphs=graphs, concurrent_prior=conc)
        for rep in range(2):
            x = torch.empty((nz, n, n), dtype=torch.float32, device=dev())
            hist = torch.zeros(iters, dtype=torch.float64, device=dev())
            plan.reconstruct(g, x, [iters], init=tomo.INIT_FBP, objective=hist)
            junk = torch.randn(1 << 20, device=dev())
            junk.mul_(2.0).sum().item()
            torch.cuda.synchronize()
            outs[conc].append((x.clone(), hist.clone()))
    for conc in (False, True):
        ref_x, ref_h = outs[conc][0]
        for x, h in outs[conc][1:]:
            assert torch.equal(x, ref_x)
            assert torch.equal(h, ref_h)
    (xs, hs), (xc, hc) = outs[False][0], outs[True][0]
    assert rel_l2(to_np(xs), to_np(xc)) < 1e-5
    # objective differences relative to F(0) = <g, g>/2, the scale of the terms that cancel in F
    assert np.max(np.abs(to_np(hs) - to_np(hc))) / abs(float(hc[0])) < 1e-5
