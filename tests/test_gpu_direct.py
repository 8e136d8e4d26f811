"""The direct (non-Toeplitz) path on the GPU: the forward projection R x (Sec. 2, Eq. 3) and the
gradient R*(R x - g) + beta grad Phi(x) evaluated with both non-uniform transforms, against
the FP64 oracle (oracle.radon, exact non-uniform DFTs), the adjoint identity between the
GPU's R and R*, and the Toeplitz gradient of the same plan (Sec. 3.1 compares the two).

Kaiser-Bessel width 8 (gridding error ~1e-7): per-operator relative L2 <= 1e-5; the
gradient normalised by ||R*R x|| + ||R* g|| + beta ||grad Phi||; objectives relative to
F(0) = <g, g>/2.
"""
import numpy as np
import pytest
import torch

from oracle import radon
from oracle import prior as qg

from gpu_util import dev, make_plan, oracle_geom, oracle_prior, problem, rel_l2, to_dev, to_np

pytestmark = pytest.mark.gpu

CASES = [  # n, nz, n_angles, n_det, center
    (32, 2, 20, 46, None), (64, 3, 45, 92, None), (100, 2, 30, 142, 70.5), (128, 1, 90, 182, None),
]


def _case(n, nz, na, nd, center, seed=5):
    sino, ang, c, phantom = problem(n, nz, na, nd, seed=seed, center=center)
    rng = np.random.default_rng(seed)
    x = (phantom + 0.05 * rng.standard_normal(phantom.shape)).astype(np.float32).astype(np.float64)
    return sino, ang, c, x


@pytest.mark.parametrize("n,nz,na,nd,center", CASES)
def test_forward_projection(n, nz, na, nd, center):
    sino, ang, c, x = _case(n, nz, na, nd, center)
    plan = make_plan(n, nz, ang, nd, center=center)
    out = torch.empty((nz, na, nd), dtype=torch.float32, device=dev())
    plan.forward_project(to_dev(x), out)
    ref = radon.forward(x, oracle_geom(n, ang, nd, center))
    assert rel_l2(to_np(out), ref) < 1e-5


@pytest.mark.parametrize("n,nz,na,nd,center", CASES)
def test_forward_and_backprojection_are_adjoint(n, nz, na, nd, center):
    sino, ang, c, x = _case(n, nz, na, nd, center, seed=7)
    plan = make_plan(n, nz, ang, nd, center=center)
    ax = torch.empty((nz, na, nd), dtype=torch.float32, device=dev())
    atg = torch.empty((nz, n, n), dtype=torch.float32, device=dev())
    xd, gd = to_dev(x), to_dev(sino)
    plan.forward_project(xd, ax)
    plan.backproject(gd, atg, ramp=False)
    lhs = float(np.vdot(to_np(ax), sino))
    rhs = float(np.vdot(x, to_np(atg)))
    scale = np.linalg.norm(to_np(ax)) * np.linalg.norm(sino)
    assert abs(lhs - rhs) / scale < 1e-6


@pytest.mark.parametrize("n,nz,na,nd,center", CASES)
@pytest.mark.parametrize("neighbours", [8, 26])
def test_direct_gradient_and_objective(n, nz, na, nd, center, neighbours):
    sino, ang, c, x = _case(n, nz, na, nd, center, seed=9)
    geom = oracle_geom(n, ang, nd, center)
    plan = make_plan(n, nz, ang, nd, center=center, neighbours=neighbours)
    grad = torch.empty((nz, n, n), dtype=torch.float32, device=dev())
    obj = torch.zeros(1, dtype=torch.float64, device=dev())
    plan.gradient_direct(to_dev(x), to_dev(sino), grad, obj)
    pr = oracle_prior(neighbours)
    ax = radon.forward(x, geom)
    r = ax - sino
    t_data = radon.adjoint(r, geom)
    gphi = qg.gradient(x, pr)
    ref = t_data + 0.01 * gphi
    norm = (np.linalg.norm(radon.adjoint(ax, geom)) + np.linalg.norm(radon.adjoint(sino, geom))
            + 0.01 * np.linalg.norm(gphi))
    assert np.linalg.norm(to_np(grad) - ref) / norm < 1e-5
    f_ref = 0.5 * float(np.vdot(r, r)) + 0.01 * qg.value(x, pr)
    assert abs(float(obj.item()) - f_ref) / (0.5 * float(np.vdot(sino, sino))) < 1e-5


@pytest.mark.parametrize("n,nz,na,nd,center", CASES)
def test_direct_and_toeplitz_gradients_agree(n, nz, na, nd, center):
    """The relative difference the paper reports between the two gradients (Sec. 3.1)."""
    sino, ang, c, x = _case(n, nz, na, nd, center, seed=11)
    plan = make_plan(n, nz, ang, nd, center=center)
    plan.precompute_psf()
    xd, gd = to_dev(x), to_dev(sino)
    b = torch.empty((nz, n, n), dtype=torch.float32, device=dev())
    plan.backproject(gd, b, ramp=False)
    g_t = torch.empty_like(b)
    g_d = torch.empty_like(b)
    o_t = torch.zeros(1, dtype=torch.float64, device=dev())
    o_d = torch.zeros(1, dtype=torch.float64, device=dev())
    tx = torch.empty_like(b)
    plan.apply_normal(xd, tx)
    plan.gradient(xd, b, g_t, o_t)
    plan.gradient_direct(xd, gd, g_d, o_d)
    gt, gdn = to_np(g_t), to_np(g_d)
    # the gradient is a difference of terms of size ||R*R x|| and ||R* g|| (each side is within
    # 1e-5 of the oracle in that measure); near the data it is much smaller than either term
    d_terms = np.linalg.norm(gdn - gt) / (np.linalg.norm(to_np(tx)) + np.linalg.norm(to_np(b)))
    d_grad = rel_l2(gdn, gt)
    half_gg = 0.5 * float(np.vdot(sino, sino))
    dl = abs(float(o_d.item()) - (float(o_t.item()) + half_gg)) / half_gg
    print(f"\n[direct vs Toeplitz] N {n}: gradient difference {d_terms:.2e} of the terms, "
          f"{d_grad:.2e} of the gradient; loss {dl:.2e}")
    assert d_terms < 2e-5 and dl < 1e-5
