"""The coefficient sigma(z) of eqs. (1)-(2) on the GPU (through the C ABI):
block solves on sine and dense axes, decomposed solves, mixed precision, the
FP64 stencil, the adjoint gradient and the batch, all against the FP64
oracle with sigma."""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint, direct, operator, separable

from parity import check

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-10, "mixed": 1e-8}


def dev(a):
    import paper_1909_01299_amd as hs
    return hs.to_device(a)


def _sig(p, rng, L=None):
    return W.with_sigma(p, W.draw_sigma(rng, L or p.nlayers))


@pytest.mark.parametrize("prec", ["c128", "mixed"])
@pytest.mark.parametrize("cfg", [dict(nx=63, ny=31, nz=40, px=0, py=0),     # sine transforms on both axes
                                 dict(nx=40, ny=36, nz=48, px=5, py=4),     # dense tables on both axes
                                 dict(nx=127, ny=20, nz=33, px=0, py=3)])
def test_sigma_block_vs_oracle(hs, prec, cfg):
    rng = np.random.default_rng(cfg["nx"] + cfg["nz"])
    p = _sig(W.random_problem(cfg["nx"], cfg["ny"], cfg["nz"], 4, rng, pml_x=cfg["px"], pml_y=cfg["py"]), rng)
    f = W.complex_normal(rng, (2,) + p.shape)
    plan = hs.Plan(p, prec, max_rhs=2, refine_steps=1 if prec == "mixed" else 0)
    u = plan.solve(dev(f)).cpu().numpy()
    check(u, separable.solve(p, f), TOL[prec])


def test_sigma_decomposed_vs_sparse_lu(hs):
    rng = np.random.default_rng(51)
    p = _sig(W.random_problem(17, 17, 6, 3, rng, sep_x=[3, 8, 13], sep_y=[3, 8, 13], pml_x=3, pml_y=3), rng)
    f = W.complex_normal(rng, (2,) + p.shape)
    u = hs.Plan(p, "c128", max_rhs=2).solve(dev(f)).cpu().numpy()
    check(u, direct.solve_splu(p, f), 1e-10, p)


@pytest.mark.parametrize("prec", ["c128", "mixed"])
def test_sigma_decomposed_pml_grid_vs_oracle(hs, prec):
    rng = np.random.default_rng(52)
    p, f = W.c2_decomposed(core_cells=64, pml_cells=8, nz=40, nlayers=8)
    p = _sig(p, rng)
    f = f + 0.1 * W.complex_normal(rng, f.shape)
    u = hs.Plan(p, prec, refine_steps=1 if prec == "mixed" else 0).solve(dev(f)).cpu().numpy()
    check(u[0], separable.solve(p, f[0]), TOL[prec], p)


def test_sigma_stencil_vs_oracle(hs):
    rng = np.random.default_rng(53)
    p = _sig(W.random_problem(20, 18, 16, 4, rng, pml_x=3, pml_y=2), rng)
    u = W.complex_normal(rng, (2,) + p.shape)
    au = hs.Plan(p, "c128", max_rhs=2).apply(dev(u)).cpu().numpy()
    ref = operator.apply_A(p, u)
    assert np.abs(au - ref).max() < 1e-12 * np.abs(ref).max()


def test_sigma_adjoint_and_gradient_vs_oracle(hs):
    import torch
    rng = np.random.default_rng(54)
    p = _sig(W.random_problem(24, 20, 30, 5, rng, pml_x=3, pml_y=3), rng)
    f = W.point_source(p.shape, 10, 9, 6)[None]
    d = separable.solve(p.with_k2(p.k2 * 1.05), f[0])[12]
    J_ref, g_ref, _, _ = adjoint.plane_misfit_grad(p, f[0], 12, d)
    plan = hs.Plan(p, "c128")
    k2 = torch.tensor(p.k2, dtype=torch.complex128, requires_grad=True)
    u = hs.helmholtz_solve(k2, dev(f), plan)
    J = 0.5 * (u[0, 12] - dev(d)).abs().pow(2).sum()
    J.backward()
    assert abs(float(J.detach()) - J_ref) < 1e-9 * abs(J_ref)
    assert np.abs(k2.grad.numpy() - g_ref).max() < 1e-8 * np.abs(g_ref).max()


def test_sigma_batch_vs_oracle_and_single_plans(hs):
    import torch
    rng = np.random.default_rng(55)
    probs = [_sig(W.uniform_problem(31, 20, 24, 3, rng), rng),
             _sig(W.random_problem(26, 33, 17, 2, rng, pml_x=3, pml_y=4), rng)]
    fs = [W.complex_normal(rng, (2,) + p.shape) for p in probs]
    plans = [hs.Plan(p, "c128", max_rhs=1) for p in probs]
    batch = hs.Batch(plans, [2, 2])
    us = batch.solve([dev(f) for f in fs])
    torch.cuda.synchronize()
    for p, f, u in zip(probs, fs, us):
        check(u.cpu().numpy(), separable.solve(p, f), 1e-10)
