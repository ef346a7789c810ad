"""Many separators per axis (through the C ABI): the second gridding of
Sec. 2, about sqrt(n) x sqrt(n) blocks of about sqrt(n) nodes per side on
general non-uniform x and y steps with stretched ends, against the oracle in
both precisions.  With more than 4 separators on an axis the right-hand side
of the global interface solve is expanded densely before the z solve; the
tests cover ragged column and row tiles of that expansion, more than one
chunk of 16 separators, axes whose counts differ (groups of the interface
contraction with no terms on one axis), the forced dense path against the
low-rank one, the adjoint and the layer gradient."""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint, direct, separable

from parity import check

pytestmark = pytest.mark.gpu

TOL128 = 1e-10
TOL64R = 1e-8


def dev(a):
    import paper_1909_01299_amd as hs
    return hs.to_device(a)


def solve(hs, p, f, prec, **kw):
    import torch
    mixed = prec == "mixed"
    plan = hs.Plan(p, prec, max_rhs=f.shape[0], refine_steps=1 if mixed else 0,
                   tol=TOL64R if mixed else TOL128, **kw)
    u = plan.solve(dev(f))
    torch.cuda.synchronize()
    plan.check()
    return plan, u.cpu().numpy()


@pytest.mark.parametrize("prec,tol", [("c128", TOL128), ("mixed", TOL64R)])
@pytest.mark.parametrize("cfg", [
    dict(nx=64, ny=49, nz=40, pml=5),     # 7 x 6 separators, blocks of 7-8 nodes
    dict(nx=100, ny=16, nz=33, pml=4),    # 9 x 3: the later contraction groups hold x terms only
    dict(nx=20, ny=324, nz=10, pml=3),    # 3 x 17: two chunks of y terms in the expansion
])
def test_gridding_b_vs_oracle(hs, prec, tol, cfg):
    rng = np.random.default_rng(cfg["nx"] * 7 + cfg["ny"])
    p = W.gridding_b_problem(cfg["nx"], cfg["ny"], cfg["nz"], 4, rng, pml=cfg["pml"])
    assert max(len(p.sep_x), len(p.sep_y)) > 4
    f = W.complex_normal(rng, (2,) + p.shape)
    _, u = solve(hs, p, f, prec)
    check(u, separable.solve(p, f), tol, p)


def test_gridding_b_vs_sparse_lu(hs):
    rng = np.random.default_rng(3)
    p = W.gridding_b_problem(36, 25, 6, 3, rng, pml=3)
    assert len(p.sep_x) == 5 and len(p.sep_y) == 4
    f = W.complex_normal(rng, (2,) + p.shape)
    _, u = solve(hs, p, f, "c128")
    check(u, direct.solve_splu(p, f), TOL128, p)


@pytest.mark.parametrize("prec", ["c128", "mixed"])
def test_dense_global_rhs_matches_low_rank_terms(hs, prec):
    """On a grid with at most 4 separators per axis the expanded global
    right-hand side (forced) and the low-rank terms inside the z solve give
    the same answer to rounding."""
    p, f = W.c2_decomposed(core_cells=48, pml_cells=6, nz=24, nlayers=4)
    rng = np.random.default_rng(9)
    f = np.concatenate([f, W.complex_normal(rng, f.shape)])
    _, u_lr = solve(hs, p, f, prec)
    _, u_dn = solve(hs, p, f, prec, dense_global=True)
    tol = 1e-12 if prec == "c128" else 1e-9
    check(u_dn, u_lr, tol)
    check(u_dn, separable.solve(p, f), TOL128 if prec == "c128" else TOL64R, p)


def test_gridding_b_large_sampled(hs):
    """255 x 255 x 48 split 16 x 16 (15 separators per axis), one source on a
    separator crossing and one inside a block, complex128 and mixed."""
    rng = np.random.default_rng(11)
    p = W.gridding_b_problem(255, 255, 48, 6, rng, pml=10)
    assert len(p.sep_x) == 15 and len(p.sep_y) == 15
    f = W.point_source_batch(p, [(int(p.sep_x[7]), int(p.sep_y[7]), 24), (100, 140, 10)])
    ref = separable.solve(p, f)
    for prec, tol in (("c128", TOL128), ("mixed", TOL64R)):
        _, u = solve(hs, p, f, prec)
        check(u, ref, tol, p, label=prec)


def test_gridding_b_adjoint_and_gradient(hs):
    import torch
    rng = np.random.default_rng(12)
    p = W.gridding_b_problem(49, 36, 20, 5, rng, pml=4)
    g = W.complex_normal(rng, (1,) + p.shape)
    plan = hs.Plan(p, "c128")
    a = plan.solve_adjoint(dev(g)).cpu().numpy()
    check(a, adjoint.solve_adjoint(p, g), TOL128, p)
    # layer gradient of a plane misfit
    f = W.point_source(p.shape, 20, 17, 6)
    d = separable.solve(p.with_k2(p.k2 * 1.05), f)[12]
    J, g_ref, u_ref, a_ref = adjoint.plane_misfit_grad(p, f, 12, d)
    u = plan.solve(dev(f[None]))
    resid = np.zeros((1,) + p.shape, complex)
    resid[0, 12] = u.cpu().numpy()[0, 12] - d
    lam = plan.solve_adjoint(dev(resid))
    gk = plan.grad_k2(u, lam).cpu().numpy()[0]
    torch.cuda.synchronize()
    assert np.abs(gk - g_ref).max() < 1e-8 * np.abs(g_ref).max()


def test_global_form_as_launch_shape(hs, tmp_path):
    """With at most 4 separators per axis the global right-hand side's form is
    a launch shape: both forms agree with each other and the oracle, the tuner
    picks one and caches it, and a grid with more separators refuses the
    low-rank form."""
    import torch
    p, f = W.c2_decomposed(core_cells=48, pml_cells=6, nz=24, nlayers=4)
    plan = hs.Plan(p, "c128")
    assert plan.info()["global_dense"] == 0
    u_lr = plan.solve(dev(f)).cpu().numpy()
    plan.set_launch({"z_chunks": 0, "sine_lines": 0, "z_fixed_rows": 0, "global_dense": 1})
    assert plan.info()["global_dense"] == 1
    u_dn = plan.solve(dev(f)).cpu().numpy()
    check(u_dn, u_lr, 1e-12)
    check(u_dn, separable.solve(p, f), TOL128, p)
    cache = str(tmp_path / "tune.jsonl")
    shapes = plan.tune(1, cache=cache)
    assert shapes["global_dense"] in (0, 1)
    assert '"global_dense": ' in open(cache).read()
    plan2 = hs.Plan(p, "c128")
    assert plan2.tune(1, cache=cache) == shapes
    u2 = plan2.solve(dev(f)).cpu().numpy()
    torch.cuda.synchronize()
    check(u2, separable.solve(p, f), TOL128, p)
    rng = np.random.default_rng(4)
    q = W.gridding_b_problem(36, 25, 6, 3, rng, pml=3)
    wide = hs.Plan(q, "c128")
    assert wide.info()["global_dense"] == 1
    with pytest.raises(hs.HSError) as e:
        wide.set_launch({"global_dense": 0})
    assert e.value.status == hs.HS_ERR_ARG
