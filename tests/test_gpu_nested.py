"""Multi-level cyclic reduction on nested partitions (through the
C ABI): a plan whose interface problem (Alg. step 5) is solved by the cyclic
reduction of a coarser plan on the same grid, to any depth, against the
oracle in both precisions; the coarsest level a single block; k^2 updates
reaching every level; the adjoint; and the argument checks of
hs_plan_set_coarse."""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint, cyclic, separable

from parity import check

pytestmark = pytest.mark.gpu

TOL128 = 1e-10
TOL64R = 1e-8


def dev(a):
    import paper_1909_01299_amd as hs
    return hs.to_device(a)


def levels_of(p, sx, sy):
    from dataclasses import replace
    return replace(p, sep_x=np.asarray(sx, np.int32), sep_y=np.asarray(sy, np.int32))


def chain(hs, problems, prec, nrhs):
    mixed = prec == "mixed"
    plans = [hs.Plan(q, prec, max_rhs=nrhs, refine_steps=1 if mixed else 0, tol=TOL64R if mixed else TOL128)
             for q in problems]
    for fine, coarse in zip(plans[:-1], plans[1:]):
        fine.set_coarse(coarse)
    return plans


@pytest.mark.parametrize("prec,tol", [("c128", TOL128), ("mixed", TOL64R)])
def test_three_levels_vs_oracle(hs, prec, tol):
    import torch
    rng = np.random.default_rng(51)
    p = W.gridding_b_problem(64, 49, 30, 4, rng, pml=5)
    sx, sy = p.sep_x.tolist(), p.sep_y.tolist()
    mid = levels_of(p, sx[1::2], sy[1::2])
    top = levels_of(p, [sx[3]], [sy[3]])
    f = W.complex_normal(rng, (2,) + p.shape)
    plans = chain(hs, [p, mid, top], prec, 2)
    u = plans[0].solve(dev(f))
    torch.cuda.synchronize()
    plans[0].check()
    un = u.cpu().numpy()
    ref = separable.solve(p, f)
    check(un, ref, tol, p)
    # the oracle's own nested form agrees with its direct solve
    check(cyclic.nested(p, f, [(sx[1::2], sy[1::2]), ([sx[3]], [sy[3]])]), ref, 1e-12)


def test_coarsest_level_a_single_block_matches_two_levels(hs):
    """A coarser plan without separators solves the interface problem on the
    whole grid in its own eigenbasis: the same answer as the global step."""
    import torch
    p, f = W.c2_decomposed(core_cells=48, pml_cells=6, nz=24, nlayers=4)
    rng = np.random.default_rng(3)
    f = np.concatenate([f, W.complex_normal(rng, f.shape)])
    two = hs.Plan(p, "c128", max_rhs=2)
    u2 = two.solve(dev(f)).cpu().numpy()
    plans = chain(hs, [p, levels_of(p, [], [])], "c128", 2)
    u = plans[0].solve(dev(f)).cpu().numpy()
    torch.cuda.synchronize()
    check(u, u2, 1e-12)
    check(u, separable.solve(p, f), TOL128, p)
    # detaching restores the global step
    plans[0].set_coarse(None)
    assert np.array_equal(plans[0].solve(dev(f)).cpu().numpy(), u2)


def test_nested_decomposed_grid_k2_update_and_adjoint(hs):
    """4 x 4 blocks whose interface problem goes to the 2 x 2 partition of
    the middle separators; k^2 set on the finest plan reaches the coarser
    one; the adjoint solve through the chain against the oracle."""
    import torch
    p, f = W.c2_decomposed(core_cells=64, pml_cells=8, nz=30, nlayers=5)
    mid = levels_of(p, [p.sep_x[1]], [p.sep_y[1]])
    plans = chain(hs, [p, mid], "c128", 1)
    fd = dev(f)
    check(plans[0].solve(fd).cpu().numpy(), separable.solve(p, f), TOL128, p)
    k2n = p.k2 * 1.3
    plans[0].set_k2(k2n)
    pn = p.with_k2(k2n)
    ref = separable.solve(pn, f)
    check(plans[0].solve(fd).cpu().numpy(), ref, TOL128, pn)
    # the coarser plan itself now solves with the new k^2
    check(plans[1].solve(fd).cpu().numpy(), ref, TOL128, mid)
    rng = np.random.default_rng(8)
    g = W.complex_normal(rng, (1,) + p.shape)
    a = plans[0].solve_adjoint(dev(g)).cpu().numpy()
    torch.cuda.synchronize()
    check(a, adjoint.solve_adjoint(pn, g), TOL128, pn)


def test_set_coarse_argument_checks(hs):
    rng = np.random.default_rng(9)
    p = W.gridding_b_problem(36, 25, 6, 3, rng, pml=3)
    fine = hs.Plan(p, "c128")

    def refused(coarse):
        with pytest.raises(hs.HSError) as e:
            fine.set_coarse(coarse)
        assert e.value.status == hs.HS_ERR_ARG

    refused(hs.Plan(levels_of(p, [int(p.sep_x[0]) + 1], []), "c128"))        # not a subset
    refused(hs.Plan(levels_of(p, [], []), "mixed"))                          # another precision
    other = p.with_k2(p.k2 * 2.0)
    refused(hs.Plan(levels_of(other, [], []), "c128"))                       # another k^2
    refused(fine)                                                            # itself
    small = hs.Plan(levels_of(p, [], []), "c128")
    big = hs.Plan(p, "c128", max_rhs=2)
    with pytest.raises(hs.HSError):
        big.set_coarse(small)                                                # max_rhs too small
    single = hs.Plan(levels_of(p, [], []), "c128")
    with pytest.raises(hs.HSError):
        single.set_coarse(hs.Plan(levels_of(p, [], []), "c128"))             # nothing to solve
    # a cycle through two plans
    a = hs.Plan(p, "c128")
    b = hs.Plan(p, "c128")
    a.set_coarse(b)
    with pytest.raises(hs.HSError):
        b.set_coarse(a)
