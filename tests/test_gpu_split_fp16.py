"""Complex64 dense transforms on fp16 matrix cores as two-term splits, against
the FP64 oracle (through the C ABI).

The split carries every operand to about 2^-22 of its group's largest value and
accumulates in FP32, so one complex64 pass has FP32-class error and a single
FP64-residual refinement step reaches the mixed-precision bar.  Cases cover
both table kinds (real sine tables, embedded complex tables), K not a multiple
of the 32-wide k step, partial panels, the largest split tables (256 complex,
512 real), an axis beyond them (FP32 matrix cores), a point source (panels of
very different magnitude) and exact power-of-two scale equivariance.
"""
import numpy as np
import pytest

import workloads as W
from oracle import operator, separable

pytestmark = pytest.mark.gpu

PASS_TOL = 2e-5      # one complex64 pass
TOL64R = 1e-8        # after refinement


def dev(a):
    import paper_1909_01299_amd as hs
    return hs.to_device(a)


def per_rhs_err(u, ref):
    return max(operator.rel_err(np.asarray(u[r]), np.asarray(ref[r])) for r in range(ref.shape[0]))


CASES = [
    # uniform: real tables on both axes (70 -> K padded to 96), partial y panels
    dict(nx=70, ny=50, nz=40, pml_x=0, pml_y=0, split=2),
    # stretched ends: embedded complex tables, n not a multiple of 16
    dict(nx=66, ny=45, nz=36, pml_x=8, pml_y=5, split=2),
    # the largest embedded table (256) and a real y table of 300 (K padded to 320)
    dict(nx=256, ny=300, nz=24, pml_x=10, pml_y=0, split=2),
    # a real x table of 500 (<= 512) and an embedded y table of 40
    dict(nx=500, ny=40, nz=30, pml_x=0, pml_y=4, split=2),
    # an embedded x table of 300 (> 256): FP32 matrix cores; y split
    dict(nx=300, ny=36, nz=32, pml_x=6, pml_y=3, split=1),
]


@pytest.mark.parametrize("cfg", CASES)
def test_one_complex64_pass_and_one_refinement(hs, cfg):
    rng = np.random.default_rng(41)
    p = W.random_problem(cfg["nx"], cfg["ny"], cfg["nz"], 3, rng, pml_x=cfg["pml_x"], pml_y=cfg["pml_y"])
    f = W.complex_normal(rng, (2,) + p.shape)
    ref = separable.solve(p, f)
    p0 = hs.Plan(p, "mixed", max_rhs=2, refine_steps=-1)
    inf = p0.info()
    assert inf["refine_steps"] == 0
    assert inf["n_split_fp16"] == cfg["split"]
    e0 = per_rhs_err(p0.solve(dev(f)).cpu().numpy(), ref)
    assert e0 < PASS_TOL, e0
    p1 = hs.Plan(p, "mixed", max_rhs=2, refine_steps=1)
    e1 = per_rhs_err(p1.solve(dev(f)).cpu().numpy(), ref)
    assert e1 < TOL64R, e1


def test_point_source_panels_of_different_magnitude(hs):
    """A point source leaves most panels orders of magnitude below the one
    that holds it; each panel takes its own scale."""
    rng = np.random.default_rng(42)
    p = W.random_problem(96, 80, 48, 4, rng, pml_x=10, pml_y=8)
    f = W.point_source_batch(p, [(30, 50, 20)])
    ref = separable.solve(p, f)
    u0 = hs.Plan(p, "mixed", refine_steps=-1).solve(dev(f)).cpu().numpy()
    assert per_rhs_err(u0, ref) < PASS_TOL
    u = hs.Plan(p, "mixed").solve(dev(f)).cpu().numpy()
    assert per_rhs_err(u, ref) < TOL64R


@pytest.mark.parametrize("e", [-60, 60])
def test_power_of_two_scaling_is_exact(hs, e):
    """Scales are powers of two chosen from the data, so scaling f by 2^e
    scales the complex64 result by exactly 2^e (no value leaves the normal
    FP32 range here)."""
    rng = np.random.default_rng(43)
    p = W.random_problem(66, 45, 36, 3, rng, pml_x=8, pml_y=5)
    f = W.complex_normal(rng, (1,) + p.shape)
    plan = hs.Plan(p, "mixed", refine_steps=-1)
    u = plan.solve(dev(f)).cpu().numpy()
    us = plan.solve(dev(f * 2.0 ** e)).cpu().numpy()
    assert np.array_equal(us, u * 2.0 ** e)
