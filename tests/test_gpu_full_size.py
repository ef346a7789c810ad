"""GPU parity at the full sizes of every workload, in the launch configuration
the benchmark times, against the FP64 oracle (through the C ABI).

Where the oracle cannot afford every output (the 64-block batch, the 16
sources of the large grid), it checks a sample of blocks and right-hand sides
one by one; elsewhere it solves the full problem.  Tolerances 1e-10
(complex128) and 1e-8 (complex64 + FP64 refinement), each applied to the
relative 2-norm error, the largest pointwise error relative to the largest
reference value, and on decomposed grids the relative error on the
separator planes alone (tests/parity.py).
"""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint, operator, separable

from parity import check

pytestmark = pytest.mark.gpu

TOL128 = 1e-10
TOL64R = 1e-8
TOL = {"c128": TOL128, "mixed": TOL64R}
# the benchmark's mixed-precision solves take one FP64-residual refinement step
REFINE = {"c128": 0, "mixed": 1}


def dev(a):
    import paper_1909_01299_amd as hs
    return hs.to_device(a)


def rel(u, ref):
    return operator.rel_err(np.asarray(u), np.asarray(ref))


@pytest.mark.parametrize("prec", ["c128", "mixed"])
def test_decomposed_287x287x200_full_vs_oracle(hs, prec):
    """Core 256 + 16 PML cells per side, n_z = 200 in 20 layers, 4x4 blocks,
    point source at the grid centre; tuned plan as in the benchmark."""
    p, f = W.c2_decomposed()
    plan = hs.Plan(p, prec, max_rhs=1, refine_steps=REFINE[prec])
    plan.tune(1)
    u = plan.solve(dev(f)).cpu().numpy()
    ref = separable.solve(p, f[0])
    check(u[0], ref, TOL[prec], p, f"287^2 {prec}")


@pytest.mark.parametrize("prec", ["c128", "mixed"])
def test_batched_64_blocks_x8_rhs_sampled_vs_oracle(hs, prec):
    """The 64-block batch at full size (8 right-hand sides per block), one
    graph per solve; the oracle checks sampled blocks (uniform and stretched,
    smallest and largest) and right-hand sides one by one."""
    import torch
    blocks = W.c3_blocks()
    nrhs = 8
    sample = {0: (0, 7), 5: (3,), 31: (0,), 32: (0, 7), 40: (5,), 63: (0,)}
    gen = torch.Generator(device="cuda")
    gen.manual_seed(190901299)
    fs = []
    for i, b in enumerate(blocks):
        if i in sample:
            fs.append(dev(W.c3_rhs(i, b.problem, nrhs)))
        else:
            shape = (nrhs,) + b.problem.shape
            fs.append(torch.complex(torch.randn(shape, generator=gen, device="cuda", dtype=torch.float64),
                                    torch.randn(shape, generator=gen, device="cuda", dtype=torch.float64)))
    plans = [hs.Plan(b.problem, prec, max_rhs=1, refine_steps=REFINE[prec]) for b in blocks]
    batch = hs.Batch(plans, [nrhs] * len(plans))
    us = batch.solve(fs)
    torch.cuda.synchronize()
    for i, rhs in sample.items():
        pb = blocks[i].problem
        f_np = W.c3_rhs(i, pb, nrhs)
        solver = separable.SeparableSolver(pb)
        for r in rhs:
            ref = solver.solve(f_np[r])
            check(us[i][r].cpu().numpy(), ref, TOL[prec], None, f"block {i} rhs {r} {prec}")


def test_adjoint_128x128x160_gradient_full_vs_oracle_and_differences(hs):
    """Adjoint workload at full size: gradient of 0.5 |P u - d|^2 with respect
    to the 40 layer values of k^2 through the autograd wrapper, against the
    oracle's adjoint gradient (all layers) and central differences of the GPU
    misfit (a sample of layers, real and imaginary directions)."""
    import torch
    p, f, k2_true, plane = W.c4_adjoint()
    d = separable.solve(p.with_k2(k2_true), f[0])[plane]
    J_ref, g_ref, _, _ = adjoint.plane_misfit_grad(p, f[0], plane, d)
    plan = hs.Plan(p, "c128")
    k2 = torch.tensor(p.k2, dtype=torch.complex128, requires_grad=True)
    fd_dev = dev(f)
    d_dev = dev(d)
    u = hs.helmholtz_solve(k2, fd_dev, plan)
    J = 0.5 * (u[0, plane] - d_dev).abs().pow(2).sum()
    J.backward()
    g = k2.grad.numpy()
    assert abs(float(J.detach()) - J_ref) < 1e-9 * abs(J_ref)
    assert np.abs(g - g_ref).max() < 1e-8 * np.abs(g_ref).max()

    def misfit(kk):
        plan.set_k2(kk)
        uu = plan.solve(fd_dev)
        return 0.5 * float((uu[0, plane] - d_dev).abs().pow(2).sum())

    for l in (0, 9, 21, 39):
        eps = 1e-6 * abs(p.k2[l])
        fd = []
        for dirn in (1.0, 1j):
            vals = []
            for sgn in (1, -1):
                kk = p.k2.copy()
                kk[l] += sgn * eps * dirn
                vals.append(misfit(kk))
            fd.append((vals[0] - vals[1]) / (2 * eps))
        fdc = fd[0] + 1j * fd[1]
        assert abs(g[l] - fdc) < 1e-5 * max(abs(fdc), 1e-3 * abs(J_ref)), l
    plan.set_k2(p.k2)


@pytest.mark.parametrize("omega", [1.0, 1.5, 2.0, 3.0])
def test_large_575x575x256_sources_vs_oracle(hs, omega):
    """Core 512 + 32 PML cells per side, n_z = 256 in 60 layers, k^2 scaled by
    omega^2, every frequency the benchmark times.  The plans are those of the
    benchmark (16 right-hand sides, one FP64 refinement step for the mixed
    solve); all 16 sources are solved and two of them, a different pair per
    frequency, are compared with the oracle."""
    import torch
    p, srcs, omegas = W.c5_multi_rhs()
    assert omega in omegas
    p = p.with_k2(p.k2 * omega ** 2)
    f = W.point_source_batch(p, srcs)
    k = omegas.index(omega)
    pick = (2 * k, 2 * k + 1)
    solver = separable.SeparableSolver(p)
    refs = {r: solver.solve(f[r]) for r in pick}
    fd = dev(f)
    # the plans check the relative residual of their result on the device
    resid_tol = {"c128": 1e-12, "mixed": 1e-8}
    for prec in ("c128", "mixed"):
        plan = hs.Plan(p, prec, max_rhs=len(srcs), refine_steps=REFINE[prec], tol=resid_tol[prec])
        u = plan.solve(fd)
        torch.cuda.synchronize()
        info = plan.info()
        assert info["converged"] == 1, (prec, info["resid_final"])
        for r in pick:
            check(u[r].cpu().numpy(), refs[r], TOL[prec], p, f"575^2 omega {omega} {prec} source {r}")
        del plan, u
        torch.cuda.empty_cache()
