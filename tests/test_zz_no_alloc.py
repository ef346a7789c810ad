"""The allocation-free gradient entry point hs_grad_k2_noalloc (through the C
ABI): the same layer gradient as hs_grad_k2, bit for bit, with its partial
sums in the library's static device scratch instead of a bound workspace."""
import ctypes

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _pair(hs, p, nrhs, seed):
    """u = A^{-1} f and a = A^{-H} g for nrhs complex-normal f, g."""
    rng = np.random.default_rng(seed)
    f = W.complex_normal(rng, (nrhs,) + p.shape)
    g = W.complex_normal(rng, (nrhs,) + p.shape)
    plan = hs.Plan(p, "c128", max_rhs=nrhs)
    u = plan.solve(hs.to_device(f))
    a = plan.solve_adjoint(hs.to_device(g))
    return plan, u, a


def test_noalloc_gradient_matches_workspace_entry_point(hs):
    import torch
    rng = np.random.default_rng(70)
    big = W.random_problem(40, 36, 48, 6, rng, pml_x=4, pml_y=3)
    small = W.random_problem(17, 12, 20, 3, rng, pml_x=2)
    plan_b, u_b, a_b = _pair(hs, big, 3, 71)
    plan_s, u_s, a_s = _pair(hs, small, 1, 72)
    # two calls in a row on one device, the second with a smaller input
    g1 = plan_b.grad_k2_noalloc(u_b, a_b)
    g2 = plan_s.grad_k2_noalloc(u_s, a_s)
    torch.cuda.synchronize()
    r1 = plan_b.grad_k2(u_b, a_b)
    r2 = plan_s.grad_k2(u_s, a_s)
    torch.cuda.synchronize()
    assert g1.shape == (3, 6) and g2.shape == (1, 3)
    assert torch.equal(g1, r1)
    assert torch.equal(g2, r2)
    # and against the definition summed on the host
    uu, aa = u_b.cpu().numpy(), a_b.cpu().numpy()
    lz = big.layer_of_z
    host = np.array([[np.sum(aa[r][lz == l] * np.conj(uu[r][lz == l])) for l in range(big.nlayers)]
                     for r in range(3)])
    assert np.abs(g1.cpu().numpy() - host).max() < 1e-12 * np.abs(host).max()


def test_noalloc_gradient_needs_no_workspace(hs):
    """A plan with no workspace bound: the workspace entry point refuses, the
    allocation-free one computes the same gradient as a bound plan."""
    import torch
    rng = np.random.default_rng(73)
    p = W.random_problem(24, 20, 30, 5, rng, pml_y=3)
    plan, u, a = _pair(hs, p, 2, 74)
    ref = plan.grad_k2(u, a)
    hx, hy, hz = (np.ascontiguousarray(x) for x in (p.hx, p.hy, p.hz))
    lz, k2 = np.ascontiguousarray(p.layer_of_z), np.ascontiguousarray(p.k2)
    grid = hs._Grid(p.nx, p.ny, p.nz, hx.ctypes.data, hy.ctypes.data, hz.ctypes.data, p.nlayers,
                    lz.ctypes.data, k2.ctypes.data)
    h = ctypes.c_void_p()
    assert hs.lib().hs_plan_create(ctypes.byref(grid), None, None, ctypes.byref(h)) == hs.HS_OK
    try:
        out = torch.zeros((2, p.nlayers), dtype=torch.complex128, device="cuda")
        s = hs._stream()
        assert hs.lib().hs_grad_k2(h, u.data_ptr(), a.data_ptr(), out.data_ptr(), 2, s) == hs.HS_ERR_STATE
        assert hs.lib().hs_grad_k2_noalloc(h, u.data_ptr(), a.data_ptr(), out.data_ptr(), 2, s) == hs.HS_OK
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
    finally:
        hs.lib().hs_plan_destroy(h)


def test_noalloc_gradient_rejects_sizes_beyond_scratch(hs):
    import torch
    rng = np.random.default_rng(75)
    p = W.uniform_problem(2, 2, 512, 4, rng)
    plan = hs.Plan(p, "c128")
    u = torch.zeros((129,) + p.shape, dtype=torch.complex128, device="cuda")
    with pytest.raises(hs.HSError) as e:
        plan.grad_k2_noalloc(u, u.clone())
    assert e.value.status == hs.HS_ERR_ARG and "scratch" in str(e.value)
    g = plan.grad_k2_noalloc(u[:128], u[:128].clone())
    torch.cuda.synchronize()
    assert g.shape == (128, 4) and torch.count_nonzero(g).item() == 0
