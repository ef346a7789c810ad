"""GPU parity of the HIP solver against the FP64 oracle (through the C ABI).

Tolerances: relative 2-norm error 1e-10 for the complex128 path and 1e-8 for
the complex64 + FP64-refinement path, per right-hand side.
"""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint, cyclic, direct, operator, separable

pytestmark = pytest.mark.gpu

TOL128 = 1e-10
TOL64R = 1e-8


def dev(a):
    import paper_1909_01299_amd as hs
    return hs.to_device(a)


def per_rhs_err(u, ref):
    u = np.asarray(u)
    ref = np.asarray(ref)
    if u.ndim == 3:
        return operator.rel_err(u, ref)
    return max(operator.rel_err(u[r], ref[r]) for r in range(u.shape[0]))


# ------------------------------------------------------------------ single block

def test_c1_single_block_vs_sparse_lu(hs):
    p, f = W.c1_single_block()
    plan = hs.Plan(p, "c128")
    u = plan.solve(dev(f)).cpu().numpy()
    ref = direct.solve_splu(p, f)
    assert per_rhs_err(u, ref) < TOL128


@pytest.mark.parametrize("shape", [(1, 1, 1), (1, 5, 3), (17, 1, 9), (33, 31, 18), (16, 48, 40)])
def test_uniform_block_shapes_vs_oracle(hs, shape):
    nx, ny, nz = shape
    rng = np.random.default_rng(nx * 1000 + ny * 10 + nz)
    p = W.uniform_problem(nx, ny, nz, max(1, min(4, nz)), rng)
    f = W.complex_normal(rng, (2,) + p.shape)
    plan = hs.Plan(p, "c128", max_rhs=2)
    u = plan.solve(dev(f)).cpu().numpy()
    assert per_rhs_err(u, separable.solve(p, f)) < TOL128


@pytest.mark.parametrize("cfg", [dict(nx=20, ny=18, nz=24, px=3, py=2),
                                 dict(nx=47, ny=33, nz=35, px=6, py=4)])
def test_nonuniform_block_vs_oracle(hs, cfg):
    rng = np.random.default_rng(cfg["nx"])
    p = W.random_problem(cfg["nx"], cfg["ny"], cfg["nz"], 4, rng, pml_x=cfg["px"], pml_y=cfg["py"])
    f = W.complex_normal(rng, (3,) + p.shape)
    plan = hs.Plan(p, "c128", max_rhs=3)
    u = plan.solve(dev(f)).cpu().numpy()
    assert per_rhs_err(u, separable.solve(p, f)) < TOL128


def test_dense_path_on_uniform_axes_matches_sine_path(hs):
    rng = np.random.default_rng(3)
    p = W.uniform_problem(40, 24, 20, 2, rng)
    f = W.complex_normal(rng, (1,) + p.shape)
    u1 = hs.Plan(p, "c128").solve(dev(f)).cpu().numpy()
    u2 = hs.Plan(p, "c128", force_dense=True).solve(dev(f)).cpu().numpy()
    assert per_rhs_err(u1, u2) < TOL128


@pytest.mark.parametrize("shape", [(15, 31, 12), (63, 127, 9), (255, 15, 6), (127, 127, 20), (511, 17, 5),
                                   (31, 511, 4), (255, 255, 3)])
def test_sine_fft_path_vs_oracle_and_dense(hs, shape):
    """Uniform axes with n + 1 a power of two (16 .. 512) take the FFT sine
    transform, along x (contiguous lines) and along y (strided lines)."""
    nx, ny, nz = shape
    rng = np.random.default_rng(nx + 7 * ny)
    p = W.uniform_problem(nx, ny, nz, 3, rng)
    f = W.complex_normal(rng, (2,) + p.shape)
    plan = hs.Plan(p, "c128", max_rhs=2)
    assert plan.info()["n_sine_axes"] >= 1
    u = plan.solve(dev(f)).cpu().numpy()
    assert per_rhs_err(u, separable.solve(p, f)) < TOL128
    u2 = hs.Plan(p, "c128", max_rhs=2, force_dense=True).solve(dev(f)).cpu().numpy()
    assert per_rhs_err(u, u2) < TOL128
    um = hs.Plan(p, "mixed", max_rhs=2).solve(dev(f)).cpu().numpy()
    assert per_rhs_err(um, u) < TOL64R


@pytest.mark.parametrize("nz", [2, 3, 31, 32, 33, 128, 129, 255, 256, 257, 300, 512])
def test_z_line_lengths_vs_oracle(hs, nz):
    """z solves split each line into up to 16 (32 beyond 256 rows) chunks;
    cover short lines, chunk-count boundaries, ragged chunks and the switch
    between 8 and 16 register rows per chunk (128 / 129 rows in 16 chunks)."""
    rng = np.random.default_rng(nz)
    p = W.random_problem(9, 7, nz, min(5, nz), rng, pml_x=2)
    f = W.complex_normal(rng, (1,) + p.shape)
    u = hs.Plan(p, "c128").solve(dev(f)).cpu().numpy()
    assert per_rhs_err(u, separable.solve(p, f)) < TOL128
    um = hs.Plan(p, "mixed").solve(dev(f)).cpu().numpy()
    assert per_rhs_err(um, u) < TOL64R


def test_nz_limit_is_an_argument_error(hs):
    rng = np.random.default_rng(0)
    p = W.uniform_problem(4, 4, 513, 1, rng)
    with pytest.raises(hs.HSError) as e:
        hs.Plan(p, "c128")
    assert e.value.status == hs.HS_ERR_ARG


def test_manufactured_solution_and_stencil(hs):
    rng = np.random.default_rng(11)
    p = W.random_problem(30, 26, 22, 3, rng, pml_x=4, pml_y=3)
    ustar = W.complex_normal(rng, p.shape)
    plan = hs.Plan(p, "c128")
    au = plan.apply(dev(ustar[None])).cpu().numpy()[0]
    ref = operator.apply_A(p, ustar)
    assert operator.rel_err(au, ref) < 1e-14
    u = plan.solve(dev(ref[None])).cpu().numpy()[0]
    assert operator.rel_err(u, ustar) < TOL128
    r = plan.residual(dev(ref[None]), dev(u[None])).cpu().numpy()[0]
    assert np.linalg.norm(r) < 1e-9 * np.linalg.norm(ref)


def test_autotune_keeps_parity_and_caches(hs, tmp_path):
    rng = np.random.default_rng(17)
    p = W.random_problem(31, 27, 70, 3, rng, pml_y=3)
    p = W.Problem(W.uniform_steps(31), p.hy, p.hz, p.layer_of_z, p.k2)
    f = W.complex_normal(rng, (2,) + p.shape)
    cache = str(tmp_path / "tune.jsonl")
    plan = hs.Plan(p, "c128", max_rhs=2)
    t1 = plan.tune(2, cache)
    assert t1["z_chunks"] in (8, 16, 32) and t1["sine_lines"] in (4, 8, 16)
    u = plan.solve(dev(f)).cpu().numpy()
    assert per_rhs_err(u, separable.solve(p, f)) < TOL128
    plan2 = hs.Plan(p, "c128", max_rhs=2)
    assert plan2.tune(2, cache) == t1          # served from the cache
    assert len(open(cache).read().splitlines()) == 1


def test_stage_profiling_all_and_single_stage(hs):
    """hipEvents around every stage, or around one named stage only (the
    benchmark's timed region); profiling leaves the result bit-identical."""
    import torch
    rng = np.random.default_rng(23)
    p = W.decomposed_problem(24, 3, 10, 2, rng)
    f = dev(W.complex_normal(rng, (1,) + p.shape))
    plan = hs.Plan(p, "c128")
    u0 = plan.solve(f).cpu().numpy()
    plan.profile(True)
    plan.profile_read()
    u1 = plan.solve(f).cpu().numpy()
    st = {s["name"]: s for s in plan.profile_read()}
    assert {"xform_x_fwd", "zsweep_blocks_v", "zsweep_global", "zsweep_blocks_u", "xform_x_inv"} <= set(st)
    assert all(s["launches"] == 1 and s["ms"] > 0 for s in st.values())
    plan.profile(True, only="zsweep_global")
    for _ in range(3):
        plan.solve(f)
    torch.cuda.synchronize()
    got = [s for s in plan.profile_read() if s["launches"] > 0]
    assert [s["name"] for s in got] == ["zsweep_global"] and got[0]["launches"] == 3
    assert got[0]["bytes_per_launch"] > 0
    with pytest.raises(hs.HSError):
        plan.profile(True, only="x" * 40)
    plan.profile(False)
    assert np.array_equal(u0, u1)


@pytest.mark.parametrize("chunks", [8, 16, 32])
@pytest.mark.parametrize("prec", ["c128", "mixed"])
def test_every_z_chunking_vs_oracle(hs, chunks, prec):
    rng = np.random.default_rng(chunks)
    p = W.random_problem(21, 17, 100, 4, rng, pml_x=3)
    f = W.complex_normal(rng, (1,) + p.shape)
    plan = hs.Plan(p, prec, z_chunks=chunks)
    assert plan.info()["z_chunks"] == chunks
    u = plan.solve(dev(f)).cpu().numpy()
    assert per_rhs_err(u, separable.solve(p, f)) < (TOL128 if prec == "c128" else TOL64R)


@pytest.mark.parametrize("chunks,nz", [(16, 256), (32, 256), (16, 128), (8, 64)])
@pytest.mark.parametrize("prec", ["c128", "mixed"])
def test_fixed_row_z_solves_vs_oracle(hs, chunks, nz, prec):
    """nz filling the chunks exactly: the fixed-row instances (straight-line
    row loops) against the oracle, on a decomposed grid so the dense-input,
    low-rank and global solves all take them, and to rounding against the
    instances with a run-time row count."""
    rng = np.random.default_rng(nz + chunks)
    p = W.random_problem(36, 30, nz, 4, rng, sep_x=[8, 20], sep_y=[14], pml_x=4, pml_y=3)
    f = W.complex_normal(rng, (2,) + p.shape)
    plan = hs.Plan(p, prec, max_rhs=2, z_chunks=chunks, refine_steps=1 if prec == "mixed" else 0)
    fd = dev(f)
    plan.set_launch({"z_chunks": chunks, "sine_lines": 0, "z_fixed_rows": 1})
    assert plan.info()["z_fixed_rows"] == 1
    u1 = plan.solve(fd).cpu().numpy()
    plan.set_launch({"z_chunks": chunks, "sine_lines": 0, "z_fixed_rows": 0})
    u0 = plan.solve(fd).cpu().numpy()
    assert per_rhs_err(u1, separable.solve(p, f)) < (TOL128 if prec == "c128" else TOL64R)
    assert per_rhs_err(u1, u0) < 1e-13


# ------------------------------------------------------------------ decomposition

DECOMP = [
    dict(nx=13, ny=11, nz=6, sx=[4, 8], sy=[5], pml=2),
    dict(nx=17, ny=17, nz=5, sx=[3, 8, 13], sy=[3, 8, 13], pml=3),
    dict(nx=40, ny=37, nz=21, sx=[5, 20, 34], sy=[18], pml=5),
]


@pytest.mark.parametrize("prec,tol", [("c128", TOL128), ("mixed", TOL64R)])
@pytest.mark.parametrize("cfg", [
    dict(nx=600, ny=24, nz=9, sx=[100, 350], sy=[11], pml=6),   # global x axis > 512 columns
    dict(nx=30, ny=530, nz=7, sx=[14], sy=[200, 400], pml=4),    # global y axis > 512 rows
])
def test_decomposed_wide_global_axis_vs_oracle(hs, prec, tol, cfg):
    """Global axes longer than one contraction workgroup's 512 columns (the
    plane is split into column slabs whose sums are added afterwards)."""
    rng = np.random.default_rng(41)
    p = W.random_problem(cfg["nx"], cfg["ny"], cfg["nz"], 3, rng, sep_x=cfg["sx"], sep_y=cfg["sy"],
                         pml_x=cfg["pml"], pml_y=cfg["pml"])
    f = W.complex_normal(rng, (1,) + p.shape)
    u = hs.Plan(p, prec).solve(dev(f)).cpu().numpy()
    assert per_rhs_err(u, separable.solve(p, f)) < tol


@pytest.mark.parametrize("cfg", DECOMP)
def test_decomposed_vs_sparse_lu(hs, cfg):
    rng = np.random.default_rng(cfg["nx"] + cfg["ny"])
    p = W.random_problem(cfg["nx"], cfg["ny"], cfg["nz"], 3, rng, sep_x=cfg["sx"], sep_y=cfg["sy"],
                         pml_x=cfg["pml"], pml_y=cfg["pml"])
    f = W.complex_normal(rng, (2,) + p.shape)
    plan = hs.Plan(p, "c128", max_rhs=2)
    u = plan.solve(dev(f)).cpu().numpy()
    assert per_rhs_err(u, direct.solve_splu(p, f)) < TOL128


def test_decomposed_reduced_c2_point_source_on_interface(hs):
    """The C2 layout at reduced size (core 32, PML 4): the centre source sits on
    a separator crossing, so the whole answer comes from the interface steps."""
    p, f = W.c2_decomposed(core_cells=32, pml_cells=4, nz=30, nlayers=5)
    assert p.sep_x[1] == p.nx // 2
    plan = hs.Plan(p, "c128")
    u = plan.solve(dev(f)).cpu().numpy()
    assert per_rhs_err(u, separable.solve(p, f)) < TOL128
    # off-interface source too
    g = W.point_source(p.shape, 10, 12, 7)[None]
    u2 = plan.solve(dev(g)).cpu().numpy()
    assert per_rhs_err(u2, separable.solve(p, g)) < TOL128


def test_decomposed_matches_seven_step_intermediates_via_result(hs):
    rng = np.random.default_rng(21)
    p = W.random_problem(23, 19, 9, 2, rng, sep_x=[6, 14], sep_y=[9], pml_x=3, pml_y=3)
    f = W.complex_normal(rng, (1,) + p.shape)
    u_ref, inter = cyclic.seven_step(p, f)
    u = hs.Plan(p, "c128").solve(dev(f)).cpu().numpy()
    on = operator.sigma_mask(p)
    # u on the interfaces equals w there (step 5), inside it equals v + w (step 7)
    assert np.abs(u[0][on] - inter["w_sigma"][0][on]).max() < 1e-10 * np.abs(u_ref).max()
    assert per_rhs_err(u, u_ref) < TOL128


# ------------------------------------------------------------------ adjoint and gradient

def test_adjoint_vs_oracle_and_dot_product(hs):
    rng = np.random.default_rng(5)
    p = W.random_problem(21, 18, 16, 3, rng, pml_x=3, pml_y=2)
    g = W.complex_normal(rng, (1,) + p.shape)
    f = W.complex_normal(rng, (1,) + p.shape)
    plan = hs.Plan(p, "c128")
    a = plan.solve_adjoint(dev(g)).cpu().numpy()
    assert per_rhs_err(a, adjoint.solve_adjoint(p, g)) < TOL128
    u = plan.solve(dev(f)).cpu().numpy()
    lhs = np.vdot(g, u)
    rhs = np.vdot(a, f)
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)


def test_adjoint_decomposed_vs_sparse_lu(hs):
    rng = np.random.default_rng(6)
    p = W.random_problem(19, 15, 8, 2, rng, sep_x=[6, 12], sep_y=[7], pml_x=3, pml_y=2)
    g = W.complex_normal(rng, (1,) + p.shape)
    a = hs.Plan(p, "c128").solve_adjoint(dev(g)).cpu().numpy()
    assert per_rhs_err(a, direct.solve_adjoint_splu(p, g)) < TOL128


def test_grad_k2_vs_oracle(hs):
    rng = np.random.default_rng(8)
    p = W.random_problem(16, 14, 20, 5, rng, pml_x=2, pml_y=2)
    f = W.point_source(p.shape, 7, 6, 3)
    d = separable.solve(p.with_k2(p.k2 * 1.07), f)[9]
    J, g_ref, u_ref, a_ref = adjoint.plane_misfit_grad(p, f, 9, d)
    plan = hs.Plan(p, "c128")
    u = plan.solve(dev(f[None]))
    resid = np.zeros((1,) + p.shape, complex)
    resid[0, 9] = u.cpu().numpy()[0, 9] - d
    a = plan.solve_adjoint(dev(resid))
    g = plan.grad_k2(u, a).cpu().numpy()[0]
    assert np.abs(g - g_ref).max() < 1e-8 * np.abs(g_ref).max()


def test_autograd_function_matches_finite_differences(hs):
    import torch
    rng = np.random.default_rng(9)
    p = W.random_problem(12, 11, 16, 4, rng)
    f = W.point_source(p.shape, 5, 5, 3)[None]
    d = separable.solve(p.with_k2(p.k2 * 0.95), f[0])[6]
    plan = hs.Plan(p, "c128")
    k2 = torch.tensor(p.k2, dtype=torch.complex128, requires_grad=True)
    u = hs.helmholtz_solve(k2, dev(f), plan)
    J = 0.5 * (u[0, 6] - dev(d)).abs().pow(2).sum()
    J.backward()
    g = k2.grad.numpy()
    for l in range(p.nlayers):
        eps = 1e-6 * abs(p.k2[l])
        fd = []
        for dirn in (1.0, 1j):
            vals = []
            for sgn in (1, -1):
                kk = p.k2.copy()
                kk[l] += sgn * eps * dirn
                Jv, _ = adjoint.plane_misfit(p.with_k2(kk), f[0], 6, d)
                vals.append(Jv)
            fd.append((vals[0] - vals[1]) / (2 * eps))
        fdc = fd[0] + 1j * fd[1]
        assert abs(g[l] - fdc) < 1e-6 * max(abs(fdc), 1e-3 * float(J))


# ------------------------------------------------------------------ mixed precision

def test_mixed_precision_single_block(hs):
    rng = np.random.default_rng(12)
    p = W.random_problem(40, 36, 48, 4, rng, pml_x=5, pml_y=4)
    f = W.complex_normal(rng, (2,) + p.shape)
    plan = hs.Plan(p, "mixed", max_rhs=2)
    u = plan.solve(dev(f)).cpu().numpy()
    assert per_rhs_err(u, separable.solve(p, f)) < TOL64R


def test_mixed_precision_near_resonance_modes_run_fp64(hs):
    """Large Re k^2 puts many low modes near resonance; their z solves switch
    to FP64 and the refined result still meets the mixed-precision bar."""
    rng = np.random.default_rng(14)
    p = W.uniform_problem(63, 47, 64, 4, rng)
    p = p.with_k2(np.array([1.5 + 0.002j, 2.0 + 0.001j, 1.2 + 0.004j, 1.8 + 0.003j]))
    f = W.complex_normal(rng, (1,) + p.shape)
    plan = hs.Plan(p, "mixed")
    assert plan.info()["n_fp64_modes"] > 0
    u = plan.solve(dev(f)).cpu().numpy()
    assert per_rhs_err(u, separable.solve(p, f)) < TOL64R
    assert hs.Plan(p, "c128").info()["n_fp64_modes"] == 0


@pytest.mark.parametrize("chunks", [8, 16, 32])
def test_mixed_near_resonance_lists_every_chunking_and_k2_update(hs, chunks):
    """The FP64 work lists exist for every chunking; a k^2 update rebuilds
    them, including to none (Re k^2 < 0 leaves no mode near resonance) and
    back, where the solve repeats bit for bit."""
    rng = np.random.default_rng(31 + chunks)
    p = W.random_problem(63, 47, 64, 4, rng, pml_x=5)
    p = p.with_k2(np.array([1.5 + 0.002j, 2.0 + 0.001j, 1.2 + 0.004j, 1.8 + 0.003j]))
    f = W.complex_normal(rng, (1,) + p.shape)
    fd = dev(f)
    plan = hs.Plan(p, "mixed", z_chunks=chunks)
    assert plan.info()["z_chunks"] == chunks and plan.info()["n_fp64_modes"] > 0
    u1 = plan.solve(fd).cpu().numpy()
    assert per_rhs_err(u1, separable.solve(p, f)) < TOL64R
    k2n = np.array([-0.5 + 0.01j, -0.2 + 0.02j, -0.4 + 0.005j, -0.3 + 0.01j])
    plan.set_k2(k2n)
    assert plan.info()["n_fp64_modes"] == 0
    un = plan.solve(fd).cpu().numpy()
    assert per_rhs_err(un, separable.solve(p.with_k2(k2n), f)) < TOL64R
    plan.set_k2(p.k2)
    assert np.array_equal(plan.solve(fd).cpu().numpy(), u1)


def test_fp64_stream_choice_same_result(hs):
    """The near-resonance FP64 z solves beside the FP32 launch on a second
    stream or before it on the solve's stream: the same workgroups write the
    same modes, so both give the same result bit for bit (decomposed grid)."""
    import torch
    p, f = W.c2_decomposed(core_cells=48, pml_cells=6, nz=40, nlayers=6)
    p = p.with_k2(p.k2 * 4.0)
    rng = np.random.default_rng(17)
    f = f + 0.1 * W.complex_normal(rng, f.shape)
    fd = dev(f)
    plan = hs.Plan(p, "mixed", refine_steps=1)
    assert plan.info()["n_fp64_modes"] > 0 and plan.info()["fp64_stream"] == 1
    u1 = plan.solve(fd).cpu().numpy()
    plan.set_launch({"z_chunks": 0, "sine_lines": 0, "z_fixed_rows": 0, "fp64_stream": 0})
    assert plan.info()["fp64_stream"] == 0
    u0 = plan.solve(fd).cpu().numpy()
    torch.cuda.synchronize()
    assert np.array_equal(u0, u1)
    assert per_rhs_err(u0, separable.solve(p, f)) < TOL64R
    shapes = plan.tune(1)
    assert shapes["fp64_stream"] in (0, 1)
    assert per_rhs_err(plan.solve(fd).cpu().numpy(), separable.solve(p, f)) < TOL64R


def test_mixed_precision_decomposed(hs):
    p, f = W.c2_decomposed(core_cells=48, pml_cells=6, nz=40, nlayers=6)
    rng = np.random.default_rng(13)
    f = f + 0.1 * W.complex_normal(rng, f.shape)
    plan = hs.Plan(p, "mixed")
    u = plan.solve(dev(f)).cpu().numpy()
    assert per_rhs_err(u, separable.solve(p, f)) < TOL64R


# ------------------------------------------------------------------ matrix-core transforms
@pytest.mark.gpu
@pytest.mark.parametrize("prec,tol", [("c128", TOL128), ("mixed", TOL64R)])
@pytest.mark.parametrize("cfg", [
    # uniform, n + 1 not a power of two: real sine table on matrix cores (x lines >= 1024)
    dict(nx=70, ny=50, nz=40, pml_x=0, pml_y=0),
    # stretched ends: embedded complex table on matrix cores, both axes
    dict(nx=66, ny=45, nz=36, pml_x=8, pml_y=5),
    # mixed: real table along x, complex along y; y panel wider than 16 columns
    dict(nx=100, ny=40, nz=33, pml_x=0, pml_y=6),
    # narrow block: complex FMA tiles along x, matrix cores along y
    dict(nx=20, ny=64, nz=70, pml_x=3, pml_y=0),
    # short stretched y axes: 16 nodes (two output tiles, four panels per
    # workgroup), 23 (three tiles, two panels; complex64 on FP32 matrix cores)
    # and 31 (four tiles, two panels; complex64 on split-fp16)
    dict(nx=33, ny=16, nz=20, pml_x=4, pml_y=3),
    dict(nx=40, ny=23, nz=24, pml_x=0, pml_y=4),
    dict(nx=28, ny=31, nz=20, pml_x=4, pml_y=4),
])
def test_dense_transform_kernels_vs_oracle(hs, prec, tol, cfg):
    """Each dense-transform kernel family (real table, embedded complex table,
    small-tile fallback) against the oracle, alone and inside a batch."""
    import torch
    rng = np.random.default_rng(31)
    p = W.random_problem(cfg["nx"], cfg["ny"], cfg["nz"], 3, rng, pml_x=cfg["pml_x"], pml_y=cfg["pml_y"])
    f = W.complex_normal(rng, (2,) + p.shape)
    plan = hs.Plan(p, prec, max_rhs=2)
    u = plan.solve(dev(f)).cpu().numpy()
    ref = separable.solve(p, f)
    assert per_rhs_err(u, ref) < tol
    batch = hs.Batch([plan], [2])
    ub = batch.solve([dev(f)])[0]
    torch.cuda.synchronize()
    assert np.array_equal(ub.cpu().numpy(), u)
