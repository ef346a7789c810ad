"""Pins of the FP64 oracle against facts that do not come from the oracle.

Every check here is fixed by the mathematics or by an independent library
routine: closed-form Dirichlet eigenpairs, exactness of the finite-volume
second difference on quadratics, the symmetry of the FV matrix of eq. (3),
LAPACK/SuperLU solves, a textbook sine-transform solver, manufactured
solutions and central finite differences.
"""
import numpy as np
import pytest
import scipy.fft
import scipy.linalg as sla
import scipy.sparse as sp

import workloads as W
from oracle import adjoint, cyclic, direct, operator, separable


def _rng(i=0):
    return np.random.default_rng(1234 + i)


# ---------------------------------------------------------------- 1D operator

@pytest.mark.parametrize("n,h", [(1, 1.0), (5, 1.0), (16, 0.5), (31, 2.0), (40, 1.0)])
def test_uniform_eigenvalues_closed_form(n, h):
    lam, Wm, Wi = separable.axis_eig(W.uniform_steps(n, h))
    m = np.arange(1, n + 1)
    exact = 2.0 * (1.0 - np.cos(np.pi * m / (n + 1))) / h ** 2
    got = np.sort(lam.real)
    assert np.max(np.abs(lam.imag)) < 1e-12 * exact.max()
    assert np.allclose(got, exact, rtol=1e-12, atol=1e-13)


def test_uniform_eigenvectors_are_sines():
    n = 12
    lam, Wm, _ = separable.axis_eig(W.uniform_steps(n))
    order = np.argsort(lam.real)
    i = np.arange(1, n + 1)
    for col, m in zip(order, range(1, n + 1)):
        s = np.sin(np.pi * m * i / (n + 1))
        v = Wm[:, col]
        c = np.vdot(s, v) / np.vdot(s, s)
        assert np.linalg.norm(v - c * s) < 1e-10 * np.linalg.norm(v)


def test_uniform_D_is_textbook_second_difference():
    n, h = 7, 0.25
    D = operator.axis_D(W.uniform_steps(n, h))
    T = (2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)) / h ** 2
    assert np.allclose(D, T, rtol=0, atol=1e-12)


@pytest.mark.parametrize("seed", range(3))
def test_fv_second_difference_exact_on_quadratics(seed):
    """For u(x) = x (X - x), vanishing at both walls, -u'' = 2; the FV scheme of
    eq. (2) reproduces this exactly on any grid, complex steps included."""
    rng = _rng(seed)
    n = 9
    h = rng.uniform(0.3, 2.0, n + 1) * (1 + 0.5j * rng.uniform(0, 1, n + 1))
    x = np.concatenate([[0], np.cumsum(h)])
    X = x[-1]
    u = x[1:-1] * (X - x[1:-1])
    D = operator.axis_D(h)
    assert np.allclose(D @ u, 2.0, rtol=0, atol=1e-12)


def test_3d_operator_on_product_of_quadratics():
    """A (qx qy qz) = 2 qy qz + 2 qx qz + 2 qx qy - k^2 qx qy qz exactly, which
    pins the Kronecker structure, the layer map and the sign of k^2."""
    rng = _rng(7)
    p = W.random_problem(6, 5, 8, 3, rng, pml_x=2, pml_y=1)

    def q(h):
        x = np.concatenate([[0], np.cumsum(h)])
        return x[1:-1] * (x[-1] - x[1:-1])

    qx, qy, qz = q(p.hx), q(p.hy), q(np.asarray(p.hz, complex))
    u = qz[:, None, None] * qy[None, :, None] * qx[None, None, :]
    k2 = p.k2[p.layer_of_z][:, None, None]
    expect = (2 * qz[:, None, None] * qy[None, :, None] + 2 * qz[:, None, None] * qx[None, None, :]
              + 2 * qy[None, :, None] * qx[None, None, :] - k2 * u)
    got = operator.apply_A(p, u)
    assert np.allclose(got, expect, rtol=1e-12, atol=1e-10)


def test_stencil_matches_kronecker_sum():
    rng = _rng(1)
    p = W.random_problem(5, 6, 7, 2, rng, pml_x=1, pml_y=2)
    u = W.complex_normal(rng, p.shape)
    A = operator.assemble_A(p)
    assert np.allclose(operator.apply_A(p, u).ravel(), A @ u.ravel(), atol=1e-12)


def test_fv_matrix_is_complex_symmetric_not_hermitian():
    """M A equals the FV matrix of eq. (3) (up to sign): symmetric, not Hermitian."""
    rng = _rng(2)
    p = W.random_problem(5, 4, 6, 2, rng, pml_x=2, pml_y=1)
    MA = sp.diags(operator.mass_diagonal(p).ravel()) @ operator.assemble_A(p)
    MA = MA.toarray()
    assert np.abs(MA - MA.T).max() < 1e-12 * np.abs(MA).max()
    assert np.abs(MA - MA.conj().T).max() > 1e-3


def test_pml_generalized_eigen_relation():
    h = W.pml_steps(16, 6)
    lam, Wm, Wi = separable.axis_eig(h)
    K = operator.axis_K(h)
    M = np.diag(operator.hhat(h))
    res = np.linalg.norm(K @ Wm - M @ Wm @ np.diag(lam)) / (np.linalg.norm(K) * np.linalg.norm(Wm))
    assert res < 1e-13
    assert np.abs(Wi @ Wm - np.eye(len(lam))).max() < 1e-10
    # PML eigenvalues lie in the lower half plane (damping)
    assert lam.imag.max() < 1e-10


@pytest.mark.parametrize("core,pml", [(256, 16), (512, 32)])
def test_global_pml_axis_tables(core, pml):
    """The global axes of the decomposed workloads (287 and 575 interior
    nodes): mirror-symmetric PML axes whose eigenvalues come in pairs that
    agree to about 1e-15.  The oracle's LAPACK eigenvectors with an explicit
    inverse must still satisfy the generalized eigen relation and invert W,
    and the eigenvalues must match a second LAPACK route (the standard
    eigenproblem of M^{-1} K, eigenvalues only)."""
    h = W.pml_steps(core, pml)
    n = len(h) - 1
    lam, Wm, Wi = separable.axis_eig(h)
    K = operator.axis_K(h)
    M = np.diag(operator.hhat(h))
    res = np.linalg.norm(K @ Wm - M @ Wm @ np.diag(lam)) / (np.linalg.norm(K) * np.linalg.norm(Wm))
    assert res < 1e-13
    assert np.abs(Wi @ Wm - np.eye(n)).max() < 1e-11
    assert np.abs(Wm @ Wi - np.eye(n)).max() < 1e-11
    lam2 = sla.eigvals(np.linalg.solve(M, K))
    scale = np.abs(lam).max()
    # every eigenvalue has a partner in the other route's spectrum and back
    assert np.abs(lam[:, None] - lam2[None, :]).min(axis=1).max() < 1e-9 * scale
    assert np.abs(lam[:, None] - lam2[None, :]).min(axis=0).max() < 1e-9 * scale
    assert lam.imag.max() < 1e-10


@pytest.mark.parametrize("core,pml,along", [(256, 16, "x"), (512, 32, "x"), (512, 32, "y")])
def test_manufactured_solution_on_global_pml_axis(core, pml, along):
    """Manufactured u* on a grid with one full global PML axis (287 or 575
    nodes) and short other axes, k^2 of the large workload's highest
    frequency (omega = 3): f = A u* by the independent stencil, and the
    separable oracle must return u*."""
    rng = _rng(20)
    long = W.pml_steps(core, pml)
    short = W.stretched_ends_steps(6, 2)
    hz = rng.uniform(0.7, 1.3, size=5)
    k2 = 9.0 * W.draw_k2(rng, 2)
    hx, hy = (long, short) if along == "x" else (short, long)
    p = W.Problem(hx, hy, hz, W.layer_map(4, 2), k2)
    ustar = W.complex_normal(rng, (2,) + p.shape)
    f = operator.apply_A(p, ustar)
    u = separable.solve(p, f)
    assert operator.rel_err(u, ustar) < 1e-11
    assert np.abs(u - ustar).max() < 1e-11 * np.abs(ustar).max()


# ---------------------------------------------------------------- z solves

def test_thomas_matches_lapack_banded():
    rng = _rng(3)
    n, m = 40, 17
    lower = W.complex_normal(rng, n)
    upper = W.complex_normal(rng, n)
    diag = 6.0 + W.complex_normal(rng, (n, m))
    lower[0] = 0
    upper[-1] = 0
    rhs = W.complex_normal(rng, (n, m))
    x = separable.thomas(lower, diag, upper, rhs)
    for j in range(m):
        ab = np.zeros((3, n), complex)
        ab[0, 1:] = upper[:-1]
        ab[1] = diag[:, j]
        ab[2, :-1] = lower[1:]
        ref = sla.solve_banded((1, 1), ab, rhs[:, j])
        assert np.allclose(x[:, j], ref, rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------------- 3D solves

SMALL = [
    dict(nx=6, ny=5, nz=7, L=2, pml_x=0, pml_y=0),
    dict(nx=9, ny=8, nz=6, L=3, pml_x=2, pml_y=2),
    dict(nx=12, ny=7, nz=9, L=4, pml_x=3, pml_y=1),
]


@pytest.mark.parametrize("cfg", SMALL)
def test_separable_matches_sparse_lu(cfg):
    rng = _rng(4)
    p = W.random_problem(cfg["nx"], cfg["ny"], cfg["nz"], cfg["L"], rng,
                         pml_x=cfg["pml_x"], pml_y=cfg["pml_y"])
    f = W.complex_normal(rng, (3,) + p.shape)
    u = separable.solve(p, f)
    ref = direct.solve_splu(p, f)
    assert operator.rel_err(u, ref) < 1e-12


def test_separable_matches_dense_numpy_solve():
    rng = _rng(5)
    p = W.random_problem(4, 3, 5, 2, rng, pml_x=1, pml_y=1)
    f = W.complex_normal(rng, p.shape)
    A = operator.assemble_A(p).toarray()
    ref = np.linalg.solve(A, f.ravel()).reshape(p.shape)
    assert operator.rel_err(separable.solve(p, f), ref) < 1e-12


def test_constant_k2_textbook_sine_solver():
    """Uniform h = 1, constant k^2: u = DST^{-1}[ DST f / (mu_x + mu_y + mu_z - k^2) ]."""
    rng = _rng(6)
    nx, ny, nz = 10, 12, 9
    k2 = 0.3 + 0.02j
    p = W.Problem(W.uniform_steps(nx), W.uniform_steps(ny), np.ones(nz + 1),
                  np.zeros(nz, np.int32), np.array([k2]))
    f = W.complex_normal(rng, p.shape)

    def mu(n):
        return 2 * (1 - np.cos(np.pi * np.arange(1, n + 1) / (n + 1)))

    den = mu(nz)[:, None, None] + mu(ny)[None, :, None] + mu(nx)[None, None, :] - k2
    fh = scipy.fft.dstn(f, type=1, norm="ortho")
    ref = scipy.fft.idstn(fh / den, type=1, norm="ortho")
    assert operator.rel_err(separable.solve(p, f), ref) < 1e-12


def test_manufactured_solution():
    rng = _rng(8)
    p = W.random_problem(20, 18, 16, 4, rng, pml_x=3, pml_y=2)
    ustar = W.complex_normal(rng, p.shape)
    f = operator.apply_A(p, ustar)
    assert operator.rel_err(separable.solve(p, f), ustar) < 1e-11


# ---------------------------------------------------------------- seven steps

DECOMP = [
    dict(nx=13, ny=11, nz=6, sx=[4, 8], sy=[5], pml=2),
    dict(nx=17, ny=17, nz=5, sx=[3, 8, 13], sy=[3, 8, 13], pml=3),
]


@pytest.mark.parametrize("cfg", DECOMP)
def test_seven_step_matches_sparse_lu(cfg):
    rng = _rng(9)
    p = W.random_problem(cfg["nx"], cfg["ny"], cfg["nz"], 3, rng, sep_x=cfg["sx"],
                         sep_y=cfg["sy"], pml_x=cfg["pml"], pml_y=cfg["pml"])
    f = W.complex_normal(rng, (2,) + p.shape)
    u, inter = cyclic.seven_step(p, f)
    ref = direct.solve_splu(p, f)
    assert operator.rel_err(u, ref) < 1e-12
    # the residual of the block solutions lives on the interfaces only
    off = ~operator.sigma_mask(p)
    assert np.abs(inter["r"][:, off]).max() < 1e-12 * np.abs(f).max()
    # w = u - v on the interfaces
    on = operator.sigma_mask(p)
    assert np.allclose(inter["w_sigma"][:, on], ref[:, on] - inter["v"][:, on], atol=1e-12)


def test_seven_step_gridding_b_matches_sparse_lu():
    """About sqrt(n) x sqrt(n) blocks on general non-uniform x and y steps
    with stretched ends (the second gridding of Sec. 2): 5 x 4 separators."""
    rng = _rng(19)
    p = W.gridding_b_problem(36, 25, 5, 3, rng, pml=3)
    assert len(p.sep_x) == 5 and len(p.sep_y) == 4
    assert len(np.unique(np.diff(np.concatenate([[-1], p.sep_x, [p.nx]])))) <= 2
    f = W.complex_normal(rng, (2,) + p.shape)
    u, _ = cyclic.seven_step(p, f)
    assert operator.rel_err(u, direct.solve_splu(p, f)) < 1e-12


def test_nested_partitions_match_sparse_lu():
    """Multi-level cyclic reduction on nested partitions: three
    levels (5 x 4 separators, then 2 x 2 of them, then one each) and two
    levels ending in a single block reproduce the direct solve."""
    rng = _rng(23)
    p = W.gridding_b_problem(36, 25, 5, 3, rng, pml=3)
    f = W.complex_normal(rng, (2,) + p.shape)
    ref = direct.solve_splu(p, f)
    sx, sy = p.sep_x.tolist(), p.sep_y.tolist()
    levels = [([sx[1], sx[3]], [sy[0], sy[2]]), ([sx[3]], [sy[2]])]
    assert operator.rel_err(cyclic.nested(p, f, levels), ref) < 1e-12
    assert operator.rel_err(cyclic.nested(p, f, [([], [])]), ref) < 1e-12
    with pytest.raises(AssertionError):
        cyclic.nested(p, f, [([sx[0] + 1], [])])


def test_block_ranges():
    assert cyclic.block_ranges(10, []) == [(0, 9)]
    assert cyclic.block_ranges(10, [3, 6]) == [(0, 2), (4, 5), (7, 9)]


# ---------------------------------------------------------------- adjoint + gradient

def test_adjoint_matches_sparse_lu_of_AH():
    rng = _rng(10)
    p = W.random_problem(8, 7, 9, 3, rng, pml_x=2, pml_y=2)
    g = W.complex_normal(rng, (2,) + p.shape)
    a = adjoint.solve_adjoint(p, g)
    assert operator.rel_err(a, direct.solve_adjoint_splu(p, g)) < 1e-12


def test_adjoint_dot_product_identity():
    rng = _rng(11)
    p = W.random_problem(10, 9, 8, 2, rng, pml_x=2, pml_y=3)
    f = W.complex_normal(rng, p.shape)
    g = W.complex_normal(rng, p.shape)
    lhs = np.vdot(g, separable.solve(p, f))
    rhs = np.vdot(adjoint.solve_adjoint(p, g), f)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_gradient_matches_central_differences():
    rng = _rng(12)
    p = W.random_problem(9, 8, 12, 4, rng, pml_x=2, pml_y=2)
    f = W.point_source(p.shape, 4, 4, 2)
    d = separable.solve(p.with_k2(p.k2 * 1.05), f)[5]
    J, g, _, _ = adjoint.plane_misfit_grad(p, f, 5, d)
    for l in range(p.nlayers):
        eps = 1e-6 * abs(p.k2[l])
        fd = []
        for direction in (1.0, 1j):
            kp = p.k2.copy()
            km = p.k2.copy()
            kp[l] += eps * direction
            km[l] -= eps * direction
            Jp, _ = adjoint.plane_misfit(p.with_k2(kp), f, 5, d)
            Jm, _ = adjoint.plane_misfit(p.with_k2(km), f, 5, d)
            fd.append((Jp - Jm) / (2 * eps))
        fd = fd[0] + 1j * fd[1]
        assert abs(g[l] - fd) < 1e-6 * max(abs(fd), 1e-3 * J)


def test_reciprocity_on_uniform_grid():
    """Uniform real steps: M is a multiple of I, so A is symmetric and
    (A^{-1})_{pq} = (A^{-1})_{qp}."""
    rng = _rng(13)
    p = W.random_problem(7, 6, 5, 2, rng)
    p = W.Problem(p.hx, p.hy, np.ones(p.nz + 1), p.layer_of_z, p.k2)
    e1 = W.point_source(p.shape, 1, 2, 3)
    e2 = W.point_source(p.shape, 5, 4, 1)
    u1 = separable.solve(p, e1)
    u2 = separable.solve(p, e2)
    assert abs(u1[1, 4, 5] - u2[3, 2, 1]) < 1e-13 * abs(u1[1, 4, 5])


# ---------------------------------------------------------------- sigma(z), eqs. (1)-(2)

def _sigma_problem(seed, nx, ny, nz, L, **kw):
    rng = _rng(seed)
    p = W.random_problem(nx, ny, nz, L, rng, **kw)
    return W.with_sigma(p, W.draw_sigma(rng, L)), rng


def test_sigma_flux_form_exact_on_product_of_quadratics():
    """u = qx qy qz with quadratics vanishing at the walls.  The x and y terms
    of eq. (2) carry sigma at the node: 2 sigma_k (qy qz + qx qz).  The z term
    is the difference of the fluxes sigma * dqz/dz at the step midpoints, which
    a central difference reproduces exactly for a quadratic; both are written
    here from their definitions, independent of the oracle's stencil."""
    p, _ = _sigma_problem(30, 6, 5, 9, 3, pml_x=2, pml_y=1)

    def nodes(h):
        return np.concatenate([[0], np.cumsum(h)])

    def q(h):
        x = nodes(h)
        return x[1:-1] * (x[-1] - x[1:-1])

    qx, qy = q(p.hx), q(p.hy)
    z = nodes(np.asarray(p.hz, complex))
    Z = z[-1]
    qz = z[1:-1] * (Z - z[1:-1])
    zmid = 0.5 * (z[:-1] + z[1:])                      # midpoints of the nz + 1 steps
    flux = p.sig_step * (Z - 2 * zmid)                 # sigma * dqz/dz there
    hh = 0.5 * (np.asarray(p.hz)[:-1] + np.asarray(p.hz)[1:])
    dz_term = -(flux[1:] - flux[:-1]) / hh             # -(sigma qz')' at the nodes
    u = qz[:, None, None] * qy[None, :, None] * qx[None, None, :]
    sig = p.sig_node[:, None, None]
    k2 = p.k2[p.layer_of_z][:, None, None]
    expect = (sig * (2 * qy[None, :, None] * qz[:, None, None] + 2 * qx[None, None, :] * qz[:, None, None])
              + dz_term[:, None, None] * qy[None, :, None] * qx[None, None, :] - k2 * u)
    got = operator.apply_A(p, u)
    assert np.abs(got - expect).max() < 1e-11 * np.abs(expect).max()


def test_sigma_constant_scaling():
    """sigma = c everywhere: A(c, k^2) = c A(1, k^2 / c), so
    u(c, k^2) = u(1, k^2 / c) / c."""
    rng = _rng(31)
    p = W.random_problem(9, 8, 7, 2, rng, pml_x=2)
    c = 1.7
    pc = W.Problem(p.hx, p.hy, p.hz, p.layer_of_z, p.k2, sigma_node=np.full(p.nz, c),
                   sigma_step=np.full(p.nz + 1, c))
    f = W.complex_normal(rng, p.shape)
    u1 = direct.solve_splu(p.with_k2(p.k2 / c), f) / c
    assert operator.rel_err(direct.solve_splu(pc, f), u1) < 1e-12
    assert operator.rel_err(separable.solve(pc, f), u1) < 1e-12


@pytest.mark.parametrize("cfg", SMALL)
def test_sigma_separable_matches_sparse_lu(cfg):
    p, rng = _sigma_problem(32, cfg["nx"], cfg["ny"], cfg["nz"], cfg["L"], pml_x=cfg["pml_x"],
                            pml_y=cfg["pml_y"])
    f = W.complex_normal(rng, (2,) + p.shape)
    assert operator.rel_err(separable.solve(p, f), direct.solve_splu(p, f)) < 1e-12


def test_sigma_stencil_matches_kronecker_and_fv_symmetry():
    p, rng = _sigma_problem(33, 7, 6, 8, 3, pml_x=2, pml_y=2)
    u = W.complex_normal(rng, p.shape)
    A = operator.assemble_A(p)
    assert np.abs(A @ u.ravel() - operator.apply_A(p, u).ravel()).max() < 1e-12 * np.abs(u).max() * 40
    MA = (sp.diags(operator.mass_diagonal(p).ravel()) @ A).toarray()
    assert np.abs(MA - MA.T).max() < 1e-12 * np.abs(MA).max()


@pytest.mark.parametrize("cfg", DECOMP)
def test_sigma_seven_step_matches_sparse_lu(cfg):
    p, rng = _sigma_problem(34, cfg["nx"], cfg["ny"], cfg["nz"], 3, sep_x=cfg["sx"], sep_y=cfg["sy"],
                            pml_x=cfg["pml"], pml_y=cfg["pml"])
    f = W.complex_normal(rng, (2,) + p.shape)
    u, inter = cyclic.seven_step(p, f)
    assert operator.rel_err(u, direct.solve_splu(p, f)) < 1e-12
    off = ~operator.sigma_mask(p)
    assert np.abs(inter["r"][:, off]).max() < 1e-12 * np.abs(f).max()


def test_sigma_adjoint_matches_sparse_lu_of_AH():
    p, rng = _sigma_problem(35, 8, 7, 9, 3, pml_x=2, pml_y=2)
    g = W.complex_normal(rng, (2,) + p.shape)
    assert operator.rel_err(adjoint.solve_adjoint(p, g), direct.solve_adjoint_splu(p, g)) < 1e-12
