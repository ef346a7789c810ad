"""The 7-point finite-volume Helmholtz operator (paper Sec. 2, eqs. (2)-(3)).

Oracle code: test infrastructure only.

Per axis with n interior nodes and steps h[0..n] (node i between h[i] and
h[i+1]), the control-volume edge of node i is hhat_i = (h[i] + h[i+1]) / 2, the
mean of its two steps (eq. (2)).  The 1D stiffness matrix is

    (K u)_i = (u_i - u_{i-1}) / h[i] - (u_{i+1} - u_i) / h[i+1],

with u_{-1} = u_n = 0 (homogeneous Dirichlet walls), the mass matrix is
M = diag(hhat), and D = M^{-1} K.  On a uniform real grid D is the textbook
tridiag(-1, 2, -1) / h^2.  The 3D operator in the D-form used throughout is

    A = Dx (x) I (x) I + I (x) Dy (x) I + I (x) I (x) (Dz - diag k^2(z)),

which is minus eq. (3) divided by the mass matrices, with sigma = 1 and the
constant lambda replaced by the layered k^2(z).  Arrays are ordered
[z][y][x] (x fastest); a right-hand-side batch is [r][z][y][x].
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def hhat(h: np.ndarray) -> np.ndarray:
    """Control-volume edges of the n interior nodes (eq. (2))."""
    h = np.asarray(h)
    return 0.5 * (h[:-1] + h[1:])


def axis_K(h: np.ndarray) -> np.ndarray:
    """Dense n x n stiffness matrix K of one axis (complex symmetric)."""
    h = np.asarray(h, dtype=np.complex128)
    n = h.shape[0] - 1
    K = np.zeros((n, n), dtype=np.complex128)
    for i in range(n):
        K[i, i] = 1.0 / h[i] + 1.0 / h[i + 1]
        if i > 0:
            K[i, i - 1] = -1.0 / h[i]
        if i + 1 < n:
            K[i, i + 1] = -1.0 / h[i + 1]
    return K


def axis_D(h: np.ndarray) -> np.ndarray:
    """Dense D = M^{-1} K of one axis."""
    return axis_K(h) / hhat(np.asarray(h, dtype=np.complex128))[:, None]


def z_tridiag(hz: np.ndarray, k2_nodes: np.ndarray):
    """Diagonals (lower, diag, upper) of Dz - diag(k^2) along z.

    lower[k] multiplies u_{k-1}, upper[k] multiplies u_{k+1}; lower[0] and
    upper[nz-1] are zero."""
    hz = np.asarray(hz, dtype=np.complex128)
    hh = hhat(hz)
    lower = -1.0 / (hh * hz[:-1])
    upper = -1.0 / (hh * hz[1:])
    diag = (1.0 / hz[:-1] + 1.0 / hz[1:]) / hh - np.asarray(k2_nodes, np.complex128)
    lower = lower.copy()
    upper = upper.copy()
    lower[0] = 0.0
    upper[-1] = 0.0
    return lower, diag, upper


def k2_nodes(problem) -> np.ndarray:
    return np.asarray(problem.k2, np.complex128)[np.asarray(problem.layer_of_z)]


def apply_A(problem, u: np.ndarray) -> np.ndarray:
    """A u by the explicit 7-point neighbour stencil (no matrices).

    u: (..., nz, ny, nx) complex.  Zero Dirichlet data on all six walls."""
    u = np.asarray(u, dtype=np.complex128)
    lead = u.shape[:-3]
    nz, ny, nx = u.shape[-3:]
    pad = [(0, 0)] * len(lead) + [(1, 1), (1, 1), (1, 1)]
    up = np.pad(u, pad)
    c = up[..., 1:-1, 1:-1, 1:-1]

    def second_diff(h, lo, hi, axis_len, shape_axis):
        hl = np.asarray(h, np.complex128)[:-1]
        hr = np.asarray(h, np.complex128)[1:]
        hh = 0.5 * (hl + hr)
        shp = [1, 1, 1]
        shp[shape_axis] = axis_len
        hl = hl.reshape(shp)
        hr = hr.reshape(shp)
        hh = hh.reshape(shp)
        return ((c - lo) / hl - (hi - c) / hr) / hh

    dx = second_diff(problem.hx, up[..., 1:-1, 1:-1, :-2], up[..., 1:-1, 1:-1, 2:], nx, 2)
    dy = second_diff(problem.hy, up[..., 1:-1, :-2, 1:-1], up[..., 1:-1, 2:, 1:-1], ny, 1)
    dz = second_diff(problem.hz, up[..., :-2, 1:-1, 1:-1], up[..., 2:, 1:-1, 1:-1], nz, 0)
    k2 = k2_nodes(problem).reshape(nz, 1, 1)
    return dx + dy + dz - k2 * c


def assemble_A(problem) -> sp.csr_matrix:
    """Sparse A as a Kronecker sum, index = (z * ny + y) * nx + x."""
    Dx = sp.csr_matrix(axis_D(problem.hx))
    Dy = sp.csr_matrix(axis_D(problem.hy))
    Dz = sp.csr_matrix(axis_D(problem.hz)) - sp.diags(k2_nodes(problem))
    Ix = sp.identity(problem.nx, dtype=np.complex128, format="csr")
    Iy = sp.identity(problem.ny, dtype=np.complex128, format="csr")
    Iz = sp.identity(problem.nz, dtype=np.complex128, format="csr")
    A = (sp.kron(Iz, sp.kron(Iy, Dx)) + sp.kron(Iz, sp.kron(Dy, Ix))
         + sp.kron(Dz, sp.kron(Iy, Ix)))
    return sp.csr_matrix(A)


def mass_diagonal(problem) -> np.ndarray:
    """Diagonal of M = Mx (x) My (x) Mz as a (nz, ny, nx) array (eq. (3))."""
    mx = hhat(problem.hx)
    my = hhat(problem.hy)
    mz = hhat(np.asarray(problem.hz, np.complex128))
    return mz[:, None, None] * my[None, :, None] * mx[None, None, :]


def sigma_mask(problem) -> np.ndarray:
    """Boolean (nz, ny, nx): True on the separator planes (the interfaces)."""
    m = np.zeros((problem.ny, problem.nx), dtype=bool)
    m[:, problem.sep_x] = True
    m[problem.sep_y, :] = True
    return np.broadcast_to(m[None], problem.shape).copy()


def rel_err(u, ref) -> float:
    u = np.asarray(u)
    ref = np.asarray(ref)
    return float(np.linalg.norm((u - ref).ravel()) / np.linalg.norm(ref.ravel()))
