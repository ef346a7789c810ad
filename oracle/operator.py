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

which is minus eq. (3) divided by the mass matrices, with the constant
lambda replaced by the layered k^2(z).  With the coefficient sigma(z) of
eqs. (1)-(2) the x and y terms of row k carry sigma at node k, and the z term
is the flux form with sigma at the two z steps of the node:

    A = diag(sigma_node) (Dx (+) Dy) + Dz^sigma - diag k^2,
    (K_z^sigma u)_k = s[k] (u_k - u_{k-1}) / h[k] - s[k+1] (u_{k+1} - u_k) / h[k+1]

(s = sigma at the steps; without sigma both are 1).  Arrays are ordered
[z][y][x] (x fastest); a right-hand-side batch is [r][z][y][x].
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def hhat(h: np.ndarray) -> np.ndarray:
    """Control-volume edges of the n interior nodes (eq. (2))."""
    h = np.asarray(h)
    return 0.5 * (h[:-1] + h[1:])


def axis_K(h: np.ndarray, w: np.ndarray = None) -> np.ndarray:
    """Dense n x n stiffness matrix K of one axis (complex symmetric); w
    (n + 1 values, default 1) weights each step's flux (sigma at the steps)."""
    h = np.asarray(h, dtype=np.complex128)
    n = h.shape[0] - 1
    w = np.ones(n + 1) if w is None else np.asarray(w)
    K = np.zeros((n, n), dtype=np.complex128)
    for i in range(n):
        K[i, i] = w[i] / h[i] + w[i + 1] / h[i + 1]
        if i > 0:
            K[i, i - 1] = -w[i] / h[i]
        if i + 1 < n:
            K[i, i + 1] = -w[i + 1] / h[i + 1]
    return K


def axis_D(h: np.ndarray, w: np.ndarray = None) -> np.ndarray:
    """Dense D = M^{-1} K of one axis."""
    return axis_K(h, w) / hhat(np.asarray(h, dtype=np.complex128))[:, None]


def z_tridiag(hz: np.ndarray, k2_nodes: np.ndarray, sig_step: np.ndarray = None):
    """Diagonals (lower, diag, upper) of Dz^sigma - diag(k^2) along z.

    lower[k] multiplies u_{k-1}, upper[k] multiplies u_{k+1}; lower[0] and
    upper[nz-1] are zero.  sig_step: sigma at the nz + 1 steps (default 1)."""
    hz = np.asarray(hz, dtype=np.complex128)
    w = np.ones(hz.shape[0]) if sig_step is None else np.asarray(sig_step, np.float64)
    hh = hhat(hz)
    lower = -w[:-1] / (hh * hz[:-1])
    upper = -w[1:] / (hh * hz[1:])
    diag = (w[:-1] / hz[:-1] + w[1:] / hz[1:]) / hh - np.asarray(k2_nodes, np.complex128)
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

    def second_diff(h, lo, hi, axis_len, shape_axis, w=None):
        hl = np.asarray(h, np.complex128)[:-1]
        hr = np.asarray(h, np.complex128)[1:]
        hh = 0.5 * (hl + hr)
        wl = np.ones(axis_len) if w is None else np.asarray(w)[:-1]
        wr = np.ones(axis_len) if w is None else np.asarray(w)[1:]
        shp = [1, 1, 1]
        shp[shape_axis] = axis_len
        hl, hr, hh = hl.reshape(shp), hr.reshape(shp), hh.reshape(shp)
        wl, wr = wl.reshape(shp), wr.reshape(shp)
        return (wl * (c - lo) / hl - wr * (hi - c) / hr) / hh

    dx = second_diff(problem.hx, up[..., 1:-1, 1:-1, :-2], up[..., 1:-1, 1:-1, 2:], nx, 2)
    dy = second_diff(problem.hy, up[..., 1:-1, :-2, 1:-1], up[..., 1:-1, 2:, 1:-1], ny, 1)
    dz = second_diff(problem.hz, up[..., :-2, 1:-1, 1:-1], up[..., 2:, 1:-1, 1:-1], nz, 0,
                     problem.sig_step)
    k2 = k2_nodes(problem).reshape(nz, 1, 1)
    sig = problem.sig_node.reshape(nz, 1, 1)
    return sig * (dx + dy) + dz - k2 * c


def assemble_A(problem) -> sp.csr_matrix:
    """Sparse A as a Kronecker sum, index = (z * ny + y) * nx + x."""
    Dx = sp.csr_matrix(axis_D(problem.hx))
    Dy = sp.csr_matrix(axis_D(problem.hy))
    Dz = sp.csr_matrix(axis_D(problem.hz, problem.sig_step)) - sp.diags(k2_nodes(problem))
    Sz = sp.diags(problem.sig_node.astype(np.complex128))
    Ix = sp.identity(problem.nx, dtype=np.complex128, format="csr")
    Iy = sp.identity(problem.ny, dtype=np.complex128, format="csr")
    A = (sp.kron(Sz, sp.kron(Iy, Dx)) + sp.kron(Sz, sp.kron(Dy, Ix))
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
