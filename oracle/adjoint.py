"""Adjoint solves and the layer gradient of a least-squares misfit.

Oracle code: test infrastructure only.  Not in the paper; the operator is
the one of Sec. 2, eq. (3).

Adjoint solve.  A = Dx (+) Dy (+) (Dz - k^2) with D_d = W_d Lambda_d W_d^{-1}
gives A^H = Dx^H (+) Dy^H (+) (Dz - k^2)^H with D_d^H = W_d^{-H} conj(Lambda_d)
W_d^H, so a = A^{-H} g is: transform by W^H along x and y, one tridiagonal
solve per mode with (Dz - k^2)^H + conj(lambda_a + mu_b), transform back by
W^{-H}.

Gradient.  With u = A(k^2)^{-1} f and J = 0.5 ||P u - d||^2, dA/dk^2_l =
-E_l (E_l selects the z nodes of layer l), so for real J the derivative is
dJ = Re(c_l dk^2_l) with c_l = sum_{z in l} conj(a) u and a = A^{-H} P^T (P u - d).
In torch's convention (dJ/dRe + i dJ/dIm) the gradient is conj(c_l) =
sum a conj(u), and the gradient with respect to f is a.
"""
from __future__ import annotations

import numpy as np

from .operator import k2_nodes, z_tridiag
from .separable import SeparableSolver, thomas, transform_x, transform_y


def solve_adjoint(problem, g: np.ndarray, solver: SeparableSolver = None) -> np.ndarray:
    g = np.asarray(g, dtype=np.complex128)
    single = g.ndim == 3
    if single:
        g = g[None]
    s = solver or SeparableSolver(problem)
    lower, zdiag, upper = z_tridiag(problem.hz, k2_nodes(problem), problem.sig_step)
    # (Dz - k^2)^H: transpose swaps lower and upper (shifted by one row), conj
    lo_h = np.zeros_like(lower)
    up_h = np.zeros_like(upper)
    lo_h[1:] = np.conj(upper[:-1])
    up_h[:-1] = np.conj(lower[1:])
    d_h = np.conj(zdiag)
    shift = np.conj(s.lam_y[:, None] + s.lam_x[None, :])
    WxH = s.Wx.conj().T
    WyH = s.Wy.conj().T
    WxiH = s.Wxi.conj().T
    WyiH = s.Wyi.conj().T
    gh = transform_y(WyH, transform_x(WxH, g))
    diag = d_h[:, None, None] + problem.sig_node[:, None, None] * shift[None]
    ah = np.empty_like(gh)
    for r in range(gh.shape[0]):
        ah[r] = thomas(lo_h, diag, up_h, gh[r])
    a = transform_y(WyiH, transform_x(WxiH, ah))
    return a[0] if single else a


def layer_sum(problem, a: np.ndarray, u: np.ndarray) -> np.ndarray:
    """grad[r, l] = sum over (x, y) and z in layer l of a * conj(u)."""
    a = np.asarray(a)
    u = np.asarray(u)
    if a.ndim == 3:
        a = a[None]
        u = u[None]
    per_z = np.sum(a * np.conj(u), axis=(2, 3))            # (R, nz)
    out = np.zeros((a.shape[0], problem.nlayers), dtype=np.complex128)
    for z, l in enumerate(problem.layer_of_z):
        out[:, l] += per_z[:, z]
    return out


def plane_misfit(problem, f, plane_z: int, d, solver: SeparableSolver = None):
    """J = 0.5 ||u[plane_z] - d||^2 with u = A^{-1} f (single RHS)."""
    s = solver or SeparableSolver(problem)
    u = s.solve(f)
    res = u[plane_z] - d
    return 0.5 * float(np.sum(np.abs(res) ** 2)), u


def plane_misfit_grad(problem, f, plane_z: int, d):
    """(J, grad_k2 (nlayers,), u, a) for the plane-sampling misfit."""
    s = SeparableSolver(problem)
    J, u = plane_misfit(problem, f, plane_z, d, s)
    g = np.zeros_like(u)
    g[plane_z] = u[plane_z] - d
    a = solve_adjoint(problem, g, s)
    return J, layer_sum(problem, a, u)[0], u, a
