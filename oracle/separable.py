"""Separable solve on the undecomposed grid (paper Sec. 2, eqs. (4)-(5)).

Oracle code: test infrastructure only.

For x and y the generalized 1D eigenproblem K W = M W Lambda with Dirichlet
walls is solved by LAPACK (scipy.linalg.eig) and W^{-1} is an explicit LU
inverse.  The paper writes the forward transform as W^*; with complex PML
steps the correct forward transform is W^{-1} (W^* = W^{-1} only for a
unitary W), which is the reading used here.  After the transform the 3D
system splits into one tridiagonal system in z per mode (a, b):

    (Dz - diag k^2 + (lambda_a + mu_b) diag sigma) u_hat(a, b, :) = f_hat(a, b, :),

solved by the Thomas algorithm (Gaussian elimination without pivoting, the
O(N_z) solve of eq. (5)), vectorised over all modes and right-hand sides.
With sigma(z) of eq. (1), Dz is the flux form with sigma at the z steps and
the modal shift is scaled by sigma at each node (sigma = 1 when absent).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .operator import axis_K, hhat, k2_nodes, z_tridiag


def axis_eig(h: np.ndarray):
    """Generalized eigenpairs of one axis: K W = M W diag(lam).

    Returns lam (n,), W (n, n) and Winv = inv(W) (explicit LU inverse)."""
    h = np.asarray(h, dtype=np.complex128)
    K = axis_K(h)
    M = np.diag(hhat(h))
    lam, W = sla.eig(K, M)
    Winv = sla.inv(W)
    return lam.astype(np.complex128), W.astype(np.complex128), Winv.astype(np.complex128)


def thomas(lower: np.ndarray, diag: np.ndarray, upper: np.ndarray, rhs: np.ndarray) -> np.ndarray:
    """Solve tridiagonal systems along axis 0 by elimination without pivoting.

    lower, upper: (n,) ; diag: (n, ...) broadcastable to rhs ; rhs: (n, ...).
    Row k reads lower[k] x[k-1] + diag[k] x[k] + upper[k] x[k+1] = rhs[k]."""
    n = rhs.shape[0]
    diag = np.broadcast_to(diag, rhs.shape)
    cp = np.empty(rhs.shape, dtype=np.complex128)
    dp = np.empty(rhs.shape, dtype=np.complex128)
    piv = diag[0]
    cp[0] = upper[0] / piv
    dp[0] = rhs[0] / piv
    for k in range(1, n):
        piv = diag[k] - lower[k] * cp[k - 1]
        cp[k] = upper[k] / piv
        dp[k] = (rhs[k] - lower[k] * dp[k - 1]) / piv
    x = np.empty(rhs.shape, dtype=np.complex128)
    x[n - 1] = dp[n - 1]
    for k in range(n - 2, -1, -1):
        x[k] = dp[k] - cp[k] * x[k + 1]
    return x


def transform_x(W: np.ndarray, u: np.ndarray) -> np.ndarray:
    """(W applied along x): out[..., a] = sum_x W[a, x] u[..., x]."""
    return np.matmul(u, W.T)


def transform_y(W: np.ndarray, u: np.ndarray) -> np.ndarray:
    """out[..., b, x] = sum_y W[b, y] u[..., y, x]."""
    return np.matmul(W, u)


class SeparableSolver:
    """Eigen tables of one grid, reusable across right-hand sides."""

    def __init__(self, problem):
        self.problem = problem
        self.lam_x, self.Wx, self.Wxi = axis_eig(problem.hx)
        self.lam_y, self.Wy, self.Wyi = axis_eig(problem.hy)
        self.lower, self.zdiag, self.upper = z_tridiag(problem.hz, k2_nodes(problem), problem.sig_step)
        self.sig = problem.sig_node

    def solve_spectral(self, fh: np.ndarray) -> np.ndarray:
        """z solves for every mode: fh is (R, nz, ny, nx) in mode space."""
        shift = self.lam_y[:, None] + self.lam_x[None, :]          # (b, a)
        diag = self.zdiag[:, None, None] + self.sig[:, None, None] * shift[None]   # (nz, b, a)
        out = np.empty_like(fh)
        for r in range(fh.shape[0]):
            out[r] = thomas(self.lower, diag, self.upper, fh[r])
        return out

    def solve(self, f: np.ndarray) -> np.ndarray:
        f = np.asarray(f, dtype=np.complex128)
        single = f.ndim == 3
        if single:
            f = f[None]
        fh = transform_y(self.Wyi, transform_x(self.Wxi, f))
        uh = self.solve_spectral(fh)
        u = transform_y(self.Wy, transform_x(self.Wx, uh))
        return u[0] if single else u


def solve(problem, f: np.ndarray) -> np.ndarray:
    """u = A^{-1} f on the whole grid (separators ignored)."""
    return SeparableSolver(problem).solve(f)
