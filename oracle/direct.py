"""Brute-force solves u = A^{-1} f and a = A^{-H} g by sparse LU.

Oracle code: test infrastructure only.  The paper's method is a direct
solver (abstract and Sec. 2): its seven steps reach exactly A^{-1} f up to
rounding, so on small grids this is the plain definition of its output.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from .operator import assemble_A


def _batched(f, shape):
    f = np.asarray(f, dtype=np.complex128)
    single = f.ndim == 3
    if single:
        f = f[None]
    assert f.shape[1:] == tuple(shape), (f.shape, shape)
    return f, single


def solve_splu(problem, f: np.ndarray) -> np.ndarray:
    f, single = _batched(f, problem.shape)
    lu = spla.splu(assemble_A(problem).tocsc())
    u = np.stack([lu.solve(fr.ravel()).reshape(problem.shape) for fr in f])
    return u[0] if single else u


def solve_adjoint_splu(problem, g: np.ndarray) -> np.ndarray:
    g, single = _batched(g, problem.shape)
    AH = assemble_A(problem).conj().T.tocsc()
    lu = spla.splu(AH)
    a = np.stack([lu.solve(gr.ravel()).reshape(problem.shape) for gr in g])
    return a[0] if single else a
