"""The seven steps of the two-level cyclic reduction, written plainly.

Oracle code: test infrastructure only.  Follows paper Sec. 2 (the block
problems of eq. (4), the interface residual, the global solve of eq. (6) and
the local correction of eq. (7)), in the paper's order:

1-2. for every block S^ij solve the Dirichlet problem A^ij v^ij = f^ij
     (v = 0 on the interfaces Sigma);
3-4. r = f - A v, which is supported on Sigma only;
5.   w = A^{-1} r on the whole grid (the global eigen-transform), kept on Sigma;
6.   for every block solve A^ij w^ij = 0 with Dirichlet data w on its
     boundary, i.e. A_II w_I = -A_{I,Sigma} w_Sigma;
7.   u = v + w inside the blocks and u = w on Sigma.

`nested` is the multi-level form of the remark that follows the cost
estimate in Sec. 2: nested partitions, with step 5 of one level
solved by the same seven steps on the next coarser partition.

Blocks are the maximal runs of interior nodes between separator planes (a
separator plane belongs to no block); A^ij is the principal sub-matrix of A
on a block, so its steps include the ones reaching the separators.
"""
from __future__ import annotations

import numpy as np

from .operator import apply_A, sigma_mask
from .separable import SeparableSolver


def block_ranges(n: int, seps) -> list:
    """Inclusive (lo, hi) runs of interior nodes between separators."""
    out = []
    start = 0
    for s in list(seps) + [n]:
        if s - 1 >= start:
            out.append((start, s - 1))
        start = s + 1
    return out


def sub_problem(problem, x0, x1, y0, y1):
    from workloads import Problem
    return Problem(problem.hx[x0:x1 + 2], problem.hy[y0:y1 + 2], problem.hz,
                   problem.layer_of_z, problem.k2, sigma_node=problem.sigma_node,
                   sigma_step=problem.sigma_step)


def _block_solve_all(problem, rhs):
    out = np.zeros_like(rhs)
    for (x0, x1) in block_ranges(problem.nx, problem.sep_x):
        for (y0, y1) in block_ranges(problem.ny, problem.sep_y):
            sub = sub_problem(problem, x0, x1, y0, y1)
            out[..., y0:y1 + 1, x0:x1 + 1] = SeparableSolver(sub).solve(
                np.ascontiguousarray(rhs[..., y0:y1 + 1, x0:x1 + 1]))
    return out


def seven_step(problem, f: np.ndarray, solve5=None):
    """Returns (u, intermediates) with intermediates v, r (full grid), w_sigma.
    solve5 (optional): the solver of step 5's A w = r on the whole grid
    (default: the global eigen-transform)."""
    f = np.asarray(f, dtype=np.complex128)
    single = f.ndim == 3
    if single:
        f = f[None]
    mask = sigma_mask(problem)[None]
    # steps 1-2
    v = _block_solve_all(problem, np.where(mask, 0.0, f))
    # steps 3-4
    r = f - apply_A(problem, v)
    # step 5
    rs = np.where(mask, r, 0.0)
    w_full = SeparableSolver(problem).solve(rs) if solve5 is None else solve5(rs)
    w_sigma = np.where(mask, w_full, 0.0)
    # step 6
    lift = -apply_A(problem, w_sigma)
    w_blocks = _block_solve_all(problem, np.where(mask, 0.0, lift))
    # step 7
    u = v + w_blocks + w_sigma
    inter = dict(v=v, r=r, w_sigma=w_sigma, w_full=w_full)
    if single:
        u = u[0]
        inter = {k: val[0] for k, val in inter.items()}
    return u, inter


def nested(problem, f: np.ndarray, coarse_levels):
    """Multi-level cyclic reduction: the seven steps on `problem`'s
    separators, whose step 5 is the same method on the next coarser
    partition coarse_levels[0] = (sep_x, sep_y), each list a subset of the
    finer one, and so on; the coarsest level's step 5 is the global
    eigen-transform.  Returns u."""
    from dataclasses import replace
    if not coarse_levels:
        return seven_step(problem, f)[0]
    sx, sy = (np.asarray(v, np.int32) for v in coarse_levels[0])
    assert set(sx.tolist()) <= set(problem.sep_x.tolist()) and set(sy.tolist()) <= set(problem.sep_y.tolist())
    coarser = replace(problem, sep_x=sx, sep_y=sy)
    rest = coarse_levels[1:]
    if len(sx) == 0 and len(sy) == 0:
        solve5 = SeparableSolver(coarser).solve
    else:
        def solve5(rhs):
            return nested(coarser, rhs, rest)
    return seven_step(problem, f, solve5)[0]

