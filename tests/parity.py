"""Parity checks of a GPU result against the oracle's, per right-hand side.

Three bounds, each at the same tolerance:
  * the relative 2-norm error over all unknowns (the metric's definition);
  * the largest pointwise error relative to the largest reference magnitude,
    so an error confined to a few nodes cannot hide in the 2-norm;
  * on decomposed grids, the relative 2-norm error over the separator planes
    alone (about 2% of the nodes, where the interface reduction writes).
"""
import numpy as np

from oracle import operator


def errors(u, ref, problem=None) -> dict:
    u = np.asarray(u)
    ref = np.asarray(ref)
    d = u - ref
    out = {"rel2": float(np.linalg.norm(d.ravel()) / np.linalg.norm(ref.ravel())),
           "relmax": float(np.abs(d).max() / np.abs(ref).max())}
    if problem is not None and (len(problem.sep_x) or len(problem.sep_y)):
        m = operator.sigma_mask(problem)
        out["rel2_sigma"] = float(np.linalg.norm(d[m]) / np.linalg.norm(ref[m]))
    return out


def check(u, ref, tol, problem=None, label=""):
    """Assert every bound for one right-hand side ([nz][ny][nx]) or for each
    right-hand side of a batch ([nrhs][nz][ny][nx])."""
    u = np.asarray(u)
    ref = np.asarray(ref)
    if u.ndim == 4:
        return [check(u[r], ref[r], tol, problem, f"{label} rhs {r}") for r in range(u.shape[0])]
    e = errors(u, ref, problem)
    for k, v in e.items():
        assert v < tol, f"{label}: {k} = {v:.3e} >= {tol:.1e} ({e})"
    return e
