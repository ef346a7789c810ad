"""Parity checks of a GPU result against the oracle's, per right-hand side.

Three bounds:
  * the relative 2-norm error over all unknowns (the metric's definition);
  * the largest pointwise error relative to the largest reference magnitude,
    so an error confined to a few nodes cannot hide in the 2-norm;
  * on decomposed grids, the relative 2-norm error over the separator planes
    alone (about 2% of the nodes, where the interface reduction writes).  Its
    bound is the tolerance, or the precision floor of an FP64 solve through
    the global eigenvector tables (1e-12 of the whole field's norm) where the
    field on the separators is so small that this floor exceeds it: for a
    source deep inside a block at the highest frequency the separator field
    is below 1e-3 of the whole, and there the oracle itself is no more exact.
"""
import numpy as np

from oracle import operator

# absolute precision floor on the separators, relative to the whole field
SIGMA_FLOOR = 1e-12


def errors(u, ref, problem=None) -> dict:
    u = np.asarray(u)
    ref = np.asarray(ref)
    d = u - ref
    out = {"rel2": float(np.linalg.norm(d.ravel()) / np.linalg.norm(ref.ravel())),
           "relmax": float(np.abs(d).max() / np.abs(ref).max())}
    if problem is not None and (len(problem.sep_x) or len(problem.sep_y)):
        m = operator.sigma_mask(problem)
        out["rel2_sigma"] = float(np.linalg.norm(d[m]) / np.linalg.norm(ref[m]))
        out["sigma_share"] = float(np.linalg.norm(ref[m]) / np.linalg.norm(ref.ravel()))
    return out


def check(u, ref, tol, problem=None, label=""):
    """Assert every bound for one right-hand side ([nz][ny][nx]) or for each
    right-hand side of a batch ([nrhs][nz][ny][nx])."""
    u = np.asarray(u)
    ref = np.asarray(ref)
    if u.ndim == 4:
        return [check(u[r], ref[r], tol, problem, f"{label} rhs {r}") for r in range(u.shape[0])]
    e = errors(u, ref, problem)
    bound = {"rel2": tol, "relmax": tol}
    if "rel2_sigma" in e:
        bound["rel2_sigma"] = max(tol, SIGMA_FLOOR / e["sigma_share"])
    for k, b in bound.items():
        assert e[k] < b, f"{label}: {k} = {e[k]:.3e} >= {b:.1e} ({e})"
    return e
