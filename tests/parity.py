"""Parity checks of a GPU result against the oracle's, per right-hand side.

Three bounds, each at the same tolerance:
  * the relative 2-norm error over all unknowns (the metric's definition);
  * the largest pointwise error relative to the largest reference magnitude,
    so an error confined to a few nodes cannot hide in the 2-norm;
  * on decomposed grids, the error on the separator planes (about 1-2% of the
    nodes, where the interface reduction writes) as an RMS per node, over the
    RMS of the whole reference field: an error confined to the separators
    must stay below the tolerance per node, sqrt(N / |Sigma|) (about 7-10)
    times stricter than the 2-norm alone.  The error relative to the
    separator field itself is reported (rel2_sigma) but not bounded: for a
    source deep inside a block at the highest frequency that field is 1e-4 of
    the whole, below what an FP64 solve through the global eigenvector tables,
    the oracle's included, resolves in relative terms.
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
        nsig, ntot = int(m.sum()), m.size
        out["rms_sigma"] = float(np.linalg.norm(d[m]) / np.sqrt(nsig)
                                 / (np.linalg.norm(ref.ravel()) / np.sqrt(ntot)))
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
    bound = {"rel2": tol, "relmax": tol}
    if "rms_sigma" in e:
        bound["rms_sigma"] = tol
    for k, b in bound.items():
        assert e[k] < b, f"{label}: {k} = {e[k]:.3e} >= {b:.1e} ({e})"
    return e
