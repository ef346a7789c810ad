"""Python binding of the MI355X separable Helmholtz solver (``libhelmsep.so``).

Argument marshalling only: every step of a solve runs in the HIP kernels of
the C library (``include/helmsep.h``).  PyTorch provides device memory
(caller-owned arrays and the plan workspace) and the current stream.

The library must be built first (``python -m paper_1909_01299_amd.build`` or
``__graft_entry__.build()``); importing this package without it raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhelmsep.so")

HS_OK, HS_ERR_ARG, HS_ERR_ALLOC, HS_ERR_DEVICE, HS_ERR_SINGULAR, HS_ERR_NOCONV, HS_ERR_STATE = range(7)
HS_C128, HS_C64_REFINE = 0, 1


class HSError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


_STATUS = {0: "HS_OK", 1: "HS_ERR_ARG", 2: "HS_ERR_ALLOC", 3: "HS_ERR_DEVICE",
           4: "HS_ERR_SINGULAR", 5: "HS_ERR_NOCONV", 6: "HS_ERR_STATE"}


class _Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("hx", ctypes.c_void_p), ("hy", ctypes.c_void_p), ("hz", ctypes.c_void_p),
                ("nlayers", ctypes.c_int32), ("layer_of_z", ctypes.c_void_p), ("k2", ctypes.c_void_p),
                ("sigma_node", ctypes.c_void_p), ("sigma_step", ctypes.c_void_p)]


class _Blocks(ctypes.Structure):
    _fields_ = [("nsep_x", ctypes.c_int32), ("sep_x", ctypes.c_void_p),
                ("nsep_y", ctypes.c_int32), ("sep_y", ctypes.c_void_p)]


class _Options(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int32), ("refine_steps", ctypes.c_int32),
                ("max_rhs", ctypes.c_int32), ("flags", ctypes.c_int32), ("tol", ctypes.c_double)]


class Info(ctypes.Structure):
    _fields_ = [("nblocks", ctypes.c_int32), ("refine_steps", ctypes.c_int32),
                ("n_dense_axes", ctypes.c_int32), ("n_sine_axes", ctypes.c_int32),
                ("kappa_max", ctypes.c_double), ("eig_resid_max", ctypes.c_double),
                ("inv_resid_max", ctypes.c_double), ("min_pivot", ctypes.c_double),
                ("plan_seconds", ctypes.c_double), ("table_bytes", ctypes.c_size_t),
                ("n_fp64_modes", ctypes.c_int64), ("z_chunks", ctypes.c_int32), ("sine_lines", ctypes.c_int32),
                ("z_fixed_rows", ctypes.c_int32), ("global_dense", ctypes.c_int32), ("fp64_stream", ctypes.c_int32), ("n_split_fp16", ctypes.c_int32), ("tol", ctypes.c_double), ("resid_first", ctypes.c_double),
                ("resid_final", ctypes.c_double), ("resid_evals", ctypes.c_int32), ("converged", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class StageTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("ms", ctypes.c_double), ("launches", ctypes.c_int64),
                ("bytes_per_launch", ctypes.c_double), ("flops_per_launch", ctypes.c_double)]


EXPORTS = {
    "hs_plan_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "hs_plan_destroy": (None, [ctypes.c_void_p]),
    "hs_plan_workspace_bytes": (ctypes.c_size_t, [ctypes.c_void_p, ctypes.c_int32]),
    "hs_plan_bind_workspace": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]),
    "hs_set_k2": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "hs_solve": (ctypes.c_int, [ctypes.c_void_p] * 3 + [ctypes.c_int32, ctypes.c_void_p]),
    "hs_solve_adjoint": (ctypes.c_int, [ctypes.c_void_p] * 3 + [ctypes.c_int32, ctypes.c_void_p]),
    "hs_grad_k2": (ctypes.c_int, [ctypes.c_void_p] * 4 + [ctypes.c_int32, ctypes.c_void_p]),
    "hs_grad_k2_noalloc": (ctypes.c_int, [ctypes.c_void_p] * 4 + [ctypes.c_int32, ctypes.c_void_p]),
    "hs_residual": (ctypes.c_int, [ctypes.c_void_p] * 4 + [ctypes.c_int32, ctypes.c_void_p]),
    "hs_apply": (ctypes.c_int, [ctypes.c_void_p] * 3 + [ctypes.c_int32, ctypes.c_void_p]),
    "hs_get_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "hs_get_residuals": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                        ctypes.c_void_p]),
    "hs_batch_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "hs_batch_workspace_bytes": (ctypes.c_size_t, [ctypes.c_void_p]),
    "hs_batch_bind_workspace": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]),
    "hs_batch_solve": (ctypes.c_int, [ctypes.c_void_p] * 4),
    "hs_batch_destroy": (None, [ctypes.c_void_p]),
    "hs_batch_tune": (ctypes.c_int, [ctypes.c_void_p] * 3 + [ctypes.c_char_p, ctypes.c_void_p]),
    "hs_plan_tune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_char_p, ctypes.c_void_p]),
    "hs_plan_set_coarse": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "hs_plan_set_launch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.c_int32]),
    "hs_profile_enable": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "hs_profile_only": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_char_p]),
    "hs_profile_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "hs_axis_eig": (ctypes.c_int, [ctypes.c_int32] + [ctypes.c_void_p] * 5),
    "hs_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "hs_last_error": (ctypes.c_char_p, []),
}

_lib = None


def lib() -> ctypes.CDLL:
    """Load the in-tree HIP library; fails loudly when it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1909_01299_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status: int):
    if status != HS_OK:
        raise HSError(status, lib().hs_last_error().decode())


def _stream(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _ptr(t) -> int:
    return int(t.data_ptr())


def _check_array(t, shape, name):
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != torch.complex128 or not t.is_cuda:
        raise TypeError(f"{name} must be a complex128 CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if tuple(t.shape[-3:]) != tuple(shape):
        raise ValueError(f"{name}: trailing shape {tuple(t.shape[-3:])} != {tuple(shape)}")


def _nrhs_of(t) -> int:
    """Right-hand sides held by an array of shape [..., nz, ny, nx]."""
    return 1 if t.dim() == 3 else int(np.prod(t.shape[:-3]))


def same_nrhs(first, second, names) -> int:
    """The right-hand-side count shared by two arrays of one call; raises
    ValueError (before anything is launched) when they differ, so a short
    output or second input is never written or read past its end."""
    n1, n2 = _nrhs_of(first), _nrhs_of(second)
    if n1 != n2:
        raise ValueError(f"{names[0]} holds {n1} right-hand sides but {names[1]} holds {n2}")
    return n1


def axis_eig(h: np.ndarray):
    """Host-only generalized eigenpairs of one axis (the plan's own eigensolver).

    Returns (lam, W, Winv, stats) with stats = (kappa, eig_resid, inv_resid)."""
    h = np.ascontiguousarray(np.asarray(h, dtype=np.complex128))
    n = h.shape[0] - 1
    lam = np.zeros(n, np.complex128)
    W = np.zeros((n, n), np.complex128)
    Wi = np.zeros((n, n), np.complex128)
    stats = np.zeros(3, np.float64)
    _check(lib().hs_axis_eig(n, h.ctypes.data, lam.ctypes.data, W.ctypes.data, Wi.ctypes.data,
                             stats.ctypes.data))
    return lam, W, Wi, stats


class Plan:
    """A solver plan for one layered grid (and optional block split).

    problem: any object with hx, hy (complex steps), hz (real steps),
    layer_of_z, k2 and optional sep_x, sep_y (numpy arrays)."""

    def __init__(self, problem, precision: str = "c128", max_rhs: int = 1, refine_steps: int = 0,
                 force_dense: bool = False, z_chunks: int = 0, tol: float = 0.0, device=None,
                 workspace=None, dense_global: bool = False):
        import torch
        self.problem = problem
        self.nx = len(problem.hx) - 1
        self.ny = len(problem.hy) - 1
        self.nz = len(problem.hz) - 1
        self.shape = (self.nz, self.ny, self.nx)
        self.nlayers = len(problem.k2)
        self.max_rhs = int(max_rhs)
        self.precision = precision
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        hx = np.ascontiguousarray(np.asarray(problem.hx, np.complex128))
        hy = np.ascontiguousarray(np.asarray(problem.hy, np.complex128))
        hz = np.ascontiguousarray(np.real(np.asarray(problem.hz)).astype(np.float64))
        lz = np.ascontiguousarray(np.asarray(problem.layer_of_z, np.int32))
        k2 = np.ascontiguousarray(np.asarray(problem.k2, np.complex128))
        sx = np.ascontiguousarray(np.asarray(getattr(problem, "sep_x", []), np.int32))
        sy = np.ascontiguousarray(np.asarray(getattr(problem, "sep_y", []), np.int32))
        sn = getattr(problem, "sigma_node", None)
        ss = getattr(problem, "sigma_step", None)
        sn = None if sn is None else np.ascontiguousarray(np.asarray(sn, np.float64))
        ss = None if ss is None else np.ascontiguousarray(np.asarray(ss, np.float64))
        grid = _Grid(self.nx, self.ny, self.nz, hx.ctypes.data, hy.ctypes.data, hz.ctypes.data,
                     self.nlayers, lz.ctypes.data, k2.ctypes.data,
                     None if sn is None else sn.ctypes.data, None if ss is None else ss.ctypes.data)
        blocks = _Blocks(len(sx), sx.ctypes.data if len(sx) else None, len(sy), sy.ctypes.data if len(sy) else None)
        prec = {"c128": HS_C128, "c64": HS_C64_REFINE, "mixed": HS_C64_REFINE}[precision]
        chunk_bits = {0: 0, 8: 1, 16: 2, 32: 3}[int(z_chunks)] << 1
        opts = _Options(prec, int(refine_steps), self.max_rhs, (1 if force_dense else 0) | chunk_bits | (8 if dense_global else 0),
                        float(tol))
        handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib().hs_plan_create(ctypes.byref(grid), ctypes.byref(blocks), ctypes.byref(opts),
                                        ctypes.byref(handle)))
        self._h = handle
        self._k2 = k2.copy()          # the plan's current k^2 (set_k2 skips an unchanged value)
        nbytes = lib().hs_plan_workspace_bytes(self._h, self.max_rhs)
        if workspace is None:
            workspace = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
        elif workspace.dtype != torch.uint8 or not workspace.is_cuda or workspace.numel() < nbytes:
            raise ValueError(f"workspace must be a CUDA uint8 tensor of at least {nbytes} bytes")
        # plans used one after another on one stream may share a workspace
        self.workspace = workspace
        _check(lib().hs_plan_bind_workspace(self._h, _ptr(self.workspace), self.workspace.numel()))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                lib().hs_plan_destroy(h)
            except Exception:
                pass
            self._h = None

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        """Plan statistics and the last solve's convergence record (a missed
        tolerance shows as converged == 0 here; check() raises for it)."""
        inf = Info()
        st = lib().hs_get_info(self._h, ctypes.byref(inf))
        if st not in (HS_OK, HS_ERR_NOCONV):
            _check(st)
        return inf.as_dict()

    def check(self):
        """Raise HSError(HS_ERR_NOCONV) when the last solve missed its
        tolerance (synchronize the solve's stream first)."""
        inf = Info()
        _check(lib().hs_get_info(self._h, ctypes.byref(inf)))

    def residuals(self) -> np.ndarray:
        """Relative residuals |f - A u_k| / |f| of the last solve, [eval][rhs]."""
        n_ev = ctypes.c_int32()
        nr = ctypes.c_int32()
        st = lib().hs_get_residuals(self._h, None, 0, ctypes.byref(n_ev), ctypes.byref(nr))
        _check(st)
        out = np.zeros(n_ev.value * nr.value, np.float64)
        _check(lib().hs_get_residuals(self._h, out.ctypes.data, out.size, ctypes.byref(n_ev), ctypes.byref(nr)))
        return out.reshape(n_ev.value, nr.value)

    def tune(self, nrhs: int = 1, cache: Optional[str] = None, stream=None):
        """Autotune launch shapes (z chunking, sine lines per workgroup, fixed
        z-solve rows, and on decomposed grids the form of the global
        right-hand side) on this plan."""
        _check(lib().hs_plan_tune(self._h, int(nrhs), cache.encode() if cache else None, _stream(stream)))
        inf = self.info()
        return {"z_chunks": inf["z_chunks"], "sine_lines": inf["sine_lines"], "z_fixed_rows": inf["z_fixed_rows"],
                "global_dense": inf["global_dense"], "fp64_stream": inf["fp64_stream"]}

    def set_coarse(self, coarse: Optional["Plan"]):
        """Solve this plan's interface problem by the cyclic reduction of a
        coarser plan on the same grid (its separators a subset of these), or
        by the global basis again (None).  The workspace is laid out anew and
        a new one is allocated and bound."""
        import torch
        _check(lib().hs_plan_set_coarse(self._h, coarse._h if coarse is not None else None))
        self._coarse = coarse   # keeps the coarser plan alive as long as this one
        nbytes = lib().hs_plan_workspace_bytes(self._h, self.max_rhs)
        self.workspace = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
        _check(lib().hs_plan_bind_workspace(self._h, _ptr(self.workspace), self.workspace.numel()))

    def set_launch(self, shapes: dict):
        """Apply launch shapes as returned by tune() (z_chunks, sine_lines,
        z_fixed_rows, global_dense, fp64_stream; a missing global_dense or
        fp64_stream keeps the plan's)."""
        _check(lib().hs_plan_set_launch(self._h, int(shapes.get("z_chunks", 0)), int(shapes.get("sine_lines", 0)),
                                        int(shapes.get("z_fixed_rows", 0)), int(shapes.get("global_dense", -1)),
                                        int(shapes.get("fp64_stream", -1))))

    def profile(self, on: bool = True, only: Optional[str] = None):
        """Record hipEvents around every stage of subsequent solves, or only
        around the stage named `only`."""
        _check(lib().hs_profile_only(self._h, None if only is None else only.encode()))
        _check(lib().hs_profile_enable(self._h, 1 if on else 0))

    def profile_read(self) -> list:
        """Per-stage accumulated time since the last read (synchronizes)."""
        buf = (StageTime * 64)()
        n = ctypes.c_int32()
        _check(lib().hs_profile_read(self._h, buf, 64, ctypes.byref(n)))
        return [dict(name=buf[i].name.decode(), ms=buf[i].ms, launches=buf[i].launches,
                     bytes_per_launch=buf[i].bytes_per_launch, flops_per_launch=buf[i].flops_per_launch)
                for i in range(min(n.value, 64))]

    def set_k2(self, k2):
        k2 = np.ascontiguousarray(np.asarray(k2, np.complex128))
        if k2.shape != (self.nlayers,):
            raise ValueError("k2 must have one value per layer")
        if np.array_equal(k2, self._k2):
            return                    # tables and pivot scan already hold this k^2
        _check(lib().hs_set_k2(self._h, k2.ctypes.data))
        self._k2 = k2.copy()
        q = getattr(self, "_coarse", None)
        while q is not None:            # the library set the coarser plans' k^2 as well
            q._k2 = k2.copy()
            q = getattr(q, "_coarse", None)

    def _nrhs(self, t):
        return _nrhs_of(t)

    def solve(self, f, out=None, stream=None):
        import torch
        _check_array(f, self.shape, "f")
        u = out if out is not None else torch.empty_like(f)
        _check_array(u, self.shape, "u")
        n = same_nrhs(f, u, ("f", "u"))
        _check(lib().hs_solve(self._h, _ptr(f), _ptr(u), n, _stream(stream)))
        return u

    def solve_adjoint(self, g, out=None, stream=None):
        import torch
        _check_array(g, self.shape, "g")
        a = out if out is not None else torch.empty_like(g)
        _check_array(a, self.shape, "a")
        n = same_nrhs(g, a, ("g", "a"))
        _check(lib().hs_solve_adjoint(self._h, _ptr(g), _ptr(a), n, _stream(stream)))
        return a

    def grad_k2(self, u, a, stream=None):
        import torch
        _check_array(u, self.shape, "u")
        _check_array(a, self.shape, "a")
        n = same_nrhs(u, a, ("u", "a"))
        grad = torch.empty((n, self.nlayers), dtype=torch.complex128, device=u.device)
        _check(lib().hs_grad_k2(self._h, _ptr(u), _ptr(a), _ptr(grad), n, _stream(stream)))
        return grad

    def grad_k2_noalloc(self, u, a, grad=None, stream=None):
        """grad_k2 through the allocation-free entry point (static device
        scratch; no workspace).  `grad` may be a preallocated (nrhs, nlayers)
        complex128 CUDA tensor."""
        import torch
        _check_array(u, self.shape, "u")
        _check_array(a, self.shape, "a")
        n = same_nrhs(u, a, ("u", "a"))
        if grad is None:
            grad = torch.empty((n, self.nlayers), dtype=torch.complex128, device=u.device)
        elif (grad.dtype != torch.complex128 or not grad.is_cuda or not grad.is_contiguous()
              or grad.numel() < n * self.nlayers):
            raise ValueError("grad must be a contiguous complex128 CUDA tensor of nrhs * nlayers values")
        _check(lib().hs_grad_k2_noalloc(self._h, _ptr(u), _ptr(a), _ptr(grad), n, _stream(stream)))
        return grad

    def residual(self, f, u, stream=None):
        import torch
        _check_array(f, self.shape, "f")
        _check_array(u, self.shape, "u")
        n = same_nrhs(f, u, ("f", "u"))
        r = torch.empty_like(f)
        _check(lib().hs_residual(self._h, _ptr(f), _ptr(u), _ptr(r), n, _stream(stream)))
        return r

    def apply(self, u, stream=None):
        import torch
        _check_array(u, self.shape, "u")
        out = torch.empty_like(u)
        _check(lib().hs_apply(self._h, _ptr(u), _ptr(out), self._nrhs(u), _stream(stream)))
        return out


class Batch:
    """Many independent single-block plans solved together: every stage is one
    batched launch over all (plan, right-hand side) pairs, enqueued as one
    captured HIP graph (re-captured only when the array pointers change)."""

    def __init__(self, plans: Sequence[Plan], nrhs: Sequence[int]):
        import torch
        self.plans = list(plans)
        self.nrhs = [int(r) for r in nrhs]
        if len(self.plans) != len(self.nrhs) or not self.plans:
            raise ValueError("one nrhs per plan")
        arr = (ctypes.c_void_p * len(self.plans))(*[p.handle.value for p in self.plans])
        rs = (ctypes.c_int32 * len(self.plans))(*self.nrhs)
        h = ctypes.c_void_p()
        _check(lib().hs_batch_create(arr, len(self.plans), rs, ctypes.byref(h)))
        self._h = h
        nbytes = lib().hs_batch_workspace_bytes(self._h)
        self.workspace = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.plans[0].device)
        _check(lib().hs_batch_bind_workspace(self._h, _ptr(self.workspace), self.workspace.numel()))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                lib().hs_batch_destroy(h)
            except Exception:
                pass
            self._h = None

    def _arrays(self, fs, us):
        for p, r, f, u in zip(self.plans, self.nrhs, fs, us):
            _check_array(f, p.shape, "f")
            _check_array(u, p.shape, "u")
            if p._nrhs(f) != r or p._nrhs(u) != r:
                raise ValueError("right-hand side count differs from the batch's")
        fa = (ctypes.c_void_p * len(fs))(*[_ptr(f) for f in fs])
        ua = (ctypes.c_void_p * len(us))(*[_ptr(u) for u in us])
        return fa, ua

    def tune(self, fs, us, cache: Optional[str] = None, stream=None):
        """Autotune the batch's launch shapes on its whole graph (us is overwritten)."""
        if len(fs) != len(self.plans) or len(us) != len(self.plans):
            raise ValueError("one f and one u per plan")
        fa, ua = self._arrays(fs, us)
        _check(lib().hs_batch_tune(self._h, fa, ua, cache.encode() if cache else None, _stream(stream)))

    def solve(self, fs, us=None, stream=None):
        import torch
        if len(fs) != len(self.plans):
            raise ValueError("one f per plan")
        if us is None:
            us = [torch.empty_like(f) for f in fs]
        if len(us) != len(self.plans):
            raise ValueError("one u per plan")
        fa, ua = self._arrays(fs, us)
        _check(lib().hs_batch_solve(self._h, fa, ua, _stream(stream)))
        return us


def _make_autograd():
    import torch

    class HelmholtzSolve(torch.autograd.Function):
        """u = A(k2)^{-1} f with gradients for k2 (per layer) and f.

        backward: a = A^{-H} grad_u (the adjoint solve reuses the forward
        kernels), grad_f = a, grad_k2[l] = sum over layer l of a * conj(u)."""

        @staticmethod
        def forward(ctx, k2, f, plan):
            plan.set_k2(k2.detach().cpu().numpy())
            u = plan.solve(f.contiguous())
            ctx.plan = plan
            ctx.save_for_backward(u)
            ctx.k2_value = k2.detach().cpu().numpy().copy()
            ctx.k2_meta = (k2.dtype, k2.device)
            return u

        @staticmethod
        def backward(ctx, grad_u):
            (u,) = ctx.saved_tensors
            plan = ctx.plan
            plan.set_k2(ctx.k2_value)
            a = plan.solve_adjoint(grad_u.contiguous())
            g = plan.grad_k2(u, a).sum(dim=0)
            dtype, device = ctx.k2_meta
            return g.to(device=device, dtype=dtype), a, None

    return HelmholtzSolve


_autograd = None


def helmholtz_solve(k2, f, plan: Plan):
    """Differentiable solve (torch.autograd.Function) for gradients w.r.t. k2 and f."""
    global _autograd
    if _autograd is None:
        _autograd = _make_autograd()
    return _autograd.apply(k2, f, plan)


def to_device(a: np.ndarray, device="cuda"):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).to(device)
