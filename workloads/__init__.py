"""Seeded synthetic inputs for the layered-media Helmholtz solver.

This module is shared by the FP64 oracle (``oracle/``) and the GPU path
(``paper_1909_01299_amd``).  It holds grid descriptions, layer maps and
random draws only: none of the solver's arithmetic lives here.

Grid convention (paper Sec. 2, the tensor grid S = S_x x S_y x S_z with per
axis steps, complex inside a PML): an axis with ``n`` interior nodes has
``n + 1`` steps ``h[0..n]``; interior node ``i`` (0-based) sits between step
``h[i]`` on its low side and ``h[i + 1]`` on its high side, and the two walls
carry homogeneous Dirichlet data.

Workload recipes (the paper prints no data sets; these stand in for the
layered-earth survey grids it describes in Sec. 2, uniform survey core plus
geometrically growing, complex-stretched PML ends):

* k^2 is piecewise constant over ``L`` layers, layer(k) = floor(k * L / nz);
  Re k^2 ~ U(0.05, 0.5), Im k^2 ~ U(0.001, 0.05) per layer.
* Complex normal entries are (N(0,1) + i N(0,1)) / sqrt(2).
* Generator: numpy PCG64, ``default_rng(190901299 + config_id)``; draw order
  k^2 real parts, k^2 imaginary parts, block sizes, right-hand sides.
* The coefficient sigma(z) of eq. (1) is optional (absent = 1).  Where it is
  drawn it is piecewise constant over the same layers, sigma ~ U(0.5, 2); the
  scheme of eq. (2) takes sigma at the nodes (x and y terms) and at the
  midpoints of the z steps (z term); a step joining two layers takes the
  harmonic mean of their values (two half-steps of the two materials in
  series), a step to a wall the value of its node's layer.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import List, Optional, Sequence

import numpy as np

SEED_BASE = 190901299


@dataclass
class Problem:
    """A layered Helmholtz problem on a tensor grid.

    hx, hy: complex steps, shapes (nx+1,), (ny+1,)
    hz:     real steps, shape (nz+1,)
    layer_of_z: int32 (nz,), values in [0, nlayers)
    k2:     complex (nlayers,)
    sep_x, sep_y: strictly increasing 0-based interior indices of the
            separator planes (block interfaces); empty = one block.
    """

    hx: np.ndarray
    hy: np.ndarray
    hz: np.ndarray
    layer_of_z: np.ndarray
    k2: np.ndarray
    sep_x: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))
    sep_y: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))
    name: str = ""
    # sigma(z) of eq. (1): real positive values at the nz nodes and at the
    # nz + 1 z steps (step k joins node k - 1 and node k); None = 1
    sigma_node: Optional[np.ndarray] = None
    sigma_step: Optional[np.ndarray] = None

    def __post_init__(self):
        self.hx = np.ascontiguousarray(self.hx, dtype=np.complex128)
        self.hy = np.ascontiguousarray(self.hy, dtype=np.complex128)
        self.hz = np.ascontiguousarray(np.real(self.hz), dtype=np.float64)
        self.layer_of_z = np.ascontiguousarray(self.layer_of_z, dtype=np.int32)
        self.k2 = np.ascontiguousarray(self.k2, dtype=np.complex128)
        self.sep_x = np.ascontiguousarray(self.sep_x, dtype=np.int32)
        self.sep_y = np.ascontiguousarray(self.sep_y, dtype=np.int32)
        if (self.sigma_node is None) != (self.sigma_step is None):
            raise ValueError("sigma_node and sigma_step are given together")
        if self.sigma_node is not None:
            self.sigma_node = np.ascontiguousarray(self.sigma_node, dtype=np.float64)
            self.sigma_step = np.ascontiguousarray(self.sigma_step, dtype=np.float64)
            assert self.sigma_node.shape == (self.nz,) and self.sigma_step.shape == (self.nz + 1,)

    @property
    def has_sigma(self) -> bool:
        return self.sigma_node is not None

    @property
    def sig_node(self) -> np.ndarray:
        """sigma at the z nodes (ones when absent)."""
        return self.sigma_node if self.sigma_node is not None else np.ones(self.nz)

    @property
    def sig_step(self) -> np.ndarray:
        """sigma at the z steps (ones when absent)."""
        return self.sigma_step if self.sigma_step is not None else np.ones(self.nz + 1)

    @property
    def nx(self) -> int:
        return self.hx.shape[0] - 1

    @property
    def ny(self) -> int:
        return self.hy.shape[0] - 1

    @property
    def nz(self) -> int:
        return self.hz.shape[0] - 1

    @property
    def nlayers(self) -> int:
        return self.k2.shape[0]

    @property
    def shape(self):
        """Array shape of one right-hand side, slowest axis first: (nz, ny, nx)."""
        return (self.nz, self.ny, self.nx)

    @property
    def unknowns(self) -> int:
        return self.nx * self.ny * self.nz

    def with_k2(self, k2) -> "Problem":
        return replace(self, k2=np.asarray(k2, np.complex128).copy())


# ----------------------------------------------------------------------------
# axis step builders
# ----------------------------------------------------------------------------

def uniform_steps(n: int, h: float = 1.0) -> np.ndarray:
    """n interior nodes, all n+1 steps equal to h (real)."""
    return np.full(n + 1, h, dtype=np.complex128)


def pml_steps(core_cells: int, pml_cells: int, ratio: float = 1.2,
              stretch: complex = 1 + 0.5j) -> np.ndarray:
    """Unit-step core of ``core_cells`` cells with ``pml_cells`` cells per side
    whose steps grow geometrically away from the core: step k (k = 1 next to
    the core) is ratio**k * stretch.  Interior nodes: core + 2*pml - 1."""
    pml = np.array([ratio ** k * stretch for k in range(1, pml_cells + 1)],
                   dtype=np.complex128)
    core = np.ones(core_cells, dtype=np.complex128)
    return np.concatenate([pml[::-1], core, pml])


def stretched_ends_steps(n: int, p: int, ratio: float = 1.2,
                         stretch: complex = 1 + 0.5j) -> np.ndarray:
    """n interior nodes; the outermost p steps at each end are stretched as in
    ``pml_steps`` (growing outward), the rest are 1."""
    h = np.ones(n + 1, dtype=np.complex128)
    for k in range(1, p + 1):
        h[p - k] = ratio ** k * stretch
        h[n - p + k] = ratio ** k * stretch
    return h


def graded_steps(n: int, rng: np.random.Generator, spread: float = 0.4, pml: int = 0,
                 ratio: float = 1.2, stretch: complex = 1 + 0.5j) -> np.ndarray:
    """n interior nodes on a general non-uniform grid: real steps
    exp(spread * s_k) with s a random sequence smoothed over five steps, so
    that no two blocks of a split share a step vector; the outermost ``pml``
    steps at each end are then stretched as in ``stretched_ends_steps``."""
    s = rng.standard_normal(n + 5)
    s = np.convolve(s, np.ones(5) / np.sqrt(5.0), mode="valid")[: n + 1]
    h = np.exp(spread * s).astype(np.complex128)
    for k in range(1, pml + 1):
        h[pml - k] *= ratio ** k * stretch
        h[n - pml + k] *= ratio ** k * stretch
    return h


def gridding_b_separators(n: int) -> np.ndarray:
    """Separators of an axis of n interior nodes split into about sqrt(n)
    blocks of about sqrt(n) nodes each (the second gridding of Sec. 2):
    round(sqrt(n)) - 1 separators, the remaining nodes shared out evenly,
    larger blocks first."""
    nsep = max(int(round(np.sqrt(n))) - 1, 0)
    nodes, nblk = n - nsep, nsep + 1
    sizes = [nodes // nblk + (1 if i < nodes % nblk else 0) for i in range(nblk)]
    seps, pos = [], -1
    for i in range(nsep):
        pos += sizes[i] + 1
        seps.append(pos)
    return np.asarray(seps, np.int32)


def layer_map(nz: int, nlayers: int) -> np.ndarray:
    """layer(k) = floor(k * L / nz) for 0-based z node k."""
    k = np.arange(nz, dtype=np.int64)
    return ((k * nlayers) // nz).astype(np.int32)


def draw_k2(rng: np.random.Generator, nlayers: int) -> np.ndarray:
    re = rng.uniform(0.05, 0.5, size=nlayers)
    im = rng.uniform(0.001, 0.05, size=nlayers)
    return re + 1j * im


def draw_sigma(rng: np.random.Generator, nlayers: int) -> np.ndarray:
    return rng.uniform(0.5, 2.0, size=nlayers)


def layered_sigma(layer_of_z: np.ndarray, sig_layers: np.ndarray):
    """(sigma_node, sigma_step) of a piecewise constant sigma: node k takes its
    layer's value; a z step between nodes of two layers the harmonic mean of
    the two, a step to a wall its node's value."""
    lz = np.asarray(layer_of_z)
    sl = np.asarray(sig_layers, dtype=np.float64)
    node = sl[lz]
    nz = lz.shape[0]
    step = np.empty(nz + 1)
    step[0] = node[0]
    step[nz] = node[nz - 1]
    a, b = node[:-1], node[1:]
    step[1:nz] = 2.0 * a * b / (a + b)
    return node, step


def with_sigma(problem: "Problem", sig_layers: np.ndarray) -> "Problem":
    node, step = layered_sigma(problem.layer_of_z, sig_layers)
    return replace(problem, sigma_node=node, sigma_step=step)


def complex_normal(rng: np.random.Generator, shape) -> np.ndarray:
    a = rng.standard_normal(size=shape)
    b = rng.standard_normal(size=shape)
    return (a + 1j * b) / np.sqrt(2.0)


def point_source(shape_zyx, x: int, y: int, z: int, amp: complex = 1.0) -> np.ndarray:
    f = np.zeros(shape_zyx, dtype=np.complex128)
    f[z, y, x] = amp
    return f


def rng_for(config_id: int, *sub: int) -> np.random.Generator:
    if sub:
        return np.random.default_rng([SEED_BASE, config_id, *sub])
    return np.random.default_rng(SEED_BASE + config_id)


# ----------------------------------------------------------------------------
# problem builders
# ----------------------------------------------------------------------------

def uniform_problem(nx: int, ny: int, nz: int, nlayers: int, rng: np.random.Generator,
                    h: float = 1.0, name: str = "") -> Problem:
    k2 = draw_k2(rng, nlayers)
    return Problem(uniform_steps(nx, h), uniform_steps(ny, h), np.full(nz + 1, 1.0),
                   layer_map(nz, nlayers), k2, name=name)


def decomposed_problem(core_cells: int, pml_cells: int, nz: int, nlayers: int,
                       rng: np.random.Generator, name: str = "",
                       ratio: float = 1.2, stretch: complex = 1 + 0.5j) -> Problem:
    """Uniform core plus PML ends on x and y, split 4 x 4: PML | core | core | PML.

    Separators (0-based interior indices): pml-1, pml-1+core/2, pml-1+core.
    """
    assert core_cells % 2 == 0
    h = pml_steps(core_cells, pml_cells, ratio, stretch)
    seps = np.array([pml_cells - 1, pml_cells - 1 + core_cells // 2,
                     pml_cells - 1 + core_cells], dtype=np.int32)
    k2 = draw_k2(rng, nlayers)
    return Problem(h, h.copy(), np.full(nz + 1, 1.0), layer_map(nz, nlayers), k2,
                   seps, seps.copy(), name=name)


def random_problem(nx: int, ny: int, nz: int, nlayers: int, rng: np.random.Generator,
                   sep_x: Sequence[int] = (), sep_y: Sequence[int] = (),
                   pml_x: int = 0, pml_y: int = 0, name: str = "") -> Problem:
    """Small test problem: optional stretched ends, random non-uniform real z
    steps in [0.7, 1.3], random layer k^2."""
    hx = stretched_ends_steps(nx, pml_x) if pml_x else uniform_steps(nx)
    hy = stretched_ends_steps(ny, pml_y) if pml_y else uniform_steps(ny)
    hz = rng.uniform(0.7, 1.3, size=nz + 1)
    k2 = draw_k2(rng, nlayers)
    return Problem(hx, hy, hz, layer_map(nz, nlayers), k2,
                   np.asarray(sep_x, np.int32), np.asarray(sep_y, np.int32), name=name)


def gridding_b_problem(nx: int, ny: int, nz: int, nlayers: int, rng: np.random.Generator,
                       pml: int = 0, spread: float = 0.4, name: str = "") -> Problem:
    """General non-uniform x and y steps (``graded_steps``, stretched ends of
    ``pml`` steps) split into about sqrt(n) x sqrt(n) blocks of about sqrt(n)
    nodes per side (``gridding_b_separators``); random real z steps in
    [0.7, 1.3] and layer k^2 as in ``random_problem``."""
    hx = graded_steps(nx, rng, spread, pml)
    hy = graded_steps(ny, rng, spread, pml)
    hz = rng.uniform(0.7, 1.3, size=nz + 1)
    k2 = draw_k2(rng, nlayers)
    return Problem(hx, hy, hz, layer_map(nz, nlayers), k2,
                   gridding_b_separators(nx), gridding_b_separators(ny), name=name)


# ----------------------------------------------------------------------------
# the five benchmark workloads
# ----------------------------------------------------------------------------

def c1_single_block():
    """32^3 uniform block, h=1, 4 layers, one complex-normal RHS, complex128."""
    rng = rng_for(0)
    p = uniform_problem(32, 32, 32, 4, rng, name="c1_single_block_32^3")
    f = complex_normal(rng, (1,) + p.shape)
    return p, f


def c2_decomposed(core_cells: int = 256, pml_cells: int = 16, nz: int = 200,
                  nlayers: int = 20, source: Optional[tuple] = None):
    """Uniform core + PML, 4x4 blocks with interface reduction; unit point source
    at the grid centre (D-form amplitude).  Defaults: 287 x 287 x 200."""
    rng = rng_for(1)
    p = decomposed_problem(core_cells, pml_cells, nz, nlayers, rng,
                           name=f"c2_decomposed_{core_cells + 2 * pml_cells - 1}^2x{nz}")
    if source is None:
        source = (p.nx // 2, p.ny // 2, nz // 2)
    f = point_source(p.shape, *source)[None]
    return p, f


@dataclass
class BatchBlock:
    problem: Problem
    uniform: bool


def c3_blocks(nblocks: int = 64, nmin: int = 32, nmax: int = 256, zmin: int = 64,
              zmax: int = 256, nlayers: int = 8) -> List[BatchBlock]:
    """Independent Dirichlet blocks of uneven sizes; the first half uniform,
    the second half with floor(n/8) stretched steps at each end of x and y."""
    rng = rng_for(2)
    sizes = []
    for _ in range(nblocks):
        nx = int(rng.integers(nmin, nmax + 1))
        ny = int(rng.integers(nmin, nmax + 1))
        nz = int(rng.integers(zmin, zmax + 1))
        sizes.append((nx, ny, nz))
    out = []
    for b, (nx, ny, nz) in enumerate(sizes):
        brng = rng_for(2, b)
        uni = b < nblocks // 2
        k2 = draw_k2(brng, nlayers)
        if uni:
            hx, hy = uniform_steps(nx), uniform_steps(ny)
        else:
            hx, hy = stretched_ends_steps(nx, nx // 8), stretched_ends_steps(ny, ny // 8)
        p = Problem(hx, hy, np.full(nz + 1, 1.0), layer_map(nz, nlayers), k2,
                    name=f"c3_block{b}_{nx}x{ny}x{nz}")
        out.append(BatchBlock(p, uni))
    return out


def c3_rhs(block_index: int, problem: Problem, nrhs: int = 8) -> np.ndarray:
    brng = rng_for(2, block_index, 1)
    return complex_normal(brng, (nrhs,) + problem.shape)


def c4_adjoint(n: int = 128, nz: int = 160, nlayers: int = 40,
               source=(64, 64, 4), plane_z: int = 9):
    """Adjoint workload: uniform n x n x nz, nlayers layers; misfit samples the
    z = plane_z plane; data come from k^2 perturbed by up to 10% (real factor)."""
    rng = rng_for(3)
    p = uniform_problem(n, n, nz, nlayers, rng, name=f"c4_adjoint_{n}^2x{nz}")
    xi = rng.uniform(-1.0, 1.0, size=nlayers)
    k2_true = p.k2 * (1.0 + 0.1 * xi)
    f = point_source(p.shape, *source)[None]
    return p, f, k2_true, plane_z


def c5_multi_rhs(core_cells: int = 512, pml_cells: int = 32, nz: int = 256,
                 nlayers: int = 60, nsrc: int = 16, omegas=(1.0, 1.5, 2.0, 3.0)):
    """Large decomposed grid; nsrc random point sources in the core, off the
    separators; k^2 scaled by omega^2 per frequency."""
    rng = rng_for(4)
    p = decomposed_problem(core_cells, pml_cells, nz, nlayers, rng,
                           name=f"c5_multi_rhs_{core_cells + 2 * pml_cells - 1}^2x{nz}")
    lo, hi = pml_cells, pml_cells + core_cells - 2
    srcs = []
    while len(srcs) < nsrc:
        x = int(rng.integers(lo, hi + 1))
        y = int(rng.integers(lo, hi + 1))
        z = int(rng.integers(0, nz))
        if x in p.sep_x or y in p.sep_y:
            continue
        srcs.append((x, y, z))
    return p, srcs, tuple(omegas)


def gridding_b_large(n: int = 575, pml: int = 32, nz: int = 256, nlayers: int = 60, nsrc: int = 4):
    """The second gridding of Sec. 2 at the large grid's size: n x n x nz with
    graded non-uniform x and y steps (spread 0.4) and stretched ends of ``pml``
    steps, split into about sqrt(n) x sqrt(n) blocks (24 x 24 of 23 nodes for
    n = 575); nsrc random point sources off the separators."""
    rng = rng_for(6)
    p = gridding_b_problem(n, n, nz, nlayers, rng, pml=pml, name=f"gridding_b_{n}^2x{nz}")
    srcs = []
    while len(srcs) < nsrc:
        x = int(rng.integers(pml, n - pml))
        y = int(rng.integers(pml, n - pml))
        z = int(rng.integers(0, nz))
        if x in p.sep_x or y in p.sep_y:
            continue
        srcs.append((x, y, z))
    return p, srcs


def point_source_batch(problem: Problem, srcs) -> np.ndarray:
    f = np.zeros((len(srcs),) + problem.shape, dtype=np.complex128)
    for r, (x, y, z) in enumerate(srcs):
        f[r, z, y, x] = 1.0
    return f
