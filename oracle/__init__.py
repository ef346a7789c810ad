"""FP64 CPU oracle for the layered-media Helmholtz block solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package: only ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` use it.  It shares no code with the HIP path
(different algorithms, different eigensolver, no common helpers); the only
common module is ``workloads`` (seeded inputs, no solver arithmetic).

What it computes (Druskin & Zaslavsky, Sec. 2):

* ``operator``  -- the 7-point finite-volume operator of eq. (2)/(3), written
  in the D-form A = Dx (x) I (x) I + I (x) Dy (x) I + I (x) I (x) (Dz - k^2(z)),
  with D_d = M_d^{-1} K_d (minus the paper's operator, sigma = 1, the constant
  lambda replaced by a layered k^2(z)), as an explicit neighbour stencil and as
  a sparse Kronecker sum.
* ``direct``    -- u = A^{-1} f by sparse LU (brute force, small grids).
* ``separable`` -- u = A^{-1} f on the undecomposed grid by the generalized
  1D eigenproblems of Sec. 2 (K W = M W Lambda, explicit inverse of W) and
  one tridiagonal solve in z per (kx, ky) mode, eq. (5).
* ``cyclic``    -- the seven steps of the two-level cyclic reduction of
  Sec. 2 written plainly, for physical-space intermediates (v next to the
  interfaces, the interface residual r, w on the interfaces).
* ``adjoint``   -- A^{-H} g and the layer gradient of a least-squares misfit.

Pins (tests/test_oracle_pins.py): closed-form Dirichlet eigenvalues, exactness
of the finite-volume second difference on quadratics, FV symmetry, a textbook
3D sine-transform solver for constant k^2, manufactured solutions, sparse LU,
LAPACK banded solves, adjoint identities and central finite differences.
"""
from . import operator, direct, separable, cyclic, adjoint  # noqa: F401
