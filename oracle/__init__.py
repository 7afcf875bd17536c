"""FP64 CPU oracle for the hp-DG subspace-correction solver.

TEST INFRASTRUCTURE. This package is the plain, slow, independent reference
that the GPU library is checked against. Only the tests, the smoke check and
the benchmark's CPU-baseline leg may import it. It shares no code with the
GPU library (paper_2009_01287_amd) and never imports it; the only common
module is hpinputs, which generates seeded inputs and holds none of the
method's arithmetic.

Modules
  gl       1D Gauss-Lobatto basis, exact 1D mass/stiffness (Sec. 2.2)
  mesh     leaves, faces, sub-entities, hanging/master relations
  dg       SIPG and BR2 operators (Sec. 2, Sec. 4.4), diagonal, sub-blocks,
           right-hand side
  precond  V_J/V_e labels, conforming prolongation, LOR, AMG, B (Sec. 3)
  pcg      PCG with Lanczos condition estimate (Sec. 3.1, Sec. 4.1)

Every function is pinned by a test under tests/ that does not re-use the
oracle's own code.
"""
from . import gl, mesh, dg, precond, pcg  # noqa: F401
from .mesh import Mesh  # noqa: F401
from .dg import Opts  # noqa: F401
