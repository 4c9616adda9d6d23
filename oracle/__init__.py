"""FP64 CPU oracle for the volume-based refined lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call, link or execute anything in this
package; only the tests, the smoke check and the CPU-baseline leg of the
benchmark do.  It shares no code, table or helper with the HIP path.

What it computes (Schornbaum & Ruede, "Massively parallel algorithms for the
lattice Boltzmann method on non-uniform grids"):

* D3Q19 lattice, incompressible equilibrium, SRT collision
  (section 2, eq. fequ, eq. fvelocity, SRT collision operator);
* acoustic scaling of time steps and the level relaxation rate
  (section 2.3, eq. omega_scaling_0 / omega_scaling);
* the forest of octrees with 2:1 balance over face, edge and corner
  neighbours (section 3.2, section 3.3);
* the recursive non-uniform time step of Algorithm 1 with homogeneous
  explosion (eq. ctof) and 1/8-average coalescence (eq. ftoc), carried out
  literally: collide, recurse, explode, stream, coalesce, and for L > 0 a
  second collide / recurse / stream / coalesce (section 4, Algorithm 1;
  section 4.3, section 4.4).

Layout: ``forest`` (leaves, 2:1 balance, canonical order), ``tables``
(per-level cell sets I_L, H_L, E_L and the index tables of the streaming,
explosion and coalescence steps, written out from their set definitions with
numpy), ``refined_oracle.c`` (the FP64 loops, plain C with OpenMP over cells)
and ``refined`` (the ctypes driver).

Readings of the paper taken here (its figures are lost, some formulas are
garbled) are listed in the module docstrings where they are used.
"""

from .refined import (RefinedOracle, omega_level, lattice, equilibrium, collide, collide_trt,  # noqa: F401
                      lambda_o_level, accel_level)
from .forest import Forest  # noqa: F401
