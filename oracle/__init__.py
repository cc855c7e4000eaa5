"""Plain, slow FP64 CPU oracle of the non-nested multilevel smoothed Schwarz
preconditioned FGMRES solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the library or its Python binding may
import, call or execute anything in this package; only the tests, the smoke
check and the benchmark's CPU-baseline leg do.  It shares no code with the
GPU path: its inputs come from the seeded generators in ``workloads`` and
everything else is written here, from the paper, with NumPy/SciPy primitives
(sparse products, LAPACK LU) as the only library steps.

Modules
  fem        P1 discretisation of -div(kappa grad u) = f (Section 2.1)
  transfer   barycentric point-location interpolation between meshes
  mls        moving-least-squares interpolation between meshes (Section 3.2)
  schwarz    coordinate-bisection partition, overlap, RAS (Section 2.2)
  ilu        ILU(k) subdomain solver (level of fill, i-k-j elimination)
  coarsen    geometry-preserving coarsening of Algorithm 1 (MIS + contraction)
  multilevel V-cycle of Algorithm 2 (Section 3.3)
  krylov     right-preconditioned flexible GMRES (Section 2.1, Section 4)
  problem    glue that builds a whole hierarchy from a workload
  elasticity P1 linear elasticity (Section 4.2) with the field-split
             interpolation of Section 3.2
"""
from . import fem, transfer, mls, ilu, coarsen, schwarz, multilevel, krylov, problem, elasticity  # noqa: F401
