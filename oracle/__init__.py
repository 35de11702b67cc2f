"""FP64 CPU oracle for two-level non-overlapping additive Schwarz PCG on the
symmetric interior penalty DG (SIPG) discretisation of -div(rho grad u) = f
on polygonal meshes.

TEST INFRASTRUCTURE ONLY. This package is the plain, slow reference that the
GPU library is checked against. Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the library never does, and the
two share no code. Everything here is NumPy/SciPy in float64.

Modules follow the paper's structure:
  quadrature  -- Gauss-Legendre and collapsed (Duffy) triangle rules
  geometry    -- polygon area/centroid/diameter/box, face extraction (Sec. 2)
  basis       -- total-degree scaled Legendre basis on cell bounding boxes (Sec. 2, V_h)
  sipg        -- SIPG matrix and load vector (Sec. 2, eq. (Ah), (lifting), (Sigma))
  clip        -- convex polygon intersection for non-nested coarse meshes
  schwarz     -- local solvers, coarse space, L2 prolongation, Galerkin A_0 (Sec. 3)
  pcg         -- ASPCG and the Lanczos condition estimate (Sec. 7 protocol)
  tet         -- the 3D case: tetrahedra, triangle faces, nested coarse transfer

Pinning status of every function is listed in each module header.
"""
from .solve import OracleSolver, solve  # noqa: F401
