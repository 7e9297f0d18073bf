"""FP64 CPU oracle for the fundamental and conventional implicit FDTD schemes.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library (no kernels, headers, helpers, tables or constants); both sides are
driven from the seeded generators in ``workloads``.

What it computes (E. L. Tan, "Fundamental Schemes for Efficient Unconditionally
Stable Implicit FDTD Methods", arXiv 2011.14043):

* ``yee``          -- the splitting operators A and B of eq. (AMat) on a Yee
                      grid in a PEC box, b and d of eq. (bd), node masks and the
                      discrete energy;
* ``tridiag``      -- the Thomas algorithm (Sec. IV, tridiagonal solving);
* ``conventional`` -- the original splitting formulae: ADI eq. (clsADI), LOD1/SS1
                      eq. (orgLOD), SS2 eq. (orgSS2), LOD2 eq. (orgLOD2) with
                      (orgLOD2i)/(orgLOD2o), D'Yakonov (orgDY), Douglas-Gunn
                      in delta form (Sec. II-E); each implicit stage solved by
                      eliminating H (a tridiagonal E system per grid line);
* ``fundamental``  -- the fundamental schemes in the paper's component form:
                      ADI Sec. III-A eqs. (fasterADIaa)-(fasterADIddh) with
                      input (fastADIi)/(uTldCol) and output (fasterADIo); LOD2
                      Sec. III-B eqs. (fastLOD2aa)-(fastLOD2dd) with
                      (fastestLOD2ex1/2), (fastLOD2i), (fastLOD2o); LOD1 (fastLOD)
                      and SS2 (fastSS2) by the same component pattern;
                      D'Yakonov (fastDY) and Douglas-Gunn ((fasterADI) with
                      the increments of (fastDGo)) of Sec. II-E;
* ``dense``        -- a dense-matrix version of every scheme for tiny grids,
                      with A and B assembled node by node from Maxwell's curl
                      equations (independent of ``yee``);
* ``crank_nicolson`` -- Crank-Nicolson without factorization, original and
                      fundamental forms (Sec. II-E), sparse direct solves;
* ``source``       -- the point-source convention for the nonhomogeneous terms
                      that the paper omits (Sec. II opening);
* ``run``          -- one entry point ``run(...)`` over schemes and forms.

Every function is pinned by tests in ``tests/test_oracle_*.py`` against
closed forms, brute-force dense solves or finite differences.
"""
from .yee import (EPS0, MU0, C0, Grid, COMPONENTS, dynamic_mask, energy,
                  apply_operator, cfl_dt)
from .tridiag import thomas
from .run import run, SCHEMES, FORMS, SPLITTINGS, UNFACTORIZED

__all__ = ["EPS0", "MU0", "C0", "Grid", "COMPONENTS", "dynamic_mask", "energy",
           "apply_operator", "cfl_dt", "thomas", "run", "SCHEMES", "FORMS", "SPLITTINGS",
           "UNFACTORIZED"]
