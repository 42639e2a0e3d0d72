"""CPU FP64 oracle for the AMR compressible-Euler hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or run
anything in this package: only the tests, the smoke check and the CPU-baseline
leg of the benchmark do.  The oracle shares no code with the HIP library and
imports nothing from the product package: it reads the plain numbers of a run
description (``geometry.Grid``) and takes initial data as a callable that
returns primitive fields at given points (the seeded generators live in their
own module, which holds none of the method's arithmetic).

Modules
  geometry  -- level geometry: cell counts, widths h_l and cell centres.
  euler     -- per-patch right-hand side: primitives (Eq. 4-7), WENO5-JS point
               interpolation, Rusanov flux (Eq. 10-12), staggered divergence
               (Eq. 9 in conservative flux form).
  riemann   -- exact Riemann solver for the 1D Euler equations (closed form
               used to pin the scheme on shock tubes).
  mesh      -- patch forest with the R1/R2 validity rules and the paper's
               refinement (Algorithm 1) and coarsening (Algorithm 2) procedures.
  solver    -- the multi-level solver: ghost fill with conservative limited
               prolongation, restriction, refluxing, CFL time step, SSP-RK3
               stages, gradient tagging and regridding.
  cnn       -- the learned refinement predictor (forward, backward, loss, Adam).
  diagnostics -- velocity-gradient tensor and density-gradient magnitude
               (numerical Schlieren) by central differences.

Parity status: every function is pinned by a test in tests/test_oracle_*.py
against closed forms, invariants or brute force, except where a function's
docstring says "parity unpinned".
"""
