"""Level geometry of the patch hierarchy, owned by the oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

A run description (any object with the attributes read in ``Grid.__init__``)
is copied into plain numbers here; every length, cell count and sample point
the oracle uses is computed from them by this module, so the oracle depends
on no other package for its geometry.

Readings (Section 2.2 places nodes at x_i = x_0 + i dx; Section 3.2 gives
every patch the same number of cells and a quadtree of children):

* the domain is [lo, hi) in every dimension; level l has
  N_l = base_cells * 2^l cells per dimension of width h_l = (hi - lo) / N_l
  (refinement ratio 2 between levels);
* cell g of level l is centred at lo + (g + 1/2) h_l (cell-centred reading);
* level l is tiled by patches of n_l cells per dimension (n_l may differ
  between levels); a level-l patch is covered by its children, so its region
  of 2 n_l level-(l+1) cells per dimension must hold a whole number of
  level-(l+1) patches, and the restriction pairs fine cells, so n_{l+1} is
  even.
"""
from __future__ import annotations

from typing import List, Sequence

import numpy as np

GHOST = 4  # ghost layers the flux-form divergence of Eq. (9) needs


class Grid:
    """Plain-number copy of a run description plus the level geometry."""

    def __init__(self, spec):
        self.dim = int(spec.dim)
        self.base_cells = int(spec.base_cells)
        self.patch_cells: List[int] = [int(n) for n in spec.patch_cells]
        self.periodic: List[bool] = [bool(p) for p in spec.periodic]
        self.lo = float(spec.lo)
        self.hi = float(spec.hi)
        self.gamma = float(spec.gamma)
        self.cfl = float(spec.cfl)
        self.weno_eps = float(spec.weno_eps)
        self.tag_theta = float(spec.tag_theta)
        self.tag_buffer = int(spec.tag_buffer)
        self.regrid_interval = int(getattr(spec, "regrid_interval", 0))
        self.max_levels = len(self.patch_cells)
        self.nvar = self.dim + 2
        self.ghost = GHOST
        self.check()

    # -- geometry ----------------------------------------------------------
    def cells(self, level: int) -> int:
        """N_l, cells per dimension of level ``level``."""
        return self.base_cells * (2 ** level)

    def h(self, level: int) -> float:
        """h_l = (hi - lo) / N_l."""
        return (self.hi - self.lo) / self.cells(level)

    def patches_per_dim(self, level: int) -> int:
        return self.cells(level) // self.patch_cells[level]

    def points(self, level: int, coord: Sequence[int]) -> List[np.ndarray]:
        """Cell centres of the interior cells of patch ``coord`` of ``level``:
        ``[x, y, z][:dim]``, each of shape ``(n,)*dim`` in array order
        (z, y, x), x varying along the last axis."""
        n = self.patch_cells[level]
        h = self.h(level)
        axes = [self.lo + (coord[j] * n + np.arange(n) + 0.5) * h for j in range(self.dim)]
        grids = np.meshgrid(*reversed(axes), indexing="ij")
        return list(reversed(grids))

    # -- structure ---------------------------------------------------------
    def check(self) -> None:
        """Raise ValueError unless the hierarchy is well formed (see the
        module docstring); the oracle needs nothing beyond that."""
        if self.dim not in (1, 2, 3):
            raise ValueError("dim must be 1, 2 or 3")
        if len(self.periodic) != self.dim:
            raise ValueError("one boundary kind per dimension")
        if not self.patch_cells or self.base_cells < 1 or not self.hi > self.lo:
            raise ValueError("empty domain or hierarchy")
        for level, n in enumerate(self.patch_cells):
            if n < 1 or self.cells(level) % n:
                raise ValueError(f"level {level}: patch edge {n} does not tile "
                                 f"{self.cells(level)} cells")
            if level > 0:
                if n % 2:
                    raise ValueError(f"level {level}: odd patch edge cannot be restricted")
                if (2 * self.patch_cells[level - 1]) % n:
                    raise ValueError(f"level {level}: patch edge {n} does not tile the "
                                     f"region of a level-{level - 1} patch")
