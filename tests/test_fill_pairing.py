"""The ghost regions that the coarse/fine fill prolongs are unions of
aligned 2^d blocks of fine cells sharing one coarse cell after the boundary
mapping.  A region of a level-l patch (l >= 1) starts at -4, 0 or n and
extends 4 or n cells in each dimension, all even for the even patch edges
the configuration rules allow, and the mapping (a periodic wrap over an even
cell count, or the clamp at a transmissive boundary) keeps each pair
(2k, 2k + 1) on one coarse cell.  The coarse-cell form of the fill computes
one coarse stencil per such block; this checks the property with the
oracle's own boundary mapping, for every region of the patches at and next
to the domain boundary and of one interior patch per level."""
import itertools

import numpy as np
import pytest

from oracle.solver import OracleAMR
from paper_2508_05020_amd import workloads as W


@pytest.mark.parametrize("d,base,cells,periodic", [
    (2, 64, [16, 32, 32], [True, False]),
    (2, 64, [32, 16, 16], [False, False]),
    (3, 32, [16, 8], [True, False, True]),
    (3, 32, [8, 8, 8], [False, False, False]),
])
def test_fill_pairs_share_coarse_cell(d, base, cells, periodic):
    cfg = W.AMRConfig(name="pair", dim=d, base_cells=base, patch_cells=cells,
                      periodic=periodic, max_patches=4096)
    o = OracleAMR(cfg)
    checked = 0
    for level in range(1, cfg.max_levels):
        n = cfg.patch_cells[level]
        npd = cfg.cells(level) // n
        near = sorted({0, 1, npd // 2, npd - 2, npd - 1} & set(range(npd)))
        for coord in itertools.product(near, repeat=d):
            for r in itertools.product((-1, 0, 1), repeat=d):
                if not any(r):
                    continue
                axes = []
                for j in range(d):
                    start = -4 if r[j] < 0 else (0 if r[j] == 0 else n)
                    axes.append(coord[j] * n + start + np.arange(4 if r[j] else n))
                g = np.meshgrid(*axes, indexing="ij")
                mapped = o.bc_map(level, g)
                for j in range(d):
                    lo = np.take(mapped[j], np.arange(0, g[j].shape[j], 2), axis=j)
                    hi = np.take(mapped[j], np.arange(1, g[j].shape[j], 2), axis=j)
                    assert np.array_equal(lo >> 1, hi >> 1), (level, coord, r, j)
                checked += 1
    assert checked > 0


def test_odd_pairing_would_fail():
    """The check is not vacuous: pairs taken from an odd start, (1, 2) and
    (3, 4), straddle coarse cells, and the comparison used above rejects
    them."""
    cfg = W.AMRConfig(name="pair", dim=1, base_cells=32, patch_cells=[8, 8],
                      periodic=[False], max_patches=64)
    o = OracleAMR(cfg)
    m = o.bc_map(1, [np.arange(1, 5)])[0]
    assert not np.array_equal(m[0::2] >> 1, m[1::2] >> 1)
