"""Input synthesis (CPU): the seeded generators evaluated on stacked patch
grids, as the batched initial-data upload calls them, give every patch the
values of the per-patch evaluation bit for bit."""
import numpy as np
import pytest

from paper_2508_05020_amd import workloads as W


@pytest.mark.parametrize("name,gen", [
    ("c1", W.shock_tube(1001)), ("c2", W.quadrants_blobs(2001)), ("implosion", W.implosion()),
    ("c3", W.blasts(3001)), ("c5", W.blasts_perturbed(5001)), ("c2", W.uniform_state(2, 3))])
def test_batched_points_equal_per_patch(name, gen):
    cfg = W.config(name)
    d = cfg.dim
    for level in range(min(2, cfg.max_levels)):
        npd = cfg.cells(level) // cfg.patch_cells[level]
        coords = [tuple((i * 7 // 3 ** j) % npd for j in range(d)) for i in range(9)]
        r, u, p = gen(W.patch_points_batch(cfg, level, coords))
        for i, c in enumerate(coords):
            r1, u1, p1 = gen(W.patch_points(cfg, level, c))
            assert np.array_equal(r[i], r1) and np.array_equal(p[i], p1)
            assert all(np.array_equal(a[i], b) for a, b in zip(u, u1))


def test_blast_refinements_stay_in_root():
    """The refinement recipe of the 3D sample mesh names one patch per level,
    each inside the region of the one before, away from the root's faces."""
    cfg = W.c5_sample_config()
    rounds = W.blast_refinements(cfg, 5001)
    assert [r[0][0] for r in rounds] == list(range(cfg.max_levels - 1))
    for (lp, cp), (lc, cc) in zip([r[0] for r in rounds], [r[0] for r in rounds[1:]]):
        ratio = 2 * cfg.patch_cells[lp] // cfg.patch_cells[lc]
        assert all(cp[j] * ratio <= cc[j] < (cp[j] + 1) * ratio for j in range(3))
