"""Pins of the oracle's patch forest (CPU only): R1/R2 after random request
sequences, Algorithm 1 against an independent fixed-point closure, the
coarsening rule, and a return to the base mesh when tags vanish."""
import itertools
import random

import pytest

from paper_2508_05020_amd import workloads as W
from oracle.mesh import Forest, MeshError


def _cfg(d, base=32, n=(8, 8, 8, 8), periodic=True):
    return W.AMRConfig(name="m", dim=d, base_cells=base, patch_cells=list(n),
                       periodic=[periodic] * d)


def _closure(forest, refine_keys):
    """Independent construction of the smallest valid refinement: repeatedly
    give children to every requested patch and to every patch whose absence
    of children leaves a missing Moore neighbour at the level above."""
    want = set()
    for k in refine_keys:
        if forest.exists(k) and forest.is_leaf(k):
            want.add(k)
    active = set(forest.parent)
    changed = True
    while changed:
        changed = False
        for k in list(want):
            for c in forest.child_keys(k):
                if c not in active:
                    active.add(c)
                    changed = True
        # R2 on the enlarged set: every patch with children needs its
        # neighbours; a missing neighbour is supplied by refining its cover
        for k in list(active):
            has_kids = any(c in active for c in forest.child_keys(k)) \
                if k[0] + 1 < forest.cfg.max_levels else False
            if not has_kids:
                continue
            for off in forest.moore_offsets():
                q = forest.shifted(k[0], k[1], off)
                if q is None or (k[0], q) in active:
                    continue
                cov = forest.covering(k[0], q)
                if cov not in want:
                    want.add(cov)
                    changed = True
    return active


@pytest.mark.parametrize("d,periodic", [(1, False), (2, True), (2, False), (3, True)])
def test_refinement_matches_closure_and_rules(d, periodic):
    rnd = random.Random(7 + d)
    base = 16 if d == 3 else 32
    cfg = _cfg(d, base=base, periodic=periodic)
    f = Forest(cfg)
    for it in range(6):
        leaves = [k for k in f.leaves() if k[0] < cfg.max_levels - 1]
        req = rnd.sample(leaves, max(1, len(leaves) // 6))
        expect = _closure(f, req)
        f.regrid(req, [])
        f.validate()
        assert set(f.parent) == expect


def test_recursive_refinement_example():
    # refining a level-1 patch whose Moore neighbour does not exist forces the
    # covering level-0 patch to be refined first (Algorithm 1)
    cfg = _cfg(2, base=32)
    f = Forest(cfg)
    f.regrid([(0, (1, 1))], [])
    # level-1 patch at the corner of the refined region
    target = (1, (2, 2))
    assert f.exists(target)
    f.regrid([target], [])
    f.validate()
    # its Moore neighbour (1, (1, 1)) lies under root (0, (0, 0))
    assert not f.is_leaf((0, (0, 0)))
    assert f.exists((2, (4, 4)))


def test_coarsening_respects_r2_and_returns_to_base():
    rnd = random.Random(3)
    cfg = _cfg(2, base=32)
    f = Forest(cfg)
    for _ in range(4):
        leaves = [k for k in f.leaves() if k[0] < cfg.max_levels - 1]
        f.regrid(rnd.sample(leaves, max(1, len(leaves) // 5)), [])
    f.validate()
    assert f.levels() >= 3
    # random coarsening requests keep the mesh valid
    for _ in range(10):
        cand = [k for k in f.keys() if not f.is_leaf(k)]
        f.regrid([], rnd.sample(cand, max(1, len(cand) // 2)))
        f.validate()
    # with every patch requested, the mesh falls back to the base level
    for _ in range(10):
        f.regrid([], [k for k in f.keys() if not f.is_leaf(k)])
        f.validate()
    assert f.levels() == 1
    assert len(f.keys()) == f.npd(0) ** 2


def test_coarsening_refused_when_children_support_finer_patch():
    cfg = _cfg(2, base=32)
    f = Forest(cfg)
    f.regrid([(0, (1, 1))], [])
    f.regrid([(1, (2, 2))], [])
    f.validate()
    # (1,(2,2)) has children; its Moore neighbours at level 1 include children
    # of (0,(0,0)) and (0,(1,0)), (0,(0,1)): those parents cannot coarsen
    assert not f.coarsening_allowed((0, (0, 0)))
    # the parent of the refined patch cannot coarsen: a child is not a leaf
    assert not f.coarsening_allowed((0, (1, 1)))
    # once the level-2 patches are gone, coarsening is allowed again
    f.regrid([], [(1, (2, 2))])
    f.validate()
    assert f.coarsening_allowed((0, (0, 0)))


def test_literal_rule_keeps_level_one():
    cfg = _cfg(2, base=32)
    f = Forest(cfg, coarsen_rule="literal")
    f.regrid([(0, (1, 1))], [])
    f.regrid([], [(0, (1, 1))])
    assert not f.is_leaf((0, (1, 1)))


def test_uneven_patch_sizes_tree():
    cfg = W.AMRConfig(name="u", dim=3, base_cells=64, patch_cells=[32, 16, 16, 8],
                      periodic=[True] * 3)
    f = Forest(cfg)
    assert f.ratio(0) == 4 and f.ratio(1) == 2 and f.ratio(2) == 4
    f.regrid([(0, (0, 0, 0))], [])
    assert len(f.children[(0, (0, 0, 0))]) == 64
    f.regrid([(1, (0, 0, 0))], [])
    f.validate()
    f.regrid([(2, (1, 1, 1))], [])
    f.validate()
    assert len(f.children[(2, (1, 1, 1))]) == 64


def test_refine_beyond_finest_rejected():
    cfg = _cfg(1, base=32, n=(8, 8))
    f = Forest(cfg)
    f.regrid([(0, (1,))], [])
    with pytest.raises(MeshError):
        f.refine((1, (2,)), [])
