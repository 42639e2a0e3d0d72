"""Patch forest with the paper's mesh-validity rules and adaptation procedures.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Section 3.2-3.3 of the paper: the base-level patches form a Cartesian layout
and each is the root of a tree (quadtree in 2D).  A patch at level l with
coordinate P covers cells ``P*n_l .. P*n_l + n_l - 1`` of level l; its children
tile the same region at level l+1.  With equal patch edges on all levels a
patch has 2^d children (the paper's ``child[4]`` in 2D); with per-level edges
it has ``(2 n_l / n_{l+1})^d``.

Rules (Section 3.3):
  R1  level-0 patches are never removed;
  R2  if a patch P at level l has children then every patch of its Moore
      neighbourhood N(P) (the 3^d - 1 same-level patches around it) is active;
      positions outside a non-periodic domain count as present (ghost patches),
      and a periodic domain wraps.

Algorithm 1 (recursive refinement) and Algorithm 2 (coarsening) are
implemented as described in the text; see ``coarsening_allowed`` for the
reading of Algorithm 2's conditions.

Keys are ``(level, coord)`` with ``coord`` a tuple in (x, y, z) order.
Deterministic orders: patches are visited by (level, z, y, x); Moore
neighbours and children are enumerated with x varying fastest.
"""
from __future__ import annotations

import itertools
from typing import Dict, List, Optional, Tuple

from .geometry import Grid

Key = Tuple[int, Tuple[int, ...]]


class MeshError(Exception):
    pass


def order_key(key: Key):
    level, coord = key
    return (level, tuple(reversed(coord)))


class Forest:
    def __init__(self, cfg, coarsen_rule: str = "text"):
        # the forest's own copy of the level geometry (a run description is
        # converted; an oracle Grid is used as it is)
        self.cfg = cfg if isinstance(cfg, Grid) else Grid(cfg)
        cfg = self.cfg
        self.d = cfg.dim
        self.coarsen_rule = coarsen_rule
        self.parent: Dict[Key, Optional[Key]] = {}
        self.children: Dict[Key, List[Key]] = {}
        for coord in self._box(self.npd(0)):
            self._add((0, coord), None)

    # -- geometry ----------------------------------------------------------
    def npd(self, level: int) -> int:
        return self.cfg.patches_per_dim(level)

    def ratio(self, level: int) -> int:
        """Children per dimension of a level-``level`` patch."""
        return 2 * self.cfg.patch_cells[level] // self.cfg.patch_cells[level + 1]

    def _box(self, m: int):
        for rev in itertools.product(range(m), repeat=self.d):
            yield tuple(reversed(rev))

    def moore_offsets(self):
        for rev in itertools.product((-1, 0, 1), repeat=self.d):
            if any(rev):
                yield tuple(reversed(rev))

    def shifted(self, level: int, coord, off):
        """Coordinate of the same-level position coord + off; None outside a
        non-periodic domain (a physical-boundary ghost patch)."""
        m = self.npd(level)
        out = []
        for j in range(self.d):
            c = coord[j] + off[j]
            if c < 0 or c >= m:
                if not self.cfg.periodic[j]:
                    return None
                c %= m
            out.append(c)
        return tuple(out)

    def covering(self, level: int, coord) -> Key:
        """The level-1 position whose region contains the level-``level`` patch."""
        n = self.cfg.patch_cells[level]
        nc = self.cfg.patch_cells[level - 1]
        return (level - 1, tuple((c * n // 2) // nc for c in coord))

    def child_keys(self, key: Key) -> List[Key]:
        level, coord = key
        r = self.ratio(level)
        out = []
        for rev in itertools.product(range(r), repeat=self.d):
            o = tuple(reversed(rev))
            out.append((level + 1, tuple(coord[j] * r + o[j] for j in range(self.d))))
        return out

    # -- state -------------------------------------------------------------
    def _add(self, key: Key, parent: Optional[Key]):
        self.parent[key] = parent
        self.children[key] = []

    def exists(self, key: Key) -> bool:
        return key in self.parent

    def is_leaf(self, key: Key) -> bool:
        return not self.children[key]

    def keys(self) -> List[Key]:
        return sorted(self.parent, key=order_key)

    def leaves(self) -> List[Key]:
        return [k for k in self.keys() if self.is_leaf(k)]

    def levels(self) -> int:
        return 1 + max(k[0] for k in self.parent)

    # -- Algorithm 1: recursive refinement ----------------------------------
    def refine(self, key: Key, created: List[Key]):
        """RefinePatch(M, p): if p is a leaf, make every missing Moore
        neighbour exist by refining the covering patch one level down
        (recursively), then create p's children."""
        if not self.exists(key):
            raise MeshError(f"refine of inactive patch {key}")
        if not self.is_leaf(key):
            return
        level, coord = key
        if level + 1 >= self.cfg.max_levels:
            raise MeshError("refinement beyond the finest level")
        for off in self.moore_offsets():
            q = self.shifted(level, coord, off)
            if q is None or self.exists((level, q)):
                continue
            if level == 0:
                raise MeshError("missing level-0 patch (violates R1)")
            r = self.covering(level, q)
            if not self.exists(r):
                raise MeshError(f"covering patch {r} of {q} missing")
            self.refine(r, created)
        for ck in self.child_keys(key):
            self._add(ck, key)
            self.children[key].append(ck)
            created.append(ck)

    # -- Algorithm 2: coarsening -------------------------------------------
    def coarsening_allowed(self, key: Key) -> bool:
        """IsCoarseningAllowed, text reading (Section 3.3): P must have children,
        all of them leaves, and no child may be a Moore neighbour of a
        same-level patch that itself has children (R2 would break).  Level-0
        patches may lose their children (R1 only protects the roots themselves).

        ``coarsen_rule == "literal"`` evaluates the printed conditions instead:
        refuse at level 0 and whenever any Moore neighbour of P has children.
        """
        if not self.exists(key) or self.is_leaf(key):
            return False
        kids = self.children[key]
        if any(not self.is_leaf(c) for c in kids):
            return False
        level, coord = key
        if self.coarsen_rule == "literal":
            if level == 0:
                return False
            for off in self.moore_offsets():
                q = self.shifted(level, coord, off)
                if q is not None and self.exists((level, q)) and not self.is_leaf((level, q)):
                    return False
            return True
        kidset = set(kids)
        for c in kids:
            for off in self.moore_offsets():
                q = self.shifted(level + 1, c[1], off)
                if q is None:
                    continue
                qk = (level + 1, q)
                if qk in kidset or not self.exists(qk):
                    continue
                if not self.is_leaf(qk):
                    return False
        return True

    def delete_children(self, key: Key, deleted: List[Key]):
        for c in self.children[key]:
            del self.parent[c]
            del self.children[c]
            deleted.append(c)
        self.children[key] = []

    # -- a regrid ----------------------------------------------------------
    def regrid(self, refine_keys, coarsen_keys):
        """Refinement pass over refine requests in (level, z, y, x) order, then
        a coarsening pass over coarsening requests in (level descending, z, y, x)
        order, each evaluated on the current mesh.  Returns (created, deleted)."""
        created: List[Key] = []
        deleted: List[Key] = []
        for key in sorted(refine_keys, key=order_key):
            if self.exists(key) and self.is_leaf(key):
                self.refine(key, created)
        newset = set(created)
        for key in sorted(coarsen_keys, key=lambda k: (-k[0], tuple(reversed(k[1])))):
            if not self.exists(key) or key in newset:
                continue
            if any(c in newset for c in self.children.get(key, [])):
                continue
            if self.coarsening_allowed(key):
                self.delete_children(key, deleted)
        return created, deleted

    # -- validity ----------------------------------------------------------
    def validate(self):
        """Raise MeshError unless R1, R2 and the tree links hold."""
        for coord in self._box(self.npd(0)):
            if not self.exists((0, coord)):
                raise MeshError(f"R1: root {coord} missing")
        for key, par in self.parent.items():
            level, coord = key
            if level == 0:
                if par is not None:
                    raise MeshError("root with a parent")
            else:
                if par != self.covering(level, coord) or not self.exists(par):
                    raise MeshError(f"bad parent link at {key}")
                if key not in self.children[par]:
                    raise MeshError(f"{key} not among its parent's children")
            kids = self.children[key]
            if kids:
                if sorted(kids, key=order_key) != sorted(self.child_keys(key), key=order_key):
                    raise MeshError(f"children of {key} do not tile it")
                for off in self.moore_offsets():
                    q = self.shifted(level, coord, off)
                    if q is not None and not self.exists((level, q)):
                        raise MeshError(f"R2: {key} has children but neighbour {q} is missing")

    def snapshot(self):
        """Canonical description: sorted (level, coord, parent, children) tuples."""
        out = []
        for k in self.keys():
            out.append((k[0], k[1], self.parent[k][1] if self.parent[k] else None,
                        tuple(sorted(c[1] for c in self.children[k]))))
        return out
