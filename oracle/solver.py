"""Multi-level AMR Euler solver: the oracle for the whole hot path.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Readings of points on which the paper is silent (each is also listed in the
design notes):

* storage: cell-centred patches with ``ng = 4`` ghost layers; three state
  buffers U^n (0), A (1), B (2);
* time stepping: one global dt for every level (no subcycling); SSP-RK3 in
  increment form (Section 2.2 names SSP-RK3):
      stage 1: A   = U^n + dt L(U^n)
      stage 2: B   = U^n + 1/4 ((A + dt L(A)) - U^n)
      stage 3: U^n = U^n + 2/3 ((B + dt L(B)) - U^n);
  only leaf patches are advanced; every non-leaf patch is overwritten by
  restriction of its children after each stage;
* ghost fill: a ghost cell takes the value of the same-level cell at its
  (periodically wrapped or, for transmissive boundaries, clamped) position when
  an active same-level patch covers it; otherwise conservative MC-limited
  linear prolongation from the level below;
* prolongation: child = phi_C + sum_j (+-1/4) MC(phi_{C+e_j} - phi_C,
  phi_C - phi_{C-e_j}) on the conserved variables, terms added in the order
  x, y, z; the slopes of a coarse cell are dropped when any of its 2^d
  children would have rho <= 0 or p <= 0;
* restriction: pairwise sum of the 2^d children in x-fastest order, times 2^-d;
* refluxing: on a face between a leaf patch and a same-level patch that has
  children, the leaf's face flux is replaced by the mean of the 2^(d-1) fine
  face fluxes (pairwise, x-fastest over the tangential directions);
* time step: dt = CFL / max over leaf cells of sum_j (|u_j| + c) / h_l;
* tagging: a cell is tagged if for some direction j and phi in {rho, p}
  |phi_{+j} - phi_{-j}| > theta (|phi_{+j}| + |phi_{-j}|); a leaf patch has a
  tag if any cell within ``tag_buffer`` cells of its interior is tagged;
  refine requests go to tagged leaves below the finest level, coarsening
  requests to patches whose children are all untagged leaves.
"""
from __future__ import annotations

import itertools
import math
from typing import Dict, List

import numpy as np

from . import euler
from .geometry import Grid
from .mesh import Forest, MeshError, order_key


def _idx(canvas_arrays, g):
    """Index a level canvas [v, (z), (y), x] at global cell indices g = [gx, gy, gz]."""
    return canvas_arrays[(slice(None),) + tuple(reversed(g))]


class OracleAMR:
    def __init__(self, cfg, coarsen_rule: str = "text", scheme: str = "weno"):
        # ``cfg`` is the run description; the oracle copies its numbers into
        # its own Grid and computes every length and sample point from those
        self.cfg = cfg
        self.grid = Grid(cfg)
        self.d = self.grid.dim
        self.ng = self.grid.ghost
        self.nvar = self.grid.nvar
        self.scheme = scheme
        self.forest = Forest(self.grid, coarsen_rule)
        self.U: List[Dict] = [{}, {}, {}]
        for key in self.forest.keys():
            self._alloc(key)
        self.t = 0.0
        self.nsteps = 0

    # ------------------------------------------------------------------ data
    def _alloc(self, key):
        n = self.grid.patch_cells[key[0]]
        shape = (self.nvar,) + (n + 2 * self.ng,) * self.d
        for b in range(3):
            self.U[b][key] = np.zeros(shape)

    def interior(self, arr):
        n = arr.shape[1] - 2 * self.ng
        return arr[(slice(None),) + (slice(self.ng, self.ng + n),) * self.d]

    def set_initial(self, key, gen, buf: int = 0):
        level, coord = key
        pts = self.grid.points(level, coord)
        rho, u, p = gen(pts)
        self.interior(self.U[buf][key])[...] = euler.conserved_from_primitive(
            rho, u, p, self.grid.gamma)

    def canvas(self, buf: int, level: int):
        """Level-wide array holding the interiors of all active patches (NaN
        elsewhere) and the presence map of level patches."""
        N = self.grid.cells(level)
        n = self.grid.patch_cells[level]
        arr = np.full((self.nvar,) + (N,) * self.d, np.nan)
        present = np.zeros((self.forest.npd(level),) * self.d, dtype=bool)
        for key, a in self.U[buf].items():
            if key[0] != level:
                continue
            coord = key[1]
            present[tuple(reversed(coord))] = True
            sl = tuple(slice(coord[j] * n, coord[j] * n + n) for j in reversed(range(self.d)))
            arr[(slice(None),) + sl] = self.interior(a)
        return arr, present

    def bc_map(self, level: int, g):
        N = self.grid.cells(level)
        out = []
        for j in range(self.d):
            if self.grid.periodic[j]:
                out.append(np.mod(g[j], N))
            else:
                out.append(np.clip(g[j], 0, N - 1))
        return out

    def _present_at(self, level, present, g):
        n = self.grid.patch_cells[level]
        return present[tuple(reversed([gj // n for gj in g]))]

    # ---------------------------------------------------------- prolongation
    def prolong(self, level: int, g, coarse):
        """Values of level-``level`` cells at mapped global indices g from the
        canvas of level-1 (conservative MC-limited linear prolongation)."""
        carr, cpres = coarse
        d = self.d
        gc = [gj // 2 for gj in g]
        sig = [np.where(gj % 2 == 1, 1.0, -1.0) for gj in g]
        need = [gc]
        for j in range(d):
            for s in (1, -1):
                gg = [c.copy() for c in gc]
                gg[j] = gg[j] + s
                need.append(self.bc_map(level - 1, gg))
        for gg in need:
            if not np.all(self._present_at(level - 1, cpres, gg)):
                raise MeshError("prolongation stencil outside the coarse level")
        phi = _idx(carr, gc)
        slopes = []
        for j in range(d):
            up = _idx(carr, need[1 + 2 * j])
            dn = _idx(carr, need[2 + 2 * j])
            a = up - phi
            b = phi - dn
            same = ((a > 0.0) & (b > 0.0)) | ((a < 0.0) & (b < 0.0))
            mag = np.minimum(np.minimum(2.0 * np.abs(a), 2.0 * np.abs(b)), 0.5 * np.abs(a + b))
            slopes.append(np.where(same, np.sign(a) * mag, 0.0))
        bad = np.zeros(phi.shape[1:], dtype=bool)
        for signs in itertools.product((-1.0, 1.0), repeat=d):
            ch = phi
            for j in range(d):
                ch = ch + (signs[j] * 0.25) * slopes[j]
            rho, _, p, _ = euler.primitives(ch, d, self.grid.gamma)
            bad |= ~((rho > 0.0) & (p > 0.0))
        val = phi
        for j in range(d):
            val = val + (sig[j] * 0.25) * np.where(bad, 0.0, slopes[j])
        return val

    # ------------------------------------------------------------ ghost fill
    def _local_grid(self, n):
        m = n + 2 * self.ng
        axes = [np.arange(-self.ng, n + self.ng)] * self.d
        grids = np.meshgrid(*axes, indexing="ij")          # (z, y, x)
        return list(reversed(grids))                       # [x, y, z]

    def fill_ghosts(self, buf: int, keys=None):
        """Fill the ghost layers of the given patches (default: all active)."""
        keys = self.forest.keys() if keys is None else keys
        canv = {}

        def get(level):
            if level not in canv:
                canv[level] = self.canvas(buf, level)
            return canv[level]

        for key in keys:
            level, coord = key
            n = self.grid.patch_cells[level]
            loc = self._local_grid(n)
            ghost = np.zeros(loc[0].shape, dtype=bool)
            for j in range(self.d):
                ghost |= (loc[j] < 0) | (loc[j] >= n)
            g = [coord[j] * n + loc[j][ghost] for j in range(self.d)]
            gm = self.bc_map(level, g)
            arr, present = get(level)
            same = self._present_at(level, present, gm)
            vals = np.empty((self.nvar, gm[0].size))
            if np.any(same):
                vals[:, same] = _idx(arr, [c[same] for c in gm])
            if not np.all(same):
                if level == 0:
                    raise MeshError("level-0 ghost without a source")
                other = ~same
                vals[:, other] = self.prolong(level, [c[other] for c in gm], get(level - 1))
            a = self.U[buf][key]
            a[(slice(None),) + tuple(np.nonzero(ghost))] = vals

    # ------------------------------------------------------------- the RHS
    def face_fluxes(self, buf: int):
        """Face fluxes of every leaf, with coarse faces on coarse/fine
        interfaces replaced by the mean of the fine face fluxes."""
        cfg, d = self.grid, self.d
        leaves = self.forest.leaves()
        faces = {k: euler.patch_faces(self.U[buf][k], d, cfg.gamma, cfg.weno_eps,
                                      self.ng, self.scheme) for k in leaves}
        fine_canvas = {}

        def fine(level, j):
            if (level, j) not in fine_canvas:
                N = cfg.cells(level)
                n = cfg.patch_cells[level]
                shape = [N] * d
                shape[j] = N + 1
                arr = np.full((self.nvar,) + tuple(reversed(shape)), np.nan)
                for k in leaves:
                    if k[0] != level:
                        continue
                    c = k[1]
                    sl = []
                    for i in reversed(range(d)):
                        ext = n + 1 if i == j else n
                        sl.append(slice(c[i] * n, c[i] * n + ext))
                    arr[(slice(None),) + tuple(sl)] = faces[k][j]
                fine_canvas[(level, j)] = arr
            return fine_canvas[(level, j)]

        for key in leaves:
            level, coord = key
            n = cfg.patch_cells[level]
            for j in range(d):
                for side in (0, 1):
                    off = [0] * d
                    off[j] = 1 if side else -1
                    q = self.forest.shifted(level, coord, off)
                    if q is None or not self.forest.exists((level, q)):
                        continue
                    if self.forest.is_leaf((level, q)):
                        continue
                    farr = fine(level + 1, j)
                    # global index of this face on level + 1; on the low side
                    # the fine patch owns it as its high face (index N, not 0,
                    # across a periodic wrap)
                    Nf = cfg.cells(level + 1)
                    F = 2 * (coord[j] * n + (n if side else 0))
                    F = F % Nf if side else (F if F > 0 else Nf)
                    tang = [i for i in range(d) if i != j]
                    local = np.meshgrid(*[np.arange(n)] * (d - 1), indexing="ij")
                    local = list(reversed(local))          # tangential, lowest dim first
                    subs = []
                    for o in itertools.product((0, 1), repeat=d - 1):
                        o = tuple(reversed(o))             # lowest tangential fastest
                        gidx = [None] * d
                        gidx[j] = np.full(local[0].shape if d > 1 else (), F)
                        for t, i in enumerate(tang):
                            gidx[i] = 2 * (coord[i] * n + local[t]) + o[t]
                        subs.append(farr[(slice(None),) + tuple(reversed(gidx))])
                    if d == 1:
                        avg = subs[0]
                    elif d == 2:
                        avg = (subs[0] + subs[1]) * 0.5
                    else:
                        avg = ((subs[0] + subs[1]) + (subs[2] + subs[3])) * 0.25
                    if np.isnan(avg).any():
                        raise MeshError("fine face flux missing at a coarse/fine face")
                    G = faces[key][j]
                    sl = [slice(None)] * (d + 1)
                    sl[euler.axis_of(j, d)] = n if side else 0
                    G[tuple(sl)] = avg
        return faces

    def rhs(self, buf: int) -> Dict:
        """L(U) on every leaf (ghosts of ``buf`` must be filled)."""
        faces = self.face_fluxes(buf)
        return {k: euler.divergence(f, self.d, self.grid.h(k[0])) for k, f in faces.items()}

    # ---------------------------------------------------------- restriction
    def restrict(self, buf: int):
        d = self.d
        for level in range(self.forest.levels() - 2, -1, -1):
            for key in self.forest.keys():
                if key[0] != level or self.forest.is_leaf(key):
                    continue
                n = self.grid.patch_cells[level]
                pin = self.interior(self.U[buf][key])
                for ck in self.forest.children[key]:
                    nf = self.grid.patch_cells[level + 1]
                    c = self.interior(self.U[buf][ck])
                    h = nf // 2
                    o = [ck[1][j] * h - key[1][j] * n for j in range(d)]
                    if d == 1:
                        avg = (c[:, 0::2] + c[:, 1::2]) * 0.5
                    elif d == 2:
                        avg = ((c[:, 0::2, 0::2] + c[:, 0::2, 1::2])
                               + (c[:, 1::2, 0::2] + c[:, 1::2, 1::2])) * 0.25
                    else:
                        avg = (((c[:, 0::2, 0::2, 0::2] + c[:, 0::2, 0::2, 1::2])
                                + (c[:, 0::2, 1::2, 0::2] + c[:, 0::2, 1::2, 1::2]))
                               + ((c[:, 1::2, 0::2, 0::2] + c[:, 1::2, 0::2, 1::2])
                                  + (c[:, 1::2, 1::2, 0::2] + c[:, 1::2, 1::2, 1::2]))) * 0.125
                    sl = tuple(slice(o[j], o[j] + h) for j in reversed(range(d)))
                    pin[(slice(None),) + sl] = avg

    # ------------------------------------------------------------ time step
    def max_rate(self, buf: int = 0) -> float:
        lam = 0.0
        for k in self.forest.leaves():
            lam = max(lam, euler.max_wave_rate(self.interior(self.U[buf][k]), self.d,
                                               self.grid.h(k[0]), self.grid.gamma))
        return lam

    def compute_dt(self, buf: int = 0) -> float:
        return self.grid.cfl / self.max_rate(buf)

    def stage(self, k: int, dt: float):
        src = {1: 0, 2: 1, 3: 2}[k]
        dst = {1: 1, 2: 2, 3: 0}[k]
        leaves = self.forest.leaves()
        self.fill_ghosts(src, leaves)
        L = self.rhs(src)
        for key in leaves:
            un = self.interior(self.U[0][key])
            ui = self.interior(self.U[src][key])
            if k == 1:
                new = un + dt * L[key]
            elif k == 2:
                new = un + 0.25 * ((ui + dt * L[key]) - un)
            else:
                new = un + (2.0 / 3.0) * ((ui + dt * L[key]) - un)
            self.interior(self.U[dst][key])[...] = new
        self.restrict(dst)

    def step(self, dt: float = None) -> float:
        if dt is None:
            dt = self.compute_dt(0)
        for k in (1, 2, 3):
            self.stage(k, dt)
        self.t += dt
        self.nsteps += 1
        return dt

    # --------------------------------------------------------------- tagging
    def coarsening_candidates(self):
        """Patches whose children are all leaves (the only ones a coarsening
        request can name)."""
        f = self.forest
        return [k for k in f.keys()
                if f.children[k] and all(f.is_leaf(c) for c in f.children[k])]

    def tag_keys(self):
        """Patches the tagger evaluates: every leaf, and every coarsening
        candidate on its restricted data."""
        return list(self.forest.leaves()) + self.coarsening_candidates()

    def tag(self, buf: int = 0):
        """Tag flag of every patch of ``tag_keys()`` and per-cell dilated tags
        (ghosts of those patches filled)."""
        cfg, d, ng = self.grid, self.d, self.ng
        b = cfg.tag_buffer
        has, cells = {}, {}
        for key in self.tag_keys():
            a = self.U[buf][key]
            n = cfg.patch_cells[key[0]]
            rho, _, p, _ = euler.primitives(a, d, cfg.gamma)
            box = tuple(slice(ng - b, ng + n + b) for _ in range(d))
            raw = np.zeros((n + 2 * b,) * d, dtype=bool)
            for j in range(d):
                ax = d - 1 - j
                for phi in (rho, p):
                    plus = [slice(ng - b, ng + n + b)] * d
                    minus = [slice(ng - b, ng + n + b)] * d
                    plus[ax] = slice(ng - b + 1, ng + n + b + 1)
                    minus[ax] = slice(ng - b - 1, ng + n + b - 1)
                    fp = phi[tuple(plus)]
                    fm = phi[tuple(minus)]
                    raw |= np.abs(fp - fm) > cfg.tag_theta * (np.abs(fp) + np.abs(fm))
            has[key] = bool(raw.any())
            dil = np.zeros((n,) * d, dtype=bool)
            for off in itertools.product(range(2 * b + 1), repeat=d):
                dil |= raw[tuple(slice(o, o + n) for o in off)]
            cells[key] = dil
        return has, cells

    def requests(self, has):
        """Refinement requests on tagged leaves below the finest level;
        coarsening requests on candidates whose children are all untagged and
        whose own restricted data are untagged too (without the last
        condition a feature that the tagger sees on a coarse level but not
        on the finer one would be refined and coarsened in turn)."""
        L = self.grid.max_levels
        refine = [k for k in self.forest.leaves() if k[0] < L - 1 and has[k]]
        coarsen = [k for k in self.coarsening_candidates()
                   if not has[k] and not any(has[c] for c in self.forest.children[k])]
        return refine, coarsen

    def regrid(self, refine, coarsen, gen=None):
        """Apply the requests, then initialise new patches level by level
        (from ``gen`` when given, else by prolongation of U^n)."""
        created, deleted = self.forest.regrid(refine, coarsen)
        for k in deleted:
            for b in range(3):
                del self.U[b][k]
        for k in created:
            self._alloc(k)
        for level in sorted({k[0] for k in created}):
            new = [k for k in created if k[0] == level]
            if gen is not None:
                for k in new:
                    self.set_initial(k, gen)
                continue
            coarse = self.canvas(0, level - 1)
            n = self.grid.patch_cells[level]
            for k in new:
                loc = self._local_grid(n)
                inner = np.ones(loc[0].shape, dtype=bool)
                for j in range(self.d):
                    inner &= (loc[j] >= 0) & (loc[j] < n)
                g = [k[1][j] * n + loc[j][inner] for j in range(self.d)]
                vals = self.prolong(level, g, coarse)
                self.U[0][k][(slice(None),) + tuple(np.nonzero(inner))] = vals
        self.forest.validate()
        return created, deleted

    def adapt(self, flags=None):
        """Fill, tag, request and regrid; ``flags`` = (refine, coarsen) keys
        replaces this side's own requests (lockstep with another solver)."""
        self.fill_ghosts(0, self.tag_keys())
        has, _ = self.tag(0)
        refine, coarsen = self.requests(has) if flags is None else flags
        return self.regrid(refine, coarsen)

    def init_from_ic(self, gen):
        """Initial hierarchy: max_levels - 1 rounds of tag and refine, new
        patches sampled from the initial data."""
        for k in self.forest.keys():
            self.set_initial(k, gen)
        history = []
        for _ in range(self.grid.max_levels - 1):
            self.fill_ghosts(0, self.tag_keys())
            has, _ = self.tag(0)
            refine, _ = self.requests(has)
            if not refine:
                break
            self.regrid(refine, [], gen)
            history.append(refine)
        return history

    def advance(self, nsteps: int, regrid: bool = True):
        for _ in range(nsteps):
            self.step()
            if regrid and self.grid.regrid_interval > 0 \
                    and self.nsteps % self.grid.regrid_interval == 0:
                self.adapt()

    # ----------------------------------------------------------- diagnostics
    def totals(self, buf: int = 0):
        """Exactly rounded sums over leaf cells of U h^d, per variable."""
        out = []
        for v in range(self.nvar):
            vals = []
            for k in self.forest.leaves():
                hd = self.grid.h(k[0]) ** self.d
                vals.extend((self.interior(self.U[buf][k])[v] * hd).ravel().tolist())
            out.append(math.fsum(vals))
        return out

    def leaf_cells(self) -> int:
        return sum(self.grid.patch_cells[k[0]] ** self.d for k in self.forest.leaves())
