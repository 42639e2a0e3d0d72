"""Full-size 3D checks (GPU): L(U), the Eq. (9) divergence of WENO5-JS +
Rusanov face fluxes (Section 2.2) with the coarse/fine flux substitution, on
the C3 hierarchy (3D blast waves, base 128^3, 4 levels, patches 32/16/16/8,
tens of millions of leaf cells) and on the C5 hierarchy (blast waves plus
the k^-2 density field, base 256^3, the same layout, about 145 M leaf
cells) in the benchmark's batched launch configuration (autotuned tile),
compared with the oracle at a seeded sample of leaf patches on every level,
half of them with coarse/fine faces.

The state is the initial data (every patch holds the generator's point
values on its own level), so the oracle builds everything it needs from the
generator: the sampled patch, its ghost layers by its own fill (same-level
copies, else its MC-limited prolongation from the coarser level), and on a
face whose same-level neighbour has children the fine face fluxes of those
children from their own ghost-filled arrays.  Only the mesh, i.e. which
patches exist, is read from the library.  1e-12 relative L-infinity per
variable over the sample."""
import itertools

import numpy as np
import pytest

from oracle import euler
from oracle.solver import OracleAMR
from paper_2508_05020_amd import workloads as W
from tests import _harness as H

pytestmark = pytest.mark.gpu

PER_LEVEL = 2   # leaves with coarse/fine faces and leaves without, per level


@pytest.fixture(scope="module")
def amr():
    import paper_2508_05020_amd.amr as A
    return A


class _LevelValues:
    """Conserved values of level-l cells at global indices, from the
    initial-data generator evaluated patch by patch on each patch's own grid
    of cell centres (the evaluation that filled the library's patches), so
    the oracle indexes the canvas its fill reads without materialising a
    level."""

    def __init__(self, grid, level, gen, cfg):
        self.grid, self.level, self.gen, self.cfg = grid, level, gen, cfg
        self.cache = {}

    def _patch(self, coord):
        if coord not in self.cache:
            rho, u, p = self.gen(W.patch_points(self.cfg, self.level, coord))
            self.cache[coord] = euler.conserved_from_primitive(rho, u, p, self.grid.gamma)
        return self.cache[coord]

    def __getitem__(self, idx):
        g = [np.asarray(a, np.int64) for a in reversed(idx[1:])]       # [gx, gy, gz]
        n = self.grid.patch_cells[self.level]
        d = len(g)
        shape = np.broadcast(*g).shape
        g = [np.broadcast_to(a, shape).ravel() for a in g]
        out = np.empty((d + 2, g[0].size))
        pc = np.stack([a // n for a in g], axis=1)
        for coord in {tuple(int(v) for v in row) for row in pc}:
            sel = np.all(pc == np.array(coord), axis=1)
            loc = [a[sel] - c * n for a, c in zip(g, coord)]
            out[:, sel] = self._patch(coord)[(slice(None),) + tuple(reversed(loc))]
        return out.reshape((d + 2,) + shape)


class _LevelPresence:
    """Which patch positions of a level hold an active patch (library mesh)."""

    def __init__(self, keys, level, npd):
        self.npd = npd
        self.codes = np.array(sorted(self._code(c) for (l, c) in keys if l == level), np.int64)

    def _code(self, c):
        return c[0] + self.npd * (c[1] + self.npd * c[2])

    def __getitem__(self, idx):
        p = [np.asarray(a, np.int64) for a in reversed(idx)]     # [px, py, pz]
        return np.isin(self._code(p), self.codes)


class _WindowOracle(OracleAMR):
    """The oracle's ghost fill and prolongation over level canvases that are
    evaluated on demand, for single patches of a large mesh."""

    def __init__(self, cfg, keys, gen):
        super().__init__(cfg.replace(base_cells=cfg.patch_cells[0]))
        self.grid = type(self.grid)(cfg)
        self.cfg = cfg
        self.keys, self.gen = set(keys), gen
        self.U = [{}, {}, {}]

    def canvas(self, buf, level):
        npd = self.grid.cells(level) // self.grid.patch_cells[level]
        return (_LevelValues(self.grid, level, self.gen, self.cfg),
                _LevelPresence(self.keys, level, npd))

    def filled(self, key):
        n = self.grid.patch_cells[key[0]]
        self.U[0][key] = np.zeros((self.nvar,) + (n + 8,) * self.d)
        self.set_initial(key, self.gen)
        self.fill_ghosts(0, [key])
        return self.U[0].pop(key)


def _reference_rhs(o, cfg, key, table_by_key, children_of):
    """L(U) of one leaf: its own face fluxes, with each face whose same-level
    neighbour has children replaced by the pairwise mean of the fine face
    fluxes (x-fastest over the tangential directions), then the divergence."""
    d = 3
    level, coord = key
    n = cfg.patch_cells[level]
    faces = euler.patch_faces(o.filled(key), d, cfg.gamma, cfg.weno_eps)
    npd = cfg.cells(level) // n
    for j in range(d):
        for side in (0, 1):
            q = list(coord)
            q[j] = (q[j] + (1 if side else -1)) % npd
            t = table_by_key.get((level, tuple(q)))
            if t is None or t["nchildren"] == 0:
                continue
            nf = cfg.patch_cells[level + 1]
            Nf = cfg.cells(level + 1)
            F = 2 * (coord[j] * n + (n if side else 0)) % Nf     # fine face index
            fine = {}                                            # tangential (a, b) -> G
            tang = [i for i in range(d) if i != j]
            for ck in children_of[t["pid"]]:
                c = ck[1]
                lo = c[j] * nf
                if side and lo != F:
                    continue
                if not side and (lo + nf) % Nf != F:
                    continue
                G = euler.patch_faces(o.filled(ck), d, cfg.gamma, cfg.weno_eps)[j]
                ax = euler.axis_of(j, d)
                G = np.take(G, 0 if side else nf, axis=ax)       # [v, (t_b), (t_a)]
                for ta, tb in itertools.product(range(nf), repeat=2):
                    fine[(c[tang[0]] * nf + ta, c[tang[1]] * nf + tb)] = G[:, tb, ta]
            Gc = faces[j]
            for ta, tb in itertools.product(range(n), repeat=2):
                ga = 2 * (coord[tang[0]] * n + ta)
                gb = 2 * (coord[tang[1]] * n + tb)
                s = [fine[(ga + oa, gb + ob)] for ob in (0, 1) for oa in (0, 1)]
                avg = ((s[0] + s[1]) + (s[2] + s[3])) * 0.25
                sl = [slice(None)] * (d + 1)
                sl[euler.axis_of(j, d)] = n if side else 0
                sl[euler.axis_of(tang[0], d)] = ta
                sl[euler.axis_of(tang[1], d)] = tb
                Gc[tuple(sl)] = avg
    return euler.divergence(faces, d, cfg.h(level))


def _has_cf_face(table_by_key, level, coord, npd):
    for j in range(len(coord)):
        for s in (-1, 1):
            q = list(coord)
            q[j] = (q[j] + s) % npd
            t = table_by_key.get((level, tuple(q)))
            if t is not None and t["nchildren"] > 0:
                return True
    return False


@pytest.mark.parametrize("name", ["c3", "c5"])
def test_full_size_rhs_sampled(name, amr):
    import gc
    import torch
    gc.collect()
    torch.cuda.empty_cache()
    cfg = W.config(name)
    gen = W.initial_data(cfg, W.seed_for(int(name[1:]), 1))
    h = amr.Hierarchy(cfg)
    amr.init_from_ic(h, gen)
    h.autotune(2)
    table = h.patch_table()
    by_key = {(t["level"], t["coord"]): t for t in table}
    key_of = {t["pid"]: (t["level"], t["coord"]) for t in table}
    children_of = {}
    for t in table:
        if t["parent"] >= 0:
            children_of.setdefault(t["parent"], []).append(key_of[t["pid"]])
    leaves = [t for t in table if t["nchildren"] == 0]
    assert sum(cfg.patch_cells[t["level"]] ** 3 for t in leaves) > 10_000_000
    rng = np.random.default_rng(3)
    sample = []
    for lev in range(cfg.max_levels):
        npd = cfg.cells(lev) // cfg.patch_cells[lev]
        for want in (True, False):
            cand = [t for t in leaves if t["level"] == lev
                    and _has_cf_face(by_key, lev, t["coord"], npd) == want]
            if cand:
                sample += [cand[i] for i in rng.choice(len(cand), min(PER_LEVEL, len(cand)),
                                                        replace=False)]
    with_cf = [t for t in sample if _has_cf_face(by_key, t["level"], t["coord"],
                                                 cfg.cells(t["level"]) // cfg.patch_cells[t["level"]])]
    assert cfg.max_levels - 1 in {t["level"] for t in sample}
    assert len({t["level"] for t in with_cf}) >= 2, "sample needs coarse/fine faces on 2 levels"
    out = h.rhs(0)
    o = _WindowOracle(cfg, by_key.keys(), gen)
    err = np.zeros(h.nvar)
    scale = np.zeros(h.nvar)
    umax = np.zeros(h.nvar)
    rate = 0.0
    for t in sample:
        lev, pid = t["level"], t["pid"]
        n = cfg.patch_cells[lev]
        key = (lev, t["coord"])
        ref = _reference_rhs(o, cfg, key, by_key, children_of)
        inner = o.filled(key)[:, 4:-4, 4:-4, 4:-4]
        rate = max(rate, euler.max_wave_rate(inner, 3, cfg.h(lev), cfg.gamma))
        off = h.offset(pid)
        full = n + 8
        got = out[off:off + h.nvar * full ** 3].cpu().numpy().reshape((h.nvar,) + (full,) * 3)
        got = got[:, 4:-4, 4:-4, 4:-4]
        for v in range(h.nvar):
            err[v] = max(err[v], np.max(np.abs(got[v] - ref[v])))
            scale[v] = max(scale[v], np.max(np.abs(ref[v])))
            umax[v] = max(umax[v], np.max(np.abs(inner[v])))
    h.close()
    del h, out
    torch.cuda.empty_cache()
    # the parity metric of L(U) (tests/_harness.rhs_error) with the sample's
    # own CFL time step
    dt = cfg.cfl / rate
    rel = err / np.maximum(np.maximum(scale, umax / dt), 1e-300)
    print(f"{name}: {len(sample)} leaves ({len(with_cf)} with coarse/fine faces): rel {rel}")
    assert np.all(rel <= H.TOL), rel
