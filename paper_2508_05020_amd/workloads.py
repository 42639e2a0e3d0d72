"""Workload descriptions and seeded synthetic initial data.

This module is shared by the HIP path's driver and by the CPU oracle.  It holds
only *input synthesis*: run configurations (mesh sizes, boundary kinds, gas and
scheme constants) and seeded generators that return primitive fields
(density, velocity, pressure) at given points.  It contains none of the
method's arithmetic: no equation of state, no conversion to conserved
variables, no fluxes.  Each consumer turns the primitive fields into its own
conserved state.

Geometry convention: the domain is the box [lo, hi) in every dimension; level
``l`` has ``base_cells * 2**l`` cells per dimension of width
``h_l = (hi - lo) / (base_cells * 2**l)``; cell ``g`` has its sample point at
``lo + (g + 1/2) h_l`` (cell-centred reading of the nodal mesh of Section 2.2).

The paper's demonstrations (Section 5) use R = 1 and gamma = 1.4; the
implosion problem is its Eq. (13).  The other generators are synthetic
stand-ins with the shapes and value ranges of the benchmark configurations:
shock tubes, four-state Riemann quadrants with density blobs, spherical blast
waves and a k^-2 density perturbation field.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Sequence

import numpy as np

# ---------------------------------------------------------------------------
# run configurations
# ---------------------------------------------------------------------------


@dataclasses.dataclass
class AMRConfig:
    name: str
    dim: int
    base_cells: int                 # level-0 cells per dimension
    patch_cells: List[int]          # patch edge (cells) per level
    periodic: List[bool]            # per dimension; False = transmissive
    lo: float = 0.0
    hi: float = 1.0
    gamma: float = 1.4
    cfl: float = 0.5
    weno_eps: float = 1e-6
    tag_theta: float = 0.02
    tag_buffer: int = 2
    regrid_interval: int = 4
    steps: int = 100
    max_patches: int = 4096
    ic: str = "uniform"
    ghost: int = 4
    # patch slots per level (0 = level 0 exact / the rest shared equally)
    level_capacity: tuple = ()

    @property
    def max_levels(self) -> int:
        return len(self.patch_cells)

    @property
    def nvar(self) -> int:
        return self.dim + 2

    def cells(self, level: int) -> int:
        return self.base_cells * (2 ** level)

    def h(self, level: int) -> float:
        return (self.hi - self.lo) / self.cells(level)

    def patches_per_dim(self, level: int) -> int:
        n = self.patch_cells[level]
        c = self.cells(level)
        if c % n:
            raise ValueError(f"level {level}: {c} cells not divisible by patch {n}")
        return c // n

    def validate(self) -> None:
        if self.dim not in (1, 2, 3):
            raise ValueError("dim must be 1, 2 or 3")
        if len(self.periodic) != self.dim:
            raise ValueError("periodic needs one entry per dimension")
        for l, n in enumerate(self.patch_cells):
            if n < 4 or n % 2:
                raise ValueError("patch edge must be even and >= 4")
            self.patches_per_dim(l)
            if l + 1 < self.max_levels:
                nf = self.patch_cells[l + 1]
                if (2 * n) % nf:
                    raise ValueError("fine patch edge must divide twice the coarse edge")

    def replace(self, **kw) -> "AMRConfig":
        return dataclasses.replace(self, **kw)


def _cfg(**kw) -> AMRConfig:
    c = AMRConfig(**kw)
    c.validate()
    return c


CONFIGS = {
    # 1D shock tube, 2 levels, 16-cell patches, transmissive, per-patch launches.
    "c1": _cfg(name="c1", dim=1, base_cells=256, patch_cells=[16, 16],
               periodic=[False], steps=200, regrid_interval=4, ic="shock_tube",
               max_patches=256),
    # 2D quadrants + blobs, 3 levels, 32/16/16 patches, periodic.
    "c2": _cfg(name="c2", dim=2, base_cells=256, patch_cells=[32, 16, 16],
               periodic=[True, True], steps=500, regrid_interval=4,
               ic="quadrants_blobs", max_patches=16384),
    # 3D blast waves, 4 levels, uneven 32/16/16/8 patches, periodic.
    "c3": _cfg(name="c3", dim=3, base_cells=128, patch_cells=[32, 16, 16, 8],
               periodic=[True] * 3, steps=50, regrid_interval=4, ic="blasts",
               max_patches=98304),
    # 2D quadrants + blobs on 512^2, 5 levels of 32^2 patches.
    "c4": _cfg(name="c4", dim=2, base_cells=512, patch_cells=[32] * 5,
               periodic=[True, True], steps=200, regrid_interval=8,
               tag_buffer=2, ic="quadrants_blobs", max_patches=65536),
    # 3D blast waves + k^-2 density perturbations, base 256^3; each refined
    # 16^3 level-2 patch has 64 children of 8^3, so level 3 holds most of the
    # 175k-250k patches of a run (150-200 M leaf cells; the pools take about
    # 200 GB).
    "c5": _cfg(name="c5", dim=3, base_cells=256, patch_cells=[32, 16, 16, 8],
               periodic=[True] * 3, steps=200, regrid_interval=8, tag_buffer=2,
               ic="blasts_perturbed", max_patches=512 + 8192 + 16384 + 327680,
               level_capacity=(512, 8192, 16384, 327680)),
    # The paper's implosion problem (Eq. (13)) on (-0.3, 0.3)^2.
    "implosion": _cfg(name="implosion", dim=2, base_cells=256,
                      patch_cells=[32, 16, 16], periodic=[True, True],
                      lo=-0.3, hi=0.3, cfl=0.45, steps=200, ic="implosion",
                      max_patches=16384),
}


def blast_refinements(cfg: AMRConfig, seed: int):
    """Refinements that build a mesh of every level of ``cfg`` around the
    first blast centre of ``seed`` (3D, at least 3 levels): the root
    holding the centre, then the level-1 patch of that root nearest the
    centre whose Moore neighbours lie in the same root (local index 1 .. m-2
    of m), then its child on the root's inner side, and so on, so that the
    neighbours the refinement rules add stay inside the root.  Returns one
    list of (level, coord) keys per refinement round."""
    c = _blast_sources(np.random.default_rng(seed), cfg.dim, cfg.lo, cfg.hi - cfg.lo)[0][0]
    span = cfg.hi - cfg.lo
    n = cfg.patch_cells
    root = tuple(int((c[j] - cfg.lo) / span * cfg.cells(0)) // n[0] for j in range(cfg.dim))
    per = 2 * n[0] // n[1]
    q = []
    for j in range(cfg.dim):
        g = int((c[j] - cfg.lo) / span * cfg.cells(1)) // n[1] - root[j] * per
        q.append(root[j] * per + min(max(g, 1), per - 2))
    rounds = [[(0, root)], [(1, tuple(q))]]
    inner = [q[j] - root[j] * per == 1 for j in range(cfg.dim)]
    for level in range(2, cfg.max_levels - 1):
        r = 2 * n[level - 1] // n[level]
        q = [r * q[j] + ((r - 1) if inner[j] else 0) for j in range(cfg.dim)]
        rounds.append([(level, tuple(q))])
    return rounds


def c5_sample_config() -> AMRConfig:
    """The 3D benchmark layout (patches 32/16/16/8 on 4 levels, blasts plus
    the k^-2 density field) on a 64^3 base; with ``blast_refinements`` it is
    a mesh of about 750 k leaf cells with coarse/fine faces on every level."""
    return AMRConfig(name="c5-sample", dim=3, base_cells=64, patch_cells=[32, 16, 16, 8],
                     periodic=[True] * 3, ic="blasts_perturbed", tag_buffer=2,
                     regrid_interval=8, max_patches=8 + 512 + 1024 + 8192,
                     level_capacity=(8, 512, 1024, 8192))


def config(name: str, **overrides) -> AMRConfig:
    c = CONFIGS[name].replace(**overrides) if overrides else CONFIGS[name]
    c.validate()
    return c


# ---------------------------------------------------------------------------
# geometry helpers (sample points only)
# ---------------------------------------------------------------------------


def patch_points(cfg: AMRConfig, level: int, coord: Sequence[int],
                 ghost: int = 0) -> List[np.ndarray]:
    """Sample points of a patch's cells, optionally including ``ghost`` layers.

    Returns ``[x, y, z][:dim]``, each of shape ``(m,)*dim`` in array axis order
    (z, y, x) with x varying along the last axis; ``m = n + 2*ghost``.
    Points of ghost cells beyond a periodic boundary are not wrapped.
    """
    n = cfg.patch_cells[level]
    h = cfg.h(level)
    d = cfg.dim
    axes = []
    for j in range(d):
        g = coord[j] * n + np.arange(-ghost, n + ghost)
        axes.append(cfg.lo + (g + 0.5) * h)
    # meshgrid in (z, y, x) order so that x is the last axis
    grids = np.meshgrid(*reversed(axes), indexing="ij")
    return list(reversed(grids))


def patch_points_batch(cfg: AMRConfig, level: int, coords) -> List[np.ndarray]:
    """Sample points of the interior cells of several patches of one level:
    ``[x, y, z][:dim]``, each of shape ``(P,) + (n,)*dim`` (patch first, then
    the array axis order of ``patch_points``)."""
    n = cfg.patch_cells[level]
    h = cfg.h(level)
    d = cfg.dim
    c = np.asarray(coords, dtype=np.int64).reshape(len(coords), d)
    out = []
    for j in range(d):
        g = c[:, j][:, None] * n + np.arange(n)[None, :]         # [P, n]
        v = cfg.lo + (g + 0.5) * h
        shp = [len(coords)] + [1] * d
        shp[d - j] = n
        out.append(np.broadcast_to(v.reshape(shp), (len(coords),) + (n,) * d))
    return out


def _min_image(dx: np.ndarray, length: float) -> np.ndarray:
    return dx - length * np.round(dx / length)


# ---------------------------------------------------------------------------
# seeded initial-data generators: each returns f(points) -> (rho, [u_j], p)
# ---------------------------------------------------------------------------

Prim = Callable[[List[np.ndarray]], tuple]


def uniform_state(dim: int, seed: int) -> Prim:
    """A constant random state: rho, p ~ U[0.2, 2], u_j ~ U[-1, 1]."""
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.2, 2.0)
    p = rng.uniform(0.2, 2.0)
    u = [rng.uniform(-1.0, 1.0) for _ in range(dim)]

    def f(pts):
        shape = pts[0].shape
        return (np.full(shape, rho), [np.full(shape, uj) for uj in u],
                np.full(shape, p))
    return f


def density_wave(dim: int, k: Sequence[int], velocity: Sequence[float],
                 amp: float = 0.2, length: float = 1.0, t: float = 0.0) -> Prim:
    """rho = 1 + amp sin(2 pi k.(x - u t)/L), u constant, p = 1 (smooth)."""

    def f(pts):
        phase = np.zeros_like(pts[0])
        for j in range(dim):
            phase = phase + k[j] * (pts[j] - velocity[j] * t)
        rho = 1.0 + amp * np.sin(2.0 * np.pi * phase / length)
        return (rho, [np.full_like(rho, velocity[j]) for j in range(dim)],
                np.ones_like(rho))
    return f


def shock_tube(seed: int) -> Prim:
    """1D Riemann problem: rho_L, p_L, rho_R, p_R ~ U[0.1, 1], x0 ~ U[0.3, 0.7], u = 0."""
    rng = np.random.default_rng(seed)
    rl, pl, rr, pr = (rng.uniform(0.1, 1.0) for _ in range(4))
    x0 = rng.uniform(0.3, 0.7)

    def f(pts):
        x = pts[0]
        left = x < x0
        return (np.where(left, rl, rr), [np.zeros_like(x)], np.where(left, pl, pr))
    f.params = dict(rho_l=rl, p_l=pl, rho_r=rr, p_r=pr, x0=x0)
    return f


def quadrants_blobs(seed: int, lo: float = 0.0, hi: float = 1.0) -> Prim:
    """Four constant Riemann states plus 8 Gaussian density blobs (periodic)."""
    rng = np.random.default_rng(seed)
    quads = []
    for _ in range(4):  # (x<1/2,y<1/2), (>=,<), (<,>=), (>=,>=)
        rho = rng.uniform(0.2, 1.5)
        p = rng.uniform(0.2, 1.5)
        u = rng.uniform(-0.5, 0.5)
        v = rng.uniform(-0.5, 0.5)
        quads.append((rho, u, v, p))
    blobs = []
    L = hi - lo
    for _ in range(8):
        cx = lo + L * rng.uniform(0.0, 1.0)
        cy = lo + L * rng.uniform(0.0, 1.0)
        amp = rng.uniform(0.1, 0.5)
        w = L * rng.uniform(0.02, 0.05)
        blobs.append((cx, cy, amp, w))
    mid = lo + 0.5 * L

    def f(pts):
        x, y = pts[0], pts[1]
        q = (x >= mid).astype(int) + 2 * (y >= mid).astype(int)
        tab = np.array(quads)
        rho = tab[q, 0].copy()
        u = tab[q, 1]
        v = tab[q, 2]
        p = tab[q, 3]
        for cx, cy, amp, w in blobs:
            dx = _min_image(x - cx, L)
            dy = _min_image(y - cy, L)
            rho = rho + amp * np.exp(-(dx * dx + dy * dy) / (w * w))
        return rho, [u, v], p
    return f


def _blast_sources(rng, dim: int, lo: float, L: float):
    src = []
    for _ in range(6):
        c = [lo + L * rng.uniform(0.0, 1.0) for _ in range(dim)]
        pj = rng.uniform(5.0, 50.0)
        rad = L * rng.uniform(0.03, 0.08)
        src.append((c, pj, rad))
    return src


def _blast_pressure(src, pts, dim: int, L: float) -> np.ndarray:
    p = np.ones_like(pts[0])
    for c, pj, rad in src:
        r2 = np.zeros_like(pts[0])
        for j in range(dim):
            dj = _min_image(pts[j] - c[j], L)
            r2 = r2 + dj * dj
        p = np.where(r2 < rad * rad, np.maximum(p, pj), p)
    return p


def _grid_axes(pts, dim: int):
    """Per-patch axis coordinates [P, m] when pts are P tensor grids stacked
    along a leading axis (as patch_points_batch makes them), else None."""
    if pts[0].ndim != dim + 1:
        return None
    vals = []
    for j in range(dim):
        ax = dim - j                      # array axis of x_j after the patch axis
        idx = [slice(None)] + [0] * dim
        idx[ax] = slice(None)
        v = pts[j][tuple(idx)]            # [P, m]
        shp = [v.shape[0]] + [1] * dim
        shp[ax] = v.shape[1]
        if not np.array_equal(np.broadcast_to(v.reshape(shp), pts[j].shape), pts[j]):
            return None
        vals.append(v)
    return vals


def _blast_pressure_grids(src, axes, dim: int, L: float) -> np.ndarray:
    """_blast_pressure on stacked tensor grids: the per-axis squared
    distances are formed once per axis and broadcast, summed in the same
    order (x, then y, then z), so every point gets the same value."""
    P, m = axes[0].shape
    full = (P,) + (m,) * dim
    p = np.ones(full)
    for c, pj, rad in src:
        r2 = np.zeros(full)
        for j in range(dim):
            dj = _min_image(axes[j] - c[j], L)
            shp = [P] + [1] * dim
            shp[dim - j] = m
            r2 = r2 + (dj * dj).reshape(shp)
        p = np.where(r2 < rad * rad, np.maximum(p, pj), p)
    return p


def blasts(seed: int, dim: int = 3, lo: float = 0.0, hi: float = 1.0) -> Prim:
    """rho = 1, u = 0, p = 1 except inside 6 spheres where p = p_jump (ratio reading)."""
    rng = np.random.default_rng(seed)
    L = hi - lo
    src = _blast_sources(rng, dim, lo, L)

    def f(pts):
        axes = _grid_axes(pts, dim)
        p = (_blast_pressure_grids(src, axes, dim, L) if axes is not None
             else _blast_pressure(src, pts, dim, L))
        return (np.ones_like(p), [np.zeros_like(p) for _ in range(dim)], p)
    return f


def blasts_perturbed(seed: int, dim: int = 3, lo: float = 0.0, hi: float = 1.0,
                     amp: float = 0.05, kmax: int = 8) -> Prim:
    """Blast waves plus a random-phase density field with shell power ~ k^-2.

    delta_rho = sum_k A_k cos(2 pi k.x / L + phi_k) over integer wave vectors
    with 1 <= |k| <= kmax in a half space, A_k ~ |k|^-2, phases ~ U[0, 2 pi);
    the amplitudes are scaled so that sum_k A_k = amp, which bounds
    max |delta_rho| by amp.
    """
    rng = np.random.default_rng(seed)
    L = hi - lo
    src = _blast_sources(rng, dim, lo, L)
    modes = []
    rngk = range(-kmax, kmax + 1)
    for kz in (rngk if dim == 3 else [0]):
        for ky in (rngk if dim >= 2 else [0]):
            for kx in rngk:
                k = (kx, ky, kz)[:dim]
                kk = sum(c * c for c in k)
                if kk == 0 or kk > kmax * kmax:
                    continue
                # half space: first nonzero component (z, y, x order) positive
                first = next(c for c in reversed(k) if c != 0)
                if first < 0:
                    continue
                modes.append((k, kk ** -1.0))
    phases = rng.uniform(0.0, 2.0 * np.pi, len(modes))
    total = sum(a for _, a in modes)
    # complex coefficients on the dense (k_z, k_y, k_x) grid; zero off the modes
    K = 2 * kmax + 1
    coef = np.zeros((K,) * dim, np.complex128)
    for (k, a), ph in zip(modes, phases):
        coef[tuple(c + kmax for c in reversed(k))] = (amp * a / total) * np.exp(1j * ph)
    ks = np.arange(-kmax, kmax + 1)

    def axis_values(pts):
        """Per-axis coordinates if pts is a tensor grid in (z, y, x) array
        order (as patch_points makes them), else None."""
        if pts[0].ndim != dim:
            return None
        vals = []
        for j in range(dim):
            ax = dim - 1 - j
            idx = [0] * dim
            idx[ax] = slice(None)
            v = pts[j][tuple(idx)]
            shp = [1] * dim
            shp[ax] = v.size
            if not np.array_equal(np.broadcast_to(v.reshape(shp), pts[j].shape), pts[j]):
                return None
            vals.append(v)
        return vals

    def perturbation(pts):
        # sum_k c_k prod_j exp(i 2 pi k_j (x_j - lo) / L), contracted one axis
        # at a time (x, then y, then z); the real part is the cosine sum
        gb = _grid_axes(pts, dim)
        if gb is not None:
            P, m = gb[0].shape
            e = [np.exp((2j * np.pi / L) * (ks[None, :, None] * (gb[j][:, None, :] - lo)))
                 for j in range(dim)]                                    # [P, k_j, m]
            # contract k_x, then k_y, then k_z, as on a single patch
            t = np.matmul(coef.reshape(-1, K)[None], e[0])              # [P, (k_z, k_y), x]
            if dim == 1:
                return t.reshape(P, m).real
            t = t.reshape((P,) + (K,) * (dim - 1) + (m,))
            t = np.matmul(np.swapaxes(t, -1, -2), e[1][:, None] if dim == 3 else e[1])
            if dim == 2:                                                 # [P, x, y]
                return np.swapaxes(t, 1, 2).real
            # t: [P, k_z, x, y] -> [P, x, y, k_z] @ [P, k_z, z] -> [P, x, y, z]
            t = np.matmul(t.transpose(0, 2, 3, 1).reshape(P, m * m, K), e[2])
            return t.reshape(P, m, m, m).transpose(0, 3, 2, 1).real
        g = axis_values(pts)
        if g is not None:
            e = [np.exp((2j * np.pi / L) * np.outer(ks, g[j] - lo)) for j in range(dim)]
            t = np.tensordot(coef, e[0], axes=([dim - 1], [0]))      # [..., k_y, x]
            for j in range(1, dim):
                # contract the last remaining wave-number axis (k_y, then k_z)
                t = np.tensordot(t, e[j], axes=([dim - 1 - j], [0]))  # new axis last
            # axes are now (x, y, z): back to (z, y, x)
            return np.transpose(t.real, tuple(range(dim - 1, -1, -1)))
        shape = pts[0].shape
        flat = [np.ravel(q) for q in pts]
        out = np.empty(flat[0].size)
        for q0 in range(0, out.size, 8192):
            sl = slice(q0, min(out.size, q0 + 8192))
            e = [np.exp((2j * np.pi / L) * np.outer(ks, flat[j][sl] - lo)) for j in range(dim)]
            t = coef.reshape(-1, K) @ e[0]
            for j in range(1, dim):
                t = (t.reshape(-1, K, e[j].shape[1]) * e[j][None]).sum(axis=1)
            out[sl] = t.reshape(-1).real
        return out.reshape(shape)

    def f(pts):
        axes = _grid_axes(pts, dim)
        p = (_blast_pressure_grids(src, axes, dim, L) if axes is not None
             else _blast_pressure(src, pts, dim, L))
        return (1.0 + perturbation(pts), [np.zeros_like(p) for _ in range(dim)], p)
    return f


def implosion(lo: float = -0.3, hi: float = 0.3) -> Prim:
    """Eq. (13): (rho, p) = (0.125, 0.14) inside |x| + |y| < 0.15, else (1, 1); at rest."""

    def f(pts):
        x, y = pts[0], pts[1]
        inside = np.abs(x) + np.abs(y) < 0.15
        rho = np.where(inside, 0.125, 1.0)
        p = np.where(inside, 0.140, 1.0)
        return rho, [np.zeros_like(x), np.zeros_like(x)], p
    return f


def initial_data(cfg: AMRConfig, seed: int) -> Prim:
    """The seeded generator named by ``cfg.ic``."""
    if cfg.ic == "shock_tube":
        return shock_tube(seed)
    if cfg.ic == "quadrants_blobs":
        return quadrants_blobs(seed, cfg.lo, cfg.hi)
    if cfg.ic == "blasts":
        return blasts(seed, cfg.dim, cfg.lo, cfg.hi)
    if cfg.ic == "blasts_perturbed":
        return blasts_perturbed(seed, cfg.dim, cfg.lo, cfg.hi)
    if cfg.ic == "implosion":
        return implosion(cfg.lo, cfg.hi)
    if cfg.ic == "uniform":
        return uniform_state(cfg.dim, seed)
    raise KeyError(cfg.ic)


def seed_for(config_index: int, run: int) -> int:
    """Seed of run ``run`` of configuration ``config_index`` (1-based)."""
    return 1000 * config_index + run
