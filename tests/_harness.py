"""Shared helpers of the GPU parity tests: build matching oracle and library
hierarchies, move the oracle's state into the library, compare results.

Data flows one way: the oracle's mesh and state are inputs to the library;
nothing computed by the library is fed to the oracle except, in lockstep runs,
the regrid requests (reported and compared, see the lockstep test)."""
from __future__ import annotations

import copy
import functools

import numpy as np

from paper_2508_05020_amd import workloads as W
from oracle.solver import OracleAMR

# Parity bar: relative L-infinity per conserved variable, max over variables.
TOL = 1e-12

# oracle scheme name -> the library's amr_config.scheme value
SCHEMES = {"weno": 0, "central": 1, "char": 2}


def case_config(name: str):
    """Small configurations spanning several tiles per patch, ratio-2 and
    ratio-4 refinements, periodic and transmissive boundaries."""
    if name == "1d":
        return W.config("c1").replace(max_patches=256), W.shock_tube(1000), None
    if name == "2d":
        cfg = W.AMRConfig(name="p2", dim=2, base_cells=64, patch_cells=[32, 16, 16],
                          periodic=[True, True], ic="quadrants_blobs", max_patches=2048)
        return cfg, W.quadrants_blobs(2001), None
    if name == "2d-wall":
        cfg = W.AMRConfig(name="p2w", dim=2, base_cells=64, patch_cells=[16, 16, 16],
                          periodic=[False, True], ic="quadrants_blobs", max_patches=2048)
        return cfg, W.quadrants_blobs(2002), None
    if name == "2d-32":
        # refined levels of 32^2 patches (the wide coarse/fine fill), one
        # transmissive direction
        cfg = W.AMRConfig(name="p2l", dim=2, base_cells=64, patch_cells=[16, 32, 32],
                          periodic=[True, False], ic="quadrants_blobs", max_patches=1024)
        picks = [[(0, (1, 1))], [(1, (1, 1))]]
        return cfg, W.quadrants_blobs(2003), picks
    if name == "implosion":
        # the paper's implosion problem (Eq. (13)) on (-0.3, 0.3)^2
        cfg = W.AMRConfig(name="pimp", dim=2, base_cells=32, patch_cells=[16, 16, 16],
                          periodic=[True, True], lo=-0.3, hi=0.3, cfl=0.45, ic="implosion",
                          max_patches=2048)
        return cfg, W.implosion(), None
    if name == "3d":
        cfg = W.AMRConfig(name="p3", dim=3, base_cells=32, patch_cells=[8, 8, 8],
                          periodic=[True] * 3, ic="blasts", max_patches=4096)
        picks = [[(0, (1, 1, 1))], [(1, (3, 3, 3))]]
        return cfg, W.blasts(3001, 3), picks
    if name == "3d-c5":
        # the layout and generator of the 3D benchmark workload (patches
        # 32/16/16/8 on 4 levels, blast waves plus the k^-2 density field) on
        # a 64^3 base; one root refined around the first blast and one patch
        # per finer level, so that every level has coarse/fine faces
        cfg = W.c5_sample_config()
        return cfg, W.blasts_perturbed(5001, 3), W.blast_refinements(cfg, 5001)
    if name == "3d-uneven":
        cfg = W.AMRConfig(name="p3u", dim=3, base_cells=32, patch_cells=[16, 8],
                          periodic=[True, False, True], ic="blasts", max_patches=4096)
        picks = [[(0, (0, 1, 1))]]
        return cfg, W.blasts(3002, 3), picks
    raise KeyError(name)


def oracle_for(name: str):
    """A fresh copy of the named case's oracle hierarchy (built once)."""
    o, gen = _oracle_for(name)
    return copy.deepcopy(o), gen


@functools.lru_cache(maxsize=4)
def _oracle_for(name: str):
    cfg, gen, picks = case_config(name)
    o = OracleAMR(cfg)
    if picks is None:
        o.init_from_ic(gen)
    else:
        for k in o.forest.keys():
            o.set_initial(k, gen)
        for keys in picks:
            o.regrid(keys, [], gen)
    return o, gen


def mirror(o: OracleAMR, h, bufs=(0, 1, 2)):
    """Refine the library's base mesh into the oracle's mesh (one regrid per
    level) and upload the oracle's state buffers.  Returns pid <-> key maps."""
    cfg = o.cfg
    for level in range(cfg.max_levels - 1):
        want = [k for k in o.forest.keys() if k[0] == level and not o.forest.is_leaf(k)]
        if not want:
            continue
        pid = {(r["level"], r["coord"]): r["pid"] for r in h.patch_table()}
        refine = np.zeros(cfg.max_patches, np.uint8)
        for k in want:
            refine[pid[k]] = 1
        h.regrid(refine, np.zeros_like(refine))
    table = h.patch_table()
    pid_of = {(r["level"], r["coord"]): r["pid"] for r in table}
    assert set(pid_of) == set(o.forest.keys()), "library mesh differs from the oracle mesh"
    key_of = {v: k for k, v in pid_of.items()}
    for r in table:
        k = key_of[r["pid"]]
        par = o.forest.parent[k]
        assert (key_of.get(r["parent"]) if r["parent"] >= 0 else None) == par
        assert r["nchildren"] == len(o.forest.children[k])
    for b in bufs:
        h.set_state(b, {pid_of[k]: o.U[b][k] for k in o.forest.keys()})
    return pid_of, key_of


def download(h, buf, pid_of):
    levels = {p: k[0] for k, p in pid_of.items()}
    got = h.get_state(buf, list(levels), levels)
    return {k: got[p] for k, p in pid_of.items()}


def tensor_patches(h, flat, pid_of):
    """Split a state-layout device tensor into per-key numpy arrays."""
    host = flat.detach().cpu().numpy()
    out = {}
    for k, p in pid_of.items():
        n = h.cfg.patch_cells[k[0]] + 8
        size = h.nvar * n ** h.cfg.dim
        off = h.offset(p)
        out[k] = host[off:off + size].reshape((h.nvar,) + (n,) * h.cfg.dim)
    return out


def rhs_error(got: dict, ref: dict, U: dict, keys, d, dt: float):
    """Parity metric of L(U), per conserved variable v: max|L_gpu - L_ref|
    over the compared cells divided by the larger of max|L_ref,v| and
    max|U_v| / dt (dt the step's CFL time step), maximum over variables.
    The second scale is the state change a stage makes per unit L: where a
    variable's L is a small difference of large flux terms (the density of
    a gas at rest with uniform density, whose L comes only from
    interpolation differences), its rounding is bounded by the stage update
    it causes rather than by its own near-zero size."""
    nv = d + 2
    num = np.zeros(nv)
    den = np.zeros(nv)
    for k in keys:
        g, r, u = got[k], ref[k], interior(U[k], d)
        for v in range(nv):
            num[v] = max(num[v], float(np.max(np.abs(g[v] - r[v]))))
            den[v] = max(den[v], float(np.max(np.abs(r[v]))), float(np.max(np.abs(u[v]))) / dt)
    return float(np.max(num / np.where(den > 0, den, 1.0)))


def interior(a, d, ng=4):
    n = a.shape[1] - 2 * ng
    return a[(slice(None),) + (slice(ng, ng + n),) * d]


def rel_linf(got: dict, ref: dict, keys, d, region="interior"):
    """max over variables of max|got - ref| / max|ref| over the given patches."""
    nv = d + 2
    num = np.zeros(nv)
    den = np.zeros(nv)
    for k in keys:
        g, r = got[k], ref[k]
        if region == "interior":
            g, r = interior(g, d), interior(r, d)
        for v in range(nv):
            num[v] = max(num[v], float(np.max(np.abs(g[v] - r[v]))))
            den[v] = max(den[v], float(np.max(np.abs(r[v]))))
    return float(np.max(num / np.where(den > 0, den, 1.0)))


def mirror_case(name: str, amr):
    """Oracle hierarchy of a named case and its mirror in a new library hierarchy."""
    o, _ = oracle_for(name)
    h = amr.Hierarchy(o.cfg)
    pid_of, key_of = mirror(o, h)
    return o, h, pid_of, key_of
