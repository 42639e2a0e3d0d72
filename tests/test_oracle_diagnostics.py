"""Pins of the velocity-gradient diagnostic's CPU reference (CPU only).

Second-order central differences are exact on quadratic fields, so a
quadratic velocity with distinct coefficients in every component and
direction, on a single-level mesh of several patches (same-level ghost
copies between them), gives the analytic gradient at every cell not next to
the transmissive boundary; a linear density gives the analytic density
gradient magnitude.  A transposed (i, j), a sign, a missing factor 2 or a
dropped direction in the magnitude fails."""
import numpy as np
import pytest

from oracle.diagnostics import velocity_gradient
from oracle.solver import OracleAMR
from paper_2508_05020_amd import workloads as W

# u_i = a_i + sum_j b_ij x_j + sum_{j<=k} c_ijk x_j x_k
RNG = np.random.default_rng(11)


def _fields(d):
    a = RNG.uniform(-0.3, 0.3, d)
    b = RNG.uniform(-1.0, 1.0, (d, d))
    c = RNG.uniform(-1.0, 1.0, (d, d, d))
    g = RNG.uniform(-0.4, 0.4, d)      # density slope

    def vel(pts):
        out = []
        for i in range(d):
            u = np.full_like(pts[0], a[i])
            for j in range(d):
                u = u + b[i, j] * pts[j]
                for k in range(j, d):
                    u = u + c[i, j, k] * pts[j] * pts[k]
            out.append(u)
        return out

    def dvel(pts):
        G = np.zeros((d, d) + pts[0].shape)
        for i in range(d):
            for j in range(d):
                g_ij = np.full_like(pts[0], b[i, j])
                for k in range(d):
                    lo, hi = min(j, k), max(j, k)
                    coef = c[i, lo, hi]
                    g_ij = g_ij + (2.0 * coef * pts[j] if k == j else coef * pts[k])
                G[i, j] = g_ij
        return G

    def gen(pts):
        rho = 2.0 + sum(g[j] * pts[j] for j in range(d))
        return rho, vel(pts), np.ones_like(pts[0])

    return gen, dvel, float(np.sqrt(np.sum(g * g)))


@pytest.mark.parametrize("d", [1, 2, 3])
def test_exact_on_quadratic_velocity_and_linear_density(d):
    base, n = {1: (64, 16), 2: (32, 8), 3: (16, 8)}[d]
    cfg = W.AMRConfig(name="q", dim=d, base_cells=base, patch_cells=[n],
                      periodic=[False] * d, max_patches=4096)
    o = OracleAMR(cfg)
    gen, dvel, grad_mag = _fields(d)
    for k in o.forest.keys():
        o.set_initial(k, gen)
    o.fill_ghosts(0, o.forest.leaves())
    out = velocity_gradient(o, 0)
    checked = 0
    for key, arr in out.items():
        assert arr.shape == (d * d + 1,) + (n,) * d
        pts = W.patch_points(cfg, key[0], key[1])
        G = dvel(pts)
        # cells whose stencil stays inside the domain
        ok = np.ones(pts[0].shape, bool)
        for j in range(d):
            gidx = key[1][j] * n + np.arange(n)
            inner = (gidx > 0) & (gidx < base - 1)
            shp = [1] * d
            shp[d - 1 - j] = n
            ok &= inner.reshape(shp)
        for i in range(d):
            for j in range(d):
                err = np.abs(arr[i * d + j] - G[i, j])[ok]
                assert np.max(err) <= 1e-11, (key, i, j, np.max(err))
        assert np.max(np.abs(arr[d * d] - grad_mag)[ok]) <= 1e-11
        checked += int(ok.sum())
    assert checked > 0


def test_boundary_cells_see_the_transmissive_copy():
    """At a transmissive boundary the ghost equals the boundary cell, so the
    x-derivative there is half the one-sided difference."""
    cfg = W.AMRConfig(name="q1", dim=1, base_cells=32, patch_cells=[16],
                      periodic=[False], max_patches=64)
    o = OracleAMR(cfg)

    def gen(pts):
        x = pts[0]
        return np.ones_like(x), [3.0 * x], np.ones_like(x)
    for k in o.forest.keys():
        o.set_initial(k, gen)
    o.fill_ghosts(0, o.forest.leaves())
    out = velocity_gradient(o, 0)
    first = out[(0, (0,))][0]
    h = cfg.h(0)
    assert first[0] == pytest.approx((3.0 * 1.5 * h - 3.0 * 0.5 * h) / (2 * h), rel=1e-12)
    assert first[5] == pytest.approx(3.0, rel=1e-12)
