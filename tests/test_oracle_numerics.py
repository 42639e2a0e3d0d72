"""Pins of the oracle's per-patch numerics (CPU only).

Each test checks the oracle against something other than its own formula:
polynomial exactness of the interpolants, the smoothness indicators as exact
integrals, the physical Euler flux, Eq. (9) of the paper written in its own
(non-flux) form, dimensional reduction and symmetry.
"""
import numpy as np
import pytest
from numpy.polynomial import polynomial as P

from oracle import euler

RNG = np.random.default_rng(12345)


def _poly_nodes(coef):
    x = np.arange(-2, 3, dtype=float)
    return [P.polyval(xi, coef) for xi in x]


def test_candidates_exact_on_quadratics():
    for _ in range(50):
        coef = RNG.normal(size=3) * 10 ** RNG.uniform(-3, 3)
        a, b, c, d, e = _poly_nodes(coef)
        exact = P.polyval(0.5, coef)
        for q in euler.weno_candidates(a, b, c, d, e):
            assert abs(q - exact) <= 1e-13 * max(1.0, np.abs(coef).sum())


def test_weno_exact_on_quadratics_any_eps():
    for eps in (1e-6, 1.0, 1e100):
        for _ in range(20):
            coef = RNG.normal(size=3)
            a, b, c, d, e = _poly_nodes(coef)
            w = euler.weno5js(a, b, c, d, e, eps)
            assert abs(w - P.polyval(0.5, coef)) < 1e-13


def test_linear_weights_give_five_point_interpolant():
    # with eps -> infinity the nonlinear weights become the linear weights and
    # the scheme is the 5-point interpolant, exact on quartics
    for _ in range(30):
        coef = RNG.normal(size=5)
        a, b, c, d, e = _poly_nodes(coef)
        w = euler.weno5js(a, b, c, d, e, 1e100)
        assert abs(w - P.polyval(0.5, coef)) < 1e-12
    vals = RNG.normal(size=5)
    fit = P.polyfit(np.arange(-2, 3), vals, 4)
    assert abs(euler.weno5js(*vals, 1e100) - P.polyval(0.5, fit)) < 1e-12


def test_smoothness_indicators_are_integrals():
    # beta_k = int_{-1/2}^{1/2} (p_k')^2 + (p_k'')^2 dx for the quadratic p_k
    # through stencil k (unit spacing), the cell around the third node.
    for _ in range(20):
        vals = RNG.normal(size=5)
        betas = euler.smoothness_indicators(*vals)
        for k in range(3):
            xs = np.arange(-2 + k, 1 + k, dtype=float)
            coef = P.polyfit(xs, vals[k:k + 3], 2)
            total = 0.0
            for order in (1, 2):
                dc = P.polyder(coef, order)
                sq = P.polymul(dc, dc)
                integ = P.polyint(sq)
                total += P.polyval(0.5, integ) - P.polyval(-0.5, integ)
            assert abs(betas[k] - total) < 1e-11 * max(1.0, total)


def test_weno_ignores_stencils_across_a_jump():
    # left-biased value at an edge just left of a jump uses the smooth stencil
    assert abs(euler.weno5js(0.0, 0.0, 0.0, 1.0, 1.0, 1e-6)) < 1e-10
    assert abs(euler.weno5js(1.0, 1.0, 1.0, 1.0, 0.0, 1e-6) - 1.0) < 1e-10


def test_central_interpolant_exact_on_cubics():
    for _ in range(20):
        coef = RNG.normal(size=4)
        a, b, c, d, e = _poly_nodes(coef)
        assert abs(euler.central4_mid(b, c, d, e) - P.polyval(0.5, coef)) < 1e-13


def _random_state(shape, d):
    rho = RNG.uniform(0.3, 2.0, shape)
    u = [RNG.uniform(-1, 1, shape) for _ in range(d)]
    p = RNG.uniform(0.3, 2.0, shape)
    return rho, u, p


@pytest.mark.parametrize("d", [1, 2, 3])
def test_primitive_roundtrip(d):
    rho, u, p = _random_state((7,), d)
    U = euler.conserved_from_primitive(rho, u, p, 1.4)
    r2, u2, p2, T2 = euler.primitives(U, d, 1.4)
    assert np.allclose(r2, rho, rtol=1e-15, atol=0)
    assert np.allclose(p2, p, rtol=1e-13, atol=0)
    assert np.allclose(T2, p / rho, rtol=1e-13, atol=0)
    for j in range(d):
        assert np.allclose(u2[j], u[j], rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("d", [1, 2, 3])
def test_rusanov_consistent_with_physical_flux(d):
    # U^L = U^R: Eq. (11) must reduce to the Euler flux of Eq. (1)-(3),
    # here evaluated from the conserved variables directly
    rho, u, p = _random_state((11,), d)
    g = 1.4
    U = euler.conserved_from_primitive(rho, u, p, g)
    for j in range(d):
        F = euler.rusanov(p, p / rho, u, p, p / rho, u, j, g)
        m = U[1:1 + d]
        E = U[d + 1]
        uj = m[j] / U[0]
        ref = [m[j]] + [m[i] * m[j] / U[0] + (p if i == j else 0) for i in range(d)] \
            + [(E + p) * uj]
        for v in range(d + 2):
            assert np.allclose(F[v], ref[v], rtol=1e-13, atol=1e-14)


def test_rusanov_dissipation_sign():
    # a stationary contact (rho jumps, u = 0, p equal): the mass flux must
    # move mass from the dense side to the light side at speed S / 2
    g = 1.4
    pL = pR = np.array([1.0])
    rL, rR = np.array([2.0]), np.array([1.0])
    u0 = [np.array([0.0])]
    F = euler.rusanov(pL, pL / rL, u0, pR, pR / rR, u0, 0, g)
    S = max(np.sqrt(g * 1.0 / 1.0), np.sqrt(g * 1.0 / 2.0))
    assert F[0][0] == pytest.approx(0.5 * S * (2.0 - 1.0), rel=1e-14)


def test_face_form_equals_eq9():
    # (G_{i+1/2} - G_{i-1/2})/h equals Eq. (9) applied to the edge values
    F = [RNG.normal(size=20)]
    h = 0.37
    G = euler.face_fluxes(F, 1, 0)[0]
    div = (G[1:] - G[:-1]) / h
    f = F[0]
    # edges e_m = m - 2 + 1/2; node i = m - 1 for G faces; Eq. (9) at node i
    eq9 = np.array([9.0 / 8.0 * (f[i + 2] - f[i + 1]) / h
                    - 1.0 / 8.0 * (f[i + 3] - f[i]) / (3.0 * h) for i in range(len(f) - 3)])
    assert np.allclose(div, eq9, rtol=1e-12, atol=1e-12)


def _patch(d, n, ng=4):
    shape = (n + 2 * ng,) * d
    rho, u, p = _random_state(shape, d)
    return euler.conserved_from_primitive(rho, u, p, 1.4)


def test_2d_constant_in_y_reduces_to_1d():
    n, ng = 12, 4
    U1 = _patch(1, n)
    m = n + 2 * ng
    U2 = np.zeros((4, m, m))
    U2[0] = U1[0][None, :]
    U2[1] = U1[1][None, :]
    U2[2] = 0.0
    U2[3] = U1[2][None, :]
    L1 = euler.patch_rhs(U1, 1, 0.1, 1.4, 1e-6)
    L2 = euler.patch_rhs(U2, 2, 0.1, 1.4, 1e-6)
    for row in range(n):
        assert np.allclose(L2[0, row], L1[0], rtol=0, atol=1e-12)
        assert np.allclose(L2[1, row], L1[1], rtol=0, atol=1e-12)
        assert np.allclose(L2[2, row], 0.0, atol=1e-12)
        assert np.allclose(L2[3, row], L1[2], rtol=0, atol=1e-12)


@pytest.mark.parametrize("d", [2, 3])
def test_transpose_symmetry(d):
    U = _patch(d, 8)
    L = euler.patch_rhs(U, d, 0.05, 1.4, 1e-6)
    # swap x and y: array axes (-1, -2) and momentum components 1 <-> 2
    perm = list(range(d + 2))
    perm[1], perm[2] = 2, 1
    Ut = np.swapaxes(U[perm], -1, -2)
    Lt = euler.patch_rhs(Ut, d, 0.05, 1.4, 1e-6)
    assert np.allclose(np.swapaxes(Lt[perm], -1, -2), L, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("d", [1, 2, 3])
def test_uniform_patch_rhs_is_exactly_zero(d):
    shape = (6 + 8,) * d
    rho = np.full(shape, 0.7)
    u = [np.full(shape, 0.3 * (j + 1)) for j in range(d)]
    p = np.full(shape, 1.3)
    U = euler.conserved_from_primitive(rho, u, p, 1.4)
    L = euler.patch_rhs(U, d, 0.01, 1.4, 1e-6)
    assert np.all(L == 0.0)
