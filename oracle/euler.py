"""Per-patch Euler right-hand side, written from Section 2 of the paper.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Plain numpy FP64; arrays are ``U[v, (z), (y), x]`` with the conserved
variables in the order (rho, rho u_x[, rho u_y[, rho u_z]], rho e) and the x
index varying fastest.  A patch array carries ``ng`` ghost layers on every
side.  No blocking, fusion or reordering: each function evaluates its
definition directly, elementwise over whole arrays.
"""
from __future__ import annotations

import numpy as np

NG = 4  # ghost layers needed by the flux-form divergence (see patch_faces)


def axis_of(j: int, d: int) -> int:
    """Array axis of spatial direction j (0 = x) in ``U[v, (z), (y), x]``."""
    return d - j


# ---------------------------------------------------------------------------
# Equation of state and primitives (Section 2.1, Eq. (4)-(7); R = 1 per Section 5)
# ---------------------------------------------------------------------------


def primitives(U: np.ndarray, d: int, gamma: float):
    """Conserved -> (rho, [u_j], p, T).

    e = e_th + u.u/2 (Eq. 4) and p = rho e_th (gamma - 1) (Eq. 6) give
    p = (gamma - 1) (E - rho u.u/2) with E = rho e.  The kinetic term is
    evaluated as 0.5 * (m_x u_x + m_y u_y + m_z u_z) with u_j = m_j / rho.
    The calorically perfect gas with R = 1 has T = p / rho.
    """
    rho = U[0]
    u = [U[1 + j] / rho for j in range(d)]
    ke = U[1] * u[0]
    for j in range(1, d):
        ke = ke + U[1 + j] * u[j]
    ke = 0.5 * ke
    p = (gamma - 1.0) * (U[d + 1] - ke)
    T = p / rho
    return rho, u, p, T


def conserved_from_primitive(rho, u, p, gamma: float) -> np.ndarray:
    """(rho, [u_j], p) -> U using E = p / (gamma - 1) + rho u.u / 2 (Eq. 4, 6)."""
    d = len(u)
    uu = u[0] * u[0]
    for j in range(1, d):
        uu = uu + u[j] * u[j]
    E = p / (gamma - 1.0) + 0.5 * rho * uu
    return np.stack([rho] + [rho * uj for uj in u] + [E])


def sound_speed(rho, p, gamma: float):
    """Eq. (7): c = sqrt(gamma p / rho)."""
    return np.sqrt(gamma * p / rho)


# ---------------------------------------------------------------------------
# WENO5-JS point interpolation at an edge (Section 2.2)
# ---------------------------------------------------------------------------

# Linear weights that combine the three 3-point candidates into the 5-point
# interpolant at the mid-point between the 3rd and 4th nodes.
WENO_D = (1.0 / 16.0, 10.0 / 16.0, 5.0 / 16.0)


def weno_candidates(a, b, c, d, e):
    """Quadratic Lagrange interpolants at x = 1/2 of the stencils
    {-2,-1,0}, {-1,0,1}, {0,1,2} (nodes a..e sit at x = -2..2)."""
    q0 = (3.0 * a - 10.0 * b + 15.0 * c) / 8.0
    q1 = (-b + 6.0 * c + 3.0 * d) / 8.0
    q2 = (3.0 * c + 6.0 * d - e) / 8.0
    return q0, q1, q2


def smoothness_indicators(a, b, c, d, e):
    """Jiang-Shu smoothness indicators of the three candidate stencils.

    beta_k = integral over the cell around node c of (p_k')^2 + (p_k'')^2
    (unit spacing), p_k the quadratic through stencil k.
    """
    b0 = 13.0 / 12.0 * (a - 2.0 * b + c) ** 2 + 0.25 * (a - 4.0 * b + 3.0 * c) ** 2
    b1 = 13.0 / 12.0 * (b - 2.0 * c + d) ** 2 + 0.25 * (b - d) ** 2
    b2 = 13.0 / 12.0 * (c - 2.0 * d + e) ** 2 + 0.25 * (3.0 * c - 4.0 * d + e) ** 2
    return b0, b1, b2


def weno5js(a, b, c, d, e, eps: float):
    """WENO5-JS value at the edge between c and d from the five nodes a..e.

    A convex combination of the candidates with weights alpha_k / sum(alpha)
    where alpha_k = d_k / (eps + beta_k)^2; on smooth data it tends to the
    5-point linear interpolant (Section 2.2).
    """
    q = weno_candidates(a, b, c, d, e)
    beta = smoothness_indicators(a, b, c, d, e)
    alpha = [WENO_D[k] / (eps + beta[k]) ** 2 for k in range(3)]
    s = alpha[0] + alpha[1] + alpha[2]
    return (alpha[0] * q[0] + alpha[1] * q[1] + alpha[2] * q[2]) / s


def central4_mid(b, c, d, e):
    """Eq. (8) solved for the mid-point: 4th-order central interpolation at the
    edge between c and d, (9 (c + d) - (b + e)) / 16 (shock-free variant)."""
    return (9.0 * (c + d) - (b + e)) / 16.0


# ---------------------------------------------------------------------------
# Rusanov edge flux (Eq. (10)-(12))
# ---------------------------------------------------------------------------


def flux_from_primitive(p, T, u, j: int, gamma: float):
    """Edge state from interpolated (p, T, u): returns (U^X list, F_j^X list, c^X).

    rho = p / T (R = 1); E = p / (gamma - 1) + rho u.u / 2;
    F_j = (rho u_j, rho u_i u_j + p delta_ij, (E + p) u_j) from Eq. (1)-(3)
    with rho h = E + p (Eq. 5).
    """
    d = len(u)
    rho = p / T
    m = [rho * ui for ui in u]
    uu = u[0] * u[0]
    for i in range(1, d):
        uu = uu + u[i] * u[i]
    E = p / (gamma - 1.0) + 0.5 * rho * uu
    Uv = [rho] + m + [E]
    F = [m[j]] + [m[i] * u[j] + (p if i == j else 0.0) for i in range(d)] + [(E + p) * u[j]]
    c = np.sqrt(gamma * T)   # Eq. (7) with p / rho = T
    return Uv, F, c


def rusanov(pL, TL, uL, pR, TR, uR, j: int, gamma: float):
    """Eq. (11) with the wave speed of Eq. (12)."""
    UL, FL, cL = flux_from_primitive(pL, TL, uL, j, gamma)
    UR, FR, cR = flux_from_primitive(pR, TR, uR, j, gamma)
    S = np.maximum(cR + np.abs(uR[j]), cL + np.abs(uL[j]))
    return [0.5 * (FR[v] + FL[v]) - 0.5 * S * (UR[v] - UL[v]) for v in range(len(FL))]


# ---------------------------------------------------------------------------
# Edge fluxes and divergence along one direction of a patch
# ---------------------------------------------------------------------------


def _shift(arr, ax: int, start: int, count: int):
    sl = [slice(None)] * arr.ndim
    sl[ax] = slice(start, start + count)
    return arr[tuple(sl)]


def _interior_cross(arr, d: int, j: int, n: int, ng: int):
    """Restrict all axes except direction j to the interior range."""
    sl = [slice(None)] * arr.ndim
    for k in range(d):
        if k != j:
            sl[arr.ndim - d + (d - 1 - k)] = slice(ng, ng + n)
    return arr[tuple(sl)]


def edge_fluxes(U: np.ndarray, d: int, j: int, gamma: float, eps: float,
                ng: int = NG, scheme: str = "weno"):
    """Riemann fluxes at the edges i+1/2, i = -2 .. n, along direction j for
    every interior line of the patch.

    The primitives p, T, u_j (the interpolated set of Section 2.2) are
    interpolated to each edge from the left-biased nodes i-2..i+2 (value L) and
    from the right-biased nodes i+3..i-1 (value R, mirrored stencil).  Where
    an interpolated p or T is not positive the edge falls back to first order
    (L from node i, R from node i+1).  Returns a list over conserved variables
    of arrays with n+3 entries along direction j.
    """
    n = U.shape[1] - 2 * ng
    rho, u, p, T = primitives(U, d, gamma)
    prims = [p, T] + u
    prims = [_interior_cross(q, d, j, n, ng) for q in prims]
    ax = axis_of(j, d) - 1          # primitives have no variable axis
    ne = n + 3
    left, right, lo1, hi1 = [], [], [], []
    for q in prims:
        s = [_shift(q, ax, ng - 4 + k, ne) for k in range(6)]  # nodes i-2 .. i+3
        if scheme == "weno":
            left.append(weno5js(s[0], s[1], s[2], s[3], s[4], eps))
            right.append(weno5js(s[5], s[4], s[3], s[2], s[1], eps))
        elif scheme == "central":
            left.append(central4_mid(s[1], s[2], s[3], s[4]))
            right.append(central4_mid(s[1], s[2], s[3], s[4]))
        else:
            raise ValueError(scheme)
        lo1.append(s[2])
        hi1.append(s[3])
    ok = (left[0] > 0.0) & (left[1] > 0.0) & (right[0] > 0.0) & (right[1] > 0.0)
    left = [np.where(ok, a, b) for a, b in zip(left, lo1)]
    right = [np.where(ok, a, b) for a, b in zip(right, hi1)]
    return rusanov(left[0], left[1], left[2:], right[0], right[1], right[2:], j, gamma)


# ---------------------------------------------------------------------------
# Characteristic-variable interpolation (shock-capturing variant, Section 2.2)
# ---------------------------------------------------------------------------


def mean_state(Ua, Ub):
    """Arithmetic mean of two conserved states: the state at which the flux
    Jacobian is decomposed for the edge between them."""
    return [0.5 * (a + b) for a, b in zip(Ua, Ub)]


def flux_eigenvectors(Ubar, d: int, j: int, gamma: float):
    """Right eigenvectors (R[v][k]: component v of vector k) and left
    eigenvectors (L[k][v], the rows of R^-1) of A_j = dF_j/dU, the Jacobian
    of the direction-j flux of Eq. (1)-(3), at the conserved state Ubar.

    Waves k in the order u_j - c, u_j (entropy), u_j (one shear wave per
    tangential direction, ascending), u_j + c.  With u = m / rho,
    q2 = u.u, p = (gamma - 1)(E - rho q2 / 2), c^2 = gamma p / rho,
    H = (E + p) / rho, b1 = (gamma - 1) / c^2 and b2 = b1 q2 / 2:
      r_- = (1, u - c e_j, H - u_j c),   r_e = (1, u, q2 / 2),
      r_t = (0, e_t, u_t),               r_+ = (1, u + c e_j, H + u_j c);
      l_- = ((b2 + u_j / c) / 2, -(b1 u + e_j / c) / 2, b1 / 2),
      l_e = (1 - b2, b1 u, -b1),          l_t = (-u_t, e_t, 0),
      l_+ = ((b2 - u_j / c) / 2, -(b1 u - e_j / c) / 2, b1 / 2).
    """
    nv = d + 2
    rho = Ubar[0]
    u = [Ubar[1 + i] / rho for i in range(d)]
    q2 = u[0] * u[0]
    for i in range(1, d):
        q2 = q2 + u[i] * u[i]
    p = (gamma - 1.0) * (Ubar[d + 1] - 0.5 * rho * q2)
    c = np.sqrt(gamma * p / rho)
    H = (Ubar[d + 1] + p) / rho
    b1 = (gamma - 1.0) / (c * c)
    b2 = 0.5 * b1 * q2
    zero = np.zeros_like(rho)
    one = np.ones_like(rho)
    tang = [t for t in range(d) if t != j]
    R = [[None] * nv for _ in range(nv)]
    L = [[None] * nv for _ in range(nv)]
    # columns of R
    cols = []
    cols.append([one] + [u[i] - c if i == j else u[i] for i in range(d)] + [H - u[j] * c])
    cols.append([one] + [u[i] for i in range(d)] + [0.5 * q2])
    for t in tang:
        cols.append([zero] + [one if i == t else zero for i in range(d)] + [u[t]])
    cols.append([one] + [u[i] + c if i == j else u[i] for i in range(d)] + [H + u[j] * c])
    for k in range(nv):
        for v in range(nv):
            R[v][k] = cols[k][v]
    # rows of L
    rows = []
    rows.append([0.5 * (b2 + u[j] / c)]
                + [-0.5 * (b1 * u[i] + (1.0 / c if i == j else 0.0)) for i in range(d)]
                + [0.5 * b1])
    rows.append([1.0 - b2] + [b1 * u[i] for i in range(d)] + [-b1])
    for t in tang:
        rows.append([-u[t]] + [one if i == t else zero for i in range(d)] + [zero])
    rows.append([0.5 * (b2 - u[j] / c)]
                + [-0.5 * (b1 * u[i] - (1.0 / c if i == j else 0.0)) for i in range(d)]
                + [0.5 * b1])
    for k in range(nv):
        for v in range(nv):
            L[k][v] = rows[k][v]
    return R, L


def _matvec(M, x):
    """sum_v M[k][v] x[v] for every k, terms added in v order."""
    out = []
    for row in M:
        acc = row[0] * x[0]
        for v in range(1, len(x)):
            acc = acc + row[v] * x[v]
        out.append(acc)
    return out


def physical_flux(U, d: int, j: int, gamma: float):
    """F_j(U) of Eq. (1)-(3) from conserved values, and |u_j| + c."""
    rho = U[0]
    u = [U[1 + i] / rho for i in range(d)]
    q2 = u[0] * u[0]
    for i in range(1, d):
        q2 = q2 + u[i] * u[i]
    p = (gamma - 1.0) * (U[d + 1] - 0.5 * rho * q2)
    F = [U[1 + j]] + [U[1 + i] * u[j] + (p if i == j else 0.0) for i in range(d)] \
        + [(U[d + 1] + p) * u[j]]
    return F, np.abs(u[j]) + np.sqrt(gamma * p / rho)


def rusanov_conserved(UL, UR, d: int, j: int, gamma: float):
    """Eq. (11) with the wave speed of Eq. (12), from conserved edge states."""
    FL, sl = physical_flux(UL, d, j, gamma)
    FR, sr = physical_flux(UR, d, j, gamma)
    S = np.maximum(sr, sl)
    return [0.5 * (FR[v] + FL[v]) - 0.5 * S * (UR[v] - UL[v]) for v in range(d + 2)]


def edge_fluxes_characteristic(U: np.ndarray, d: int, j: int, gamma: float, eps: float,
                               ng: int = NG):
    """Riemann fluxes at the edges i+1/2, i = -2 .. n, along direction j, from
    characteristic variables: the conserved states of the window nodes
    i-2 .. i+3 are projected on the left eigenvectors of A_j at the mean of
    nodes i and i+1, each characteristic field is interpolated by WENO5-JS
    (left value from nodes i-2..i+2, right value from the mirrored stencil
    i+3..i-1), and the values are projected back with the right
    eigenvectors.  An edge where an interpolated rho or p is not positive on
    either side falls back to first order (the conserved states of nodes i
    and i+1)."""
    n = U.shape[1] - 2 * ng
    nv = d + 2
    Uc = [_interior_cross(U[v], d, j, n, ng) for v in range(nv)]
    ax = axis_of(j, d) - 1
    ne = n + 3
    s = [[_shift(Uc[v], ax, ng - 4 + k, ne) for v in range(nv)] for k in range(6)]
    R, L = flux_eigenvectors(mean_state(s[2], s[3]), d, j, gamma)
    W = [_matvec(L, s[k]) for k in range(6)]
    WL = [weno5js(W[0][k], W[1][k], W[2][k], W[3][k], W[4][k], eps) for k in range(nv)]
    WR = [weno5js(W[5][k], W[4][k], W[3][k], W[2][k], W[1][k], eps) for k in range(nv)]
    UL = _matvec(R, WL)
    UR = _matvec(R, WR)
    ok = np.ones(UL[0].shape, dtype=bool)
    for X in (UL, UR):
        rho = X[0]
        ke = X[1] * (X[1] / rho)
        for i in range(1, d):
            ke = ke + X[1 + i] * (X[1 + i] / rho)
        p = (gamma - 1.0) * (X[d + 1] - 0.5 * ke)
        ok &= (rho > 0.0) & (p > 0.0)
    UL = [np.where(ok, a, b) for a, b in zip(UL, s[2])]
    UR = [np.where(ok, a, b) for a, b in zip(UR, s[3])]
    return rusanov_conserved(UL, UR, d, j, gamma)


def face_fluxes(F, d: int, j: int):
    """Conservative face flux G at faces -1/2 .. n-1/2 from the edge fluxes
    at i+1/2, i = -2..n:  G_{i+1/2} = F_{i+1/2} - (F_{i-1/2} - 2 F_{i+1/2} + F_{i+3/2}) / 24.

    The difference (G_{i+1/2} - G_{i-1/2}) / dx equals the 4th-order staggered
    difference of Eq. (9) exactly (in exact arithmetic).
    """
    ax = d - 1 - j
    out = []
    for Fv in F:
        ne = Fv.shape[ax]
        m = ne - 2
        Fm = _shift(Fv, ax, 0, m)
        F0 = _shift(Fv, ax, 1, m)
        Fp = _shift(Fv, ax, 2, m)
        out.append(F0 - ((Fm - 2.0 * F0) + Fp) / 24.0)
    return out


def patch_faces(U: np.ndarray, d: int, gamma: float, eps: float, ng: int = NG,
                scheme: str = "weno"):
    """Face fluxes G of every direction: list over j of arrays [v, ...] with
    n+1 faces along direction j and n interior lines in the others."""
    def edges(j):
        if scheme == "char":
            return edge_fluxes_characteristic(U, d, j, gamma, eps, ng)
        return edge_fluxes(U, d, j, gamma, eps, ng, scheme)
    return [np.stack(face_fluxes(edges(j), d, j)) for j in range(d)]


def divergence(faces, d: int, h: float) -> np.ndarray:
    """L(U) = - sum_j (G_{i+1/2} - G_{i-1/2}) / h, accumulated in the order x, y, z."""
    L = None
    for j in range(d):
        G = faces[j]
        ax = axis_of(j, d)
        n = G.shape[ax] - 1
        dG = _shift(G, ax, 1, n) - _shift(G, ax, 0, n)
        L = -(dG / h) if L is None else L - dG / h
    return L


def patch_rhs(U: np.ndarray, d: int, h: float, gamma: float, eps: float,
              ng: int = NG, scheme: str = "weno") -> np.ndarray:
    """L(U) on the interior of one patch whose ghost layers are filled."""
    return divergence(patch_faces(U, d, gamma, eps, ng, scheme), d, h)


def max_wave_rate(U: np.ndarray, d: int, h: float, gamma: float) -> float:
    """max over cells of sum_j (|u_j| + c) / h (interior array, no ghosts)."""
    rho, u, p, T = primitives(U, d, gamma)
    c = sound_speed(rho, p, gamma)
    s = np.abs(u[0]) + c
    for j in range(1, d):
        s = s + (np.abs(u[j]) + c)
    return float(np.max(s / h))
