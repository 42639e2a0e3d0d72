"""CPU reference of the velocity-gradient diagnostic (TEST INFRASTRUCTURE
ONLY, see ``oracle/__init__.py``).

The paper's task-fusion listing (§4.1) shows a task that reads the conserved
variables and writes a velocity-gradient region; its body is elided, and §5
images the shear-layer flow by numerical Schlieren.  Reading taken here: at
every interior cell of a leaf patch, with ghost cells filled,

    G[i][j] = (u_i(x + h e_j) - u_i(x - h e_j)) / (2 h),   u_i = m_i / rho,
    S       = sqrt(sum_j ((rho(x + h e_j) - rho(x - h e_j)) / (2 h))^2),

second-order central differences on the cell's own level (h = h_l); S is the
density-gradient magnitude a numerical Schlieren image is drawn from.  The sum
in S runs over j in the order x, y, z.
"""
from __future__ import annotations

from typing import Dict

import numpy as np


def _shift(a: np.ndarray, axis: int, s: int, ng: int) -> np.ndarray:
    """Interior block of ``a`` (spatial axes 1..d) displaced by s cells along
    spatial axis ``axis`` (0 = the last array axis, x)."""
    d = a.ndim - 1
    sl = [slice(None)]
    for ax in range(d):
        j = d - 1 - ax            # array axis ax holds spatial direction j
        off = s if j == axis else 0
        sl.append(slice(ng + off, a.shape[ax + 1] - ng + off))
    return a[tuple(sl)]


def velocity_gradient(o, buf: int) -> Dict:
    """Per leaf key, an array [d*d + 1, n, ...] (interior cells, array axes
    z, y, x): G[i][j] at component i*d + j, then S."""
    d = o.grid.dim
    ng = o.grid.ghost
    out = {}
    for key in o.forest.leaves():
        U = o.U[buf][key]
        h = o.grid.h(key[0])
        rho = U[0]
        vel = [U[1 + i] / rho for i in range(d)]
        comps = []
        grad_rho = []
        for i in range(d):
            for j in range(d):
                up = _shift(vel[i][None], j, +1, ng)[0]
                um = _shift(vel[i][None], j, -1, ng)[0]
                comps.append((up - um) / (2.0 * h))
        for j in range(d):
            rp = _shift(rho[None], j, +1, ng)[0]
            rm = _shift(rho[None], j, -1, ng)[0]
            grad_rho.append((rp - rm) / (2.0 * h))
        s2 = grad_rho[0] * grad_rho[0]
        for j in range(1, d):
            s2 = s2 + grad_rho[j] * grad_rho[j]
        comps.append(np.sqrt(s2))
        out[key] = np.stack(comps)
    return out
