"""Step 4 of Algorithm 1 (Sec. 4): xi = zeta / V0, then c from
xi = 1/c0^2 - 1/c^2 (Sec. 2, Assumption 5; the paper's sign).

Oracle (test infrastructure only).

Reading for the case the paper leaves open: where 1/c0^2 - xi < 1e-6/c0^2
(including <= 0, where no real c exists) the argument is clamped to 1e-6/c0^2
and the cell is counted.
"""
from __future__ import annotations

import numpy as np

CLAMP_REL = 1e-6


def xi_from_zeta(zeta, V0):
    return np.asarray(zeta, dtype=np.float64) / np.asarray(V0, dtype=np.float64)


def c_from_xi(xi, c0):
    floor = CLAMP_REL / (c0 * c0)
    arg = 1.0 / (c0 * c0) - np.asarray(xi, dtype=np.float64)
    clamped = arg < floor
    arg = np.where(clamped, floor, arg)
    return 1.0 / np.sqrt(arg), int(clamped.sum())


def recover(zeta, V0, c0):
    """Returns (xi, c, n_clamped)."""
    xi = xi_from_zeta(zeta, V0)
    c, n = c_from_xi(xi, c0)
    return xi, c, n
