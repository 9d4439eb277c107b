"""Synthetic data through the paper's own linear operator.

Oracle (test infrastructure only).

By Remark 1 (Eq. (7)) the difference data 2 pi (dV2/dz - dV2^(0)/dz) on Y equal
A zeta with zeta = xi V0 (Sec. 2), so the data are F = A(xi V0) + e.  The
noise e is a given draw rescaled so that ||e|| = delta_rel ||A zeta||, and
delta = ||e|| is the level of Sec. 3 (||v - v_delta|| <= delta).  Sec. 6
synthesises its data the same way, through the discretised operator.
"""
from __future__ import annotations

import numpy as np

from .geometry import Geom, v0
from .operator import forward_circulant, forward_direct


def make_data(g: Geom, xi, noise, delta_rel, direct=False, A0=1.0):
    V0 = v0(g, A0)
    zeta = np.asarray(xi, dtype=np.float64) * V0
    AF = forward_direct(g, zeta) if direct else forward_circulant(g, zeta)
    e = np.asarray(noise, dtype=np.float64)
    e = e * (delta_rel * np.linalg.norm(AF) / np.linalg.norm(e))
    return dict(F=AF + e, delta=float(np.linalg.norm(e)), zeta=zeta, V0=V0, AF=AF)
