"""Algorithm 1 as the paper runs it (Sec. 5): a 2D transform in the lateral
variables and, for every lateral frequency, a dense M x M' system in z
(Eq. (14)), regularised per frequency.

Oracle (test infrastructure only).

Readings (each also listed in the design notes):
* Lateral axes: the same circulant embedding as the 3D path (P = 2n per
  lateral axis, zero slot at offset index n), so the lateral convolution is
  the exact discrete one.  The z axis is not embedded: the system matrix of
  lateral frequency (kx, ky) is A[i][j] = k~(kx, ky; i - j), Y layer i
  (height D + i cells), R layer j (height j cells), where k~(.; dz) is the 2D
  DFT of the wrapped lateral samples h^2 hz K(ox h, oy h, (D + dz) hz).  M = M' =
  nz.  K is even in x and y, so k~ and every A are real.
* One alpha for all frequencies, chosen by the discrepancy principle on the
  residual over Y (Sec. 4 rule applied to the whole data set); or, reading
  Algorithm 1 step 2 per frequency (``solve_per_frequency``), one alpha per
  system by the same rule on that system's own residual.
* Regularising algorithms (Sec. 5: standard and iterated Tikhonov, TSVD),
  through the SVD A = U S V^T with filter factors phi(s):
  Tikhonov s^2/(s^2 + a), iterated Tikhonov of order m 1 - (a/(s^2 + a))^m
  (evaluated as s^2/(s^2 + a) sum_{j<m} (a/(s^2 + a))^j), TSVD [s^2 >= a];
  x^ = V diag(phi/s) U^T f^ (0 where s = 0) and the residual A x^ - f^.
"""
from __future__ import annotations

import numpy as np

from .geometry import Geom, kernel_fn, offset_of_index
from .tikhonov import ITERATED, TIKHONOV, TSVD


def lateral_kernel_spectrum(g: Geom):
    """k~[l][ky][kx] for l = dz + nz - 1, dz in (-nz, nz): 2D DFT over the
    wrapped lateral offset table at z offset (D + dz) hz, weight h^2 hz."""
    py, px = 2 * g.ny, 2 * g.nx
    ox, vx = offset_of_index(np.arange(px), g.nx, px)
    oy, vy = offset_of_index(np.arange(py), g.ny, py)
    dz = np.arange(-(g.nz - 1), g.nz)
    K = g.h * g.h * g.hv * kernel_fn(g.kind)(ox[None, None, :] * g.h, oy[None, :, None] * g.h,
                                             (g.d + dz[:, None, None]) * g.hv)
    K = K * (vx[None, None, :] & vy[None, :, None])
    return np.fft.fft2(K, axes=(1, 2))


def system_matrices(g: Geom, kt):
    """A for every lateral frequency: real array [Py][Px][nz][nz]."""
    i = np.arange(g.nz)[:, None]
    j = np.arange(g.nz)[None, :]
    A = kt[i - j + g.nz - 1].real            # [nz][nz][Py][Px]
    return np.ascontiguousarray(np.moveaxis(A, (0, 1), (2, 3)))


def lateral_spectrum(g: Geom, u):
    """2D DFT of every layer of an nz x ny x nx field, zero-padded laterally."""
    up = np.zeros((g.nz, 2 * g.ny, 2 * g.nx))
    up[:, : g.ny, : g.nx] = u
    return np.fft.fft2(up, axes=(1, 2))


def filter_factors(s, a: float, method: int = TIKHONOV, order: int = 1):
    lam = s * s
    if method == TIKHONOV:
        return lam / (lam + a)
    if method == ITERATED:
        # 1 - q^m = (1 - q) sum_{j<m} q^j with 1 - q = lam/(lam + a): no cancellation for small lam
        q = a / (lam + a)
        return lam / (lam + a) * sum(q ** j for j in range(order))
    if method == TSVD:
        return (lam >= a).astype(np.float64)
    raise ValueError(f"unknown method {method}")


def solve_layered(g: Geom, kt, F, alpha: float, method: int = TIKHONOV, order: int = 1):
    """Regularised estimate at alpha; zeta on R, r on Y and their norms."""
    A = system_matrices(g, kt)
    fh = np.moveaxis(lateral_spectrum(g, np.asarray(F, dtype=np.float64)), 0, 2)   # [Py][Px][nz]
    U, S, Vt = np.linalg.svd(A)
    phi = filter_factors(S, alpha, method, order)
    gain = np.where(S > 0, phi / np.where(S > 0, S, 1.0), 0.0)
    b = np.einsum("...ij,...i->...j", U, fh)             # U^T f
    xh = np.einsum("...ji,...j->...i", Vt, gain * b)      # V (gain b)
    rh = np.einsum("...ij,...j->...i", A, xh) - fh        # A x - f
    xs = np.fft.ifft2(np.moveaxis(xh, 2, 0), axes=(1, 2))
    rs = np.fft.ifft2(np.moveaxis(rh, 2, 0), axes=(1, 2))
    zeta = xs.real[:, : g.ny, : g.nx]
    r = rs.real[:, : g.ny, : g.nx]
    return dict(zeta=zeta, r=r, zeta_norm=float(np.sqrt(np.sum(zeta * zeta))),
                r_norm=float(np.sqrt(np.sum(r * r))),
                imag_max=float(max(np.abs(xs.imag).max(), np.abs(rs.imag).max())),
                singular_values=S)


def forward_layered(g: Geom, kt, zeta):
    """A zeta through the per-frequency systems: F^ = A^(m) zeta^ for every (kx, ky)."""
    A = system_matrices(g, kt)
    zh = np.moveaxis(lateral_spectrum(g, np.asarray(zeta, dtype=np.float64)), 0, 2)
    yh = np.einsum("...ij,...j->...i", A, zh)
    return np.fft.ifft2(np.moveaxis(yh, 2, 0), axes=(1, 2)).real[:, : g.ny, : g.nx]


def assembled_operator(g: Geom):
    """The laterally embedded, z-exact operator as one explicit matrix from
    R's layers over the padded lateral box to Y's: rows (i, y, x), columns
    (j, y', x'), entry h^2 hz K(wrapped offset (x - x', y - y'), (D + i - j) hz).
    No transform; for tiny grids only."""
    py, px = 2 * g.ny, 2 * g.nx
    n = g.nz * py * px
    C = np.zeros((n, n))
    K = kernel_fn(g.kind)
    for i in range(g.nz):
        for y in range(py):
            for x in range(px):
                row = (i * py + y) * px + x
                for j in range(g.nz):
                    for y2 in range(py):
                        oy, vy = offset_of_index((y - y2) % py, g.ny, py)
                        if not vy:
                            continue
                        for x2 in range(px):
                            ox, vx = offset_of_index((x - x2) % px, g.nx, px)
                            if not vx:
                                continue
                            C[row, (j * py + y2) * px + x2] = g.h * g.h * g.hv * K(
                                float(ox) * g.h, float(oy) * g.h, (g.d + i - j) * g.hv)
    return C


def dense_layered(g: Geom, F, alpha: float, method: int = TIKHONOV):
    """Tikhonov (normal equations) or TSVD (SVD with cut alpha) of the
    assembled operator for data F on Y's footprint; zeta and r restricted to
    the footprints of R and Y."""
    C = assembled_operator(g)
    py, px = 2 * g.ny, 2 * g.nx
    f = np.zeros((g.nz, py, px))
    f[:, : g.ny, : g.nx] = F
    f = f.ravel()
    if method == TIKHONOV:
        u = np.linalg.solve(C.T @ C + alpha * np.eye(C.shape[1]), C.T @ f)
    elif method == TSVD:
        Uc, Sc, Vtc = np.linalg.svd(C)
        keep = Sc * Sc >= alpha
        u = Vtc[keep].T @ ((Uc[:, keep].T @ f) / Sc[keep])
    else:
        raise ValueError("dense form for Tikhonov and TSVD only")
    res = (C @ u - f).reshape(g.nz, py, px)
    u = u.reshape(g.nz, py, px)
    return dict(zeta=u[:, : g.ny, : g.nx], r=res[:, : g.ny, : g.nx])


def solve_per_frequency(g: Geom, kt, F, delta: float, tau: float = 1.0, lo: float = -8.0, hi: float = 0.0,
                        tol: float = 1e-3, max_steps: int = 40, method: int = TIKHONOV, order: int = 1):
    """Algorithm 1 step 2 read per lateral frequency: every system gets its own
    alpha, chosen by the plain discrepancy rule (bisection in log10 alpha) on
    its own residual ||A x^ - f^|| against tau delta.  Units: the unnormalised
    lateral DFT, in which white noise of norm delta on Y has expected energy
    delta^2 at every frequency (Parseval: the PxPy frequencies carry PxPy
    delta^2).  Returns dict(zeta, r, zeta_norm, r_norm, alphas [Py][Px],
    flags [Py][Px])."""
    from . import discrepancy
    A = system_matrices(g, kt)
    fh = np.moveaxis(lateral_spectrum(g, np.asarray(F, dtype=np.float64)), 0, 2)   # [Py][Px][nz]
    py, px = fh.shape[:2]
    U, S, Vt = np.linalg.svd(A)
    xh = np.zeros_like(fh)
    alphas = np.zeros((py, px))
    flags = np.zeros((py, px), dtype=np.int64)
    for iy in range(py):
        for ix in range(px):
            Am, f = A[iy, ix], fh[iy, ix]
            b = U[iy, ix].T @ f

            def solve(a):
                phi = filter_factors(S[iy, ix], a, method, order)
                gain = np.where(S[iy, ix] > 0, phi / np.where(S[iy, ix] > 0, S[iy, ix], 1.0), 0.0)
                return Vt[iy, ix].T @ (gain * b)

            def ev(a):
                x = solve(a)
                return float(np.linalg.norm(Am @ x - f)), float(np.linalg.norm(x))
            res = discrepancy.bisection(ev, delta, lo=lo, hi=hi, max_steps=max_steps, tol=tol, tau=tau)
            alphas[iy, ix] = res["alpha"]
            flags[iy, ix] = res["flags"]
            xh[iy, ix] = solve(res["alpha"])
    rh = np.einsum("...ij,...j->...i", A, xh) - fh
    xs = np.fft.ifft2(np.moveaxis(xh, 2, 0), axes=(1, 2))
    rs = np.fft.ifft2(np.moveaxis(rh, 2, 0), axes=(1, 2))
    zeta = xs.real[:, : g.ny, : g.nx]
    r = rs.real[:, : g.ny, : g.nx]
    return dict(zeta=zeta, r=r, zeta_norm=float(np.sqrt(np.sum(zeta * zeta))),
                r_norm=float(np.sqrt(np.sum(r * r))), alphas=alphas, flags=flags,
                imag_max=float(max(np.abs(xs.imag).max(), np.abs(rs.imag).max())))
