"""Exact discrete solutions of the cell-centred 5-point operator (TEST
INFRASTRUCTURE ONLY; part of the oracle).

The discrete problem the multigrid iteration converges to (pyro paper,
Sec. 3.3, Eq. (helmholtz)) is

    alpha phi_ij - beta/h^2 (phiE + phiW + phiN + phiS - 4 phi_ij) = f_ij

with the out-of-domain neighbour replaced by its ghost value:
Dirichlet ghost = -phi (own cell), Neumann ghost = +phi, periodic = the cell
on the opposite side.  Two independent ways to get its solution:

* ``dense_solve``: assemble the n^2 x n^2 matrix entry by entry and call
  ``numpy.linalg.solve`` (``lstsq`` plus a zero-mean row when singular);
* ``transform_solve``: diagonalise with the transform whose basis vectors are
  the operator's eigenvectors -- FFT for periodic, DST-II for Dirichlet,
  DCT-II for Neumann, one axis at a time -- and divide by
  alpha - beta (lam_x + lam_y).

Arrays of valid cells are indexed [j, i] (y, x).
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft

from . import DIRICHLET, NEUMANN, PERIODIC, bc_codes


def assemble(n: int, h: float, alpha: float, beta: float, bc) -> np.ndarray:
    """Dense matrix of (alpha - beta Lap_h) with ghost cells eliminated.
    Unknown ordering k = j*n + i."""
    bc = bc_codes(bc)
    A = np.zeros((n * n, n * n))
    c = beta / (h * h)
    for j in range(n):
        for i in range(n):
            k = j * n + i
            A[k, k] += alpha + 4.0 * c
            # neighbours: (di, dj, side index when it leaves the domain)
            for di, dj, side in ((-1, 0, 0), (1, 0, 1), (0, -1, 2), (0, 1, 3)):
                ii, jj = i + di, j + dj
                if 0 <= ii < n and 0 <= jj < n:
                    A[k, jj * n + ii] -= c
                elif bc[side] == PERIODIC:
                    A[k, (jj % n) * n + (ii % n)] -= c
                elif bc[side] == DIRICHLET:
                    A[k, k] -= c * (-1.0)
                else:  # Neumann
                    A[k, k] -= c * (+1.0)
    return A


def is_singular(alpha: float, bc) -> bool:
    return alpha == 0.0 and DIRICHLET not in bc_codes(bc)


def dense_solve(f: np.ndarray, h: float, alpha: float, beta: float, bc) -> np.ndarray:
    n = f.shape[0]
    A = assemble(n, h, alpha, beta, bc)
    b = f.reshape(-1)
    if is_singular(alpha, bc):
        # constant null space: append the zero-mean condition
        A2 = np.vstack([A, np.ones((1, n * n))])
        b2 = np.concatenate([b, [0.0]])
        x = np.linalg.lstsq(A2, b2, rcond=None)[0]
    else:
        x = np.linalg.solve(A, b)
    return x.reshape(n, n)


def eigenvalues_1d(n: int, h: float, kind: int) -> np.ndarray:
    """Eigenvalues of the 1-d second difference (phi[i+1] - 2 phi[i] + phi[i-1])/h^2
    in the order of the matching scipy transform's output."""
    if kind == PERIODIC:
        k = np.fft.fftfreq(n, d=1.0 / n)  # integer wavenumbers
        return -(4.0 / h**2) * np.sin(np.pi * k / n) ** 2
    if kind == DIRICHLET:  # DST-II basis sin(pi k x), k = 1..n
        k = np.arange(1, n + 1)
        return -(4.0 / h**2) * np.sin(np.pi * k / (2 * n)) ** 2
    if kind == NEUMANN:  # DCT-II basis cos(pi k x), k = 0..n-1
        k = np.arange(0, n)
        return -(4.0 / h**2) * np.sin(np.pi * k / (2 * n)) ** 2
    raise ValueError(kind)


def _fwd(a, axis, kind):
    if kind == PERIODIC:
        return sfft.fft(a, axis=axis)
    if kind == DIRICHLET:
        return sfft.dst(a, type=2, axis=axis, norm="ortho")
    return sfft.dct(a, type=2, axis=axis, norm="ortho")


def _inv(a, axis, kind):
    if kind == PERIODIC:
        return sfft.ifft(a, axis=axis)
    if kind == DIRICHLET:
        return sfft.idst(a, type=2, axis=axis, norm="ortho")
    return sfft.idct(a, type=2, axis=axis, norm="ortho")


def transform_solve(f: np.ndarray, h: float, alpha: float, beta: float, bc) -> np.ndarray:
    """Exact solve when each axis has the same type on both sides."""
    bc = bc_codes(bc)
    if bc[0] != bc[1] or bc[2] != bc[3]:
        raise ValueError("transform_solve needs the same type on both sides of an axis")
    n = f.shape[0]
    kx, ky = bc[0], bc[2]
    lam = eigenvalues_1d(n, h, ky)[:, None] + eigenvalues_1d(n, h, kx)[None, :]
    den = alpha - beta * lam
    g = _fwd(_fwd(f.astype(np.complex128 if PERIODIC in (kx, ky) else np.float64), 1, kx), 0, ky)
    zero = np.abs(den) < 1e-300
    den = np.where(zero, 1.0, den)
    u = g / den
    u = np.where(zero, 0.0, u)  # singular mode -> zero-mean solution
    x = _inv(_inv(u, 0, ky), 1, kx)
    return np.real(x) if np.iscomplexobj(x) else x


def apply_operator(phi: np.ndarray, h: float, alpha: float, beta: float, bc) -> np.ndarray:
    """(alpha - beta Lap_h) phi on valid cells (array form, for invariants)."""
    bc = bc_codes(bc)
    n = phi.shape[0]
    g = np.zeros((n + 2, n + 2))
    g[1:-1, 1:-1] = phi
    for side, (sl_ghost, sl_in, sl_opp) in enumerate((
            ((slice(1, -1), 0), (slice(1, -1), 1), (slice(1, -1), n)),
            ((slice(1, -1), n + 1), (slice(1, -1), n), (slice(1, -1), 1)),
            ((0, slice(1, -1)), (1, slice(1, -1)), (n, slice(1, -1))),
            ((n + 1, slice(1, -1)), (n, slice(1, -1)), (1, slice(1, -1))))):
        if bc[side] == PERIODIC:
            g[sl_ghost] = g[sl_opp]
        elif bc[side] == DIRICHLET:
            g[sl_ghost] = -g[sl_in]
        else:
            g[sl_ghost] = g[sl_in]
    c = g[1:-1, 1:-1]
    lap = ((g[1:-1, 2:] - c) + (g[1:-1, :-2] - c) + (g[2:, 1:-1] - c) + (g[:-2, 1:-1] - c)) / h**2
    return alpha * c - beta * lap


def relative_residual(phi: np.ndarray, f: np.ndarray, h: float, alpha: float, beta: float,
                      bc) -> float:
    r = f - apply_operator(phi, h, alpha, beta, bc)
    return float(np.sqrt(np.sum(r * r)) / np.sqrt(np.sum(f * f)))
