"""Non-Cartesian forward operator (eq. forward with F a non-uniform Fourier
transform, the in-vivo spiral setting), FP64 reference.

Test infrastructure only.

The exact non-uniform DFT written from its definition (no gridding, no
kernel): for a sample at k = (ky, kx) cycles per pixel of frame t,
    y(k) = (ny nx)^(-1/2) sum_{ry, rx} X_t[ry, rx] exp(-2 pi i (ky ry + kx rx))
over pixels ry in [0, ny), rx in [0, nx); the adjoint is the conjugate
transpose.  At grid frequencies k = (kappa_y/ny, kappa_x/nx) it equals the
unitary 2-D DFT of ``fourier`` (pinned in the tests).  Coils as in
``fourier``: S_q X per coil, samples coil-major, conj(S_q) in the adjoint.
The GPU approximates this operator by gridding (a NUFFT); the tests compare
within that approximation's error bound.
"""
from __future__ import annotations

import numpy as np


def _factors(k: np.ndarray, ny: int, nx: int):
    """exp(-2 pi i ky ry) [m][ny] and exp(-2 pi i kx rx) [m][nx]: the
    exponential of the sum is the product of these two, so y = sum_ry
    ey[ry] sum_rx ex[rx] X[ry][rx]."""
    k = np.asarray(k, dtype=np.float64)
    ey = np.exp(-2j * np.pi * np.outer(k[:, 0], np.arange(ny)))
    ex = np.exp(-2j * np.pi * np.outer(k[:, 1], np.arange(nx)))
    return ey, ex


def forward(X: np.ndarray, off: np.ndarray, coords: np.ndarray) -> np.ndarray:
    """A(X): X frame-major [S][L][ny][nx] -> samples [M] in CSR order."""
    S, L, ny, nx = X.shape
    out = np.empty(int(off[-1]), dtype=np.complex128)
    for s in range(S):
        for t in range(L):
            p = s * L + t
            ey, ex = _factors(coords[off[p]:off[p + 1]], ny, nx)
            rows = ey @ np.asarray(X[s, t], dtype=np.complex128)          # [m][nx]: sum over ry
            out[off[p]:off[p + 1]] = np.sum(rows * ex, axis=1) / np.sqrt(ny * nx)
    return out


def adjoint(R: np.ndarray, off: np.ndarray, coords: np.ndarray, S: int, L: int, ny: int, nx: int) -> np.ndarray:
    """A^H(R): X[ry][rx] = (ny nx)^(-1/2) sum_i conj(ey_i[ry] ex_i[rx]) R_i."""
    R = np.asarray(R, dtype=np.complex128)
    out = np.empty((S, L, ny, nx), dtype=np.complex128)
    for s in range(S):
        for t in range(L):
            p = s * L + t
            ey, ex = _factors(coords[off[p]:off[p + 1]], ny, nx)
            out[s, t] = ey.conj().T @ (R[off[p]:off[p + 1], None] * ex.conj()) / np.sqrt(ny * nx)
    return out


def forward_coils(X, off, coords, smaps):
    c = smaps.shape[1]
    return np.stack([forward(smaps[:, q, None] * X, off, coords) for q in range(c)])


def adjoint_coils(R, off, coords, S, L, ny, nx, smaps):
    out = np.zeros((S, L, ny, nx), dtype=np.complex128)
    for q in range(smaps.shape[1]):
        out += np.conj(smaps[:, q, None]) * adjoint(R[q], off, coords, S, L, ny, nx)
    return out
