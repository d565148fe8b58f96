"""Forward operator A = P_Omega F S and its adjoint (eq. forward).

Test infrastructure only.

F is the unitary 2-D DFT of each frame (1/sqrt(ny*nx) normalisation, the
reading under which the paper's step sizes mu = 1 and mu = n/m are
admissible).  S = I for one coil; with c coils S maps a frame to its c
copies weighted pixel-wise by the coil sensitivity maps (the same maps for
every frame), and the one pattern of each (slice, frame) samples every
coil.  P_Omega keeps the samples listed per (slice, frame) in the CSR
pattern; its adjoint scatters them back into a zero-filled k-space.  The
FFT is numpy's (a library routine used as one step); the tests pin it
against the DFT sum written out.
"""
from __future__ import annotations

import numpy as np


def fft2_unitary(x: np.ndarray) -> np.ndarray:
    return np.fft.fft2(np.asarray(x, dtype=np.complex128), norm="ortho")


def ifft2_unitary(k: np.ndarray) -> np.ndarray:
    return np.fft.ifft2(np.asarray(k, dtype=np.complex128), norm="ortho")


def forward(X: np.ndarray, off: np.ndarray, idx: np.ndarray) -> np.ndarray:
    """A(X): X frame-major [S][L][ny][nx] -> samples [M] in CSR order."""
    S, L, ny, nx = X.shape
    out = np.empty(int(off[-1]), dtype=np.complex128)
    for s in range(S):
        k = fft2_unitary(X[s]).reshape(L, ny * nx)
        for t in range(L):
            p = s * L + t
            out[off[p]:off[p + 1]] = k[t, idx[off[p]:off[p + 1]]]
    return out


def adjoint(R: np.ndarray, off: np.ndarray, idx: np.ndarray, S: int, L: int,
            ny: int, nx: int) -> np.ndarray:
    """A^H(R): samples [M] -> frame-major image [S][L][ny][nx]."""
    R = np.asarray(R, dtype=np.complex128)
    out = np.empty((S, L, ny, nx), dtype=np.complex128)
    for s in range(S):
        k = np.zeros((L, ny * nx), dtype=np.complex128)
        for t in range(L):
            p = s * L + t
            k[t, idx[off[p]:off[p + 1]]] = R[off[p]:off[p + 1]]
        out[s] = ifft2_unitary(k.reshape(L, ny, nx))
    return out


def forward_coils(X: np.ndarray, off: np.ndarray, idx: np.ndarray, smaps: np.ndarray) -> np.ndarray:
    """A(X) = P_Omega F S(X) with c coils: smaps [S][c][ny][nx]; returns the
    samples coil-major, [c][M] (row q: the samples of F(S_q X_t))."""
    c = smaps.shape[1]
    return np.stack([forward(smaps[:, q, None] * X, off, idx) for q in range(c)])


def adjoint_coils(R: np.ndarray, off: np.ndarray, idx: np.ndarray, S: int, L: int, ny: int, nx: int,
                  smaps: np.ndarray) -> np.ndarray:
    """A^H(R) = sum_q conj(S_q) F^H P_Omega^T R_q for R [c][M]."""
    out = np.zeros((S, L, ny, nx), dtype=np.complex128)
    for q in range(smaps.shape[1]):
        out += np.conj(smaps[:, q, None]) * adjoint(R[q], off, idx, S, L, ny, nx)
    return out


def frame_to_voxel(X: np.ndarray) -> np.ndarray:
    """[S][L][ny][nx] -> voxel-major rows [n][L] (v = s*ny*nx + y*nx + x)."""
    S, L, ny, nx = X.shape
    return X.transpose(0, 2, 3, 1).reshape(S * ny * nx, L)


def voxel_to_frame(V: np.ndarray, S: int, ny: int, nx: int) -> np.ndarray:
    L = V.shape[1]
    return V.reshape(S, ny, nx, L).transpose(0, 3, 1, 2)
