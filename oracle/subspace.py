"""Temporal subspace compression, FP64 reference.

Test infrastructure only.

Section "Dimension-reduced subspace matched-filtering" (eq. CS1, eq.
gradupdate, eq. gradcompression) and the compressed step rule of the
Algorithm 2 discussion:
  * V_s = the s dominant eigenvectors of sum_j D_j D_j^H, here over the
    normalised atoms (the GPU's FP32 normalised atoms, widened to FP64), each
    eigenvector multiplied by a unit phase so that its entry of largest
    magnitude (the lowest row among equal magnitudes) is real and positive;
  * compressed atoms Dtilde_j = V_s^H D_j (rows: a_j conj(V_s));
  * a voxel's time series x_v = V_s xtilde_v, xtilde_v = V_s^H x_v; for
    frame-major images X_t = sum_k V_s[t, k] Xtilde_k and
    Xtilde_k = sum_t conj(V_s[t, k]) X_t (the Fourier transform acts per
    frame, so it commutes with both);
  * the compressed operator is A(expand(.)) and its adjoint
    compress(A^H(.)).
"""
from __future__ import annotations

import numpy as np

from . import mf


def dominant_subspace(atoms: np.ndarray, s: int):
    """(V [L][s] complex128, eigenvalues [s] descending) of
    sum_j Dhat_j Dhat_j^H over the FP32-rounded normalised atoms."""
    a = mf.normalised_atoms_f32(atoms).astype(np.complex128)
    G = a.T @ a.conj()                       # G[t, t'] = sum_j a_j[t] conj(a_j[t'])
    lam, U = np.linalg.eigh(G)               # ascending, orthonormal columns
    lam, U = lam[::-1][:s].copy(), U[:, ::-1][:, :s].copy()
    for k in range(s):
        mag = np.abs(U[:, k])
        i = int(np.flatnonzero(mag == mag.max())[0])
        U[:, k] *= np.conj(U[i, k]) / mag[i]
    return U, lam


def compress_atoms(atoms: np.ndarray, V: np.ndarray) -> np.ndarray:
    """Dtilde_j = V^H Dhat_j for the FP32-rounded normalised atoms."""
    return mf.normalised_atoms_f32(atoms).astype(np.complex128) @ V.conj()


def expand(Xc: np.ndarray, V: np.ndarray) -> np.ndarray:
    """[S][s][ny][nx] -> [S][L][ny][nx]: X_t = sum_k V[t, k] Xc_k."""
    return np.einsum("tk,skyx->styx", V, Xc)


def compress(X: np.ndarray, V: np.ndarray) -> np.ndarray:
    """[S][L][ny][nx] -> [S][s][ny][nx]: Xc_k = sum_t conj(V[t, k]) X_t."""
    return np.einsum("tk,styx->skyx", V.conj(), X)
