"""Exact matched filter: the cone projection P_cone(D) of eq. exactP / exactPs.

Test infrastructure only (see package docstring).

For a voxel Z_v (complex, length L) and atoms D_j:
    j*   = argmin_j || Z_v - D_j/||D_j|| ||                 (nearest neighbour)
    gamma_v = max( Re<Z_v, D_j*> / ||D_j*||^2 , 0 )         (proton density)
    X_v  = gamma_v D_j*                                      (rescaling)
Expanding the distance, ||Z_v - D^_j||^2 = ||Z_v||^2 - 2 Re<Z_v, D^_j> + 1,
so j* is the (lowest-index) maximiser of c_j = Re<Z_v, D_j>/||D_j||.  The
tests pin this identity by brute-force distances on small inputs.

Readings where the paper is silent: ties go to the lowest atom index; a voxel
with ||Z_v|| = 0 keeps its warm index (else 0) with gamma = 0 and corr = 0;
corr_v = c_j* / ||Z_v|| is the normalised correlation reported per voxel.
Real atoms (FISP) use Re(Z_v) in the inner product, and ||Z_v|| is always the
full complex norm.
"""
from __future__ import annotations

import numpy as np


def atom_norms(atoms: np.ndarray) -> np.ndarray:
    """Euclidean norm of every atom, FP64."""
    a = np.asarray(atoms)
    return np.sqrt(np.sum(np.abs(a.astype(np.complex128 if np.iscomplexobj(a) else np.float64)) ** 2, axis=1))


def normalised_atoms_f32(atoms: np.ndarray) -> np.ndarray:
    """D_j / ||D_j|| computed in FP64 and rounded once to FP32 (complex64 for
    complex atoms): the normalised dictionary the GPU scores against."""
    a = np.asarray(atoms)
    nrm = atom_norms(a)
    if np.iscomplexobj(a):
        return (a.astype(np.complex128) / nrm[:, None]).astype(np.complex64)
    return (a.astype(np.float64) / nrm[:, None]).astype(np.float32)


def correlations(Z: np.ndarray, atoms: np.ndarray, norms=None) -> np.ndarray:
    """c[v, j] = Re<Z_v, D_j> / ||D_j|| in FP64 (matrix product as one step).

    Re<Z_v, D_j> = sum_t Re(Z_vt) Re(D_jt) + Im(Z_vt) Im(D_jt); for real atoms
    only the first sum remains."""
    Z = np.asarray(Z).astype(np.complex128)
    a = np.asarray(atoms)
    nrm = atom_norms(a) if norms is None else norms
    zr = np.ascontiguousarray(Z.real)
    if np.iscomplexobj(a):
        zi = np.ascontiguousarray(Z.imag)
        s = zr @ np.ascontiguousarray(a.real, dtype=np.float64).T
        s += zi @ np.ascontiguousarray(a.imag, dtype=np.float64).T
    else:
        s = zr @ np.ascontiguousarray(a, dtype=np.float64).T
    return s / nrm[None, :]


def exact_mf(Z: np.ndarray, atoms: np.ndarray, warm_idx=None, block: int = 2048,
             want_X: bool = False):
    """Exact matched filter of every row of Z ([n][L]) against atoms ([d][L]).

    Returns a dict with idx [n] (int64), gamma [n] (the PD of eq. exactPs),
    score [n] = c_j* (= Re<Z_v, D_j*>/||D_j*||), corr [n] = score/||Z_v||,
    gap [n] = (c_max - c_second)/||Z_v|| (near-tie measure) and, if asked,
    X [n][L] = gamma_v D_j*.
    """
    Z = np.asarray(Z).astype(np.complex128)
    a = np.asarray(atoms)
    n = Z.shape[0]
    nrm = atom_norms(a)
    idx = np.zeros(n, dtype=np.int64)
    score = np.zeros(n)
    gap = np.full(n, np.inf)
    for s0 in range(0, n, block):
        c = correlations(Z[s0:s0 + block], a, nrm)
        j = np.argmax(c, axis=1)                 # first maximiser = lowest index
        idx[s0:s0 + block] = j
        best = c[np.arange(c.shape[0]), j]
        score[s0:s0 + block] = best
        if c.shape[1] > 1:
            c2 = c.copy()
            c2[np.arange(c.shape[0]), j] = -np.inf
            gap[s0:s0 + block] = best - c2.max(axis=1)
    znorm = np.sqrt(np.sum(np.abs(Z) ** 2, axis=1))
    zero = znorm == 0.0
    if np.any(zero):
        idx[zero] = 0 if warm_idx is None else np.asarray(warm_idx)[zero]
        score[zero] = 0.0
    gamma = np.maximum(score, 0.0) / nrm[idx]
    corr = np.where(zero, 0.0, score / np.where(zero, 1.0, znorm))
    gap = np.where(zero, np.inf, gap / np.where(zero, 1.0, znorm))
    out = dict(idx=idx, gamma=gamma, score=score, corr=corr, gap=gap, znorm=znorm)
    if want_X:
        out["X"] = gamma[:, None] * a[idx].astype(np.complex128)
    return out


def index_ok(Z: np.ndarray, atoms: np.ndarray, idx_test: np.ndarray, tol: float = 1e-6):
    """Near-tie acceptance of a candidate index per voxel: True where the
    normalised correlation of idx_test is within ``tol`` of the maximum."""
    Z = np.asarray(Z).astype(np.complex128)
    c = correlations(Z, atoms)
    znorm = np.sqrt(np.sum(np.abs(Z) ** 2, axis=1))
    zn = np.where(znorm == 0, 1.0, znorm)
    best = c.max(axis=1) / zn
    got = c[np.arange(c.shape[0]), np.asarray(idx_test)] / zn
    return got >= best - tol
