"""Complex proton density by temporal phase alignment, FP64 reference.

Test infrastructure only.

The phase-alignment extension of Section "CoverBLIP algorithm" (the
paragraph after the compressed step rule: complex-valued PD, aligned with
the phases of the first principal component of the dictionary):
  * u = the dominant eigenvector of sum_j Dhat_j Dhat_j^H (the first column
    of ``subspace.dominant_subspace``, phase convention included); for a
    temporally compressed dictionary whose basis starts with u, u is the
    first unit vector of the compressed coordinates;
  * atom phases: c_j = u^H Dhat_j, aligned atoms Dhat_j e^{-i angle(c_j)}
    (for real atoms the factor is the sign of c_j, so they stay real; a zero
    coefficient leaves the atom as it is);
  * voxel phases: theta_v = angle(u^H Z_v) (0 where the coefficient is 0);
    the search runs on Z_v e^{-i theta_v} against the aligned atoms
    (eq. exactP, real PD gamma_v of eq. exactPs);
  * X_v = gamma_v e^{i theta_v} Dhat^a_j*: with the aligned atom
    Dhat^a_j = e^{-i phi_j} Dhat_j, the complex PD on the normalised atom
    Dhat_j* is rho_v = gamma_v e^{i (theta_v - phi_j*)}.
"""
from __future__ import annotations

import numpy as np

from . import mf, subspace


def dominant_vector(atoms: np.ndarray) -> np.ndarray:
    """u [L] complex128: the dominant eigenvector with the phase convention."""
    V, _ = subspace.dominant_subspace(atoms, 1)
    return V[:, 0]


def atom_factors(atoms_n: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Per-atom unit factors f_j with aligned atom = f_j Dhat_j, for the
    normalised atoms ``atoms_n`` (complex: conj(c_j)/|c_j|; real: sign(Re c_j);
    1 where c_j = 0)."""
    a = np.asarray(atoms_n)
    c = a.astype(np.complex128) @ np.conj(u)
    if np.iscomplexobj(a):
        m = np.abs(c)
        return np.where(m > 0, np.conj(c) / np.where(m > 0, m, 1.0), 1.0 + 0j)
    return np.where(c.real < 0, -1.0, 1.0)


def aligned_atoms(atoms: np.ndarray, u: np.ndarray):
    """(aligned normalised atoms in FP64, factors f_j) from the FP32-rounded
    normalised atoms the GPU holds."""
    a = mf.normalised_atoms_f32(atoms)
    f = atom_factors(a, u)
    wide = a.astype(np.complex128 if np.iscomplexobj(a) else np.float64)
    return wide * f[:, None], f


def voxel_factors(Z: np.ndarray, u: np.ndarray) -> np.ndarray:
    """e^{i theta_v} with theta_v = angle(u^H Z_v) (1 where u^H Z_v = 0)."""
    c = np.asarray(Z, dtype=np.complex128) @ np.conj(u)
    m = np.abs(c)
    return np.where(m > 0, c / np.where(m > 0, m, 1.0), 1.0 + 0j)


def project_aligned(Z: np.ndarray, atoms_aligned: np.ndarray, u: np.ndarray, warm_idx=None):
    """Phase-aligned matched filter of voxel rows Z [n][L] against aligned
    atoms.  Returns exact_mf's dict on the aligned voxels plus 'vphase'
    (e^{i theta_v}) and X = gamma_v e^{i theta_v} Dhat^a_j*."""
    e = voxel_factors(Z, u)
    res = mf.exact_mf(np.asarray(Z, dtype=np.complex128) * np.conj(e)[:, None], atoms_aligned,
                      warm_idx=warm_idx, want_X=True)
    res["vphase"] = e
    res["X"] = res["X"] * e[:, None]
    return res


def pd_phase(res, factors: np.ndarray) -> np.ndarray:
    """Phase of the complex PD rho_v = gamma_v e^{i theta_v} f_j* (the aligned
    atom is f_j* Dhat_j*), wrapped to (-pi, pi]."""
    return np.angle(res["vphase"] * factors[res["idx"]])
