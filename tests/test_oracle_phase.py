"""Pins of the phase-aligned (complex PD) projection: noiseless voxels with a
complex PD are recovered exactly (index, |rho|, phase, X) where the real-PD
projection is not; rotating a voxel by a global phase rotates X and the PD
phase and leaves the index and |rho|; real atoms stay real and are flipped
by the sign of their first principal coefficient; the compressed
dictionary's first coordinate gives the same atom phases as the
uncompressed first principal direction; a full-sampling step recovers a
complex-PD image exactly."""
import numpy as np

from oracle import ipg, mf, phase, subspace
from synth import rng, workloads


def _noiseless_complex(D, n, seed):
    a = mf.normalised_atoms_f32(D.atoms).astype(np.complex128)
    j = (rng.uniform(seed, "j", n) * D.d).astype(np.int64)
    mag = rng.uniform(seed, "mag", n, 0.3, 1.0)
    ang = rng.uniform(seed, "ang", n, -np.pi, np.pi)
    rho = mag * np.exp(1j * ang)
    return rho[:, None] * a[j], j, rho


def test_noiseless_complex_pd_recovered():
    D = workloads.bssfp_dictionary(L=40, n_t1=10, n_t2=10, n_df=5, seed=3)
    u = phase.dominant_vector(D.atoms)
    Da, f = phase.aligned_atoms(D.atoms, u)
    Z, j, rho = _noiseless_complex(D, 300, 1)
    res = phase.project_aligned(Z, Da, u)
    np.testing.assert_array_equal(res["idx"], j)
    np.testing.assert_allclose(res["gamma"], np.abs(rho), rtol=1e-12)
    d = np.angle(np.exp(1j * (phase.pd_phase(res, f) - np.angle(rho))))
    assert np.max(np.abs(d)) < 1e-10
    np.testing.assert_allclose(res["X"], Z, atol=1e-12)
    # the real-PD projection loses the voxels whose PD phase is far from 0
    plain = mf.exact_mf(Z, mf.normalised_atoms_f32(D.atoms).astype(np.complex128), want_X=True)
    assert np.mean(plain["idx"] == j) < 0.9
    assert np.max(np.abs(plain["X"] - Z)) > 0.1


def test_global_phase_equivariance():
    D = workloads.bssfp_dictionary(L=30, n_t1=8, n_t2=8, n_df=3, seed=4)
    u = phase.dominant_vector(D.atoms)
    Da, f = phase.aligned_atoms(D.atoms, u)
    g = rng.normal(4, "z", 2 * 200 * 30).reshape(200, 30, 2)
    Z = g[..., 0] + 1j * g[..., 1]
    psi = 1.234
    r0 = phase.project_aligned(Z, Da, u)
    r1 = phase.project_aligned(Z * np.exp(1j * psi), Da, u)
    np.testing.assert_array_equal(r0["idx"], r1["idx"])
    np.testing.assert_allclose(r0["gamma"], r1["gamma"], rtol=1e-10)
    np.testing.assert_allclose(r1["X"], r0["X"] * np.exp(1j * psi), atol=1e-10)
    d = np.angle(np.exp(1j * (phase.pd_phase(r1, f) - phase.pd_phase(r0, f) - psi)))
    assert np.max(np.abs(d[r0["gamma"] > 0])) < 1e-9


def test_real_atoms_flip_sign_and_recover_complex_pd():
    D = workloads.fisp_dictionary(L=50, n_t1=10, n_t2=10)
    u = phase.dominant_vector(D.atoms)
    Da, f = phase.aligned_atoms(D.atoms, u)
    assert not np.iscomplexobj(Da)
    assert set(np.unique(f)) <= {-1.0, 1.0}
    assert np.all((Da @ u.real) >= 0)
    Z, j, rho = _noiseless_complex(D, 200, 2)
    res = phase.project_aligned(Z, Da, u)
    # FISP atoms of neighbouring T2 can be nearly parallel: accept near-ties
    assert np.all(mf.index_ok(Z * np.conj(res["vphase"])[:, None], Da, j, tol=1e-9))
    np.testing.assert_allclose(res["X"], Z, atol=1e-9)


def test_compressed_first_coordinate_gives_the_same_phases():
    D = workloads.bssfp_dictionary(L=40, n_t1=8, n_t2=8, n_df=4, seed=5)
    V, _ = subspace.dominant_subspace(D.atoms, 6)
    u = V[:, 0]
    f_full = phase.atom_factors(mf.normalised_atoms_f32(D.atoms), u)
    Dc = subspace.compress_atoms(D.atoms, V)
    Dc_n = Dc / np.linalg.norm(Dc, axis=1, keepdims=True)
    e1 = np.zeros(6, dtype=np.complex128)
    e1[0] = 1.0
    f_comp = phase.atom_factors(Dc_n, e1)
    np.testing.assert_allclose(f_comp, f_full, atol=1e-12)
    np.testing.assert_allclose(u, phase.dominant_vector(D.atoms), atol=1e-12)


def test_full_sampling_step_recovers_complex_pd_image():
    """A^H A = I: one step from zero at mu = 1 projects the image itself, so
    the aligned projection returns a complex-PD image exactly and the
    real-PD projection does not."""
    D = workloads.bssfp_dictionary(L=24, n_t1=8, n_t2=8, n_df=3, seed=6)
    S, ny, nx = 1, 16, 16
    a = mf.normalised_atoms_f32(D.atoms).astype(np.complex128)
    n = ny * nx
    j = (rng.uniform(6, "j", n) * D.d).astype(np.int64)
    rho = rng.uniform(6, "m", n, 0.3, 1.0) * np.exp(1j * rng.uniform(6, "p", n, -np.pi, np.pi))
    Xv = rho[:, None] * a[j]
    X0 = Xv.reshape(S, ny, nx, D.L).transpose(0, 3, 1, 2)
    full = workloads.random_lines(6, S, D.L, ny, nx, ny)
    Y = workloads.simulate_kspace(X0, full, None, 6)
    u = phase.dominant_vector(D.atoms)
    Da, f = phase.aligned_atoms(D.atoms, u)
    X1, res, st = ipg.ipg_step(Y, full.off, full.idx, Da, np.zeros_like(X0), 1.0, u=u)
    np.testing.assert_array_equal(res["idx"], j)
    assert np.max(np.abs(X1 - X0)) < 1e-10
    Xp, resp, stp = ipg.ipg_step(Y, full.off, full.idx, a, np.zeros_like(X0), 1.0)
    assert np.max(np.abs(Xp - X0)) > 0.1
