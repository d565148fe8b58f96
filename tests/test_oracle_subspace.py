"""Pins of the temporal-subspace oracle (eq. CS1, eq. gradupdate, eq.
gradcompression): orthonormal basis and the trace identity, the phase
convention, s = L reducing to the uncompressed IPG step, an exactly rank-s
dictionary giving the full matched filter, the adjoint identity of the
compressed operator."""
import numpy as np

from oracle import fourier, ipg, mf, subspace
from synth import rng, workloads


def _cg(seed, tag, shape):
    n = int(np.prod(shape))
    g = rng.normal(seed, tag, 2 * n).reshape(tuple(shape) + (2,))
    return g[..., 0] + 1j * g[..., 1]


def test_basis_orthonormal_trace_and_phase():
    D = workloads.bssfp_dictionary(L=24, n_t1=6, n_t2=6, n_df=5, seed=2)
    V, lam = subspace.dominant_subspace(D.atoms, 24)
    np.testing.assert_allclose(V.conj().T @ V, np.eye(24), atol=1e-12)
    assert np.all(np.diff(lam) <= 1e-9)
    # trace of sum_j Dhat_j Dhat_j^H = sum_j ||Dhat_j||^2 = d (unit atoms, FP32-rounded)
    a = mf.normalised_atoms_f32(D.atoms).astype(np.complex128)
    assert abs(lam.sum() - np.sum(np.abs(a) ** 2)) < 1e-9 * D.d
    for k in range(24):
        i = int(np.argmax(np.abs(V[:, k])))
        assert abs(V[i, k].imag) < 1e-15 and V[i, k].real > 0
    # truncation keeps the leading eigenpairs of the same matrix
    V5, lam5 = subspace.dominant_subspace(D.atoms, 5)
    np.testing.assert_allclose(lam5, lam[:5], rtol=1e-12)
    np.testing.assert_allclose(np.abs(V5.conj().T @ V[:, :5]), np.eye(5), atol=1e-8)


def test_full_rank_step_equals_uncompressed_step():
    """s = L: V is unitary, so the compressed step is the uncompressed step in
    the rotated basis (same indices, same step statistics)."""
    D = workloads.fisp_dictionary(L=16, n_t1=8, n_t2=10)
    S, L, ny, nx = 1, 16, 8, 8
    V, _ = subspace.dominant_subspace(D.atoms, L)
    Dc = subspace.compress_atoms(D.atoms, V)
    smp = workloads.random_lines(3, S, L, ny, nx, 3)
    X0 = _cg(3, "x", (S, L, ny, nx)) * 0.1
    Y = fourier.forward(X0, smp.off, smp.idx) + 0.01 * _cg(3, "y", (smp.M,))
    Xp = _cg(3, "xp", (S, L, ny, nx))
    atoms32 = mf.normalised_atoms_f32(D.atoms).astype(np.complex128)
    X1, r1, s1 = ipg.ipg_step(Y, smp.off, smp.idx, atoms32, Xp, 0.7)
    X2, r2, s2 = ipg.ipg_step(Y, smp.off, smp.idx, Dc, subspace.compress(Xp, V), 0.7, V=V)
    np.testing.assert_array_equal(r1["idx"], r2["idx"])
    np.testing.assert_allclose(subspace.expand(X2, V), X1, atol=1e-10)
    for k in ("dx2", "adx2", "f_old", "f_new"):
        assert abs(s1[k] - s2[k]) <= 1e-9 * max(1.0, abs(s1[k]))


def test_rank_s_dictionary_gives_full_matched_filter():
    """Atoms spanning exactly s dimensions: compressing loses nothing, so the
    matched filter of compressed voxels equals the full one."""
    L, s, d = 40, 6, 300
    B = _cg(4, "basis", (s, L))
    atoms = _cg(4, "coef", (d, s)) @ B
    V, lam = subspace.dominant_subspace(atoms, s)
    Dc = subspace.compress_atoms(atoms, V)
    Z = _cg(4, "c", (50, s)) @ B + 0.0
    full = mf.exact_mf(Z, mf.normalised_atoms_f32(atoms).astype(np.complex128))
    comp = mf.exact_mf(Z @ V.conj(), Dc)
    np.testing.assert_array_equal(comp["idx"], full["idx"])
    np.testing.assert_allclose(comp["gamma"], full["gamma"], rtol=1e-9)


def test_compressed_operator_adjoint_identity():
    D = workloads.fisp_dictionary(L=20, n_t1=6, n_t2=8)
    V, _ = subspace.dominant_subspace(D.atoms, 5)
    S, ny, nx = 2, 16, 16
    smp = workloads.random_lines(5, S, 20, ny, nx, 4)
    x = _cg(5, "x", (S, 5, ny, nx))
    y = _cg(5, "y", (smp.M,))
    lhs = np.vdot(y, ipg.op_forward(x, smp.off, smp.idx, V))
    rhs = np.vdot(ipg.op_adjoint(y, smp.off, smp.idx, S, 5, ny, nx, V), x)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
