"""Pins of the multi-coil forward model (eq. forward with c coils): one coil
with unit maps is the single-coil operator, the adjoint identity, c equal
maps 1/sqrt(c) give the single-coil normal operator, sum-of-squares
normalised maps with full sampling give A^H A = I (one-step recovery of a
noiseless fingerprint image), the gradient by central differences, and the
coil maps' normalisation."""
import numpy as np

from oracle import fourier, ipg, mf
from synth import rng, workloads


def _cg(seed, tag, shape):
    n = int(np.prod(shape))
    g = rng.normal(seed, tag, 2 * n).reshape(tuple(shape) + (2,))
    return g[..., 0] + 1j * g[..., 1]


def test_coil_maps_sum_of_squares():
    sm = workloads.coil_maps(3, 2, 6, 32, 16)
    assert sm.shape == (2, 6, 32, 16)
    np.testing.assert_allclose(np.sum(np.abs(sm) ** 2, axis=1), 1.0, atol=1e-12)
    # smooth, genuinely coil-dependent profiles
    assert np.std(np.abs(sm[0, 0])) > 0.05 and np.max(np.abs(sm[0, 0] - sm[0, 1])) > 0.1


def test_one_unit_coil_is_single_coil():
    S, L, ny, nx = 2, 3, 16, 16
    smp = workloads.random_lines(1, S, L, ny, nx, 5)
    X = _cg(1, "x", (S, L, ny, nx))
    ones = np.ones((S, 1, ny, nx), dtype=np.complex128)
    np.testing.assert_array_equal(fourier.forward_coils(X, smp.off, smp.idx, ones)[0],
                                  fourier.forward(X, smp.off, smp.idx))
    R = _cg(1, "r", (smp.M,))
    np.testing.assert_allclose(fourier.adjoint_coils(R[None], smp.off, smp.idx, S, L, ny, nx, ones),
                               fourier.adjoint(R, smp.off, smp.idx, S, L, ny, nx), atol=1e-15)


def test_coil_adjoint_identity():
    S, L, ny, nx, c = 2, 4, 16, 32, 5
    smp = workloads.random_lines(2, S, L, ny, nx, 6)
    sm = workloads.coil_maps(2, S, c, ny, nx)
    X = _cg(2, "x", (S, L, ny, nx))
    R = _cg(2, "r", (c, smp.M))
    lhs = np.vdot(R, ipg.op_forward(X, smp.off, smp.idx, smaps=sm))
    rhs = np.vdot(ipg.op_adjoint(R, smp.off, smp.idx, S, L, ny, nx, smaps=sm), X)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_equal_maps_give_single_coil_normal_operator():
    """S_q = 1/sqrt(c) for all q: sum_q |S_q|^2 = 1, so A^H A and ||A X||^2
    equal the single-coil ones although each coil sees X / sqrt(c)."""
    S, L, ny, nx, c = 1, 3, 16, 16, 4
    smp = workloads.random_lines(3, S, L, ny, nx, 4)
    sm = np.full((S, c, ny, nx), 1.0 / np.sqrt(c), dtype=np.complex128)
    X = _cg(3, "x", (S, L, ny, nx))
    AX = ipg.op_forward(X, smp.off, smp.idx, smaps=sm)
    AX1 = fourier.forward(X, smp.off, smp.idx)
    assert abs(np.sum(np.abs(AX) ** 2) - np.sum(np.abs(AX1) ** 2)) <= 1e-12 * np.sum(np.abs(AX1) ** 2)
    np.testing.assert_allclose(ipg.op_adjoint(AX, smp.off, smp.idx, S, L, ny, nx, smaps=sm),
                               fourier.adjoint(AX1, smp.off, smp.idx, S, L, ny, nx), atol=1e-12)


def test_full_sampling_one_step_recovery_with_coils():
    """Every k-space location sampled and sum_q |S_q|^2 = 1: A^H A = I, so
    from X = 0 one step at mu = 1 projects X0 itself and recovers a
    noiseless image built from atoms exactly (indices and PD)."""
    D = workloads.fisp_dictionary(L=12, n_t1=6, n_t2=6)
    S, ny, nx, c = 1, 16, 16, 4
    ph = workloads.disc_phantom(D, seed=4, size=16, radius=6.0, snap=True)
    X0 = ph.X0
    full = workloads.random_lines(4, S, D.L, ny, nx, ny)
    sm = workloads.coil_maps(4, S, c, ny, nx)
    Y = workloads.simulate_kspace(X0, full, None, 4, smaps=sm)
    atoms = mf.normalised_atoms_f32(D.atoms).astype(np.complex128)
    X1, res, st = ipg.ipg_step(Y, full.off, full.idx, atoms, np.zeros_like(X0), 1.0, smaps=sm)
    inside = ph.idx >= 0
    np.testing.assert_array_equal(res["idx"][inside], ph.idx[inside])
    assert np.max(np.abs(X1 - X0)) < 1e-6 * np.max(np.abs(X0))
    assert st["f_new"] < 1e-12 * st["f_old"]


def test_coil_gradient_central_differences():
    """f(X) = ||A X - Y||_W^2 with coils and DCF weights: the directional
    derivative along E equals 2 Re<G, E> for G = A^H W (A X - Y)."""
    S, L, ny, nx, c = 1, 3, 8, 8, 3
    smp = workloads.random_lines(5, S, L, ny, nx, 3)
    sm = workloads.coil_maps(5, S, c, ny, nx)
    w = rng.uniform(5, "w", smp.M, 0.5, 2.0)
    X = _cg(5, "x", (S, L, ny, nx))
    Y = _cg(5, "y", (c, smp.M))
    E = _cg(5, "e", (S, L, ny, nx))
    G, _ = ipg.gradient(X, Y, smp.off, smp.idx, w, smaps=sm)

    def f(Xt):
        R = ipg.op_forward(Xt, smp.off, smp.idx, smaps=sm) - Y
        return float(np.sum(w * np.abs(R) ** 2))

    h = 1e-5
    fd = (f(X + h * E) - f(X - h * E)) / (2 * h)
    assert abs(fd - 2 * np.real(np.vdot(G, E))) <= 1e-7 * abs(fd)
