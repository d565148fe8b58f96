"""Pins of the non-Cartesian forward model (eq. forward with a non-uniform
Fourier transform): a brute-force triple loop on a tiny case, equality with
the unitary DFT at grid frequencies, the adjoint identity (with coils), the
synthetic k-space generator against the oracle, and the spiral's Voronoi
density compensation (mean 1, small at the dense centre)."""
import numpy as np

from oracle import fourier, ipg, nudft
from synth import rng, workloads


def _cg(seed, tag, shape):
    n = int(np.prod(shape))
    g = rng.normal(seed, tag, 2 * n).reshape(tuple(shape) + (2,))
    return g[..., 0] + 1j * g[..., 1]


def test_brute_force_tiny():
    ny, nx = 4, 8
    X = _cg(1, "x", (1, 1, ny, nx))
    k = rng.uniform(1, "k", 10, -0.5, 0.5).reshape(5, 2)
    off = np.array([0, 5])
    got = nudft.forward(X, off, k)
    for i in range(5):
        acc = 0j
        for y in range(ny):
            for x in range(nx):
                acc += X[0, 0, y, x] * np.exp(-2j * np.pi * (k[i, 0] * y + k[i, 1] * x))
        assert abs(got[i] - acc / np.sqrt(ny * nx)) < 1e-12


def test_grid_frequencies_give_the_unitary_dft():
    S, L, ny, nx = 2, 3, 16, 32
    smp = workloads.random_lines(2, S, L, ny, nx, 5)
    ky, kx = smp.idx // nx, smp.idx % nx
    k = np.stack([ky / ny, kx / nx], axis=1)
    k = np.where(k >= 0.5, k - 1.0, k)          # the same frequencies in [-0.5, 0.5)
    X = _cg(2, "x", (S, L, ny, nx))
    np.testing.assert_allclose(nudft.forward(X, smp.off, k), fourier.forward(X, smp.off, smp.idx), atol=1e-12)
    R = _cg(2, "r", (smp.M,))
    np.testing.assert_allclose(nudft.adjoint(R, smp.off, k, S, L, ny, nx),
                               fourier.adjoint(R, smp.off, smp.idx, S, L, ny, nx), atol=1e-12)


def test_adjoint_identity_with_coils():
    S, L, ny, nx, c = 1, 3, 16, 16, 3
    tr = workloads.spiral_trajectory(S, L, ny, nx, frac=0.3)
    sm = workloads.coil_maps(3, S, c, ny, nx)
    X = _cg(3, "x", (S, L, ny, nx))
    R = _cg(3, "r", (c, tr.M))
    lhs = np.vdot(R, ipg.op_forward(X, tr.off, None, smaps=sm, coords=tr.coords))
    rhs = np.vdot(ipg.op_adjoint(R, tr.off, None, S, L, ny, nx, smaps=sm, coords=tr.coords), X)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_simulated_kspace_matches_the_oracle():
    S, L, ny, nx = 1, 2, 16, 16
    tr = workloads.spiral_trajectory(S, L, ny, nx, frac=0.2)
    X = _cg(4, "x", (S, L, ny, nx))
    np.testing.assert_allclose(workloads.simulate_kspace_nc(X, tr, None, 4), nudft.forward(X, tr.off, tr.coords),
                               atol=1e-12)


def test_spiral_density_compensation():
    tr = workloads.spiral_trajectory(1, 2, 64, 64, frac=0.05)
    assert tr.coords.dtype == np.float32
    assert np.all(tr.coords >= -0.5) and np.all(tr.coords < 0.5)
    for p in range(2):
        w = tr.dcf[tr.off[p]:tr.off[p + 1]]
        r = np.hypot(*tr.coords[tr.off[p]:tr.off[p + 1]].T)
        assert abs(w.mean() - 1.0) < 1e-12
        # denser sampling near the centre gets smaller weights
        assert np.median(w[r < 0.1]) < 0.5 * np.median(w[r > 0.3])
