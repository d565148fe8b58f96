"""Pins of the FP64 oracle against what the paper and the mathematics fix:
brute force on tiny inputs, closed forms, invariants and special cases."""
import numpy as np
import pytest

from oracle import fourier, ipg, mf, quant
from synth import rng, workloads


def _rand_complex(seed, tag, shape):
    n = int(np.prod(shape))
    g = rng.normal(seed, tag, 2 * n).reshape(tuple(shape) + (2,))
    return g[..., 0] + 1j * g[..., 1]


# --- exact matched filter (eq. exactP, exactPs) -----------------------------
def _brute_force_projection(z, atoms):
    """Definition written out: nearest normalised atom by Euclidean distance,
    then gamma = max(Re<z, D>/||D||^2, 0) with explicit sums."""
    best, bj = np.inf, -1
    for j in range(atoms.shape[0]):
        nj = np.sqrt(sum(abs(a) ** 2 for a in atoms[j]))
        dist = np.sqrt(sum(abs(z[t] - atoms[j][t] / nj) ** 2 for t in range(len(z))))
        if dist < best:
            best, bj = dist, j
    nj2 = sum(abs(a) ** 2 for a in atoms[bj])
    inner = sum(z[t] * np.conj(atoms[bj][t]) for t in range(len(z)))
    gamma = max(inner.real / nj2, 0.0)
    return bj, gamma


@pytest.mark.parametrize("complex_atoms", [True, False])
def test_mf_matches_brute_force(complex_atoms):
    d, L, n = 23, 9, 40
    atoms = _rand_complex(1, "a", (d, L)) if complex_atoms else rng.normal(1, "a", d * L).reshape(d, L)
    atoms = atoms * rng.uniform(1, "s", d, 0.2, 3.0)[:, None]
    Z = _rand_complex(1, "z", (n, L))
    res = mf.exact_mf(Z, atoms, want_X=True)
    for v in range(n):
        j, g = _brute_force_projection(Z[v] if complex_atoms else Z[v], atoms)
        if not complex_atoms:
            # real atoms: the distance to a real atom ranks like that of Re(z)
            j, g = _brute_force_projection(Z[v].real + 0j, atoms)
        assert res["idx"][v] == j
        assert abs(res["gamma"][v] - g) <= 1e-12 * max(1.0, g)
        assert np.allclose(res["X"][v], g * atoms[j], atol=1e-12)


def test_mf_against_library_product():
    d, L, n = 64, 33, 200
    atoms = _rand_complex(2, "a", (d, L))
    Z = _rand_complex(2, "z", (n, L))
    res = mf.exact_mf(Z, atoms)
    A = atoms / np.linalg.norm(atoms, axis=1, keepdims=True)
    ip = np.real(np.conj(A) @ Z.T).T               # <Z, D^> = sum Z conj(D^)
    assert np.array_equal(res["idx"], np.argmax(ip, axis=1))


def test_mf_noiseless_recovers_atom_and_pd():
    D = workloads.fisp_dictionary(L=100)
    j = rng.randint(3, "j", 300, D.d)
    pd = rng.uniform(3, "pd", 300, 0.3, 1.0)
    Z = pd[:, None] * D.atoms[j]
    res = mf.exact_mf(Z.astype(np.complex128), D.atoms)
    assert np.array_equal(res["idx"], j)
    assert np.max(np.abs(res["gamma"] - pd) / pd) < 1e-14


def test_mf_invariances():
    d, L, n = 31, 12, 50
    atoms = _rand_complex(4, "a", (d, L))
    Z = _rand_complex(4, "z", (n, L))
    r1 = mf.exact_mf(Z, atoms)
    r2 = mf.exact_mf(3.7 * Z, atoms)
    assert np.array_equal(r1["idx"], r2["idx"])
    assert np.allclose(r2["gamma"], 3.7 * r1["gamma"], rtol=1e-13)
    # Z = -D_j: every correlation with D_j is negative, so gamma = 0 for it
    r3 = mf.exact_mf(-atoms[:1], atoms[:1])
    assert r3["gamma"][0] == 0.0
    # duplicated atoms: the lowest index wins
    dup = np.concatenate([atoms, atoms[5:6]], axis=0)
    r4 = mf.exact_mf(atoms[5:6] * 2.0, dup)
    assert r4["idx"][0] == 5
    # zero voxel keeps its warm index, gamma 0, corr 0
    r5 = mf.exact_mf(np.zeros((2, L), complex), atoms, warm_idx=np.array([7, 3]))
    assert list(r5["idx"]) == [7, 3] and np.all(r5["gamma"] == 0) and np.all(r5["corr"] == 0)


def test_mf_real_part_not_magnitude():
    # a voxel equal to i*D_j has |<z, D_j>| maximal but Re<z, D_j> = 0:
    # the projection uses the real part (PD real and positive)
    atoms = np.array([[1.0, 0.0], [0.6, 0.8]], dtype=complex)
    z = np.array([[1j, 0.0]])
    res = mf.exact_mf(z, atoms)
    assert res["idx"][0] == 0 and res["gamma"][0] == 0.0
    z2 = np.array([[0.0, 1.0 + 0j]])
    assert mf.exact_mf(z2, atoms)["idx"][0] == 1


# --- Fourier operator --------------------------------------------------------
@pytest.mark.parametrize("ny,nx", [(8, 8), (16, 16), (8, 16)])
def test_fft_equals_dft_sum(ny, nx):
    x = _rand_complex(5, "x", (ny, nx))
    ref = np.zeros((ny, nx), dtype=complex)
    for ky in range(ny):
        for kx in range(nx):
            acc = 0j
            for y in range(ny):
                for xx in range(nx):
                    acc += x[y, xx] * np.exp(-2j * np.pi * (ky * y / ny + kx * xx / nx))
            ref[ky, kx] = acc / np.sqrt(ny * nx)
    assert np.max(np.abs(fourier.fft2_unitary(x) - ref)) < 1e-12
    assert np.max(np.abs(fourier.ifft2_unitary(ref) - x)) < 1e-12


def test_parseval_and_adjoint():
    S, L, ny, nx = 2, 5, 16, 16
    smp = workloads.random_lines(7, S, L, ny, nx, 4)
    X = _rand_complex(7, "x", (S, L, ny, nx))
    Yr = _rand_complex(7, "y", (smp.M,))
    assert abs(np.linalg.norm(fourier.fft2_unitary(X)) - np.linalg.norm(X)) < 1e-12 * np.linalg.norm(X)
    AX = fourier.forward(X, smp.off, smp.idx)
    AhY = fourier.adjoint(Yr, smp.off, smp.idx, S, L, ny, nx)
    lhs = np.vdot(Yr, AX)          # <Ax, y>
    rhs = np.vdot(AhY, X)          # <x, A^H y>
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)


# --- projected gradient ------------------------------------------------------
def _small_problem(seed=11, L=20, size=16, nlines=4, snr=None):
    D = workloads.fisp_dictionary(L=L, n_t1=12, n_t2=10)
    ph = workloads.disc_phantom(D, seed=seed, size=size, radius=6.5)
    smp = workloads.random_lines(seed, 1, L, size, size, nlines)
    Y = workloads.simulate_kspace(ph.X0, smp, snr, seed)
    return D, ph, smp, Y


def test_ipg_full_sampling_one_step_recovers_truth():
    D, ph, _, _ = _small_problem()
    smp = workloads.random_lines(1, 1, D.L, 16, 16, 16)       # every line
    Y = workloads.simulate_kspace(ph.X0, smp, None, 1)
    X, idx, gamma, hist = ipg.ipg_solve(Y, smp.off, smp.idx, (1, D.L, 16, 16), D.atoms,
                                        mu0=1.0, adaptive=False, max_iter=1, rel_tol=0)
    assert np.max(np.abs(X - ph.X0)) < 1e-12
    inside = ph.idx >= 0
    assert np.array_equal(idx[inside], ph.idx[inside])


def test_ipg_truth_is_fixed_point():
    D, ph, smp, Y = _small_problem()
    X, res, st = ipg.ipg_step(Y, smp.off, smp.idx, D.atoms, ph.X0, mu=16 / 4)
    assert np.max(np.abs(X - ph.X0)) < 1e-12
    assert st["f_old"] < 1e-24 and st["dx2"] < 1e-24


def test_ipg_template_matching_is_first_iteration():
    D, ph, smp, Y = _small_problem(snr=30.0)
    S, L, ny, nx = 1, D.L, 16, 16
    X1, _, _, _ = ipg.ipg_solve(Y, smp.off, smp.idx, (S, L, ny, nx), D.atoms, mu0=1.0,
                                adaptive=False, max_iter=1, rel_tol=0)
    bpi = fourier.adjoint(Y, smp.off, smp.idx, S, L, ny, nx)       # A^H Y
    Xtm, _ = ipg.project(bpi, D.atoms)
    assert np.max(np.abs(X1 - Xtm)) < 1e-12


def test_ipg_adaptive_monotone():
    D, ph, smp, Y = _small_problem(snr=25.0, nlines=3)
    S, L, ny, nx = 1, D.L, 16, 16
    X, idx, gamma, hist = ipg.ipg_solve(Y, smp.off, smp.idx, (S, L, ny, nx), D.atoms,
                                        mu0=16 / 3, zeta=2.0, adaptive=True, max_iter=12, rel_tol=0)
    f = [h["f"] for h in hist]
    assert all(f[i + 1] <= f[i] * (1 + 1e-12) for i in range(len(f) - 1))
    for h in hist:
        assert h["dx2"] == 0 or h["adx2"] == 0 or h["mu"] < h["dx2"] / h["adx2"]


def test_dcf_gradient_is_weighted_least_squares_gradient():
    # eq. blip_dcf: the gradient of f(X) = sum w |A X - Y|^2 is 2 A^H W (A X - Y);
    # checked by central differences along random directions
    S, L, ny, nx = 1, 3, 8, 8
    smp = workloads.spiral_sampling(S, L, ny, nx, frac=0.3)
    X = _rand_complex(9, "x", (S, L, ny, nx))
    Y = _rand_complex(9, "y", (smp.M,))
    w = smp.dcf

    def f(Xv):
        r = fourier.forward(Xv, smp.off, smp.idx) - Y
        return float(np.sum(w * np.abs(r) ** 2))

    G, _ = ipg.gradient(X, Y, smp.off, smp.idx, w)
    for k in range(3):
        Dir = _rand_complex(9, f"d{k}", X.shape)
        h = 1e-6
        num = (f(X + h * Dir) - f(X - h * Dir)) / (2 * h)
        ana = 2 * np.real(np.vdot(G, Dir))
        assert abs(num - ana) < 1e-6 * max(1.0, abs(ana))


# --- precision forms ---------------------------------------------------------
def test_bf16_matches_library_conversion():
    import torch
    bits = np.concatenate([
        (np.arange(-2 ** 20, 2 ** 20, 37, dtype=np.int64) + (e << 23)) for e in (1, 60, 126, 127, 128, 200, 253)
    ]).astype(np.uint32)
    x = bits.view(np.float32)
    x = np.concatenate([x, -x])
    x = x[np.isfinite(x)]
    ref = torch.from_numpy(x.copy()).to(torch.bfloat16).float().numpy()
    assert np.array_equal(quant.bf16_round(x), ref)


def test_e4m3_matches_library_conversion():
    import torch
    x = np.concatenate([np.linspace(-448, 448, 200001), 2.0 ** -np.arange(0, 12, 0.01),
                        (2.0 ** -9) * np.arange(0, 20, 0.5)]).astype(np.float32)
    v = quant.e4m3_value(x)
    t = torch.from_numpy(x.copy()).to(torch.float8_e4m3fn)
    assert np.array_equal(v, t.float().numpy().astype(np.float64))
    assert np.array_equal(quant.e4m3_code(v), t.view(torch.uint8).numpy())
    assert np.array_equal(quant.e4m3_decode(quant.e4m3_code(v)), v)
    # saturation beyond the largest finite value
    assert quant.e4m3_value(np.array([1e6, -900.0], np.float32)).tolist() == [448.0, -448.0]


def test_quantised_match_full_topk_is_exact():
    # with k = d every atom is rescored, so the answer is the exact matched
    # filter of the FP32 operands
    d, L, n = 40, 16, 60
    atoms = _rand_complex(12, "a", (d, L))
    Z = _rand_complex(12, "z", (n, L)).astype(np.complex64)
    Dhat = mf.normalised_atoms_f32(atoms)
    for prec in ("bf16", "fp8"):
        r = quant.quantised_match(quant.as_real_rows(Z), quant.as_real_rows(Dhat), prec, topk=d)
        ex = mf.exact_mf(Z.astype(np.complex128), Dhat.astype(np.complex128))
        assert np.array_equal(r["idx"], ex["idx"])


def test_quantised_match_recovers_noiseless_atoms():
    D = workloads.bssfp_dictionary(L=40, n_t1=8, n_t2=8, n_df=5, seed=2)
    j = rng.randint(13, "j", 200, D.d)
    Z = (rng.uniform(13, "pd", 200, 0.3, 1.0)[:, None] * D.atoms[j]).astype(np.complex64)
    Dhat = mf.normalised_atoms_f32(D.atoms)
    for prec in ("bf16", "fp8"):
        r = quant.quantised_match(quant.as_real_rows(Z), quant.as_real_rows(Dhat), prec, topk=8)
        assert np.array_equal(r["idx"], j)


def test_quantised_score_error_bound():
    """The certificate's bound on reduced-precision scores: with q the decoded
    voxel row and r_j the decoded atom row, |<q, r_j> - <z, d_j>| <=
    ||z - q|| ||r_j|| + ||z|| ||d_j - r_j|| (Cauchy-Schwarz on the two error
    terms of q r - z d = (q - z) r + z (r - d)).  Checked on every pair of a
    coherent dictionary; dropping either term is caught."""
    D = workloads.bssfp_dictionary(L=60, n_t1=12, n_t2=12, n_df=7, seed=2)
    Z, _, _, _ = workloads.random_voxels(D, 300, seed=14, snr_db_range=(10.0, 40.0))
    zr = quant.as_real_rows(Z.astype(np.complex64)).astype(np.float32)
    dr = quant.as_real_rows(mf.normalised_atoms_f32(D.atoms)).astype(np.float32)
    s = zr.astype(np.float64) @ dr.astype(np.float64).T
    for prec in ("bf16", "fp8"):
        if prec == "bf16":
            zq, dq = quant.bf16_round(zr).astype(np.float64), quant.bf16_round(dr).astype(np.float64)
        else:
            zq, dq = quant.quantise_rows_e4m3(zr)[2], quant.quantise_rows_e4m3(dr)[2]
        err = np.abs(zq @ dq.T - s)
        ez = np.linalg.norm(zr - zq, axis=1)[:, None]
        qn = np.linalg.norm(dq, axis=1)[None, :]
        zn = np.linalg.norm(zr, axis=1)[:, None]
        ed = np.linalg.norm(dr - dq, axis=1)[None, :]
        bound = ez * qn + zn * ed
        assert np.all(err <= bound * (1 + 1e-12))
        # the bound is not vacuous: it is within two orders of the worst error
        assert np.max(err / bound) > 0.01
    # each term is needed: with BF16-exact atoms (d = r) only the voxel term
    # remains, with BF16-exact voxels (z = q) only the atom term, and both
    # errors are non-zero
    db = quant.bf16_round(dr)
    zb = quant.bf16_round(zr)
    err_v = np.abs(quant.bf16_round(zr).astype(np.float64) @ db.astype(np.float64).T
                   - zr.astype(np.float64) @ db.astype(np.float64).T)
    err_a = np.abs(zb.astype(np.float64) @ quant.bf16_round(dr).astype(np.float64).T
                   - zb.astype(np.float64) @ dr.astype(np.float64).T)
    assert np.max(err_v) > 0 and np.max(err_a) > 0
