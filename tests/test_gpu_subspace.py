"""GPU parity of the temporal subspace compression (eq. CS1, eq. gradupdate,
eq. gradcompression) against the FP64 oracle, through the C ABI: the basis
V and its eigenvalues, the compressed atoms, the matched filter of
compressed voxels, a teacher-forced compressed projected-gradient step and a
short compressed solve."""
import numpy as np
import pytest

from gpu_helpers import banner, c64, dev, host
from oracle import fourier, ipg, mf, subspace
from synth import rng, workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def m():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1810_01967_amd as pkg
    pkg.lib()
    return pkg


def _cg(seed, tag, shape):
    n = int(np.prod(shape))
    g = rng.normal(seed, tag, 2 * n).reshape(tuple(shape) + (2,))
    return g[..., 0] + 1j * g[..., 1]


def _rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300)


def _check_basis(Vg, lg, Vo, lo):
    """Eigenvalues to FP64 rounding of the Gram matrix; the projector always;
    each column where its eigenvalue is separated from its neighbours."""
    s = Vo.shape[1]
    np.testing.assert_allclose(lg, lo, rtol=0, atol=1e-10 * lo[0])
    np.testing.assert_allclose(Vg.conj().T @ Vg, np.eye(s), atol=1e-10)
    assert np.linalg.norm(Vg @ Vg.conj().T - Vo @ Vo.conj().T) < 1e-7
    for k in range(s):
        gap = min(abs(lo[k] - lo[k - 1]) if k > 0 else np.inf, abs(lo[k] - lo[k + 1]) if k + 1 < s else np.inf)
        if gap > 1e-6 * lo[0]:
            np.testing.assert_allclose(Vg[:, k], Vo[:, k], atol=1e-8 * lo[0] / gap + 1e-12)


@pytest.mark.parametrize("kind,s", [("fisp", 10), ("fisp", 100), ("bssfp", 12)])
def test_compress_basis_and_atoms(m, kind, s):
    banner(f"subspace basis {kind} s={s}")
    if kind == "fisp":   # real atoms
        Dd = workloads.fisp_dictionary(L=100)
    else:                # complex atoms
        Dd = workloads.bssfp_dictionary(L=60, n_t1=12, n_t2=12, n_df=5, seed=2)
    atoms = Dd.atoms
    D = m.Dictionary(atoms, Dd.params, grid_dims=Dd.grid_dims)
    C = D.compress(s)
    inf = C.info()
    assert (inf.L, inf.L_full, inf.is_complex, inf.d) == (s, atoms.shape[1], 1, atoms.shape[0])
    Vg, lg = C.subspace()
    Vo, lo = subspace.dominant_subspace(atoms, s)
    _check_basis(Vg, lg, Vo, lo)
    # compressed atoms as stored (FP32 rows of the FP64-normalised V^H Dhat_j)
    got = host(m.mrf_dict_copy_atoms(C, "fp32")).view(np.complex64).astype(np.complex128)
    ref = subspace.compress_atoms(atoms, Vo)
    ref /= np.linalg.norm(ref, axis=1, keepdims=True)
    # coordinates on the well-separated eigenvectors; all of them through the
    # (basis-independent) expansion V Dtilde_j
    sep = [k for k in range(s) if min(abs(lo[k] - lo[k - 1]) if k else np.inf,
                                      abs(lo[k] - lo[k + 1]) if k + 1 < s else np.inf) > 1e-6 * lo[0]]
    assert np.max(np.abs(got[:, sep] - ref[:, sep])) < 2e-6
    assert np.max(np.abs(got @ Vg.T - ref @ Vo.T)) < 2e-6


def test_compressed_matched_filter(m):
    """Noisy atoms compressed with the oracle's V: the GPU filter over the
    compressed dictionary against the oracle's filter over the compressed
    atoms (indices up to near ties, PD)."""
    banner("subspace matched filter FISP L=100 s=10, 3000 voxels")
    Dd = workloads.fisp_dictionary(L=100)
    D = m.Dictionary(Dd.atoms, Dd.params, grid_dims=Dd.grid_dims)
    C = D.compress(10)
    Vo, _ = subspace.dominant_subspace(Dd.atoms, 10)
    Z, _, _, _ = workloads.random_voxels(Dd, 3000, seed=4)
    Zc = Z.astype(np.complex128) @ Vo.conj()
    out = m.mrf_match(C, dev(c64(Zc)))
    Dc = subspace.compress_atoms(Dd.atoms, Vo)
    ref = mf.exact_mf(Zc, Dc)
    gidx = host(out["idx"]).astype(np.int64)
    diff = gidx != ref["idx"]
    print(f"compressed filter: {int(diff.sum())} index differences of {len(gidx)}")
    assert diff.mean() < 0.01
    if diff.any():
        assert np.all(mf.index_ok(c64(Zc[diff]), Dc, gidx[diff], tol=1e-6))
    np.testing.assert_allclose(host(out["pd"])[~diff], ref["gamma"][~diff], rtol=1e-4, atol=1e-6)


def _fisp_problem(seed=1, L=100, size=64, nlines=6, snr=30.0, S=1):
    Dd = workloads.fisp_dictionary(L=L)
    if S == 1:
        ph = workloads.disc_phantom(Dd, seed=seed, size=size, snap=True)
    else:
        ph = workloads.smooth_phantom(Dd, seed=seed, S=S, size=size)
    smp = workloads.random_lines(seed, S, L, size, size, nlines)
    Y = workloads.simulate_kspace(ph.X0, smp, snr, seed)
    return Dd, ph, smp, c64(Y)


@pytest.mark.parametrize("S,s", [(1, 10), (2, 20)])
def test_compressed_step_teacher_forced(m, S, s):
    """One compressed step from the same compressed iterate on both sides:
    objective, projection indices (near-tie rule), PD, X~' and the step
    statistics of the compressed step rule."""
    banner(f"subspace ipg step teacher-forced S={S} 64x64 L=100 s={s}")
    Dd, ph, smp, Y = _fisp_problem(S=S)
    D = m.Dictionary(Dd.atoms, Dd.params, grid_dims=Dd.grid_dims)
    C = D.compress(s)
    A = m.Operator.from_sampling(smp)
    Vo, _ = subspace.dominant_subspace(Dd.atoms, s)
    Dc = subspace.compress_atoms(Dd.atoms, Vo)
    X1, _, _, _ = ipg.ipg_solve(Y, smp.off, smp.idx, (S, s, 64, 64), Dc, mu0=1.0, adaptive=False, max_iter=1,
                                rel_tol=0, V=Vo)
    Xk = c64(X1)
    for mu in (1.0, 64 / 6):
        Xn, idx, pd, st = m.mrf_ipg_step(C, A, dev(Y), dev(Xk), mu)
        Xr, res, sr = ipg.ipg_step(Y, smp.off, smp.idx, Dc, Xk.astype(np.complex128), mu, V=Vo)
        gidx = host(idx)
        diff = gidx != res["idx"]
        Zv = fourier.frame_to_voxel(res["Z"])
        print(f"mu={mu:.3f}: {int(diff.sum())} index differences; f_in {st.f_in:.6e} / {sr['f_old']:.6e}")
        assert abs(st.f_in - sr["f_old"]) <= 2e-5 * sr["f_old"]
        if diff.any():
            assert np.all(mf.index_ok(Zv[diff], Dc, gidx[diff], tol=1e-6))
        np.testing.assert_allclose(host(pd)[~diff], res["gamma"][~diff], rtol=1e-4, atol=1e-6)
        if not diff.any():
            assert _rel(host(Xn), Xr) < 1e-5
            for k, g in (("dx2", st.dx2), ("adx2", st.adx2), ("f_new", st.f_out)):
                assert abs(g - sr[k]) <= 1e-4 * abs(sr[k]) + 1e-12, (k, g, sr[k])


def test_compressed_full_rank_matches_uncompressed(m):
    """s = L: V is unitary, so the compressed step expands to the
    uncompressed step (same indices up to near ties, same statistics)."""
    banner("subspace s = L step vs uncompressed step, 64x64 L=100")
    Dd, ph, smp, Y = _fisp_problem()
    D = m.Dictionary(Dd.atoms, Dd.params, grid_dims=Dd.grid_dims)
    C = D.compress(100)
    A = m.Operator.from_sampling(smp)
    Vg, _ = C.subspace()
    X0 = c64(_cg(7, "x", (1, 100, 64, 64)) * 0.01)
    Xu, iu, pu, su = m.mrf_ipg_step(D, A, dev(Y), dev(X0), 2.0)
    X0c = c64(subspace.compress(X0.astype(np.complex128), Vg))
    Xc, ic, pc, sc = m.mrf_ipg_step(C, A, dev(Y), dev(X0c), 2.0)
    agree = np.mean(host(iu) == host(ic))
    print(f"s = L: index agreement {agree:.5f}; f_in {su.f_in:.6e} / {sc.f_in:.6e}; dx2 {su.dx2:.6e} / {sc.dx2:.6e}")
    assert agree > 0.995
    assert abs(su.f_in - sc.f_in) <= 1e-4 * su.f_in
    assert abs(su.f_out - sc.f_out) <= 1e-3 * su.f_out
    assert _rel(subspace.expand(host(Xc).astype(np.complex128), Vg), host(Xu)) < 0.03


@pytest.mark.parametrize("adaptive", [False, True])
def test_compressed_solve(m, adaptive):
    """Ten iterations of the compressed solve against the oracle's compressed
    solve (mu = 1 fixed, or adaptive from mu0 = n/m), and the reconstruction
    error against the uncompressed GPU solve.  At a fixed mu the two runs
    follow the same path (indices, objective history); with the adaptive
    rule, FP32 / FP64 argmax flips at near-ties (frequent among compressed
    atoms, whose T2 neighbours differ little in 10 dimensions) change later
    step sizes, so the end states are compared by objective and error (each
    single step is checked teacher-forced above)."""
    banner(f"subspace ipg solve 64x64 L=100 s=10 adaptive={adaptive}")
    Dd, ph, smp, Y = _fisp_problem()
    D = m.Dictionary(Dd.atoms, Dd.params, grid_dims=Dd.grid_dims)
    C = D.compress(10)
    A = m.Operator.from_sampling(smp)
    Vo, _ = subspace.dominant_subspace(Dd.atoms, 10)
    Dc = subspace.compress_atoms(Dd.atoms, Vo)
    mu0 = 64 / 6 if adaptive else 1.0
    Xc, idx, pd, params, hist = m.mrf_ipg_solve(C, A, dev(Y), mu0=mu0, zeta=2.0, adaptive=adaptive, max_iter=10,
                                                rel_tol=0.0)
    Xr, idr, gr, hr = ipg.ipg_solve(Y, smp.off, smp.idx, (1, 10, 64, 64), Dc, mu0=mu0, zeta=2.0,
                                    adaptive=adaptive, max_iter=10, rel_tol=0, V=Vo)
    Xu, iu, pu, _, hu = m.mrf_ipg_solve(D, A, dev(Y), mu0=mu0, zeta=2.0, adaptive=adaptive, max_iter=10,
                                        rel_tol=0.0)
    Vg, _ = C.subspace()
    gidx = host(idx)
    inside = ph.idx >= 0
    fr = np.array([h["f"] for h in hr])
    nm_c = _rel(subspace.expand(host(Xc).astype(np.complex128), Vg), ph.X0)
    nm_o = _rel(subspace.expand(Xr, Vo), ph.X0)
    nm_u = _rel(host(Xu), ph.X0)
    agree = np.mean(gidx[inside] == idr[inside])
    print(f"compressed solve: object agreement {agree:.4f}; f gpu {np.array2string(hist['f'], precision=4)} "
          f"oracle {np.array2string(fr, precision=4)}; nmse compressed {nm_c:.4e} oracle {nm_o:.4e} "
          f"uncompressed {nm_u:.4e}; {hist['ms']:.1f} ms vs {hu['ms']:.1f} ms uncompressed")
    assert hist["iters"] == 10
    np.testing.assert_array_equal(host(params), Dd.params[gidx].astype(np.float32))
    if not adaptive:
        assert agree > 0.99
        np.testing.assert_allclose(hist["f"], fr, rtol=2e-3)
        assert abs(nm_c - nm_o) < 0.05 * nm_o + 1e-4
    else:
        assert np.all(np.diff(hist["f"]) <= 1e-6 * hist["f"][:-1])
        assert abs(hist["f"][-1] - fr[-1]) < 0.03 * fr[-1]
        assert abs(nm_c - nm_o) < 0.2 * nm_o
        assert nm_c < 1.25 * nm_u


def test_compress_argument_errors(m):
    banner("subspace argument errors")
    Dd = workloads.fisp_dictionary(L=20, n_t1=6, n_t2=8)
    D = m.Dictionary(Dd.atoms, Dd.params)
    for bad in (0, 21, -3):
        with pytest.raises(m.MrfError):
            D.compress(bad)
    C = D.compress(5)
    with pytest.raises(m.MrfError):
        C.compress(3)
    with pytest.raises(m.MrfError):
        D.subspace()
    smp = workloads.random_lines(2, 1, 5, 16, 16, 3)   # operator of 5 frames, C expects 20
    A = m.Operator.from_sampling(smp)
    import torch
    X = torch.zeros((1, 5, 16, 16), dtype=torch.complex64, device="cuda")
    Y = torch.zeros(smp.M, dtype=torch.complex64, device="cuda")
    with pytest.raises(m.MrfError):
        m.mrf_ipg_step(C, A, Y, X, 1.0)
