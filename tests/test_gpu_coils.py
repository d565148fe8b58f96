"""GPU parity of the multi-coil forward model (eq. forward with c coils and
sensitivity maps) against the FP64 oracle, through the C ABI: operator
forward / adjoint, teacher-forced projected-gradient steps (plain, DCF,
temporally compressed) and a short solve."""
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


@pytest.mark.parametrize("S,L,ny,nx,c,kind", [(2, 5, 64, 64, 4, "lines"), (1, 6, 32, 16, 3, "spiral"),
                                              (3, 3, 16, 32, 1, "lines"), (1, 4, 128, 128, 8, "lines")])
def test_coil_operator_forward_adjoint(m, S, L, ny, nx, c, kind):
    banner(f"coil operator S={S} L={L} {ny}x{nx} c={c} {kind}")
    smp = (workloads.random_lines(41, S, L, ny, nx, max(2, ny // 10)) if kind == "lines"
           else workloads.spiral_sampling(S, L, ny, nx, frac=0.2))
    sm = workloads.coil_maps(41, S, c, ny, nx)
    A = m.Operator.from_sampling(smp, smaps=sm)
    smc = c64(sm).astype(np.complex128)          # the maps as the device holds them
    X = c64(_cg(41, "x", (S, L, ny, nx)))
    Y = c64(_cg(41, "y", (c, smp.M)))
    R, nrm = m.mrf_op_forward(A, dev(X), dev(Y), want_norm=True)
    ref = ipg.op_forward(X.astype(np.complex128), smp.off, smp.idx, smaps=smc) - Y
    assert host(R).shape == (c, smp.M)
    assert _rel(host(R), ref) < 3e-6
    w = smp.dcf if smp.dcf is not None else np.ones(smp.M)
    assert abs(nrm - np.sum(w * np.abs(ref) ** 2)) < 1e-5 * np.sum(w * np.abs(ref) ** 2)
    G = m.mrf_op_adjoint(A, dev(Y), apply_dcf=True)
    gref = ipg.op_adjoint(Y.astype(np.complex128) * w, smp.off, smp.idx, S, L, ny, nx, smaps=smc)
    assert _rel(host(G), gref) < 3e-6
    AX = host(m.mrf_op_forward(A, dev(X))).astype(np.complex128)
    AhY = host(m.mrf_op_adjoint(A, dev(Y), apply_dcf=False)).astype(np.complex128)
    lhs = np.vdot(Y.astype(np.complex128), AX)
    rhs = np.vdot(AhY, X.astype(np.complex128))
    assert abs(lhs - rhs) < 1e-5 * abs(lhs)


def test_unit_single_coil_equals_no_maps(m):
    """One coil with a unit map runs the coil kernels; its results equal the
    map-free operator's bit for bit (multiplications by 1 are exact)."""
    banner("coil c=1 unit map vs no maps")
    S, L, ny, nx = 2, 4, 32, 32
    smp = workloads.random_lines(42, S, L, ny, nx, 5)
    A0 = m.Operator.from_sampling(smp)
    A1 = m.Operator.from_sampling(smp, smaps=np.ones((S, 1, ny, nx)))
    X = dev(c64(_cg(42, "x", (S, L, ny, nx))))
    Y = c64(_cg(42, "y", (smp.M,)))
    np.testing.assert_array_equal(host(m.mrf_op_forward(A1, X, dev(Y))).reshape(-1),
                                  host(m.mrf_op_forward(A0, X, dev(Y))))
    np.testing.assert_array_equal(host(m.mrf_op_adjoint(A1, dev(Y))), host(m.mrf_op_adjoint(A0, dev(Y))))


def _coil_problem(seed=1, L=100, size=64, nlines=4, c=4, snr=30.0, spiral=False):
    Dd = workloads.fisp_dictionary(L=L)
    ph = workloads.disc_phantom(Dd, seed=seed, size=size, snap=True)
    smp = (workloads.spiral_sampling(1, L, size, size, frac=0.04) if spiral
           else workloads.random_lines(seed, 1, L, size, size, nlines))
    sm = c64(workloads.coil_maps(seed, 1, c, size, size)).astype(np.complex128)
    Y = workloads.simulate_kspace(ph.X0, smp, snr, seed, smaps=sm)
    return Dd, ph, smp, sm, c64(Y)


@pytest.mark.parametrize("spiral", [False, True])
def test_coil_step_teacher_forced(m, spiral):
    """One step from the oracle's first iterate on both sides: objective,
    indices (near-tie rule), PD and step statistics; DCF weights on the
    spiral-like pattern."""
    banner(f"coil ipg step teacher-forced 64x64 L=100 c=4 spiral={spiral}")
    Dd, ph, smp, sm, Y = _coil_problem(spiral=spiral)
    D = m.Dictionary(Dd.atoms, Dd.params, grid_dims=Dd.grid_dims)
    A = m.Operator.from_sampling(smp, smaps=sm)
    w = smp.dcf
    X1, _, _, _ = ipg.ipg_solve(Y, smp.off, smp.idx, (1, Dd.L, 64, 64), Dd.atoms, mu0=1.0, adaptive=False,
                                max_iter=1, rel_tol=0, w=w, smaps=sm)
    Xk = c64(X1)
    for mu in (1.0, 2.0):
        Xn, idx, pd, st = m.mrf_ipg_step(D, A, dev(Y), dev(Xk), mu)
        Xr, res, sr = ipg.ipg_step(Y, smp.off, smp.idx, Dd.atoms, Xk.astype(np.complex128), mu, w=w, smaps=sm)
        gidx = host(idx)
        diff = gidx != res["idx"]
        print(f"mu={mu}: {int(diff.sum())} index differences; f_in {st.f_in:.6e} / {sr['f_old']:.6e}")
        assert abs(st.f_in - sr["f_old"]) <= 2e-5 * sr["f_old"]
        if diff.any():
            assert np.all(mf.index_ok(fourier.frame_to_voxel(res["Z"])[diff], Dd.atoms, gidx[diff], tol=1e-6))
        np.testing.assert_allclose(host(pd)[~diff], res["gamma"][~diff], rtol=1e-4, atol=1e-6)
        if not diff.any():
            assert _rel(host(Xn), Xr) < 1e-5
            for k, g in (("dx2", st.dx2), ("adx2", st.adx2), ("f_new", st.f_out)):
                assert abs(g - sr[k]) <= 1e-4 * abs(sr[k]) + 1e-12, (k, g, sr[k])


def test_coil_compressed_step_teacher_forced(m):
    """Coils and temporal compression together (s = 10)."""
    banner("coil + subspace ipg step teacher-forced 64x64 L=100 c=4 s=10")
    Dd, ph, smp, sm, Y = _coil_problem()
    D = m.Dictionary(Dd.atoms, Dd.params, grid_dims=Dd.grid_dims)
    C = D.compress(10)
    A = m.Operator.from_sampling(smp, smaps=sm)
    Vo, _ = subspace.dominant_subspace(Dd.atoms, 10)
    Dc = subspace.compress_atoms(Dd.atoms, Vo)
    X1, _, _, _ = ipg.ipg_solve(Y, smp.off, smp.idx, (1, 10, 64, 64), Dc, mu0=1.0, adaptive=False, max_iter=1,
                                rel_tol=0, V=Vo, smaps=sm)
    Xk = c64(X1)
    Xn, idx, pd, st = m.mrf_ipg_step(C, A, dev(Y), dev(Xk), 1.0)
    Xr, res, sr = ipg.ipg_step(Y, smp.off, smp.idx, Dc, Xk.astype(np.complex128), 1.0, V=Vo, smaps=sm)
    gidx = host(idx)
    diff = gidx != res["idx"]
    print(f"{int(diff.sum())} index differences; f_in {st.f_in:.6e} / {sr['f_old']:.6e}")
    assert abs(st.f_in - sr["f_old"]) <= 2e-5 * sr["f_old"]
    if diff.any():
        assert np.all(mf.index_ok(fourier.frame_to_voxel(res["Z"])[diff], Dc, gidx[diff], tol=1e-6))
    np.testing.assert_allclose(host(pd)[~diff], res["gamma"][~diff], rtol=1e-4, atol=1e-6)
    if not diff.any():
        assert _rel(host(Xn), Xr) < 1e-5
        for k, g in (("dx2", st.dx2), ("adx2", st.adx2), ("f_new", st.f_out)):
            assert abs(g - sr[k]) <= 1e-4 * abs(sr[k]) + 1e-12, (k, g, sr[k])


def test_coil_solve_fixed_mu(m):
    """Ten iterations at mu = 1 with four coils against the oracle's solve:
    objective history, error and object indices (FP32 / FP64 argmax flips
    at near-ties propagate along the iterations; each single step is checked
    teacher-forced above)."""
    banner("coil ipg solve 64x64 L=100 c=4 8 lines 10 iterations mu=1")
    Dd, ph, smp, sm, Y = _coil_problem(nlines=8)
    D = m.Dictionary(Dd.atoms, Dd.params, grid_dims=Dd.grid_dims)
    A = m.Operator.from_sampling(smp, smaps=sm)
    X, idx, pd, params, hist = m.mrf_ipg_solve(D, A, dev(Y), mu0=1.0, adaptive=False, max_iter=10, rel_tol=0.0)
    Xr, idr, gr, hr = ipg.ipg_solve(Y, smp.off, smp.idx, (1, Dd.L, 64, 64), Dd.atoms, mu0=1.0, adaptive=False,
                                    max_iter=10, rel_tol=0, smaps=sm)
    gidx = host(idx)
    inside = ph.idx >= 0
    agree = np.mean(gidx[inside] == idr[inside])
    fr = np.array([h["f"] for h in hr])
    nm_g, nm_o = _rel(host(X), ph.X0), _rel(Xr, ph.X0)
    print(f"coil solve: object agreement {agree:.5f}; f gpu {hist['f'][-1]:.6e} oracle {fr[-1]:.6e}; "
          f"nmse gpu {nm_g:.4e} oracle {nm_o:.4e}; {hist['ms']:.1f} ms")
    assert hist["iters"] == 10
    assert agree > 0.98
    np.testing.assert_allclose(hist["f"], fr, rtol=2e-3)
    assert abs(nm_g - nm_o) < 0.05 * nm_o + 1e-4
    np.testing.assert_array_equal(host(params), Dd.params[gidx].astype(np.float32))


def test_coil_argument_errors(m):
    banner("coil argument errors")
    import ctypes
    smp = workloads.random_lines(43, 1, 3, 16, 16, 3)
    A = m.Operator.from_sampling(smp, smaps=np.ones((1, 2, 16, 16)))
    import torch
    X = torch.zeros((1, 3, 16, 16), dtype=torch.complex64, device="cuda")
    bad = m.mrf.Op.from_buffer_copy(A.c)
    bad.smaps = None
    R = torch.empty((2, smp.M), dtype=torch.complex64, device="cuda")
    st = m.lib().mrf_op_forward(ctypes.byref(bad), X.data_ptr(), None, R.data_ptr(), None, None)
    assert st == -1
    bad = m.mrf.Op.from_buffer_copy(A.c)
    bad.ncoils = 65
    assert m.lib().mrf_op_forward(ctypes.byref(bad), X.data_ptr(), None, R.data_ptr(), None, None) == -1
