"""Pins of the oracle's CoverBLIP projection (Algorithm 2 with Algorithm 1 in
place of the exhaustive argmax) against what does not depend on the tree:
at eps = 0 it is the exact matched filter (eq. exactP) computed by brute
force; at eps > 0 every answer satisfies Definition 3.1 and is no farther
from the query than the warm start; zero voxels keep their warm index; and
an IPG solve with the eps = 0 tree projection repeats the exact solve."""
import numpy as np
import pytest

from oracle import covertree as ct
from oracle import ipg, mf
from synth import rng, workloads


@pytest.fixture(scope="module", params=["fisp", "bssfp"])
def small(request):
    if request.param == "fisp":
        Dd = workloads.fisp_dictionary(L=24, n_t1=8, n_t2=10)
    else:
        Dd = workloads.bssfp_dictionary(L=16, n_t1=6, n_t2=6, n_df=5, seed=2)
    t = ct.build(ct.atom_rows(Dd.atoms))
    return Dd, t


def _brute_dist(Z, atoms):
    P = ct.query_rows(Z, np.iscomplexobj(atoms))
    A = ct.atom_rows(atoms)
    return np.linalg.norm(P[:, None, :] - A[None, :, :], axis=2)


def test_eps0_is_exact_matched_filter(small):
    Dd, t = small
    Z, j, pd, snr = workloads.random_voxels(Dd, 300, seed=31, snr_db_range=(0.0, 30.0))
    Z[7] = 0.0
    warm = rng.randint(31, "warm", 300, Dd.d)
    r = ct.tree_mf(Z, Dd.atoms, t, 0.0, warm_idx=warm)
    ex = mf.exact_mf(Z, Dd.atoms, warm_idx=warm, want_X=True)
    clear = ex["gap"] > 1e-9
    np.testing.assert_array_equal(r["idx"][clear], ex["idx"][clear])
    assert np.all(mf.index_ok(Z, Dd.atoms, r["idx"], tol=1e-9))
    same = r["idx"] == ex["idx"]
    np.testing.assert_allclose(r["gamma"][same], ex["gamma"][same], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(r["X"][same], ex["X"][same], rtol=1e-12, atol=1e-15)
    assert r["idx"][7] == warm[7] and r["gamma"][7] == 0.0 and not np.any(r["X"][7])


@pytest.mark.parametrize("eps", [0.2, 0.8, 1.6])
def test_eps_answers_satisfy_definition(small, eps):
    Dd, t = small
    Z, j, pd, snr = workloads.random_voxels(Dd, 200, seed=32, snr_db_range=(-5.0, 30.0))
    warm = rng.randint(32, "warm", 200, Dd.d)
    r = ct.tree_mf(Z, Dd.atoms, t, eps, warm_idx=warm)
    dist = _brute_dist(Z, Dd.atoms)
    got = dist[np.arange(200), r["idx"]]
    assert np.all(got <= (1 + eps) * dist.min(axis=1) + 1e-12)       # Definition 3.1
    assert np.all(got <= dist[np.arange(200), warm] + 1e-12)          # never worse than the warm start
    # PD from the returned atom's own correlation (not the best one's)
    a = Dd.atoms[r["idx"]]
    c = np.real(np.sum(Z * np.conj(a), axis=1))
    np.testing.assert_allclose(r["gamma"], np.maximum(c, 0) / np.sum(np.abs(a) ** 2, axis=1), rtol=1e-12)
    assert np.all(r["evals"] >= 2) and np.all(r["evals"] <= t.X.shape[0] + 2)


def test_coverblip_solve_eps0_repeats_exact_solve():
    Dd = workloads.fisp_dictionary(L=24, n_t1=8, n_t2=10)
    ph = workloads.disc_phantom(Dd, seed=5, size=16, radius=6.0, snap=True)
    smp = workloads.random_lines(5, 1, Dd.L, 16, 16, 3)
    Y = workloads.simulate_kspace(ph.X0, smp, 30.0, 5)
    t = ct.build(ct.atom_rows(Dd.atoms))
    dims = (1, Dd.L, 16, 16)
    Xe, ie, ge, he = ipg.ipg_solve(Y, smp.off, smp.idx, dims, Dd.atoms, mu0=1.0, adaptive=True, max_iter=4,
                                   rel_tol=0)
    Xt, it, gt, ht = ipg.ipg_solve(Y, smp.off, smp.idx, dims, Dd.atoms, mu0=1.0, adaptive=True, max_iter=4,
                                   rel_tol=0, tree=t, eps=0.0)
    np.testing.assert_array_equal(it, ie)
    np.testing.assert_allclose([h["f"] for h in ht], [h["f"] for h in he], rtol=1e-12)
    np.testing.assert_allclose(Xt, Xe, rtol=0, atol=1e-12 * np.abs(Xe).max())
    assert all(h["evals"] > 0 for h in ht)
