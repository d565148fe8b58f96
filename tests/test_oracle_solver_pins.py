"""Pins of the oracle's optional solver branches and of the near-tie
acceptance rule against what the paper fixes:

* the kappa rescaling of the first iterate (section "CoverBLIP algorithm",
  the paragraph after eq. steprule): kappa = ||Y|| / ||A X^1|| with plain
  norms, X^1 <- kappa X^1 and the initial step mu <- kappa mu;
* the relative-progress stop (section "Numerical experiments", computational
  cost paragraph): stop at the first k with (f_k - f_{k+1}) / f_k < tol;
* the step-size shrink cap of Algorithm 2's adaptive rule;
* the near-tie rule: a candidate index is accepted iff its normalised
  correlation is within tol of the maximum (it must also reject).
"""
import numpy as np
import pytest

from oracle import fourier, ipg, mf
from synth import rng, workloads


def _dcf_problem(snr=30.0, seed=7):
    """16 x 16 FISP disc, 20 frames, spiral-like points with Voronoi DCF
    weights (w != 1, so weighted and plain norms differ)."""
    D = workloads.fisp_dictionary(L=20, n_t1=12, n_t2=10)
    ph = workloads.disc_phantom(D, seed=seed, size=16, radius=6.5)
    smp = workloads.spiral_sampling(1, D.L, 16, 16, frac=0.3)
    Y = workloads.simulate_kspace(ph.X0, smp, snr, seed)
    return D, ph, smp, Y


def _plain_norm(x):
    return float(np.sqrt(np.sum(np.abs(np.asarray(x)) ** 2)))


def test_kappa_rescales_first_iterate_with_plain_norms():
    D, ph, smp, Y = _dcf_problem()
    dims = (1, D.L, 16, 16)
    common = dict(mu0=1.0, adaptive=False, rel_tol=0, w=smp.dcf)
    X1, idx1, g1, h1 = ipg.ipg_solve(Y, smp.off, smp.idx, dims, D.atoms, max_iter=1, **common)
    X1k, idx1k, g1k, h1k = ipg.ipg_solve(Y, smp.off, smp.idx, dims, D.atoms, max_iter=1, kappa=True, **common)
    # X^1 <- kappa X^1: the same atoms, every voxel scaled by one scalar
    assert np.array_equal(idx1, idx1k)
    kap = np.vdot(X1, X1k).real / np.vdot(X1, X1).real
    assert np.max(np.abs(X1k - kap * X1)) < 1e-12 * np.max(np.abs(X1k))
    np.testing.assert_allclose(g1k, kap * g1, rtol=1e-12, atol=0)
    # kappa = ||Y|| / ||A X^1|| in the plain norm: after the rescaling the
    # forward model of the iterate has the measurements' energy
    AX = fourier.forward(X1k, smp.off, smp.idx)
    assert abs(_plain_norm(AX) - _plain_norm(Y)) < 1e-12 * _plain_norm(Y)
    # ... and not in the DCF-weighted norm (a weighted kappa would fail above)
    w = np.sqrt(smp.dcf)
    assert abs(_plain_norm(w * AX) - _plain_norm(w * Y)) > 1e-3 * _plain_norm(w * Y)
    assert kap > 1.0 + 1e-3 or kap < 1.0 - 1e-3
    # the step size of the next iteration starts from kappa mu0
    _, _, _, h2 = ipg.ipg_solve(Y, smp.off, smp.idx, dims, D.atoms, max_iter=2, kappa=True, **common)
    assert h2[0]["mu"] == 1.0
    assert abs(h2[1]["mu"] - kap) < 1e-12 * kap
    # with the adaptive rule every trial of iteration 2 is kappa mu0 / zeta^s
    _, _, _, h3 = ipg.ipg_solve(Y, smp.off, smp.idx, dims, D.atoms, mu0=4.0, zeta=2.0, adaptive=True,
                                max_iter=3, rel_tol=0, w=smp.dcf, kappa=True)
    X1a, _, _, _ = ipg.ipg_solve(Y, smp.off, smp.idx, dims, D.atoms, mu0=4.0, zeta=2.0, adaptive=True,
                                 max_iter=1, rel_tol=0, w=smp.dcf)
    X1ak, _, _, _ = ipg.ipg_solve(Y, smp.off, smp.idx, dims, D.atoms, mu0=4.0, zeta=2.0, adaptive=True,
                                  max_iter=1, rel_tol=0, w=smp.dcf, kappa=True)
    ka = np.vdot(X1a, X1ak).real / np.vdot(X1a, X1a).real
    for h in h3[1:]:
        assert abs(h["mu"] - 4.0 * ka / 2.0 ** h["shrinks"]) < 1e-12 * h["mu"]


def test_kappa_off_leaves_the_solve_unchanged():
    D, ph, smp, Y = _dcf_problem()
    dims = (1, D.L, 16, 16)
    a = ipg.ipg_solve(Y, smp.off, smp.idx, dims, D.atoms, mu0=1.0, adaptive=False, max_iter=3,
                      rel_tol=0, w=smp.dcf)
    b = ipg.ipg_solve(Y, smp.off, smp.idx, dims, D.atoms, mu0=1.0, adaptive=False, max_iter=3,
                      rel_tol=0, w=smp.dcf, kappa=False)
    assert np.array_equal(a[0], b[0])
    assert all(x["mu"] == 1.0 for x in a[3])


def _progress(Y, w, hist):
    """Relative decrease per accepted iteration, r_k = (f_{k-1} - f_k) / f_{k-1},
    with f_0 = ||Y||_W^2 (the objective of X^0 = 0), from the history."""
    f0 = float(np.sum((1.0 if w is None else w) * np.abs(Y) ** 2))
    f = np.array([f0] + [h["f"] for h in hist])
    return (f[:-1] - f[1:]) / f[:-1]


def pick_tolerance(r, m_min=2):
    """A tolerance that the relative-progress rule first meets at iteration m
    (r[m] < tol <= every earlier r[i]), and that the variant with f_{k+1} as
    denominator, r/(1 - r) > r + r^2, would not meet there.  Returns (m, tol)
    or None."""
    for m in range(m_min, len(r)):
        lo = float(np.min(r[:m]))
        if r[m] > 0 and lo > r[m]:
            return m, float(r[m] + 0.5 * min(r[m] ** 2, lo - r[m]))
    return None


def test_relative_progress_stop_is_first_small_decrease():
    D, ph, smp, Y = _dcf_problem(snr=25.0)
    dims = (1, D.L, 16, 16)
    common = dict(mu0=1.0, zeta=2.0, adaptive=True, w=smp.dcf)
    _, _, _, full = ipg.ipg_solve(Y, smp.off, smp.idx, dims, D.atoms, max_iter=12, rel_tol=0, **common)
    r = _progress(Y, smp.dcf, full)
    picked = pick_tolerance(r)
    assert picked is not None, r
    m, tol = picked
    assert r[m] < tol and np.all(r[:m] >= tol)
    assert r[m] / (1 - r[m]) >= tol   # the other denominator would not stop here
    _, _, _, stopped = ipg.ipg_solve(Y, smp.off, smp.idx, dims, D.atoms, max_iter=12, rel_tol=tol, **common)
    assert len(stopped) == m + 1
    for a, b in zip(stopped, full[:m + 1]):
        assert a["f"] == b["f"] and a["mu"] == b["mu"]
    # a tolerance below every decrease never stops early
    _, _, _, never = ipg.ipg_solve(Y, smp.off, smp.idx, dims, D.atoms, max_iter=12,
                                   rel_tol=0.5 * float(np.min(r[r > 0])), **common)
    assert len(never) == len(full)


def test_relative_progress_stop_on_non_monotone_runs():
    # fixed steps above the safe one: at mu = 1.5 the objective decreases by
    # alternating large and small amounts, at mu = 2 it goes up at every
    # other iteration; the rule stops at the first k whose relative decrease
    # is below tol (a negative one included), not at the smallest one
    D, ph, smp, Y = _dcf_problem(snr=25.0)
    dims = (1, D.L, 16, 16)
    for mu, tols in ((1.5, (0.3, 0.26, 0.24, 0.2)), (2.0, (1e-9, 0.05))):
        common = dict(mu0=mu, adaptive=False, w=smp.dcf)
        _, _, _, full = ipg.ipg_solve(Y, smp.off, smp.idx, dims, D.atoms, max_iter=10, rel_tol=0, **common)
        r = _progress(Y, smp.dcf, full)
        stops = set()
        for tol in tols:
            first = np.nonzero(r < tol)[0]
            expect = (int(first[0]) + 1) if first.size else len(full)
            stops.add(expect)
            _, _, _, h = ipg.ipg_solve(Y, smp.off, smp.idx, dims, D.atoms, max_iter=10, rel_tol=tol, **common)
            assert len(h) == expect, (mu, tol, r)
        assert len(stops) == len(tols) or mu == 2.0   # the tolerances probe different stops


def test_zero_data_stops_after_one_iteration():
    # Y = 0 and X^0 = 0: the gradient vanishes, every voxel projects to zero,
    # Delta X = 0 exactly and the solve ends after the first iteration
    D, ph, smp, Y = _dcf_problem()
    X, idx, g, hist = ipg.ipg_solve(np.zeros_like(Y), smp.off, smp.idx, (1, D.L, 16, 16), D.atoms,
                                    mu0=1.0, adaptive=True, max_iter=10, rel_tol=1e-6, w=smp.dcf)
    assert len(hist) == 1 and hist[0]["dx2"] == 0.0
    assert not np.any(X) and not np.any(g)


def test_shrink_cap_raises_no_convergence():
    D, ph, smp, Y = _dcf_problem()
    dims = (1, D.L, 16, 16)
    with pytest.raises(ipg.NoConvergence):
        ipg.ipg_solve(Y, smp.off, smp.idx, dims, D.atoms, mu0=1e6, adaptive=True, max_iter=2,
                      rel_tol=0, max_shrinks=0, w=smp.dcf)
    # the same start is accepted after enough shrinks
    _, _, _, h = ipg.ipg_solve(Y, smp.off, smp.idx, dims, D.atoms, mu0=1e6, adaptive=True, max_iter=1,
                               rel_tol=0, max_shrinks=60, w=smp.dcf)
    assert h[0]["shrinks"] > 0
    assert h[0]["mu"] < h[0]["dx2"] / h[0]["adx2"]


# --- near-tie acceptance ------------------------------------------------------
def _two_atoms(cos_t):
    """Two unit atoms at angle t in the plane of e0, e1 (L = 6, complex), and
    the voxel z = 3 e0, whose normalised correlations are 1 and cos t."""
    sin_t = np.sqrt(1.0 - cos_t ** 2)
    a = np.zeros((2, 6), np.complex128)
    a[0, 0] = 1.0
    a[1, 0], a[1, 1] = cos_t, sin_t
    z = np.zeros((1, 6), np.complex128)
    z[0, 0] = 3.0
    return z, a


@pytest.mark.parametrize("below,ok", [(2e-6, False), (1.5e-6, False), (0.5e-6, True), (0.0, True)])
def test_index_ok_accepts_only_within_tolerance(below, ok):
    z, a = _two_atoms(1.0 - below)
    assert bool(mf.index_ok(z, a, np.array([1]), tol=1e-6)[0]) is ok
    assert bool(mf.index_ok(z, a, np.array([0]), tol=1e-6)[0])


def test_index_ok_rejects_a_wrong_atom_on_random_voxels():
    d, L, n = 50, 12, 40
    g = rng.normal(21, "a", 2 * d * L).reshape(d, L, 2)
    atoms = g[..., 0] + 1j * g[..., 1]
    g = rng.normal(21, "z", 2 * n * L).reshape(n, L, 2)
    Z = g[..., 0] + 1j * g[..., 1]
    res = mf.exact_mf(Z, atoms)
    c = mf.correlations(Z, atoms) / res["znorm"][:, None]
    order = np.argsort(-c, axis=1)
    second = order[:, 1]
    gap = c[np.arange(n), res["idx"]] - c[np.arange(n), second]
    ok = mf.index_ok(Z, atoms, second, tol=1e-6)
    assert np.array_equal(ok, gap <= 1e-6)
    assert not np.all(ok)
    assert np.all(mf.index_ok(Z, atoms, res["idx"], tol=1e-6))
