"""Pins of the learned-proposal oracle (MLP, Adam, grid mapping) and of the
local matched filter with fallback: finite differences, closed forms,
special cases that reduce to the exhaustive filter, brute force."""
import math

import numpy as np
import pytest

from oracle import local, mf, mlp
from synth import grids, rng, workloads


def _params(seed, I, H, P, scale=1.0):
    def w(tag, shape, fan):
        return rng.normal(seed, tag, int(np.prod(shape))).reshape(shape) * scale * math.sqrt(2.0 / fan)
    return {"W1": w("W1", (H, I), I), "b1": 0.1 * rng.normal(seed, "b1", H),
            "W2": w("W2", (H, H), H), "b2": 0.1 * rng.normal(seed, "b2", H),
            "W3": w("W3", (P, H), H), "b3": 0.1 * rng.normal(seed, "b3", P)}


def test_gelu_identities():
    a = np.linspace(-6, 6, 1001)
    # Phi(a) + Phi(-a) = 1  =>  gelu(a) - gelu(-a) = a
    assert np.max(np.abs(mlp.gelu(a) - mlp.gelu(-a) - a)) < 1e-14
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    # exact form at 1: Phi(1) = 0.8413447460685429...
    assert abs(mlp.gelu(np.array([1.0]))[0] - 0.8413447460685429) < 1e-15
    h = 1e-6
    num = (mlp.gelu(a + h) - mlp.gelu(a - h)) / (2 * h)
    assert np.max(np.abs(num - mlp.gelu_grad(a))) < 1e-8


def test_bf16_forward_special_cases():
    """The BF16 inference form: on operands already representable in BF16
    (multiples of 2^-6 of magnitude < 2) and without the hidden rounding it
    is the FP64 forward; the hidden rounding moves each h1 entry by at most
    half a BF16 spacing (2^-9 relative), so y moves by at most
    2^-9 sum_n |h1_n| max_p sum_j |W3_pj| |W2_jn| * max gelu' (< 1.13)."""
    I, H, P, B = 16, 8, 3, 11
    q = lambda a: np.round(np.asarray(a) * 64) / 64
    prm = _params(7, I, H, P)
    prm["W1"], prm["W2"] = q(np.clip(prm["W1"], -1.9, 1.9)), q(np.clip(prm["W2"], -1.9, 1.9))
    X = q(np.clip(rng.normal(7, "x", B * I).reshape(B, I), -1.9, 1.9))
    y, (_, a1, h1, _, _) = mlp.forward(prm, X)
    np.testing.assert_allclose(mlp.forward_bf16(prm, X, round_hidden=False), y, rtol=0, atol=1e-13)
    yb = mlp.forward_bf16(prm, X)
    gain = (np.abs(prm["W3"]) @ np.abs(prm["W2"])).max(axis=0)        # [H]
    bound = 1.13 * 2.0 ** -9 * (np.abs(h1) @ gain) + 1e-13
    assert np.all(np.abs(yb - y) <= bound[:, None])
    assert np.any(np.abs(yb - y) > 1e-12)                               # the rounding acts


def test_mlp_gradients_central_differences():
    I, H, P, B = 7, 5, 3, 6
    prm = _params(1, I, H, P)
    X = rng.normal(1, "x", B * I).reshape(B, I)
    T = rng.normal(1, "t", B * P).reshape(B, P)
    loss, g = mlp.loss_and_grads(prm, X, T)
    h = 1e-6
    for k in mlp.NAMES:
        flat = prm[k].reshape(-1)
        for i in range(flat.size):
            old = flat[i]
            flat[i] = old + h
            lp, _ = mlp.loss_and_grads(prm, X, T)
            flat[i] = old - h
            lm, _ = mlp.loss_and_grads(prm, X, T)
            flat[i] = old
            num = (lp - lm) / (2 * h)
            ana = g[k].reshape(-1)[i]
            assert abs(num - ana) <= 1e-6 * max(1.0, abs(ana)) + 1e-9, (k, i, num, ana)


def test_adam_first_step_is_signed_lr():
    prm = _params(2, 4, 3, 2)
    g = {k: rng.normal(2, "g" + k, prm[k].size).reshape(prm[k].shape) for k in mlp.NAMES}
    st = {"m": {k: np.zeros_like(prm[k]) for k in mlp.NAMES}, "v": {k: np.zeros_like(prm[k]) for k in mlp.NAMES}}
    new = mlp.adam_step(prm, g, st, 1, lr=1e-3, eps=0.0)
    for k in mlp.NAMES:
        np.testing.assert_allclose(new[k] - prm[k], -1e-3 * np.sign(g[k]), rtol=1e-12, atol=1e-15)


def test_loss_decreases_with_adam():
    I, H, P, B = 20, 16, 3, 64
    prm = _params(3, I, H, P)
    X = rng.normal(3, "x", B * I).reshape(B, I)
    T = rng.normal(3, "t", B * P).reshape(B, P)
    st = {"m": {k: np.zeros_like(prm[k]) for k in mlp.NAMES}, "v": {k: np.zeros_like(prm[k]) for k in mlp.NAMES}}
    l0, _ = mlp.loss_and_grads(prm, X, T)
    for t in range(1, 201):
        _, g = mlp.loss_and_grads(prm, X, T)
        prm = mlp.adam_step(prm, g, st, t, lr=1e-2)
    l1, _ = mlp.loss_and_grads(prm, X, T)
    assert l1 < 0.1 * l0


def test_nearest_cells_on_grid_values():
    t1 = grids.log_grid(100, 4000, 60)
    df = grids.lin_grid(-40, 40, 28)
    table = grids.product_grid([t1, df])
    u, mean, std = mlp.standardise(table, [True, False])
    cells = mlp.nearest_cells(u, mean, std, [True, False], [t1, df])
    np.testing.assert_array_equal(grids.grid_index(cells, (60, 28)), np.arange(table.shape[0]))


def test_box_atoms_clipping_and_order():
    dims = (10, 8, 6)
    b = local.box_atoms((0, 0, 0), dims, 3)
    assert len(b) == 4 ** 3 and np.all(np.diff(b) > 0)
    b = local.box_atoms((5, 4, 3), dims, 3)
    assert len(b) == 7 * 7 * 6
    sub = grids.grid_sub(b, dims)
    assert sub[:, 0].min() == 2 and sub[:, 0].max() == 8


def test_local_search_special_cases_reduce_to_exhaustive():
    D = workloads.bssfp_dictionary(L=30, n_t1=9, n_t2=8, n_df=5, seed=2)
    Z, j, pd, snr = workloads.random_voxels(D, 60, seed=4, snr_db_range=(10.0, 30.0))
    ex = mf.exact_mf(Z, D.atoms)
    cells = grids.grid_sub(rng.randint(4, "c", 60, D.d), D.grid_dims)
    # a box that covers the whole grid is the exhaustive filter
    r_all = local.local_match(Z, D.atoms, D.grid_dims, cells, r=20, threshold=-1.0)
    np.testing.assert_array_equal(r_all["idx"], ex["idx"])
    # threshold above any correlation: every voxel falls back
    r_fb = local.local_match(Z, D.atoms, D.grid_dims, cells, r=1, threshold=1.5)
    assert r_fb["fallback"].all()
    np.testing.assert_array_equal(r_fb["idx"], ex["idx"])
    # brute force over the box
    r1 = local.local_match(Z, D.atoms, D.grid_dims, cells, r=1, threshold=-1.0)
    for v in range(60):
        box = local.box_atoms(cells[v], D.grid_dims, 1)
        c = [np.real(np.vdot(D.atoms[k], Z[v])) / np.linalg.norm(D.atoms[k]) for k in box]
        assert r1["idx"][v] == box[int(np.argmax(c))]


def test_local_search_recentre_walks_to_the_optimum():
    D = workloads.bssfp_dictionary(L=60, n_t1=20, n_t2=20, n_df=9, seed=2)
    dims = D.grid_dims
    j = rng.randint(5, "j", 40, D.d)
    Z = D.atoms[j] * 0.7
    sub = grids.grid_sub(j, dims)
    # proposals off by 5 cells in T1 (clipped to the grid)
    cells = sub.copy()
    cells[:, 0] = np.clip(sub[:, 0] + np.where(sub[:, 0] < 10, 5, -5), 0, dims[0] - 1)
    r0 = local.local_match(Z, D.atoms, dims, cells, r=3, threshold=-1.0, recentre=0)
    r3 = local.local_match(Z, D.atoms, dims, cells, r=3, threshold=-1.0, recentre=3)
    assert np.mean(r0["idx"] == j) < 0.5
    np.testing.assert_array_equal(r3["idx"], j)


def test_local_search_warm_start_safeguard():
    """With a warm index the local search is never worse than the warm atom:
    a box far from the optimum plus the exact answer as warm start gives the
    exact matched filter; a poor warm atom changes nothing."""
    D = workloads.fisp_dictionary(L=30, n_t1=12, n_t2=14)
    Z, j, pd, snr = workloads.random_voxels(D, 40, seed=9, snr_db_range=(20.0, 40.0))
    ex = mf.exact_mf(Z, D.atoms)
    far = np.zeros((40, 2), dtype=np.int64)                 # boxes in the grid corner
    far[:, 0] = np.where(grids.grid_sub(ex["idx"], D.grid_dims)[:, 0] > 6, 0, 11)
    out = local.local_match(Z, D.atoms, D.grid_dims, far, r=1, threshold=-1.0, warm=ex["idx"])
    np.testing.assert_array_equal(out["idx"], ex["idx"])
    base = local.local_match(Z, D.atoms, D.grid_dims, far, r=1, threshold=-1.0)
    worst = np.argmin(mf.correlations(Z, D.atoms), axis=1)
    out2 = local.local_match(Z, D.atoms, D.grid_dims, far, r=1, threshold=-1.0, warm=worst)
    np.testing.assert_array_equal(out2["idx"], base["idx"])
