"""Pins of the seeded input generators against what the paper and the
mathematics fix (closed forms, printed grid sizes, brute force)."""
import numpy as np
import pytest

from synth import bloch, grids, rng, sequences, workloads


# --- grids: atom counts printed in the paper --------------------------------
def test_brainweb_grid_size():
    # Section "Numerical Brainweb phantom": d = 314160 fingerprints
    t1, t2, b0 = grids.brainweb_axes()
    assert (len(t1), len(t2), len(b0)) == (68, 84, 55)
    assert grids.product_grid([t1, t2, b0]).shape == (314160, 3)


def test_invivo_grid_size_needs_t2_le_t1():
    # Section "In-vivo data": d = 363624 fingerprints; only the T2 <= T1
    # filtered product reaches that count
    t1, t2, b0 = grids.invivo_axes()
    assert (len(t1), len(t2), len(b0)) == (106, 36, 109)
    full = grids.product_grid([t1, t2, b0])
    assert full.shape[0] == 106 * 36 * 109
    filt = grids.product_grid([t1, t2, b0], t2_lt_t1=True, inclusive=True)
    assert filt.shape[0] == 363624


def test_fisp_grid_counts():
    t1 = grids.log_grid(100, 4000, 40)
    t2 = grids.log_grid(10, 600, 50)
    assert grids.product_grid([t1, t2]).shape[0] == 2000
    assert grids.product_grid([t1, t2], t2_lt_t1=True).shape[0] == 1776
    assert t1[0] == 100 and abs(t1[-1] - 4000) < 1e-9
    assert np.allclose(np.diff(np.log(t1)), np.log(40) / 39)


def test_grid_index_roundtrip():
    dims = (5, 7, 3)
    idx = np.arange(5 * 7 * 3)
    sub = grids.grid_sub(idx, dims)
    assert np.array_equal(grids.grid_index(sub, dims), idx)
    # last parameter fastest, matching product_grid
    p = grids.product_grid([np.arange(5), np.arange(7), np.arange(3)])
    assert np.array_equal(p.astype(int), sub)


# --- closed-form trajectories of Section "Bloch dynamic model" ---------------
def test_inversion_recovery_closed_form():
    # no excitation after an ideal inversion: Mz(t TR) = 1 - 2 exp(-t TR / T1)
    T1 = np.array([300.0, 800.0, 2500.0])
    T2 = np.array([50.0, 80.0, 200.0])
    L, TR = 60, 10.0
    _, mz = bloch.fisp_epg(T1, T2, np.zeros(L), TR, TE=5.0, TI=0.0, return_mz_end=True)
    t = np.arange(1, L + 1)
    ref = 1.0 - 2.0 * np.exp(-t[None, :] * TR / T1[:, None])
    assert np.max(np.abs(mz - ref)) < 1e-13


def test_t2_decay_closed_form():
    # a 90 degree pulse then no excitation: |Mxy(t TR)| = exp(-t TR / T2)
    T1 = np.array([900.0, 1500.0])
    T2 = np.array([40.0, 120.0])
    L, TR = 30, 10.0
    alpha = np.zeros(L)
    alpha[0] = 90.0
    sig = bloch.bssfp(T1, T2, np.array([0.0, 17.0]), alpha, np.zeros(L), TR, TE=TR, TI=0.0)
    t = np.arange(1, L + 1)
    ref = np.exp(-t[None, :] * TR / T2[:, None])
    assert np.max(np.abs(np.abs(sig) - ref)) < 1e-13


def _isochromat_fisp(T1, T2, alpha_deg, TR, TE, TI):
    """Brute force: mean transverse signal of N = 2L+1 isochromats whose
    phases advance by 2 pi q / N per TR (the dephasing gradient)."""
    L = len(alpha_deg)
    N = 2 * L + 1
    th = 2 * np.pi * np.arange(N) / N
    mx = np.zeros(N)
    my = np.zeros(N)
    mz = np.full(N, -np.exp(-TI / T1) + 1 - np.exp(-TI / T1))
    out = np.zeros(L, dtype=np.complex128)
    for t in range(L):
        a = np.deg2rad(alpha_deg[t])
        my, mz = my * np.cos(a) - mz * np.sin(a), my * np.sin(a) + mz * np.cos(a)
        e1, e2 = np.exp(-TE / T1), np.exp(-TE / T2)
        mx, my, mz = mx * e2, my * e2, mz * e1 + 1 - e1
        out[t] = np.mean(mx + 1j * my)
        e1, e2 = np.exp(-(TR - TE) / T1), np.exp(-(TR - TE) / T2)
        mx, my, mz = mx * e2, my * e2, mz * e1 + 1 - e1
        c, s = np.cos(th), np.sin(th)
        mx, my = mx * c - my * s, mx * s + my * c
    return out


def test_epg_equals_isochromat_average():
    L = 24
    alpha = sequences.fisp_train(L) + rng.uniform(7, "fa", L, -20, 20)
    for T1, T2 in [(800.0, 50.0), (1500.0, 300.0), (300.0, 30.0)]:
        atom = bloch.fisp_epg([T1], [T2], alpha, 10.0, 5.0, 10.0)[0]
        assert bloch.fisp_epg.last_max_abs_real < 1e-14     # echo purely imaginary
        ref = _isochromat_fisp(T1, T2, alpha, 10.0, 5.0, 10.0)
        assert np.max(np.abs(ref.real)) < 1e-12
        assert np.max(np.abs(ref.imag - atom)) < 1e-12


def test_bssfp_steady_state_fixed_point():
    """Constant flip angle with alternating phase converges to the fixed
    point of the affine two-TR map, solved directly."""
    T1, T2, df, TR, TE, a = 800.0, 60.0, 13.0, 10.0, 5.0, np.deg2rad(35.0)

    def rz(t):
        return np.array([[np.cos(t), -np.sin(t), 0], [np.sin(t), np.cos(t), 0], [0, 0, 1.0]])

    def rx(t):
        return np.array([[1.0, 0, 0], [0, np.cos(t), -np.sin(t)], [0, np.sin(t), np.cos(t)]])

    def free(tau):
        e1, e2 = np.exp(-tau / T1), np.exp(-tau / T2)
        A = np.diag([e2, e2, e1]) @ rz(-2 * np.pi * df * tau * 1e-3)
        return A, np.array([0, 0, 1 - e1])

    def tr_map(phi):
        R = rz(phi) @ rx(a) @ rz(-phi)
        A1, b1 = free(TE)
        A2, b2 = free(TR - TE)
        return A2 @ A1 @ R, A2 @ b1 + b2

    A0, b0 = tr_map(0.0)
    Api, bpi = tr_map(np.pi)
    A = Api @ A0
    b = Api @ b0 + bpi
    s = np.linalg.solve(np.eye(3) - A, b)           # state at the start of a phase-0 TR
    A1, b1 = free(TE)
    ste = A1 @ (rx(a) @ s) + b1
    ref = ste[0] + 1j * ste[1]
    L = 2000
    sig = bloch.bssfp([T1], [T2], [df], np.full(L, 35.0), sequences.alternating_phase(L), TR, TE, 10.0)[0]
    assert abs(sig[-2] - ref) < 1e-12                # even index = phase 0


def test_bssfp_b1_scales_flip():
    L = 50
    alpha = sequences.halfsine_train(L, 3)
    ph = sequences.alternating_phase(L)
    a = bloch.bssfp([900.0], [70.0], [5.0], 1.3 * alpha, ph, 10.0, 5.0, 10.0)[0]
    b = bloch.bssfp([900.0], [70.0], [5.0], alpha, ph, 10.0, 5.0, 10.0, B1=[1.3])[0]
    assert np.max(np.abs(a - b)) < 1e-14


# --- sequences ---------------------------------------------------------------
def test_halfsine_train_structure():
    L = 1000
    a = sequences.halfsine_train(L, 2)
    t0 = np.arange(L)
    gap = (t0 % 300) >= 250
    assert np.all(a[gap] == 0)
    clean = sequences.halfsine_train(L, 2, noise_std=0.0)
    assert abs(clean[124] - 60.0) < 1e-12        # peak of the first lobe (u = 125)
    assert abs(clean[300 + 124] - 30.0) < 1e-12  # second lobe peaks at 30 degrees
    noise = (a - clean)[~gap]
    assert abs(np.std(noise) - 5.0) < 0.5
    assert np.max(np.abs(noise)) <= 5.0 * np.sqrt(3) + 1e-12


def test_fisp_train_formula():
    a = sequences.fisp_train(100)
    assert abs(a[0] - (10 + 50 * abs(np.sin(np.pi / 125)))) < 1e-12
    assert abs(a[99] - (10 + 50 * abs(np.sin(100 * np.pi / 125)))) < 1e-12


# --- RNG ---------------------------------------------------------------------
def test_rng_counter_based():
    a = rng.uniform(5, "x", 1000)
    b = rng.uniform(5, "x", 500, offset=500)
    assert np.array_equal(a[500:], b)
    assert not np.array_equal(a, rng.uniform(5, "y", 1000))
    u = rng.uniform(1, "m", 200000)
    assert abs(u.mean() - 0.5) < 5e-3 and abs(u.var() - 1 / 12) < 2e-3
    g = rng.normal(1, "g", 200000)
    assert abs(g.mean()) < 1e-2 and abs(g.std() - 1) < 1e-2
    # SplitMix64 published first output for state 0: 0xE220A8397B1DCDAF
    assert int(rng.mix64(np.array([0x9E3779B97F4A7C15], dtype=np.uint64))[0]) == 0xE220A8397B1DCDAF


# --- workloads ---------------------------------------------------------------
def test_random_voxels_snr():
    D = workloads.fisp_dictionary(L=100)
    Z, j, pd, snr = workloads.random_voxels(D, 4000, seed=3, snr_db_range=(30.0, 30.0))
    x = pd[:, None] * D.atoms[j]
    noise = Z - x
    ratio = np.sum(np.abs(noise) ** 2) / np.sum(np.abs(x) ** 2)
    assert abs(10 * np.log10(1 / ratio) - 30.0) < 0.2


def test_masks_unique_and_sized():
    smp = workloads.random_lines(1, 2, 5, 64, 64, [6, 9])
    assert smp.off[-1] == 5 * 6 * 64 + 5 * 9 * 64
    for p in range(10):
        seg = smp.idx[smp.off[p]:smp.off[p + 1]]
        assert len(np.unique(seg)) == len(seg)
    sp = workloads.spiral_sampling(1, 4, 64, 64)
    for p in range(4):
        seg = sp.idx[sp.off[p]:sp.off[p + 1]]
        assert len(np.unique(seg)) == len(seg) == 205
    assert sp.dcf is not None and np.all(sp.dcf > 0)
    # the spiral is denser at the centre: central samples get smaller weights
    seg = sp.idx[: sp.off[1]]
    ky = ((seg // 64 + 32) % 64) - 32
    kx = ((seg % 64 + 32) % 64) - 32
    r = np.hypot(ky, kx)
    w = sp.dcf[: sp.off[1]]
    assert w[r < 8].mean() < w[r > 20].mean()


def test_kspace_noise_level():
    D = workloads.fisp_dictionary(L=20)
    ph = workloads.disc_phantom(D, seed=1)
    smp = workloads.random_lines(1, 1, 20, 64, 64, 6)
    Y0 = workloads.simulate_kspace(ph.X0, smp, None, 1)
    Y = workloads.simulate_kspace(ph.X0, smp, 30.0, 1)
    snr = 10 * np.log10(np.sum(np.abs(Y0) ** 2) / np.sum(np.abs(Y - Y0) ** 2))
    assert abs(snr - 30.0) < 0.3
