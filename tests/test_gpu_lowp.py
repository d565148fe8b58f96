"""GPU parity of the reduced-precision forms of the matched filter: the BF16
and FP8-E4M3 encoders bit-exact against the oracle's encoders; certified
BF16 / FP8 scoring exact against the FP64 oracle; uncertified scoring against
the oracle's precision form."""
import numpy as np
import pytest

from gpu_helpers import banner, c64, dev, host
from oracle import mf, quant
from synth import rng, workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def m():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1810_01967_amd as pkg
    pkg.lib()
    return pkg


def _edge_rows():
    """FP32 values around every binade and rounding boundary, plus zeros."""
    base = np.concatenate([
        np.array([0.0, -0.0, 1.0, -1.0, 448.0, 464.0, 480.0, 2 ** -6, 2 ** -9, 2 ** -10, 3 * 2 ** -11]),
        np.ldexp(1.0 + np.arange(0, 1, 1 / 64), np.arange(-12, 12).repeat(1)[:, None]).reshape(-1),
        rng.normal(41, "v", 4000) * np.exp(rng.uniform(41, "e", 4000, -12, 6)),
    ]).astype(np.float32)
    # halfway cases for BF16 (low 16 bits = 0x8000) and neighbours
    hw = (rng.raw64(41, "h", 3000) & np.uint64(0x3FFF0000)).astype(np.uint32) | np.uint32(0x8000)
    hw = np.concatenate([hw, hw + 1, hw - 1]).view(np.float32)
    vals = np.concatenate([base, hw, -hw])
    K = 128
    r = len(vals) // K
    return vals[: r * K].reshape(r, K)


def test_quantize_bf16_bit_exact(m):
    banner("quantize bf16 bit-exact")
    x = _edge_rows()
    q, _ = m.mrf_quantize_rows(dev(x), "bf16", out_pitch=256)
    got = host(q).view(np.uint16)
    ref = (quant.bf16_round(x).view(np.uint32) >> 16).astype(np.uint16)
    np.testing.assert_array_equal(got[:, :128], ref)
    assert np.all(got[:, 128:] == 0)


def test_quantize_fp8_bit_exact(m):
    banner("quantize fp8 e4m3 bit-exact")
    x = _edge_rows()
    x[0] = 0.0          # all-zero row -> scale 1, codes 0
    q, sc = m.mrf_quantize_rows(dev(x), "fp8", out_pitch=256)
    codes, scales, _ = quant.quantise_rows_e4m3(x)
    np.testing.assert_array_equal(host(sc), scales)
    np.testing.assert_array_equal(host(q)[:, :128], codes)
    assert np.all(host(q)[:, 128:] == 0)


def test_dictionary_copies_match_encoders(m):
    banner("dictionary fp32/bf16/fp8 copies vs oracle encoders")
    Dd = workloads.bssfp_dictionary(L=50, n_t1=10, n_t2=10, n_df=5, seed=2)
    D = m.Dictionary(Dd.atoms, Dd.params, store_bf16=True, store_fp8=True)
    f32 = host(m.mrf_dict_copy_atoms(D, "fp32"))
    ref = quant.as_real_rows(mf.normalised_atoms_f32(Dd.atoms))
    # FP64 norms summed in a different order may move a value by one ulp
    assert np.max(np.abs(f32 - ref)) <= np.max(np.abs(ref)) * 2 ** -23
    b = host(m.mrf_dict_copy_atoms(D, "bf16")).view(np.uint16)
    np.testing.assert_array_equal(b, (quant.bf16_round(f32).view(np.uint32) >> 16).astype(np.uint16))
    c, s = m.mrf_dict_copy_atoms(D, "fp8")
    codes, scales, _ = quant.quantise_rows_e4m3(f32)
    np.testing.assert_array_equal(host(s), scales)
    np.testing.assert_array_equal(host(c), codes)


def _lowp_case(m, kind):
    if kind == "fisp":
        Dd = workloads.fisp_dictionary(L=100)
        n = 4096
    else:
        Dd = workloads.bssfp_dictionary(L=60, n_t1=20, n_t2=20, n_df=9, seed=2)
        n = 3000
    D = m.Dictionary(Dd.atoms, Dd.params, store_bf16=True, store_fp8=True)
    Z, j, pd, snr = workloads.random_voxels(Dd, n, seed=7, snr_db_range=(15.0, 40.0))
    return Dd, D, c64(Z)


@pytest.mark.parametrize("precision", ["bf16", "fp8"])
@pytest.mark.parametrize("kind", ["fisp", "bssfp"])
def test_lowp_certified_is_exact(m, precision, kind):
    """Certified reduced-precision scoring (the default) returns the exact
    matched filter: index equal to the FP64 oracle's outside near-ties, PD
    and corr from the exact score."""
    banner(f"lowp certified match {precision} {kind}")
    Dd, D, Z = _lowp_case(m, kind)
    out = m.mrf_match(D, dev(Z), precision=precision, stats=True)
    st = out["stats"]
    gidx = host(out["idx"]).astype(np.int64)
    exact = mf.exact_mf(Z.astype(np.complex128), Dd.atoms)
    diff = gidx != exact["idx"]
    if np.any(diff):
        ok = mf.index_ok(Z[diff].astype(np.complex128), Dd.atoms, gidx[diff], tol=1e-6)
        assert np.all(ok), f"{np.sum(~ok)} index mismatches beyond the near-tie rule"
    same = ~diff
    np.testing.assert_allclose(host(out["pd"])[same], exact["gamma"][same], rtol=2e-5,
                               atol=1e-6 * exact["gamma"].max())
    print(f"{precision}/{kind}: certified, {int(diff.sum())} near-tie differences; candidates rescored "
          f"{st.cert_rescored} ({st.cert_rescored / Z.shape[0]:.1f} per voxel), FP32 rescans {st.cert_rescanned}, "
          f"full scans {st.cert_scanned}")
    # the FP32 and split-BF16 certified filters return the same answers
    ref = m.mrf_match(D, dev(Z), precision="fp32")
    np.testing.assert_array_equal(gidx, host(ref["idx"]))
    np.testing.assert_array_equal(host(out["pd"]), host(ref["pd"]))


@pytest.mark.parametrize("precision", ["bf16", "fp8"])
@pytest.mark.parametrize("kind", ["fisp", "bssfp"])
def test_lowp_uncertified_parity(m, precision, kind):
    """Without the certificate: the reduced-precision argmax (the oracle's
    precision form with one candidate, same FP32 operands), its PD from the
    exact score.  The GPU accumulates the quantised products in FP32, the
    oracle in FP64, so the two may differ only where the oracle's quantised
    scores of the two picks are within the FP32 accumulation bound."""
    banner(f"lowp uncertified match {precision} {kind}")
    Dd, D, Z = _lowp_case(m, kind)
    out = m.mrf_match(D, dev(Z), precision=precision, certify=False)
    gidx = host(out["idx"]).astype(np.int64)
    f32 = host(m.mrf_dict_copy_atoms(D, "fp32"))
    Zr = quant.as_real_rows(Z) if Dd.is_complex else np.ascontiguousarray(Z.real)
    ref = quant.quantised_match(Zr, f32, precision, topk=1)
    exact = mf.exact_mf(Z.astype(np.complex128), Dd.atoms)
    agree_q = np.mean(gidx == ref["idx"])
    ok_x = mf.index_ok(Z.astype(np.complex128), Dd.atoms, gidx, tol=1e-6)
    print(f"{precision}/{kind}: agreement with the oracle's precision form {agree_q:.5f}, exact FP64 within "
          f"near-tie {np.mean(ok_x):.5f}")
    diff = gidx != ref["idx"]
    if np.any(diff):
        if precision == "bf16":
            zq, dq = quant.bf16_round(Zr).astype(np.float64), quant.bf16_round(f32).astype(np.float64)
        else:
            zq, dq = quant.quantise_rows_e4m3(Zr)[2], quant.quantise_rows_e4m3(f32)[2]
        K = Zr.shape[1]
        g = 2 * (K + 1) * 2.0 ** -24
        a = np.einsum("nk,nk->n", zq[diff], dq[gidx[diff]])
        b = np.einsum("nk,nk->n", zq[diff], dq[ref["idx"][diff]])
        bound = g * np.linalg.norm(zq[diff], axis=1) * np.max(np.linalg.norm(dq, axis=1))
        assert np.all(np.abs(a - b) <= 2 * bound)
    # PD from the exact score of the returned atom
    sc = np.einsum("nk,nk->n", Zr.astype(np.float64), f32[gidx].astype(np.float64))
    inv = 1.0 / mf.atom_norms(Dd.atoms)
    np.testing.assert_allclose(host(out["pd"]), np.maximum(sc, 0) * inv[gidx], rtol=2e-5, atol=1e-7)
