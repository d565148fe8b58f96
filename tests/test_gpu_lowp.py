"""GPU parity of the reduced-precision forms of the matched filter: the BF16
and FP8-E4M3 encoders bit-exact against the oracle's encoders, and the
candidate scoring + FP32 rescore against the oracle's precision form and the
exact FP64 matched filter."""
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


@pytest.mark.parametrize("precision", ["bf16", "fp8"])
@pytest.mark.parametrize("kind", ["fisp", "bssfp"])
def test_lowp_match_parity(m, precision, kind):
    """Against the oracle's precision form (same FP32 operands): the final
    index is the oracle's or a near-tie of it (rescore within 1e-6), and the
    rescored candidate beats or equals the 8th candidate of the oracle.  The
    agreement with the exact FP64 matched filter is reported."""
    banner(f"lowp match {precision} {kind}")
    if kind == "fisp":
        Dd = workloads.fisp_dictionary(L=100)
        n = 4096
    else:
        Dd = workloads.bssfp_dictionary(L=60, n_t1=20, n_t2=20, n_df=9, seed=2)
        n = 3000
    D = m.Dictionary(Dd.atoms, Dd.params, store_bf16=True, store_fp8=True)
    Z, j, pd, snr = workloads.random_voxels(Dd, n, seed=7, snr_db_range=(15.0, 40.0))
    Z = c64(Z)
    out = m.mrf_match(D, dev(Z), precision=precision, topk=8)
    gidx = host(out["idx"]).astype(np.int64)
    f32 = host(m.mrf_dict_copy_atoms(D, "fp32"))
    Zr = quant.as_real_rows(Z) if Dd.is_complex else np.ascontiguousarray(Z.real)
    ref = quant.quantised_match(Zr, f32, precision, topk=8)
    exact = mf.exact_mf(Z.astype(np.complex128), Dd.atoms)
    agree_q = np.mean(gidx == ref["idx"])
    agree_x = np.mean(gidx == exact["idx"])
    ok_x = mf.index_ok(Z.astype(np.complex128), Dd.atoms, gidx, tol=1e-6)
    print(f"{precision}/{kind}: agreement with oracle precision form {agree_q:.5f}, with exact FP64 "
          f"{agree_x:.5f} (within near-tie {np.mean(ok_x):.5f})")
    # differences from the oracle's precision form may only come from the
    # top-8 boundary: the GPU's pick must score (FP64 rescore) at least as
    # well as the oracle's 8th candidate, and equal the oracle where the
    # oracle's pick is far inside the top-8 set
    diff = gidx != ref["idx"]
    if np.any(diff):
        zz = Zr[diff].astype(np.float64)
        got = np.einsum("nk,nk->n", zz, f32[gidx[diff]].astype(np.float64))
        eighth = np.einsum("nk,nk->n", zz, f32[ref["cand"][diff, -1]].astype(np.float64))
        assert np.all(got >= eighth - 1e-6 * np.linalg.norm(zz, axis=1))
    assert agree_q > 0.995
    # the agreement with the exact FP64 filter is a measured property of the
    # precision form (coherent dictionaries reorder beyond the top 8); it is
    # reported, not pinned

