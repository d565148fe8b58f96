"""mrf_match_noalloc (the exhaustive FP32 filter on the library's fixed device
workspace) against mrf_match through the C ABI: identical idx / pd / corr /
X / params on two calls in a row, the second smaller, in both layouts and
with and without the certificate; calls past the workspace are refused
before any device work."""
import ctypes

import numpy as np
import pytest

from gpu_helpers import banner, c64, dev, host
from synth import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def m():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1810_01967_amd as pkg
    pkg.lib()
    return pkg


def _outputs(torch, n, nparam, Z):
    return {"idx": torch.full((n,), -7, dtype=torch.int32, device="cuda"),
            "pd": torch.full((n,), -7.0, dtype=torch.float32, device="cuda"),
            "corr": torch.full((n,), -7.0, dtype=torch.float32, device="cuda"),
            "X": torch.zeros_like(Z),
            "params": torch.full((n, nparam), -7.0, dtype=torch.float32, device="cuda")}


def _same(a, b):
    for k in ("idx", "pd", "corr", "X", "params"):
        np.testing.assert_array_equal(host(a[k]), host(b[k]), err_msg=k)


@pytest.mark.parametrize("certify", [True, False])
def test_noalloc_equals_match_voxel_major(m, certify):
    import torch
    Dd = workloads.fisp_dictionary()
    D = m.Dictionary(Dd.atoms, Dd.params, grid_dims=Dd.grid_dims)
    Z, _, _, _ = workloads.random_voxels(Dd, 3001, seed=41, snr_db_range=(15.0, 40.0))
    for n in (3001, 700):  # the second call is smaller and reuses the workspace
        banner(f"noalloc vs mrf_match: FISP d=2000 L=100 n={n} voxel-major certify={certify}")
        Zd = dev(c64(Z[:n]))
        ref = m.mrf_match(D, Zd, want_X=True, want_params=True, certify=certify)
        got = m.mrf_match_noalloc(D, Zd, _outputs(torch, n, Dd.params.shape[1], Zd), certify=certify)
        _same(ref, got)


def test_noalloc_equals_match_frame_major(m):
    import torch
    Dd = workloads.bssfp_dictionary(L=100, n_t1=20, n_t2=20, n_df=9, seed=2)
    D = m.Dictionary(Dd.atoms, Dd.params, grid_dims=Dd.grid_dims)
    for S, ny, nx in ((2, 32, 32), (1, 16, 24)):
        n = S * ny * nx
        banner(f"noalloc vs mrf_match: bSSFP d={Dd.d} L=100 frame-major {S}x{ny}x{nx}")
        Zv, _, _, _ = workloads.random_voxels(Dd, n, seed=42 + S, snr_db_range=(10.0, 40.0))
        Zf = c64(Zv.reshape(S, ny, nx, Dd.L).transpose(0, 3, 1, 2))
        Zd = dev(Zf)
        ref = m.mrf_match(D, Zd, layout="frame", slice_voxels=ny * nx, want_X=True, want_params=True)
        got = m.mrf_match_noalloc(D, Zd, _outputs(torch, n, Dd.params.shape[1], Zd), layout="frame",
                                  slice_voxels=ny * nx)
        _same(ref, got)


def test_noalloc_refuses_oversized_and_other_paths(m):
    import torch
    banner("noalloc: refused calls")
    Dd = workloads.bssfp_dictionary(L=500, n_t1=6, n_t2=6, n_df=4, seed=2)
    D = m.Dictionary(Dd.atoms, Dd.params, grid_dims=Dd.grid_dims)
    n = 16384  # 16,384 x 1,008 x 4 bytes of packed rows alone exceed 32 MiB
    Zd = torch.zeros((n, Dd.L), dtype=torch.complex64, device="cuda")
    out = {"idx": torch.full((n,), -7, dtype=torch.int32, device="cuda")}
    with pytest.raises(m.MrfError) as e:
        m.mrf_match_noalloc(D, Zd, out)
    assert e.value.status == -1
    assert "workspace" in str(e.value)
    assert int(host(out["idx"]).min()) == -7  # nothing was written
    opts = m.mrf.match_opts("bf16x3", 8, 0)
    st = m.lib().mrf_match_noalloc(D.handle, ctypes.byref(opts), 4, Zd.data_ptr(), 0, 0, None,
                                   out["idx"].data_ptr(), None, None, None, None, None)
    assert st == -4
