"""The multi-parametric dictionary: L = 1000 complex frames, IR-bSSFP on
T1 (80) x T2 (80) x B1 in [0.6, 1.4] (17) x df in [-40, 40] Hz (11) =
1,196,800 atoms (9.6 GB FP32, 4.8 GB BF16 on the device), a four-output
network and a 7^4 = 2,401-atom local box.

* standalone: 4,096 noisy atoms, the learned path (split-BF16 local search)
  against the certified exhaustive split-BF16 filter (the exact argmax over
  all 1.2 M atoms), at most 0.1 % index mismatch, the certified answers
  checked against the FP64 oracle on sampled voxels and on every voxel
  where the two paths disagree (near-tie rule, gap 1e-6);
* one projected-gradient step batched over 16 slices of 32 x 32 with uneven
  masks (2 + s/2 of 32 lines per frame in slice s): learned against the
  certified exhaustive projection (same objective; at most 0.1 % of the
  tissue voxels where the learned atom's FP64 correlation falls more than
  1e-6 below the certified one), the certified answers graded on sampled
  voxels against the oracle's projection of the oracle's gradient step.

The voxel counts are reduced from the 256 x 256 x 16 workload to keep the
oracle's share (2.4 GFLOP per voxel in FP64 over all atoms) small; the
device side at the full shape (1,048,576 voxels: 16.5 s for the uncertified
split-BF16 filter, 0.13 s for the learned path) is timed by the bench's
multi-parametric rows."""
import numpy as np
import pytest

from gpu_helpers import banner, c64, dev, host
from oracle import ipg, mf
from synth import rng, workloads

pytestmark = pytest.mark.gpu

L = 1000


@pytest.fixture(scope="module")
def big():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1810_01967_amd as m
    banner("1,196,800-atom dictionary: generate, upload, train a 4-output network")
    Dd = workloads.bssfp_dictionary(L=L, n_t1=80, n_t2=80, n_df=11, b1_axis=np.linspace(0.6, 1.4, 17),
                                    dtype=np.complex64)
    assert Dd.atoms.shape == (1_196_800, L) and tuple(Dd.grid_dims) == (80, 80, 17, 11)
    D = m.Dictionary(Dd.atoms, Dd.params, grid_dims=Dd.grid_dims, store_bf16=True)
    net = m.Net(2 * L, 4, hidden=256, seed=11)
    tr = m.mrf_net_train(net, D, samples=2_000_000, batch=4096, epochs=4, lr=1e-3, lr_min=1e-5, snr_lo=15.0,
                         snr_hi=40.0, seed=12)
    print(f"training loss {tr['first_loss']:.3f} -> {tr['last_loss']:.5f} in {tr['ms'] / 1e3:.1f} s")
    return m, Dd, D, net


def _exact(Z, atoms, chunk=40000):
    """FP64 oracle over all atoms in chunks: best normalised correlation and
    its lowest index."""
    best = np.full(Z.shape[0], -np.inf)
    arg = np.zeros(Z.shape[0], dtype=np.int64)
    for a0 in range(0, atoms.shape[0], chunk):
        c = mf.correlations(Z, atoms[a0:a0 + chunk])
        j = np.argmax(c, axis=1)
        v = c[np.arange(Z.shape[0]), j]
        upd = v > best
        best[upd], arg[upd] = v[upd], a0 + j[upd]
    zn = np.linalg.norm(Z, axis=1)
    return best / zn, arg


def _corr(Z, atoms, idx):
    a = atoms[idx].astype(np.complex128)
    return np.real(np.sum(np.conj(a) * Z, axis=1)) / np.linalg.norm(a, axis=1) / np.linalg.norm(Z, axis=1)


def test_bigdict_learned_vs_bf16(big):
    m, Dd, D, net = big
    banner("1.2M atoms: learned (split BF16) vs the certified exhaustive filter, 4,096 voxels")
    n = 4096
    Z, j, pd, snr = workloads.random_voxels(Dd, n, seed=5)
    Z = c64(Z)
    Zd = dev(Z)
    ob = m.mrf_match(D, Zd, precision="bf16x3", stats=True)  # certified: the exact argmax
    ol = m.mrf_match(D, Zd, net=net, precision="bf16x3", box_radius=3, fallback_corr=0.98, recentre=2,
                     stats=True)
    ib, il = host(ob["idx"]).astype(np.int64), host(ol["idx"]).astype(np.int64)
    st = ol["stats"]
    mism = float(np.mean(ib != il))
    print(f"certified exhaustive {ob['stats'].ms:.1f} ms ({ob['stats'].cert_rescanned} rescanned, "
          f"{ob['stats'].cert_scanned} scanned); learned {st.ms:.2f} ms ({st.first_box_atoms / n:.0f} box "
          f"atoms per voxel, {st.fallbacks} fallbacks, {st.recentred} re-centred); index mismatch {mism:.4f}")
    # grade on the FP64 oracle over all atoms: 48 random voxels and every
    # voxel where the two paths disagree
    sample = np.union1d(rng.permutation(5, "sample", n)[:48], np.flatnonzero(ib != il))
    Zs = Z[sample].astype(np.complex128)
    best, arg = _exact(Zs, Dd.atoms)
    cl, cb = _corr(Zs, Dd.atoms, il[sample]), _corr(Zs, Dd.atoms, ib[sample])
    ok_l, ok_b = cl >= best - 1e-6, cb >= best - 1e-6
    dis = np.isin(sample, np.flatnonzero(ib != il))
    print(f"FP64 oracle on {len(sample)} voxels ({int(dis.sum())} where the paths disagree): learned exact on "
          f"{ok_l.mean():.3f} (disagreements {ok_l[dis].mean() if dis.any() else 1:.3f}), certified on "
          f"{ok_b.mean():.3f}")
    assert np.all(ok_b)        # the certified filter is exact (near-tie rule)
    # the learned path is exact within its box; a voxel whose best atom lies
    # outside the box while its correlation stays above the fallback
    # threshold keeps the box's best: at most 0.1 % of the voxels
    assert mism <= 0.001


def test_bigdict_batched_step_uneven_masks(big):
    m, Dd, D, net = big
    banner("1.2M atoms: one IPG step over 16 slices of 32 x 32 with uneven masks")
    import torch
    S, size = 16, 32
    ph = workloads.smooth_phantom(Dd, seed=6, S=S, size=size)
    smp = workloads.random_lines(6, S, L, size, size, [2 + s // 2 for s in range(S)])
    Y = workloads.simulate_kspace(ph.X0, smp, 30.0, seed=6)
    A = m.Operator.from_sampling(smp)
    Yd = dev(c64(Y))
    X0 = torch.zeros((S, L, size, size), dtype=torch.complex64, device="cuda")
    Xe, ie, pde, ste = m.mrf_ipg_step(D, A, Yd, X0, 1.0, precision="bf16x3")  # certified
    Xl, il, pdl, stl = m.mrf_ipg_step(D, A, Yd, X0, 1.0, net=net, precision="bf16x3", recentre=2)
    ie, il = host(ie).astype(np.int64), host(il).astype(np.int64)
    head = ph.idx >= 0
    agree = float(np.mean(ie[head] == il[head]))
    print(f"step: |dX|^2 exhaustive {ste.dx2:.5e} learned {stl.dx2:.5e}; f exhaustive {ste.f_out:.6e} "
          f"learned {stl.f_out:.6e}; tissue indices learned = exhaustive {agree:.4f}")
    # oracle: Z = X0 - mu G = -G at X0 = 0, projected exactly on 32 random
    # tissue voxels and up to 64 voxels where the two projections disagree
    G, _ = ipg.gradient(np.zeros((S, L, size, size)), Y, smp.off, smp.idx, None)
    Zv = (-G).transpose(0, 2, 3, 1).reshape(S * size * size, L)
    tissue = np.flatnonzero(head)
    dis = tissue[ie[tissue] != il[tissue]]
    vox = np.union1d(tissue[rng.permutation(6, "sample", tissue.size)[:32]],
                     dis[rng.permutation(6, "dis", dis.size)[:64]])
    best, arg = _exact(Zv[vox], Dd.atoms)
    ok_l = _corr(Zv[vox], Dd.atoms, il[vox]) >= best - 1e-6
    ok_b = _corr(Zv[vox], Dd.atoms, ie[vox]) >= best - 1e-6
    isdis = np.isin(vox, dis)
    print(f"FP64 oracle on {vox.size} voxels ({int(isdis.sum())} disagreements): learned exact on {ok_l.mean():.3f} "
          f"(disagreements {ok_l[isdis].mean() if isdis.any() else 1:.3f}), certified on {ok_b.mean():.3f}")
    # the device's gradient step is FP32: its Z differs from the oracle's by
    # ~1e-7 relative, so a certified index may differ from the oracle's where
    # the oracle's own gap is below that; count only larger gaps
    assert np.mean(ok_b) >= 0.99
    assert abs(stl.f_out - ste.f_out) <= 0.001 * ste.f_out
    # from X = 0 the correlation landscape is flat and many voxels hold
    # near-ties: every tissue voxel where the two projections disagree is
    # graded in FP64 (the learned atom against the certified one), and at
    # most 0.1 % of the tissue may fall more than 1e-6 below it
    c_l, c_e = _corr(Zv[dis], Dd.atoms, il[dis]), _corr(Zv[dis], Dd.atoms, ie[dis])
    below = int(np.sum(c_l < c_e - 1e-6))
    print(f"tissue voxels {tissue.size}: {dis.size} disagreements, {below} more than 1e-6 below the certified atom")
    assert below <= 0.001 * tissue.size
