"""Benchmark: matched-filter voxels/s at ~100k atoms, L = 500 (one GPU);
learned proposal + local search vs exhaustive.

Workload: 256 x 256 = 65,536 voxels, L = 500 complex64 frames, IR-bSSFP
dictionary T1 60 x T2 60 x df 28 = 100,800 atoms.  Voxels are random atoms
scaled by PD ~ U(0.3, 1) with complex Gaussian noise at SNR ~ U(20, 40) dB
(seeded, synthetic).  One step = one mrf_match call over all voxels: the
whole projection, inputs resident in HBM:
  * exhaustive: voxel packing, [quantisation,] scoring with the fused argmax
    / top-k, split merge, [FP32 rescore,] rescaling and look-up;
  * learned: voxel packing, network proposal, cell mapping, grouping, local
    search, re-centring, exhaustive fallback, rescaling and look-up.
Dictionary generation, upload, cover-tree build and network training are
outside the timed region (their times are reported).  The cover-tree
comparator (Algorithm 1, batched) is timed the same way over an eps sweep
with its recall@1 against the exhaustive FP32 filter.  The headline value is the learned
path when its index mismatch against the exhaustive FP32 filter is at most
0.1 %, else the exhaustive FP32 path.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

TRAFFIC = os.path.join(HERE, "profiles", "local_score_bf16x3_65536vox_traffic.json")


def measured_traffic(kernel_source):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE, each scaled by what the counter reads
    for a copy of known size), or None when the kernel's source has changed
    since the counters were taken."""
    import hashlib
    try:
        t = json.load(open(TRAFFIC))
        src = open(os.path.join(HERE, "paper_1810_01967_amd", "csrc", kernel_source), "rb").read()
    except (OSError, ValueError):
        return None
    if hashlib.sha256(src).hexdigest() != t.get("source_sha256"):
        return None
    return t["fetch_bytes_per_launch"] + t["write_bytes_per_launch"]


# MI355X published dense peaks
PEAK = {"fp32": 157.3, "bf16": 2500.0, "fp8": 5000.0}   # TFLOP/s
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--variants", type=int, default=1, help="also time BF16 / FP8 exhaustive scoring")
    ap.add_argument("--learned", type=int, default=1, help="train the network and time the learned path")
    ap.add_argument("--net-cache", default="",
                    help="network file: loaded if it exists (no training), else written after training; lets a "
                         "profiled run time the very network of an earlier run")
    ap.add_argument("--train-samples", type=int, default=2_000_000)
    ap.add_argument("--train-epochs", type=int, default=4)
    ap.add_argument("--recentre", type=int, default=1, help="re-centring rounds of the local search")
    ap.add_argument("--box-radius", type=int, default=2, help="local-search box radius (grid cells)")
    ap.add_argument("--learned-precisions", default="bf16x3,fp32",
                    help="local-search arithmetic(s) of the learned path")
    ap.add_argument("--tree", type=int, default=1, help="build the cover tree and run the eps sweep")
    ap.add_argument("--iteration", type=int, default=1,
                    help="time projected-gradient steps: Cartesian 1 / 4 coils, spiral non-uniform FFT with "
                         "6 coils and DCF (also compressed, s = 200), phase-aligned")
    ap.add_argument("--subspace", default="20,200",
                    help="temporal subspace sizes s for the compressed matched filter ('' to skip)")
    ap.add_argument("--cpu-baseline", type=int, default=1, help="time the FP64 oracle on a sample")
    ap.add_argument("--cpu-sample", type=int, default=32768, help="voxels in the oracle sample")
    ap.add_argument("--splits", type=int, default=0, help="atom splits (0 = library default)")
    ap.add_argument("--n", type=int, default=65536)
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="run one 1 GiB device-to-device copy (reference for HBM byte counters)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the matched filter runs on one GPU; runs on several GPUs are not "
                                   "supported",
                          "n_gpus": args.gpus}), flush=True)
        return 2
    import torch
    import paper_1810_01967_amd as m
    from synth import workloads

    t0 = time.time()
    Dd = workloads.bssfp_dictionary(L=500)
    Z, jtrue, pd_true, snr = workloads.random_voxels(Dd, args.n, seed=2)
    Z = Z.astype(np.complex64)
    log(f"inputs generated in {time.time() - t0:.1f}s: d={Dd.d} L={Dd.L} n={args.n}")
    t1 = time.time()
    D = m.Dictionary(Dd.atoms, Dd.params, grid_dims=Dd.grid_dims, store_bf16=True, store_fp8=True)
    Zd = torch.from_numpy(Z).cuda()
    torch.cuda.synchronize()
    log(f"dictionary built and uploaded in {time.time() - t1:.1f}s")
    n, d, K = args.n, Dd.d, 2 * Dd.L
    flops = 2.0 * n * d * K               # algorithmic: one real MAC per (voxel, atom, real dim)

    def run(steps, warmup, D_=None, **kw):
        """Time `steps` calls as a caller makes them (no per-call statistics:
        those record device events and read them back, which synchronises the
        stream).  Three more calls after the timed region request the
        statistics (stage and kernel times, counts); they are averaged."""
        DD = D if D_ is None else D_
        o = {}
        for _ in range(warmup):
            o = m.mrf_match(DD, Zd, atom_splits=args.splits, want_corr=False, out=o, **kw)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(steps):
            o = m.mrf_match(DD, Zd, atom_splits=args.splits, want_corr=False, out=o, **kw)
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / steps
        st = []
        for _ in range(3):
            o = m.mrf_match(DD, Zd, atom_splits=args.splits, want_corr=False, out=o, stats=True, **kw)
            s = o["stats"]
            st.append((s.score_ms, s.proposal_ms, s.fallback_ms, s.fallbacks, s.recentred, s.local_atoms,
                       s.search_ms, s.first_box_atoms))
        return ms, np.mean(np.array(st, dtype=np.float64), axis=0), o

    ms32, st32, o32 = run(args.steps, args.warmup, precision="fp32")
    idx32 = o32["idx"].cpu().numpy()
    answers = {"exhaustive_fp32": (idx32, o32["pd"].cpu().numpy())}   # checked against FP64 on the sample
    score_ms32 = float(st32[0])
    log(f"exhaustive fp32: {ms32:.3f} ms/step, scoring kernel {score_ms32:.3f} ms, "
        f"splits {o32['stats'].splits}")
    exhaustive = {"voxels_per_s": n / (ms32 * 1e-3), "ms_per_step": ms32, "score_kernel_ms": score_ms32,
                  "mfma_frac": flops / (score_ms32 * 1e-3) / 1e12 / PEAK["fp32"],
                  "recovered_generating_atom": float(np.mean(idx32 == jtrue))}
    variants = {}
    if args.variants:
        for p in ("bf16x3", "bf16", "fp8"):
            vms, vst, vo = run(max(3, args.steps // 2), 1, precision=p)
            vidx = vo["idx"].cpu().numpy()
            answers[f"exhaustive_{p}"] = (vidx, vo["pd"].cpu().numpy())
            # split BF16 executes three BF16 products per algorithmic one
            mult, pk = (3.0, PEAK["bf16"]) if p == "bf16x3" else (1.0, PEAK[p])
            variants[p] = {"voxels_per_s": n / (vms * 1e-3), "ms_per_step": vms,
                           "score_kernel_ms": float(vst[0]),
                           "algorithmic_tflops": flops / (float(vst[0]) * 1e-3) / 1e12,
                           "mfma_frac": mult * flops / (float(vst[0]) * 1e-3) / 1e12 / pk,
                           "index_mismatch_vs_fp32": float(np.mean(vidx != idx32))}
            log(f"exhaustive {p}: {vms:.3f} ms/step, scoring kernel {vst[0]:.3f} ms, "
                f"mismatch vs fp32 {variants[p]['index_mismatch_vs_fp32']:.5f}")
    learned = None
    if args.learned:
        t2 = time.time()
        if args.net_cache and os.path.exists(args.net_cache):
            net = m.Net.load(args.net_cache)
            log(f"network loaded from {args.net_cache}")
            learned = {"training": {"loaded": args.net_cache}}
        else:
            net = m.Net(K, Dd.params.shape[1], hidden=256, seed=11)
            tr = m.mrf_net_train(net, D, samples=args.train_samples, batch=4096, epochs=args.train_epochs,
                                 lr=1e-3, lr_min=1e-5, snr_lo=15.0, snr_hi=40.0, seed=12)
            log(f"network trained in {time.time() - t2:.1f}s ({tr['steps']} steps, loss "
                f"{tr['first_loss']:.4f} -> {tr['last_loss']:.5f})")
            learned = {"training": {"samples": args.train_samples, "epochs": args.train_epochs,
                                    "steps": tr["steps"], "seconds": tr["ms"] / 1e3,
                                    "loss_first": tr["first_loss"], "loss_last": tr["last_loss"]}}
            if args.net_cache:
                net.save(args.net_cache)
        fastest = min([ms32] + [v["ms_per_step"] for v in variants.values()
                                if v["index_mismatch_vs_fp32"] <= 1e-3])
        for lp in args.learned_precisions.split(","):
            lms, lst, lo = run(args.steps, args.warmup, net=net, box_radius=args.box_radius, fallback_corr=0.98,
                               recentre=args.recentre, precision=lp)
            lidx = lo["idx"].cpu().numpy()
            answers[f"learned_{lp}"] = (lidx, lo["pd"].cpu().numpy())
            mism = float(np.mean(lidx != idx32))
            # algorithmic work of the first local-search launch: 2 K flops per
            # (voxel, atom of its clipped box)
            box_flops = 2.0 * K * float(lst[7])
            learned[lp] = {"voxels_per_s": n / (lms * 1e-3), "ms_per_step": lms,
                           "index_mismatch_vs_exhaustive_fp32": mism,
                           "local_score_kernel_ms": float(lst[0]), "local_search_ms": float(lst[6]),
                           "proposal_ms": float(lst[1]),
                           "fallback_ms": float(lst[2]), "fallbacks_per_step": float(lst[3]),
                           "recentred_per_step": float(lst[4]), "local_atoms_scored": float(lst[5]),
                           "first_launch_box_atoms": float(lst[7]),
                           "speedup_vs_exhaustive_fp32": ms32 / lms,
                           "speedup_vs_fastest_exhaustive_within_0.1pct": fastest / lms,
                           "box_flop_first_launch": box_flops}
            log(f"learned ({lp}): {lms:.3f} ms/step (local search {lst[6]:.3f}, first scoring kernel "
                f"{lst[0]:.3f}, proposal {lst[1]:.3f}, fallback {lst[2]:.3f} ms, {lst[3]:.0f} fallbacks, "
                f"{lst[4]:.0f} re-centred, {lst[7] / n:.1f} box atoms per voxel), mismatch {mism:.5f}")

    tree = None
    DT = None
    if args.tree:
        t3 = time.time()
        DT = m.Dictionary(Dd.atoms, Dd.params, grid_dims=Dd.grid_dims, cover_tree=True)
        tb = time.time() - t3
        ti = DT.tree_info()
        log(f"cover tree built in {tb:.1f}s: {ti.unique_atoms} unique atoms, {ti.imax + 1} levels, "
            f"{ti.entries} entries")
        tree = {"build_seconds": tb, "levels": ti.imax + 1, "entries": int(ti.entries), "sweep": []}
        for eps in (0.0, 0.1, 0.2, 0.4, 0.8, 1.6):
            tms, tst, to = run(max(3, args.steps // 2), 1, D_=DT, eps=eps)
            tidx = to["idx"].cpu().numpy()
            answers[f"cover_tree_eps{eps}"] = (tidx, to["pd"].cpu().numpy())
            evals = to["stats"].distance_evals / n
            row = {"eps": eps, "voxels_per_s": n / (tms * 1e-3), "ms_per_step": tms,
                   "search_ms": float(tst[6]), "recall_at_1_vs_exhaustive_fp32": float(np.mean(tidx == idx32)),
                   "distance_evals_per_voxel": evals, "distance_reduction_vs_exhaustive": d / evals,
                   "fallbacks": int(to["stats"].fallbacks)}
            tree["sweep"].append(row)
            log(f"cover tree eps={eps}: {tms:.3f} ms/step, recall@1 {row['recall_at_1_vs_exhaustive_fp32']:.4f}, "
                f"{evals:.0f} distances per voxel, {row['fallbacks']} fallbacks")

    subspace = None
    if args.subspace:
        subspace = []
        for sdim in [int(x) for x in args.subspace.split(",") if x]:
            t4 = time.time()
            C = D.compress(sdim)
            torch.cuda.synchronize()
            tb = time.time() - t4
            V, lam = C.subspace()
            # voxels arrive compressed (Z~ = V^H Z per voxel), prepared on the host
            Zc = torch.from_numpy((Z @ V.conj().astype(np.complex64)).astype(np.complex64)).cuda()
            row = {"s": sdim, "build_seconds": tb,
                   "energy_kept": float(lam.sum() / d)}
            for p in ("fp32", "bf16x3"):
                o = {}
                for _ in range(2):
                    o = m.mrf_match(C, Zc, precision=p, want_corr=False, out=o)
                torch.cuda.synchronize()
                ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                ksteps = max(3, args.steps)
                ev0.record()
                for _ in range(ksteps):
                    o = m.mrf_match(C, Zc, precision=p, want_corr=False, out=o)
                ev1.record()
                torch.cuda.synchronize()
                cms = ev0.elapsed_time(ev1) / ksteps
                cidx = o["idx"].cpu().numpy()
                answers[f"subspace{sdim}_{p}"] = (cidx, o["pd"].cpu().numpy())
                row[p] = {"voxels_per_s": n / (cms * 1e-3), "ms_per_step": cms,
                          "index_agreement_vs_full_fp32": float(np.mean(cidx == idx32)),
                          "recovered_generating_atom": float(np.mean(cidx == jtrue))}
                log(f"subspace s={sdim} {p}: {cms:.3f} ms/step, agreement with the full filter "
                    f"{row[p]['index_agreement_vs_full_fp32']:.4f}, generating atom "
                    f"{row[p]['recovered_generating_atom']:.4f}")
            subspace.append(row)
            del C, Zc

    iteration = None
    if args.iteration:
        iteration = iteration_bench(m, torch, D, Dd, net if args.learned else None, args, DT)

    ok = [lp for lp in args.learned_precisions.split(",")
          if learned is not None and learned[lp]["index_mismatch_vs_exhaustive_fp32"] <= 1e-3]
    if ok:
        lp = min(ok, key=lambda p: learned[p]["ms_per_step"])
        L_ = learned[lp]
        ms = L_["ms_per_step"]
        path = f"learned-proposal+local-search ({'split-BF16 MFMA' if lp == 'bf16x3' else 'FP32 MFMA'})"
        dt = "bf16x3" if lp == "bf16x3" else "f32"
        pk = PEAK["bf16"] if lp == "bf16x3" else PEAK["fp32"]
        # dominant kernel: the first local-search scoring launch.  Its
        # algorithmic intensity (2 K flops per box atom over the bytes of
        # every voxel row and every dictionary row read once, 4 bytes per
        # element in FP32 or split BF16) is ~60 flop/byte, below both MFMA
        # ridges, so its roofline is HBM bandwidth
        kern_ms = L_["local_score_kernel_ms"]
        alg_bytes = 4.0 * K * (n + d) + 8.0 * n
        achieved = alg_bytes / (kern_ms * 1e-3) / 1e9
        tf = L_["box_flop_first_launch"] / (kern_ms * 1e-3) / 1e12
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS,
                "traffic": measured_traffic("k_local.hip") if lp == "bf16x3" else None,
                "kernel": f"k_local_score<{'split-BF16' if lp == 'bf16x3' else 'FP32'}> (first launch)",
                "algorithmic_bytes_per_launch": alg_bytes, "kernel_ms": kern_ms,
                "flop_view": {"algorithmic_flop_per_launch": L_["box_flop_first_launch"], "achieved_tflops": tf,
                              "peak_tflops": pk, "frac": tf / pk}}
    else:
        ms, path, dt = ms32, "exhaustive FP32 MFMA", "f32"
        achieved = flops / (score_ms32 * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": PEAK["fp32"], "unit": "TFLOP/s",
                "frac": achieved / PEAK["fp32"], "traffic": None, "kernel": "k_score_f32",
                "algorithmic_flop_per_launch": flops, "kernel_ms": score_ms32}
    res = {
        "metric": "matched-filter voxels/s at 100k atoms, L=500; learned+local vs exhaustive",
        "value": n / (ms * 1e-3),
        "unit": "voxels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dt,
        "data": "synthetic",
        "config": {"workload": "matched filter, 256x256 voxels, L=500 complex, T1 60 x T2 60 x df 28 "
                               "= 100,800 IR-bSSFP atoms, SNR 20-40 dB",
                   "path": path, "voxels": n, "atoms": d, "L": Dd.L},
        "roofline": roof,
        "exhaustive_fp32": exhaustive,
        "variants": variants,
    }
    if learned is not None:
        res["learned"] = learned
    if tree is not None:
        res["cover_tree"] = tree
    if subspace is not None:
        res["subspace"] = subspace
    if iteration is not None:
        res["iteration"] = iteration
    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        res["copy_calibration_bytes"] = {"read": 1 << 30, "write": 1 << 30}
    if args.cpu_baseline:
        res["cpu_baseline"], res["vs_fp64_oracle_on_sample"] = cpu_baseline(Dd, Z, args.cpu_sample, answers)
    print(json.dumps(res), flush=True)
    return 0


def iteration_bench(m, torch, D, Dd, net, args, DT=None):
    """Projected-gradient steps (eq. blip / eq. blip_dcf) on the headline
    dictionary (100,800 atoms, L = 500) with the exhaustive split-BF16
    projection (and the learned one on the Cartesian case): ms per step, and
    the operator alone (A then A^H) per step.  Inputs: smooth bSSFP phantoms,
    k-space simulated on the host with noise at 30 dB."""
    from synth import workloads
    out = {}
    t0 = time.time()
    ph256 = workloads.smooth_phantom(Dd, seed=7, S=1, size=256)
    smp = workloads.random_lines(7, 1, Dd.L, 256, 256, 26)
    sm4 = workloads.coil_maps(7, 1, 4, 256, 256)
    ph128 = workloads.smooth_phantom(Dd, seed=8, S=1, size=128)
    tr = workloads.spiral_trajectory(1, Dd.L, 128, 128, frac=1.0 / 48)
    sm6 = workloads.coil_maps(8, 1, 6, 128, 128)
    Ycart = workloads.simulate_kspace(ph256.X0, smp, 30.0, 7)
    Y4 = workloads.simulate_kspace(ph256.X0, smp, 30.0, 7, smaps=sm4)
    Ysp = workloads.simulate_kspace_nc(ph128.X0, tr, 30.0, 8, smaps=sm6)
    log(f"iteration inputs generated in {time.time() - t0:.1f}s")
    Dc = D.compress(200)
    Da = D.align()
    A1 = m.Operator.from_sampling(smp)
    A4 = m.Operator.from_sampling(smp, smaps=sm4)
    As = m.Operator.from_trajectory(tr, smaps=sm6)
    cases = [("cartesian_256_1coil", D, A1, Ycart, 256, Dd.L, {}),
             ("cartesian_256_4coils", D, A4, Y4, 256, Dd.L, {}),
             ("cartesian_256_1coil_phase_aligned", Da, A1, Ycart, 256, Dd.L, {}),
             ("spiral_128_6coils_dcf_nufft", D, As, Ysp, 128, Dd.L, {}),
             ("spiral_128_6coils_dcf_nufft_s200", Dc, As, Ysp, 128, 200, {})]
    if net is not None:
        cases.insert(1, ("cartesian_256_1coil_learned", D, A1, Ycart, 256, Dd.L,
                         {"net": net, "recentre": args.recentre}))
        if DT is not None:  # the same dictionary with its cover tree: tree fallback (eps = 0, exact)
            cases.insert(2, ("cartesian_256_1coil_learned_tree_fallback", DT, A1, Ycart, 256, Dd.L,
                             {"net": net, "recentre": args.recentre, "eps": 0.0}))
    if DT is not None:  # CoverBLIP: the cover tree as the projection (Algorithm 1 inside Algorithm 2)
        for eps in (0.0, 0.4):
            cases.append((f"cartesian_256_1coil_covertree_eps{eps:g}", DT, A1, Ycart, 256, Dd.L, {"eps": eps}))
        # the paper's fast compressed setting (s = 20): exhaustive, and CoverBLIP on the compressed atoms' tree
        t1 = time.time()
        D20 = D.compress(20, cover_tree=True)
        log(f"s = 20 dictionary with its cover tree built in {time.time() - t1:.1f}s")
        cases.append(("cartesian_256_1coil_s20", D20, A1, Ycart, 256, 20, {}))
        cases.append(("cartesian_256_1coil_s20_covertree_eps0.4", D20, A1, Ycart, 256, 20, {"eps": 0.4}))
    for name, DD, A, Y, size, F, kw in cases:
        Yd = torch.from_numpy(np.ascontiguousarray(Y.astype(np.complex64))).cuda()
        X = torch.zeros((1, F, size, size), dtype=torch.complex64, device="cuda")
        X1, I1, _, _ = m.mrf_ipg_step(DD, A, Yd, X, 1.0, precision="bf16x3", stats=False, **kw)
        torch.cuda.synchronize()
        steps = 3
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(steps):  # warm-started at the previous iterate's atoms, as inside a solve
            X2, _, _, st = m.mrf_ipg_step(DD, A, Yd, X1, 1.0, idx_in=I1, precision="bf16x3", stats=False, **kw)
        ev1.record()
        torch.cuda.synchronize()
        step_ms = ev0.elapsed_time(ev1) / steps
        # the operator alone: forward of the full-frame image, then the adjoint
        Xf = torch.zeros((1, Dd.L, size, size), dtype=torch.complex64, device="cuda")
        m.mrf_op_forward(A, Xf)
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(steps):
            R = m.mrf_op_forward(A, Xf, Yd)
            m.mrf_op_adjoint(A, R)
        ev1.record()
        torch.cuda.synchronize()
        op_ms = ev0.elapsed_time(ev1) / steps
        extra = {}
        if "net" in kw or "eps" in kw:  # fallback share and tree distance counts along a solve
            _, _, _, _, h = m.mrf_ipg_solve(DD, A, Yd, X0=X1, mu0=1.0, adaptive=False, max_iter=steps, rel_tol=0.0,
                                            precision="bf16x3", **kw)
            if "net" in kw:
                extra = {"fallbacks_per_step": h["fallbacks"] / steps,
                         "fallback_fraction": h["fallbacks"] / steps / (size * size)}
            if h["distance_evals"]:
                extra["distance_evals_per_voxel_per_iteration"] = h["distance_evals"] / steps / (size * size)
        out[name] = {"ms_per_step": step_ms, "operator_ms_full_frames": op_ms, "voxels": size * size,
                     "frames": F, "samples_per_coil": int(A.M), "coils": max(A.ncoils, 1),
                     "projection": (("cover tree, eps = %g (Algorithm 1)" % kw["eps"] if "eps" in kw else
                                     "exhaustive split BF16") if "net" not in kw else
                                    "learned + split-BF16 local search + " +
                                    ("cover-tree fallback" if "eps" in kw else "exhaustive fallback")), **extra}
        log(f"iteration {name}: {step_ms:.2f} ms per step, operator (A, A^H on {Dd.L} frames) {op_ms:.2f} ms"
            + "".join(f", {k} {v:.3f}" for k, v in extra.items()))
    return out


def cpu_baseline(Dd, Z, sample, answers):
    """The FP64 oracle (exact matched filter, numpy) on the first `sample`
    voxels of the same workload, on the host cores; its answers also grade
    every GPU path on that sample: strict index mismatch, mismatch outside
    near-ties (a GPU index is accepted when its normalised correlation is
    within 1e-6 of the maximum), and T1 / T2 / PD relative errors."""
    from oracle import mf
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        cores = max([i.get("num_threads", 1) for i in info if i.get("user_api") == "blas"] or [1])
    except Exception:
        cores = os.cpu_count() or 1
    Zs = Z[:sample].astype(np.complex128)
    t = time.time()
    ref = mf.exact_mf(Zs, Dd.atoms)
    dt = time.time() - t
    log(f"cpu oracle: {sample} voxels in {dt:.1f}s on {cores} threads")
    base = {"value": sample / dt, "unit": "voxels/s", "cores": int(cores), "kind": "oracle",
            "sample": f"first {sample} of the 65,536 voxels, FP64 numpy oracle (exact matched "
                      f"filter over all 100,800 atoms, BLAS matrix product), {dt:.1f} s"}
    nrm = mf.atom_norms(Dd.atoms)
    near = int(np.sum(ref["gap"] < 1e-6))
    grade = {"voxels": sample, "near_ties": near}
    for name, (idx, pd) in answers.items():
        j = idx[:sample].astype(np.int64)
        # normalised correlation of the GPU's atom, in FP64
        c = np.real(np.sum(Zs * np.conj(Dd.atoms[j]), axis=1)) / nrm[j] / np.maximum(ref["znorm"], 1e-300)
        ok = c >= ref["corr"] - 1e-6
        tr = Dd.params[ref["idx"], :2]
        relp = np.abs(Dd.params[j, :2] - tr) / tr
        # a compressed handle's atoms are the compressed normalised atoms: its PD is the
        # one of a unit-norm atom, max(score, 0), not that of the raw atom
        gref = np.maximum(ref["score"], 0.0) if name.startswith("subspace") else ref["gamma"]
        pde = np.abs(pd[:sample].astype(np.float64) - gref) / np.maximum(gref, 1e-12)
        grade[name] = {"index_mismatch": float(np.mean(j != ref["idx"])),
                       "index_mismatch_outside_near_ties": float(np.mean(~ok)),
                       "t1_rel_err_max": float(relp[:, 0].max()), "t2_rel_err_max": float(relp[:, 1].max()),
                       "pd_rel_err_median": float(np.median(pde)), "pd_rel_err_max": float(pde.max())}
    return base, grade


if __name__ == "__main__":
    sys.exit(main())
