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
    ap.add_argument("--cfg3", type=int, default=1,
                    help="precision forms inside Algorithm 2 on the 64 x 64 FISP spiral workload")
    ap.add_argument("--cfg4", type=int, default=1,
                    help="learned against exhaustive projections inside Algorithm 2 on 8 x 256 x 256 voxels")
    ap.add_argument("--cfg5", type=int, default=1,
                    help="16 x 256 x 256 voxels against the 1,196,800-atom L = 1000 dictionary")
    ap.add_argument("--cfg5-sample", type=int, default=256, help="random tissue voxels graded against FP64 (cfg5)")
    ap.add_argument("--dict-workers", type=int, default=min(16, os.cpu_count() or 1),
                    help="processes generating the 1,196,800-atom dictionary")
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
    D5 = None
    if args.cfg5:  # generated in forked processes before the GPU is touched
        t5 = time.time()
        D5 = cfg5_atoms(args.dict_workers)
        log(f"1,196,800-atom dictionary generated in {time.time() - t5:.1f}s on {args.dict_workers} processes")
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
                       s.search_ms, s.first_box_atoms, s.cert_rescored, s.cert_rescanned))
        return ms, np.mean(np.array(st, dtype=np.float64), axis=0), o

    ms32, st32, o32 = run(args.steps, args.warmup, precision="fp32")
    idx32 = o32["idx"].cpu().numpy()
    answers = {"exhaustive_fp32": (idx32, o32["pd"].cpu().numpy())}   # checked against FP64 on the sample
    score_ms32 = float(st32[0])
    log(f"exhaustive fp32: {ms32:.3f} ms/step, scoring kernel {score_ms32:.3f} ms, "
        f"splits {o32['stats'].splits}")
    exhaustive = {"voxels_per_s": n / (ms32 * 1e-3), "ms_per_step": ms32, "score_kernel_ms": score_ms32,
                  "certified": True, "rescored_per_voxel": float(st32[8]) / n, "rescanned": float(st32[9]),
                  "mfma_frac": flops / (score_ms32 * 1e-3) / 1e12 / PEAK["fp32"],
                  "recovered_generating_atom": float(np.mean(idx32 == jtrue))}
    variants = {}
    if args.variants:
        # certified (exact argmax) and uncertified (the scoring arithmetic's own argmax) forms
        for p, cert in (("bf16x3", True), ("bf16", True), ("fp8", True), ("fp32", False), ("bf16x3", False),
                        ("bf16", False), ("fp8", False)):
            key = p if cert else p + "_uncertified"
            vms, vst, vo = run(max(3, args.steps // 2), 1, precision=p, certify=cert)
            vidx = vo["idx"].cpu().numpy()
            answers[f"exhaustive_{key}"] = (vidx, vo["pd"].cpu().numpy())
            # split BF16 executes three BF16 products per algorithmic one
            mult, pk = (3.0, PEAK["bf16"]) if p == "bf16x3" else (1.0, PEAK[p])
            variants[key] = {"voxels_per_s": n / (vms * 1e-3), "ms_per_step": vms, "certified": cert,
                             "score_kernel_ms": float(vst[0]),
                             "algorithmic_tflops": flops / (float(vst[0]) * 1e-3) / 1e12,
                             "mfma_frac": mult * flops / (float(vst[0]) * 1e-3) / 1e12 / pk,
                             "index_mismatch_vs_fp32": float(np.mean(vidx != idx32)),
                             "rescored_per_voxel": float(vst[8]) / n, "rescanned": float(vst[9])}
            log(f"exhaustive {key}: {vms:.3f} ms/step, scoring kernel {vst[0]:.3f} ms, "
                f"mismatch vs certified fp32 {variants[key]['index_mismatch_vs_fp32']:.5f}, rescored "
                f"{variants[key]['rescored_per_voxel']:.2f} per voxel, {vst[9]:.0f} rescanned")
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
        cases = [(lp, args.box_radius, lp, False) for lp in args.learned_precisions.split(",")]
        if args.box_radius != 3:  # the +-3 box the learned form names, beside the default one
            cases.append(("bf16x3", 3, "bf16x3_r3", False))
        # certified local search: exact (FP64) argmax over each box and warm atom
        cases += [(lp, args.box_radius, f"{lp}_certified", True) for lp in args.learned_precisions.split(",")]
        for lp, radius, key, cl in cases:
            lms, lst, lo = run(args.steps, args.warmup, net=net, box_radius=radius, fallback_corr=0.98,
                               recentre=args.recentre, precision=lp, certify_local=cl)
            lidx = lo["idx"].cpu().numpy()
            answers[f"learned_{key}"] = (lidx, lo["pd"].cpu().numpy())
            mism = float(np.mean(lidx != idx32))
            # algorithmic work of the first local-search launch: 2 K flops per
            # (voxel, atom of its clipped box)
            box_flops = 2.0 * K * float(lst[7])
            learned[key] = {"voxels_per_s": n / (lms * 1e-3), "ms_per_step": lms, "box_radius": radius,
                            "certified_local": cl,
                           "index_mismatch_vs_exhaustive_fp32": mism,
                           "local_score_kernel_ms": float(lst[0]), "local_search_ms": float(lst[6]),
                           "proposal_ms": float(lst[1]),
                           "fallback_ms": float(lst[2]), "fallbacks_per_step": float(lst[3]),
                           "recentred_per_step": float(lst[4]), "local_atoms_scored": float(lst[5]),
                           "first_launch_box_atoms": float(lst[7]),
                           "speedup_vs_exhaustive_fp32": ms32 / lms,
                           "speedup_vs_fastest_exhaustive_within_0.1pct": fastest / lms,
                           "box_flop_first_launch": box_flops,
                           "rescored_per_voxel": float(lst[8]) / n, "rescanned": float(lst[9])}
            log(f"learned ({key}, radius {radius}): {lms:.3f} ms/step (local search {lst[6]:.3f}, first scoring kernel "
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
                   "energy_kept": float(lam.sum() / d),
                   "voxels": "pre-compressed on the host (V^H Z outside the timed region; the projected-gradient "
                             "rows of 'iteration' include the compression)"}
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
                   "path": path, "voxels": n, "atoms": d, "L": Dd.L,
                   "box_radius": args.box_radius if ok else None},
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
    if args.cfg3:
        res["cfg3_precision_ipg"] = cfg3_bench(m, torch)
    if args.cfg4 and args.learned:
        res["cfg4_multislice_ipg"] = cfg4_bench(m, torch, D, Dd, net)
    if args.cpu_baseline:
        res["cpu_baseline"], res["vs_fp64_oracle_on_sample"] = cpu_baseline(Dd, Z, args.cpu_sample, answers)
    if D5 is not None:
        del D, DT
        torch.cuda.empty_cache()
        res["cfg5_multiparametric"] = cfg5_bench(m, torch, D5, args)
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
             ("cartesian_256_1coil_certified", D, A1, Ycart, 256, Dd.L, {"certify": True}),
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
        # the projections inside the iteration are the uncertified split-BF16
        # filter (its own argmax) unless the case asks for the certificate
        kw = dict({"certify": False}, **kw)
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
                                     "exhaustive split BF16" + (" certified" if kw["certify"] else "")) if "net" not in kw
                                    else "learned + split-BF16 local search + " +
                                    ("cover-tree fallback" if "eps" in kw else "exhaustive fallback")), **extra}
        log(f"iteration {name}: {step_ms:.2f} ms per step, operator (A, A^H on {Dd.L} frames) {op_ms:.2f} ms"
            + "".join(f", {k} {v:.3f}" for k, v in extra.items()))
    return out


def cfg3_bench(m, torch):
    """The precision forms inside Algorithm 2 on the 64 x 64 FISP workload
    (2,000 real atoms, L = 100): a variable-density spiral of 5 % of k-space
    per frame rasterised to the grid, rotated 7.5 degrees per frame, with
    Voronoi density compensation (eq. blip_dcf); 20 adaptive iterations
    (zeta = 2) from mu0 = n / m.  The projection scores in FP32, BF16 or FP8
    (certified: exact) and, for BF16 / FP8, also uncertified.  Graded against
    the FP64 oracle: teacher-forced (each GPU step from the oracle's iterate
    and step size, its indices against the oracle's projection) and the full
    solve (indices and T1 / T2 / PD against the oracle's solve)."""
    from oracle import ipg
    from synth import workloads
    t0 = time.time()
    Dd = workloads.fisp_dictionary()
    size = 64
    ph = workloads.disc_phantom(Dd, seed=3, size=size, radius=28.0, snap=False)
    smp = workloads.spiral_sampling(1, Dd.L, size, size, frac=0.05)
    Y = workloads.simulate_kspace(ph.X0, smp, 30.0, 3)
    mu0 = size * size / (smp.M / Dd.L)
    iters = 20
    # the oracle: 20 accepted iterations, then the same steps one at a time
    Xo, io, go, ho = ipg.ipg_solve(Y, smp.off, smp.idx, (1, Dd.L, size, size), Dd.atoms, mu0, 2.0, adaptive=True,
                                   max_iter=iters, rel_tol=0.0, w=smp.dcf)
    forced = []
    X = np.zeros((1, Dd.L, size, size))
    warm = None
    for h in ho:
        Xn, res, _ = ipg.ipg_step(Y, smp.off, smp.idx, Dd.atoms, X, h["mu"], w=smp.dcf, warm_idx=warm)
        forced.append((X, warm, h["mu"], res["idx"], res["gap"]))
        X, warm = Xn, res["idx"]
    oracle_s = time.time() - t0
    log(f"cfg3 oracle: {len(ho)} iterations in {oracle_s:.1f}s (mu0 {mu0:.2f}, {sum(h['shrinks'] for h in ho)} "
        "step-size shrinks)")
    D = m.Dictionary(Dd.atoms, Dd.params, grid_dims=Dd.grid_dims, store_bf16=True, store_fp8=True)
    A = m.Operator.from_sampling(smp)
    Yd = torch.from_numpy(Y.astype(np.complex64)).cuda()
    tissue = np.isfinite(ph.params[:, 0])
    out = {"workload": "64x64 FISP disc phantom (off-grid classes), L=100, 2,000 atoms; spiral 5% per frame, "
                       "Voronoi DCF; 20 adaptive iterations from mu0 = n/m",
           "mu0": mu0, "oracle_seconds": oracle_s, "oracle_shrinks": int(sum(h["shrinks"] for h in ho))}
    for prec, cert in (("fp32", True), ("bf16", True), ("fp8", True), ("bf16", False), ("fp8", False)):
        key = prec if cert else prec + "_uncertified"
        agree, outside = [], []
        for Xk, wk, mu, oidx, ogap in forced:
            Xd = torch.from_numpy(np.ascontiguousarray(Xk.astype(np.complex64))).cuda()
            wd = None if wk is None else torch.from_numpy(wk.astype(np.int32)).cuda()
            _, gi, _, _ = m.mrf_ipg_step(D, A, Yd, Xd, mu, idx_in=wd, precision=prec, certify=cert)
            gi = gi.cpu().numpy().astype(np.int64)
            agree.append(float(np.mean(gi == oidx)))
            outside.append(float(np.mean((gi != oidx) & (ogap >= 1e-6))))
        m.mrf_ipg_solve(D, A, Yd, mu0=mu0, zeta=2.0, adaptive=True, max_iter=iters, rel_tol=0.0, precision=prec,
                        certify=cert)
        torch.cuda.synchronize()
        t1 = time.time()
        X, idx, pd, prm, hist = m.mrf_ipg_solve(D, A, Yd, mu0=mu0, zeta=2.0, adaptive=True, max_iter=iters,
                                                rel_tol=0.0, precision=prec, certify=cert)
        torch.cuda.synchronize()
        solve_ms = (time.time() - t1) * 1e3
        gi = idx.cpu().numpy().astype(np.int64)
        gp = pd.cpu().numpy().astype(np.float64)
        # the accept / reject decisions of the step rule compare two nearly
        # equal quantities, so an FP32 and an FP64 solve may take different
        # step sizes from some iteration on; up to there they must agree
        kd = next((k for k in range(min(len(ho), len(hist["mu"])))
                   if abs(hist["mu"][k] - ho[k]["mu"]) > 1e-6 * ho[k]["mu"]), len(ho))
        common = None
        if kd > 0:
            _, ic, _, _, _ = m.mrf_ipg_solve(D, A, Yd, mu0=mu0, zeta=2.0, adaptive=True, max_iter=kd, rel_tol=0.0,
                                             precision=prec, certify=cert)
            ic = ic.cpu().numpy().astype(np.int64)
            common = {"iterations": kd, "index_agreement_vs_fp64": float(np.mean(ic == forced[kd - 1][3])),
                      "mismatch_outside_near_ties": float(np.mean((ic != forced[kd - 1][3]) &
                                                                  (forced[kd - 1][4] >= 1e-6)))}
        pe, po = Dd.params[gi[tissue]], Dd.params[io[tissue]]
        rel = np.abs(pe - po) / po
        pde = np.abs(gp[tissue] - go[tissue]) / np.maximum(go[tissue], 1e-12)
        tru = np.abs(pe - ph.params[tissue]) / ph.params[tissue]
        out[key] = {"teacher_forced_index_agreement_mean": float(np.mean(agree)),
                    "teacher_forced_index_agreement_min": float(np.min(agree)),
                    "teacher_forced_mismatch_outside_near_ties_max": float(np.max(outside)),
                    "solve_ms": solve_ms, "iterations": int(hist["iters"]),
                    "shrinks": int(hist["total_shrinks"]),
                    "final_index_agreement_vs_fp64_solve": float(np.mean(gi[tissue] == io[tissue])),
                    "t1_rel_err_vs_fp64_mean": float(rel[:, 0].mean()), "t1_rel_err_vs_fp64_max": float(rel[:, 0].max()),
                    "t2_rel_err_vs_fp64_mean": float(rel[:, 1].mean()), "t2_rel_err_vs_fp64_max": float(rel[:, 1].max()),
                    "pd_rel_err_vs_fp64_median": float(np.median(pde)), "pd_rel_err_vs_fp64_max": float(pde.max()),
                    "f_final_rel_diff_vs_fp64": float(abs(hist["f"][-1] - ho[-1]["f"]) / ho[-1]["f"]),
                    "first_iteration_with_other_step_size": kd if kd < len(ho) else None,
                    "solve_until_then": common,
                    "t1_rel_err_vs_truth_mean": float(tru[:, 0].mean()),
                    "t2_rel_err_vs_truth_mean": float(tru[:, 1].mean())}
        log(f"cfg3 {key}: teacher-forced agreement {np.mean(agree):.5f} (min {np.min(agree):.5f}, outside near-ties "
            f"<= {np.max(outside):.5f}), solve {solve_ms:.1f} ms, final agreement "
            f"{out[key]['final_index_agreement_vs_fp64_solve']:.5f}, PD err median {np.median(pde):.2e}")
    return out


def kspace_on_device(torch, X0, smp, snr_db, gen):
    """Y = P_Omega F X0 + noise for a frame-major device image X0 [S][L][ny][nx]
    (unitary 2-D DFT per frame, torch's FFT), the samples in the CSR order of
    `smp`, circular complex Gaussian noise from the seeded generator `gen` at
    the given SNR over all samples."""
    off = torch.from_numpy(smp.off).cuda()
    npix = smp.ny * smp.nx
    pairs = torch.repeat_interleave(torch.arange(smp.S * smp.L, device="cuda", dtype=torch.int64), off[1:] - off[:-1])
    flat = pairs * npix + torch.from_numpy(smp.idx.astype(np.int64)).cuda()
    K = torch.fft.fft2(X0, norm="ortho").reshape(-1)
    Y = K[flat]
    del K, flat, pairs
    s2 = torch.sum(torch.abs(Y) ** 2) / Y.numel() * 10.0 ** (-snr_db / 10.0) / 2.0
    return Y + torch.sqrt(s2) * torch.complex(torch.randn(Y.shape, generator=gen, device="cuda"),
                                              torch.randn(Y.shape, generator=gen, device="cuda"))


def cfg4_bench(m, torch, D, Dd, net):
    """Learned against exhaustive projections inside Algorithm 2 on 8 slices
    of 256 x 256 (524,288 voxels) with the 100,800-atom L = 500 dictionary: a
    smooth six-tissue phantom per slice with a df ramp, 26 of 256 random ky
    lines per frame, k-space noise at 30 dB, 20 adaptive iterations (zeta = 2)
    from mu0 = n / m.  Exhaustive: the uncertified split-BF16 filter; learned:
    network proposal + split-BF16 local search (+-2 box, re-centring), warm
    started, exhaustive fallback below 0.98 (and below 0.9)."""
    from synth import workloads
    S, size, L, iters = 8, 256, Dd.L, 20
    t0 = time.time()
    ph = workloads.smooth_phantom(Dd, seed=4, S=S, size=size, dtype=np.complex64)
    smp = workloads.random_lines(4, S, L, size, size, 26)
    X0 = torch.from_numpy(ph.X0).cuda()
    del ph.X0
    g = torch.Generator(device="cuda")
    g.manual_seed(4)
    Yd = kspace_on_device(torch, X0, smp, 30.0, g)
    A = m.Operator.from_sampling(smp)
    n = S * size * size
    mu0 = float(n * L) / smp.M
    head = ph.idx >= 0
    log(f"cfg4 inputs in {time.time() - t0:.1f}s")
    out = {"workload": "8 x 256 x 256 voxels, L=500, 100,800 atoms, 26/256 lines per frame, SNR 30 dB, 20 adaptive "
                       "iterations from mu0 = n/m", "voxels": n, "mu0": mu0}
    ref = None
    for name, kw in (("exhaustive_bf16x3", dict(precision="bf16x3", certify=False)),
                     ("learned_bf16x3", dict(net=net, precision="bf16x3", box_radius=2, recentre=1,
                                             certify=False)),
                     ("learned_bf16x3_fallback0.9", dict(net=net, precision="bf16x3", box_radius=2, recentre=1,
                                                         fallback_corr=0.9, certify=False))):
        torch.cuda.synchronize()
        t1 = time.time()
        X, idx, pd, _, hist = m.mrf_ipg_solve(D, A, Yd, mu0=mu0, zeta=2.0, adaptive=True, max_iter=iters,
                                              rel_tol=0.0, want_params=False, **kw)
        torch.cuda.synchronize()
        dt = time.time() - t1
        nmse = float(torch.linalg.vector_norm(X - X0) / torch.linalg.vector_norm(X0))
        ii = idx.cpu().numpy().astype(np.int64)
        trials = hist["iters"] + hist["total_shrinks"]
        row = {"seconds": dt, "ms_per_projection": dt * 1e3 / trials, "iterations": int(hist["iters"]),
               "step_size_shrinks": int(hist["total_shrinks"]), "nmse": nmse, "f_final": float(hist["f"][-1]),
               "tissue_on_generating_atom": float(np.mean(ii[head] == ph.idx[head]))}
        if "net" in kw:
            row["fallback_fraction"] = hist["fallbacks"] / (n * trials)
            row["tissue_index_agreement_with_exhaustive"] = float(np.mean(ii[head] == ref[head]))
            row["speedup_vs_exhaustive"] = out["exhaustive_bf16x3"]["seconds"] / dt
        else:
            ref = ii
        out[name] = row
        log(f"cfg4 {name}: {dt:.2f} s ({row['ms_per_projection']:.1f} ms per projection), NMSE {nmse:.4e}, "
            f"f {row['f_final']:.6e}" + (f", fallbacks {row['fallback_fraction']:.3f}" if "net" in kw else ""))
        del X
    return out


def cfg5_atoms(workers):
    """The multi-parametric dictionary: IR-bSSFP, L = 1000, T1 80 x T2 80 x
    B1 17 in [0.6, 1.4] x df 11 in [-40, 40] Hz = 1,196,800 atoms (complex64
    on the host)."""
    from synth import workloads
    return workloads.bssfp_dictionary(L=1000, n_t1=80, n_t2=80, n_df=11, b1_axis=np.linspace(0.6, 1.4, 17),
                                      dtype=np.complex64, workers=workers)


def cfg5_bench(m, torch, Dd, args):
    """The multi-parametric scale-up: 16 slices of 256 x 256 (1,048,576
    voxels) against 1,196,800 atoms of L = 1000 complex frames.
    * standalone mrf_match over every voxel (the phantom's voxels with
      voxel-domain noise at 30 dB): the learned path (4-output network, split
      BF16 local search over the 7^4 box, exhaustive fallback below 0.98) and
      the uncertified split-BF16 and BF16 filters (their own argmax, exact
      PD), graded against the FP64 oracle over all atoms on a sample of
      voxels and every voxel where learned and split BF16 disagree (at most
      256); the certified split-BF16 filter timed on the first slice (its
      derived bound, 4.1e-4 ||Z|| at K = 2000, leaves many near-degenerate
      atoms of this dictionary to rescan);
    * one projected-gradient step batched over the 16 slices in one launch,
      slice s sampling 16 + 2 s of 256 lines per frame (k-space noise 30 dB),
      from X = 0 with mu = 1: learned and uncertified split-BF16 projections."""
    from oracle import mf
    from synth import workloads
    L, S, size = Dd.L, 16, 256
    n = S * size * size
    out = {"workload": "16 x 256 x 256 voxels, L=1000 complex, T1 80 x T2 80 x B1 17 x df 11 = 1,196,800 "
                       "IR-bSSFP atoms", "voxels": n, "atoms": Dd.d}
    t0 = time.time()
    D = m.Dictionary(Dd.atoms, Dd.params, grid_dims=Dd.grid_dims, store_bf16=True)
    torch.cuda.synchronize()
    out["dictionary_upload_seconds"] = time.time() - t0
    t0 = time.time()
    net = m.Net(2 * L, Dd.params.shape[1], hidden=256, seed=11)
    tr = m.mrf_net_train(net, D, samples=args.train_samples, batch=4096, epochs=args.train_epochs, lr=1e-3,
                         lr_min=1e-5, snr_lo=15.0, snr_hi=40.0, seed=12)
    out["training"] = {"samples": args.train_samples, "epochs": args.train_epochs, "seconds": time.time() - t0,
                       "loss_first": tr["first_loss"], "loss_last": tr["last_loss"]}
    log(f"cfg5: dictionary uploaded in {out['dictionary_upload_seconds']:.1f}s, network trained in "
        f"{out['training']['seconds']:.1f}s")
    t0 = time.time()
    ph = workloads.smooth_phantom(Dd, seed=9, S=S, size=size, dtype=np.complex64)
    X0 = torch.from_numpy(ph.X0).cuda()
    del ph.X0
    g = torch.Generator(device="cuda")
    g.manual_seed(9)
    # voxel-domain noise: per voxel E|xi|^2 per entry = ||x_v||^2 / L 10^(-3)
    sig = torch.sqrt(torch.sum(torch.abs(X0) ** 2, dim=1, keepdim=True) / L * 1e-3 / 2.0)
    Zd = X0 + sig * torch.complex(torch.randn(X0.shape, generator=g, device="cuda"),
                                  torch.randn(X0.shape, generator=g, device="cuda"))
    del sig
    log(f"cfg5: phantom and voxels in {time.time() - t0:.1f}s")
    tissue = ph.idx >= 0
    res = {}

    def timed(name, **kw):
        t1 = time.time()
        o = m.mrf_match(D, Zd, layout="frame", slice_voxels=size * size, want_corr=False, stats=True, **kw)
        log(f"cfg5 {name}: first call {time.time() - t1:.1f}s")
        t1 = time.time()
        o = m.mrf_match(D, Zd, layout="frame", slice_voxels=size * size, want_corr=False, out=o, stats=True, **kw)
        ms = (time.time() - t1) * 1e3
        log(f"cfg5 {name}: {ms:.0f} ms")
        return o, ms

    ol, ms_l = timed("learned", net=net, precision="bf16x3", box_radius=3, fallback_corr=0.98, recentre=2)
    ox, ms_x = timed("exhaustive split BF16 uncertified", precision="bf16x3", certify=False)
    ob, ms_b = timed("exhaustive BF16 uncertified", precision="bf16", certify=False)
    t1 = time.time()
    oc = m.mrf_match(D, Zd[:1].contiguous(), layout="frame", slice_voxels=size * size, want_corr=False, stats=True,
                     precision="bf16x3")
    ms_c = (time.time() - t1) * 1e3
    ic = oc["idx"].cpu().numpy().astype(np.int64)
    log(f"cfg5 certified split BF16 on one slice: {ms_c:.0f} ms, {oc['stats'].cert_rescanned} rescanned, "
        f"{oc['stats'].cert_scanned} scanned")
    il, ix, ib = (o["idx"].cpu().numpy().astype(np.int64) for o in (ol, ox, ob))
    res["learned_bf16x3_r3"] = {"ms": ms_l, "voxels_per_s": n / (ms_l * 1e-3),
                                "fallbacks": int(ol["stats"].fallbacks),
                                "box_atoms_per_voxel": float(ol["stats"].first_box_atoms) / n,
                                "index_mismatch_vs_split_bf16": float(np.mean(il != ix)),
                                "index_mismatch_vs_split_bf16_tissue": float(np.mean(il[tissue] != ix[tissue]))}
    res["exhaustive_bf16x3_uncertified"] = {"ms": ms_x, "voxels_per_s": n / (ms_x * 1e-3)}
    res["exhaustive_bf16_uncertified"] = {"ms": ms_b, "voxels_per_s": n / (ms_b * 1e-3),
                                          "index_mismatch_vs_split_bf16": float(np.mean(ib != ix))}
    res["exhaustive_bf16x3_certified_first_slice"] = {
        "voxels": size * size, "ms": ms_c, "rescored": int(oc["stats"].cert_rescored),
        "rescanned": int(oc["stats"].cert_rescanned), "scanned": int(oc["stats"].cert_scanned),
        "index_mismatch_vs_uncertified": float(np.mean(ic != ix[:size * size]))}
    res["learned_speedup_vs_split_bf16"] = ms_x / ms_l
    res["learned_speedup_vs_bf16"] = ms_b / ms_l
    log(f"cfg5 match: learned {ms_l:.1f} ms ({res['learned_bf16x3_r3']['fallbacks']} fallbacks, mismatch vs split "
        f"BF16 {res['learned_bf16x3_r3']['index_mismatch_vs_split_bf16']:.5f}), split BF16 {ms_x:.0f} ms, BF16 "
        f"{ms_b:.0f} ms (mismatch {res['exhaustive_bf16_uncertified']['index_mismatch_vs_split_bf16']:.5f})")
    # FP64 grading: sampled tissue voxels and learned / exact disagreements
    t0 = time.time()
    tis = np.flatnonzero(tissue)
    dis = np.flatnonzero(il != ix)
    from synth import rng
    sample = np.union1d(tis[rng.permutation(5, "cfg5-sample", tis.size)[:args.cfg5_sample]],
                        dis[rng.permutation(5, "cfg5-dis", dis.size)[:256]])
    pix = sample % (size * size)
    sl = sample // (size * size)
    Zs = Zd[torch.from_numpy(sl).cuda(), :, torch.from_numpy(pix // size).cuda(),
            torch.from_numpy(pix % size).cuda()].cpu().numpy().astype(np.complex128)
    nrm = mf.atom_norms(Dd.atoms)
    best = np.full(sample.size, -np.inf)
    arg = np.zeros(sample.size, dtype=np.int64)
    for a0 in range(0, Dd.d, 40000):
        c = mf.correlations(Zs, Dd.atoms[a0:a0 + 40000], nrm[a0:a0 + 40000])
        j = np.argmax(c, axis=1)
        v = c[np.arange(sample.size), j]
        up = v > best
        best[up], arg[up] = v[up], a0 + j[up]
    zn = np.linalg.norm(Zs, axis=1)
    best = best / zn
    isdis = np.isin(sample, dis)
    grade = {"voxels": int(sample.size), "disagreements_graded": int(isdis.sum()),
             "oracle_seconds": time.time() - t0}
    for name, ii in (("learned_bf16x3_r3", il), ("exhaustive_bf16x3_uncertified", ix),
                     ("exhaustive_bf16_uncertified", ib)):
        j = ii[sample]
        cj = np.real(np.sum(Zs * np.conj(Dd.atoms[j].astype(np.complex128)), axis=1)) / nrm[j] / zn
        ok = cj >= best - 1e-6
        pr = np.abs(Dd.params[j] - Dd.params[arg]) / np.abs(Dd.params[arg]).clip(1e-12)
        grade[name] = {"index_mismatch": float(np.mean(j != arg)),
                       "index_mismatch_outside_near_ties": float(np.mean(~ok)),
                       "index_mismatch_outside_near_ties_on_random_sample": float(np.mean(~ok[~isdis])),
                       "t1_rel_err_max": float(pr[:, 0].max()), "t2_rel_err_max": float(pr[:, 1].max())}
    res["vs_fp64_oracle"] = grade
    log(f"cfg5 FP64 grading on {sample.size} voxels ({int(isdis.sum())} disagreements) in "
        f"{grade['oracle_seconds']:.1f}s: " + ", ".join(f"{k} {v['index_mismatch_outside_near_ties']:.4f}"
                                                      for k, v in grade.items() if isinstance(v, dict)))
    out["match"] = res
    del Zd
    # one batched step over the 16 slices with uneven masks
    t0 = time.time()
    smp = workloads.random_lines(9, S, L, size, size, [16 + 2 * s for s in range(S)])
    Yd = kspace_on_device(torch, X0, smp, 30.0, g)
    A = m.Operator.from_sampling(smp)
    log(f"cfg5: sampling ({smp.M} samples) and k-space in {time.time() - t0:.1f}s")
    Xz = torch.zeros_like(X0)
    del X0
    step = {}
    for name, kw in (("learned_bf16x3_r3", dict(net=net, precision="bf16x3", box_radius=3, recentre=2)),
                     ("exhaustive_bf16x3_uncertified", dict(precision="bf16x3", certify=False))):
        t1 = time.time()
        m.mrf_ipg_step(D, A, Yd, Xz, 1.0, **kw)
        torch.cuda.synchronize()
        log(f"cfg5 step {name}: first call {time.time() - t1:.1f}s")
        t1 = time.time()
        Xs, ii, _, st = m.mrf_ipg_step(D, A, Yd, Xz, 1.0, **kw)
        torch.cuda.synchronize()
        step[name] = {"ms": (time.time() - t1) * 1e3, "f_out": st.f_out, "dx2": st.dx2,
                      "idx": ii.cpu().numpy().astype(np.int64)}
        del Xs
    il, ix = step["learned_bf16x3_r3"].pop("idx"), step["exhaustive_bf16x3_uncertified"].pop("idx")
    step["learned_index_mismatch_vs_split_bf16_tissue"] = float(np.mean(il[tissue] != ix[tissue]))
    step["learned_objective_rel_diff"] = abs(step["learned_bf16x3_r3"]["f_out"] -
                                             step["exhaustive_bf16x3_uncertified"]["f_out"]) / \
        step["exhaustive_bf16x3_uncertified"]["f_out"]
    step["samples"] = int(smp.M)
    step["lines_per_frame"] = [16 + 2 * s for s in range(S)]
    out["ipg_step"] = step
    log(f"cfg5 step: learned {step['learned_bf16x3_r3']['ms']:.0f} ms, split BF16 "
        f"{step['exhaustive_bf16x3_uncertified']['ms']:.0f} ms, tissue mismatch "
        f"{step['learned_index_mismatch_vs_split_bf16_tissue']:.5f}")
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
