"""Host-side checks of bench.py: it refuses more than one GPU before touching
a device, and the dominant kernel's traffic figure is taken from the
committed counter summary only while the kernel source is the one counted."""
import hashlib
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["n_gpus"] == 2 and "one GPU" in out["error"]


@pytest.fixture
def bench_module():
    sys.path.insert(0, ROOT)
    import bench
    return bench


def test_traffic_follows_the_counted_source(bench_module, tmp_path, monkeypatch):
    b = bench_module
    src_dir = tmp_path / "paper_1810_01967_amd" / "csrc"
    src_dir.mkdir(parents=True)
    (src_dir / "k.hip").write_bytes(b"kernel source")
    summary = tmp_path / "traffic.json"
    summary.write_text(json.dumps({"source_sha256": hashlib.sha256(b"kernel source").hexdigest(),
                                   "fetch_bytes_per_launch": 2.0e9, "write_bytes_per_launch": 6.0e6}))
    monkeypatch.setattr(b, "HERE", str(tmp_path))
    monkeypatch.setattr(b, "TRAFFIC", str(summary))
    assert b.measured_traffic("k.hip") == pytest.approx(2.006e9)
    (src_dir / "k.hip").write_bytes(b"kernel source, changed")
    assert b.measured_traffic("k.hip") is None
    summary.unlink()
    assert b.measured_traffic("k.hip") is None



def test_grading_of_compressed_pd(bench_module):
    """The bench grades each path's PD against the oracle's: the full
    dictionary's PD is that of the raw atom (eq. exactPs), a compressed
    handle's is that of its unit-norm compressed atom, max(score, 0).  The
    oracle's own answers in each convention grade as exact."""
    import numpy as np
    from oracle import mf
    from synth import workloads
    Dd = workloads.bssfp_dictionary(L=40, n_t1=8, n_t2=8, n_df=3, seed=2)
    Z, _, _, _ = workloads.random_voxels(Dd, 64, seed=3)
    ref = mf.exact_mf(Z.astype(np.complex128), Dd.atoms)
    answers = {"exhaustive_fp32": (ref["idx"], ref["gamma"]),
               "subspace20_fp32": (ref["idx"], np.maximum(ref["score"], 0.0)),
               "subspace200_fp32": (ref["idx"], ref["gamma"])}
    _, grade = bench_module.cpu_baseline(Dd, Z, 64, answers)
    assert grade["exhaustive_fp32"]["pd_rel_err_max"] == 0.0
    assert grade["subspace20_fp32"]["pd_rel_err_max"] == 0.0
    # the raw atom's PD is not a compressed handle's: the atoms here are not unit-norm
    assert grade["subspace200_fp32"]["pd_rel_err_median"] > 1e-3
    for g in (grade["exhaustive_fp32"], grade["subspace20_fp32"]):
        assert g["index_mismatch"] == 0.0 and g["t1_rel_err_max"] == 0.0
