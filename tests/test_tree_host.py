"""The library's host cover-tree builder (an exact pruned evaluation of the
greedy nested nets) against the oracle's direct construction: identical
node sets, insertion levels and parents; maxdist to FP32 rounding; and the
flattened per-level form the device traverses is consistent with the tree."""
import os
import subprocess

import numpy as np
import pytest

from oracle import covertree as ct
from synth import rng, workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


# the driver is built twice: optimised, and with the address and
# undefined-behaviour sanitizers (any report aborts the run)
SANITIZE = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


@pytest.fixture(scope="module", params=["O2", "asan-ubsan"])
def driver(tmp_path_factory, request):
    exe = tmp_path_factory.mktemp("tree") / "tree_driver"
    opt = ["-O2"] if request.param == "O2" else SANITIZE
    subprocess.run(["g++", *opt, "-std=c++17", "-pthread", os.path.join(ROOT, "tests", "tree_driver.cpp"),
                    os.path.join(ROOT, "paper_1810_01967_amd", "csrc", "covertree.cpp"), "-o", str(exe)],
                   check=True)
    return str(exe)


def _run(driver, X, tmp_path):
    inp = tmp_path / "x.bin"
    with open(inp, "wb") as f:
        np.array([X.shape[0], X.shape[1]], dtype=np.int64).tofile(f)
        np.ascontiguousarray(X, dtype=np.float64).tofile(f)
    out = tmp_path / "t.txt"
    subprocess.run([driver, str(inp), str(out)], check=True)
    lines = open(out).read().split("\n")
    sigma, imax, u, E = lines[0].split()
    sigma, imax, u, E = float(sigma), int(imax), int(u), int(E)
    tab = np.array([list(map(int, l.split())) for l in lines[1:1 + u]])
    nmd = sum(1 for _ in range(0))
    rest = lines[1 + u:]
    return sigma, imax, tab, rest, E


def _cases():
    c = rng.normal(1, "c", 8 * 10).reshape(8, 10)
    x = c[rng.randint(1, "l", 400, 8)] + 0.1 * rng.normal(1, "x", 400 * 10).reshape(400, 10)
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    x = np.concatenate([x, x[[5, 17]]])          # exact duplicates
    D = workloads.fisp_dictionary(L=60, n_t1=16, n_t2=20)
    f = D.atoms / np.linalg.norm(D.atoms, axis=1, keepdims=True)
    B = workloads.bssfp_dictionary(L=40, n_t1=10, n_t2=10, n_df=7, seed=2)
    a = B.atoms / np.linalg.norm(B.atoms, axis=1, keepdims=True)
    b = np.empty((a.shape[0], 80))
    b[:, 0::2], b[:, 1::2] = a.real, a.imag
    return {"clustered": x, "fisp": f, "bssfp": b}


@pytest.mark.parametrize("name", ["clustered", "fisp", "bssfp"])
def test_host_builder_equals_oracle(driver, tmp_path, name):
    X = _cases()[name]
    sigma, imax, tab, rest, E = _run(driver, X, tmp_path)
    t = ct.build(X)
    assert abs(sigma - t.sigma) <= 1e-14 * t.sigma
    assert imax == t.imax
    np.testing.assert_array_equal(tab[:, 0], t.rep)
    u = len(t.rep)
    # insertion level and parent of every unique atom
    ins = np.full(u, -1)
    for i, lev in enumerate(t.levels):
        for q in lev:
            if ins[q] < 0:
                ins[q] = i
    np.testing.assert_array_equal(tab[:, 1], ins)
    par = np.full(u, -1)
    for i in range(1, t.imax + 1):
        for q, p in t.parent[i].items():
            if ins[q] == i:
                par[q] = p
    np.testing.assert_array_equal(tab[:, 2], par)
    nmd = sum(len(l) for l in t.levels)
    md = np.array([float(x) for x in rest[:nmd]])
    ref = np.concatenate([[t.maxdist[i][int(q)] for q in t.levels[i]] for i in range(t.imax + 1)])
    np.testing.assert_allclose(md, ref, rtol=1e-6, atol=1e-7)
    # flattened form: every entry's child range holds exactly its children (self included)
    ent = np.array([list(map(int, l.split())) for l in rest[nmd:nmd + E]])
    lb = np.array([int(l) for l in rest[nmd + E:nmd + E + imax + 2]])
    for i in range(imax):
        for e in range(lb[i], lb[i + 1]):
            q = ent[e, 0]
            kids = sorted(ent[ent[e, 1]:ent[e, 2], 0]) if ent[e, 2] > ent[e, 1] else []
            assert kids == t.children(i, q)
            for c in range(ent[e, 1], ent[e, 2]):
                assert ent[c, 3] == (1 if ent[c, 0] == q else 0)
