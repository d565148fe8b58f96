"""Host pieces of the non-uniform FFT plan, compiled with g++: the
deapodisation transform phihat against adaptive quadrature of its definition
(scipy), and the per-pair bin sorting of the samples (a stable permutation by
bin, consistent offsets, bins recomputed independently from the
coordinates)."""
import os
import subprocess

import numpy as np
import pytest
from scipy import integrate

from synth import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


# the driver is built twice: optimised, and with the address and
# undefined-behaviour sanitizers (any report aborts the run)
SANITIZE = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


@pytest.fixture(scope="module", params=["O2", "asan-ubsan"])
def driver(tmp_path_factory, request):
    exe = tmp_path_factory.mktemp("nufft") / "nufft_driver"
    opt = ["-O2"] if request.param == "O2" else SANITIZE
    subprocess.run(["g++", *opt, "-std=c++17", os.path.join(ROOT, "tests", "nufft_driver.cpp"), "-o", str(exe)],
                   check=True)
    return str(exe)


def _run(driver, tmp_path, W, Ny, Nx, xi, tr):
    inp = tmp_path / "in.bin"
    npairs = len(tr.off) - 1
    with open(inp, "wb") as f:
        np.array([W, Ny, Nx, len(xi), npairs], dtype=np.int64).tofile(f)
        np.asarray(xi, dtype=np.float64).tofile(f)
        np.asarray(tr.off, dtype=np.int64).tofile(f)
        np.ascontiguousarray(tr.coords, dtype=np.float32).tofile(f)
    out = tmp_path / "out.txt"
    subprocess.run([driver, str(inp), str(out)], check=True)
    lines = open(out).read().split("\n")
    ph = np.array([float(v) for v in lines[:len(xi)]])
    bperm = np.array(lines[len(xi)].split(), dtype=np.int64)
    boff = np.array(lines[len(xi) + 1].split(), dtype=np.int64)
    return ph, bperm, boff


@pytest.mark.parametrize("W", [5, 7, 8])
def test_phihat_and_bins(driver, tmp_path, W):
    ny = nx = 32
    Ny, Nx = 2 * ny, 2 * nx
    tr = workloads.spiral_trajectory(2, 3, ny, nx, frac=0.2)
    xi = (np.arange(ny) - ny // 2) / Ny
    ph, bperm, boff = _run(driver, tmp_path, W, Ny, Nx, xi, tr)
    beta = 2.30 * W

    def phi(u):
        z = 2.0 * u / W
        return np.exp(beta * (np.sqrt(max(0.0, 1.0 - z * z)) - 1.0)) if abs(z) < 1 else 0.0

    for x, got in zip(xi, ph):
        ref, _ = integrate.quad(lambda u: phi(u) * np.cos(2 * np.pi * u * x), -W / 2, W / 2, limit=200,
                                epsabs=1e-13, epsrel=1e-12)
        # Simpson on 4,096 intervals; the kernel's derivative is singular at the
        # support edge, where phi = e^-beta: 3e-9 at W = 5, far below the
        # transform's own 1e-4 there
        assert abs(got - ref) <= 1e-8 * abs(ref)
    # bins recomputed from the coordinates: floor of the fine position mod N over 8
    k = tr.coords.astype(np.float64)
    uy, ux = np.mod(k[:, 0] * Ny, Ny), np.mod(k[:, 1] * Nx, Nx)
    nby, nbx = Ny // 8, Nx // 8
    binid = np.minimum(uy // 8, nby - 1).astype(int) * nbx + np.minimum(ux // 8, nbx - 1).astype(int)
    nb = nby * nbx
    for p in range(len(tr.off) - 1):
        b, e = tr.off[p], tr.off[p + 1]
        perm = bperm[b:e]
        assert sorted(perm.tolist()) == list(range(b, e))
        bins = binid[perm]
        assert np.all(np.diff(bins) >= 0)
        for q in np.unique(bins):                       # ties keep the sample order
            assert np.all(np.diff(perm[bins == q]) > 0)
        bo = boff[p * (nb + 1):(p + 1) * (nb + 1)]
        np.testing.assert_array_equal(bo, np.concatenate([[0], np.cumsum(np.bincount(bins, minlength=nb))]))
