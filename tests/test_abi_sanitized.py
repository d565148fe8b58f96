"""The library's host code built with the address and undefined-behaviour
sanitizers (host side only; the device objects are the regular build's),
driven through the C ABI by tests/abi_driver.cpp: argument validation of
every entry point, the host passes over the caller's arrays that precede any
device call, and the error paths a machine without a GPU takes.  Any
sanitizer report aborts the driver (no recovery)."""
import concurrent.futures
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1810_01967_amd", "csrc")
HOST_SOURCES = ["mrf_api.cpp", "mrf_net.cpp", "mrf_tree.cpp", "covertree.cpp", "mrf_subspace.cpp",
                "mrf_nufft.cpp"]
# each sanitizer flag applies to the host compilation only
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all"]


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    pytest.skip("hipcc not available")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    from paper_1810_01967_amd import build as lib_build
    kernels = [os.path.join(ROOT, "paper_1810_01967_amd", "_build", os.path.splitext(s)[0] + ".o")
               for s in lib_build.SOURCES if s.startswith("k_")]
    kernels = [k for k in kernels if os.path.exists(k)]
    assert kernels, "build the library first (paper_1810_01967_amd.build.build())"
    out = tmp_path_factory.mktemp("abi_san")
    hipcc = _hipcc()
    common = ["-O1", "-g", "-std=c++17", "-fPIC", "-fno-omit-frame-pointer", "--offload-arch=gfx950",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *HOST_SAN,
              "-I", os.path.join(ROOT, "include")]

    def compile_one(src):
        obj = str(out / (os.path.basename(src) + ".o"))
        r = subprocess.run([hipcc, *common, "-x", "hip", "-c", src, "-o", obj], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr
        return obj

    srcs = [os.path.join(CSRC, s) for s in HOST_SOURCES] + [os.path.join(ROOT, "tests", "abi_driver.cpp")]
    with concurrent.futures.ThreadPoolExecutor(max_workers=4) as ex:
        objs = list(ex.map(compile_one, srcs))
    exe = str(out / "abi_driver")
    r = subprocess.run([hipcc, "--offload-arch=gfx950", *HOST_SAN, "-o", exe, *objs, *kernels,
                        "-L/opt/rocm/lib", "-lrocsolver", "-lrocblas", "-Wl,-rpath,/opt/rocm/lib"],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def test_abi_validation_under_sanitizers(driver):
    env = dict(os.environ)
    # leak reports would name the HIP runtime's own start-up allocations
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1"
    r = subprocess.run([driver], capture_output=True, text=True, env=env, timeout=300)
    print(r.stdout[-3000:])
    assert "ERROR: AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    assert "runtime error" not in r.stderr, r.stderr[-4000:]
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
    assert "0 failure(s)" in r.stdout
