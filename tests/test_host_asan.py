"""The library built with AddressSanitizer on its host code (device code unchanged),
driven through the C ABI on the CPU by tests/asan_driver.cpp: the host utilities on
ragged, empty and edge-case inputs (the visibility order with no, density and
continuous preconditioners; the density counts; the Daubechies filters) and the
argument checks of hs_create.  Any invalid host access aborts the driver."""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1806_04596_amd", "csrc")
SOURCES = ["hs_api.cpp", "hs_plan.cpp", "k_nufft.hip", "k_wavelet.hip", "k_nuclear.hip", "k_misc.hip"]


def _hipcc():
    p = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
    return p if os.path.exists(p) else shutil.which("hipcc")


@pytest.mark.slow
def test_host_code_under_address_sanitizer(tmp_path):
    hipcc = _hipcc()
    if not hipcc:
        pytest.skip("hipcc not found")
    # -fsanitize only for the host pass of each compilation
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]
    flags = ["-x", "hip", "--offload-arch=gfx950", "-O1", "-std=c++17", "-I", os.path.join(ROOT, "include"),
             "-I", CSRC, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-result", "-Wno-unused-value", *san]

    def compile_one(src):
        obj = str(tmp_path / (os.path.splitext(src)[0] + ".o"))
        extra = ["-ffp-contract=off"] if src == "hs_plan.cpp" else []
        r = subprocess.run([hipcc, *flags, *extra, "-c", os.path.join(CSRC, src), "-o", obj],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        return obj

    with ThreadPoolExecutor(max_workers=6) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    drv = str(tmp_path / "asan_driver.o")
    r = subprocess.run([hipcc, "-O1", "-std=c++17", "-I", os.path.join(ROOT, "include"), *san, "-c",
                        os.path.join(ROOT, "tests", "asan_driver.cpp"), "-o", drv], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    exe = str(tmp_path / "asan_driver")
    r = subprocess.run([hipcc, "--offload-arch=gfx950", *san, "-o", exe, *objs, drv], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "ok (0 failures)" in r.stdout
