"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

tests/host_sanitize_driver.cpp drives the host stages of the C ABI (geometry,
spaces, cluster trees, block partitions, near pairs, CSR patterns and tiles,
size models, error paths, handle destruction) on a host-only context; it is
built here with the sanitizers on the host compilation only (-Xarch_host) and
must run to its end with no report, leaks included.  No GPU is used.
"""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2306_11324_amd", "csrc")


@pytest.mark.slow
def test_host_stages_clean_under_sanitizers(tmp_path):
    from paper_2306_11324_amd import build as b
    from paper_2306_11324_amd import inputs as I
    hipcc = b.hipcc()
    if shutil.which("ld.lld") is None and not os.path.exists("/opt/rocm/llvm/bin/ld.lld"):
        pytest.skip("no linker for hipcc")
    exe = str(tmp_path / "driver")
    cmd = [hipcc, f"--offload-arch={b.ARCH}", "-O1", "-g", "-std=c++17",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument",
           "-I", os.path.join(ROOT, "include"), "-o", exe, os.path.join(ROOT, "tests", "host_sanitize_driver.cpp")]
    cmd += [os.path.join(CSRC, f) for f in b.SOURCES]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    pth = str(tmp_path / "sphere.bin")
    with open(pth, "wb") as f:
        P = I.sphere_patches()
        f.write(struct.pack("i", len(P)))
        for p in P:
            f.write(struct.pack("4i", p.deg_u, p.deg_v, p.ncp_u, p.ncp_v))
            for a in (p.knots_u, p.knots_v, p.cpw):
                f.write(np.ascontiguousarray(a, dtype=np.float64).tobytes())
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe, pth], capture_output=True, text=True, env=env, timeout=900)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert r.stdout.strip().endswith("ok")
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr[-4000:]
