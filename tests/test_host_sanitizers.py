"""libdg's host code (dg_api.hip, dg_vec.hip host parts) under
AddressSanitizer and UndefinedBehaviorSanitizer on the CPU: workspace
queries, the N_dof limit, null-argument and missing-workspace paths."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
BUILD = os.path.join(ROOT, "paper_1911_01492_amd", "_build")
CSRC = os.path.join(ROOT, "paper_1911_01492_amd", "csrc")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
@pytest.mark.skipif(not all(os.path.exists(os.path.join(BUILD, f + ".o"))
                            for f in ("dg_affine", "dg_mfma", "dg_ppd", "dg_trilinear", "dg_geom")),
                    reason="library objects not built")
def test_host_code_under_asan_ubsan(tmp_path):
    objs = []
    for f in ("dg_api", "dg_vec"):
        o = str(tmp_path / (f + ".o"))
        subprocess.run([HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC"] + SAN +
                       ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                        "-I" + os.path.join(ROOT, "include"), "-c", os.path.join(CSRC, f + ".hip"), "-o", o],
                       check=True, capture_output=True)
        objs.append(o)
    drv = str(tmp_path / "drv.o")
    subprocess.run([HIPCC, "-O1", "-g", "-std=c++17"] + SAN + ["-I" + os.path.join(ROOT, "include"),
                   "-x", "c++", "-c", os.path.join(ROOT, "tests", "host_sanitize_driver.cpp"), "-o", drv],
                   check=True, capture_output=True)
    exe = str(tmp_path / "drv")
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-fsanitize=address", "-fsanitize=undefined",
                    "-fno-gpu-sanitize", drv] + objs +
                   [os.path.join(BUILD, f + ".o") for f in ("dg_affine", "dg_mfma", "dg_ppd", "dg_trilinear", "dg_geom")] +
                   ["-o", exe],
                   check=True, capture_output=True)
    # the HIP runtime's own allocations are not this library's: leak checking off
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "host driver: ok" in r.stdout
