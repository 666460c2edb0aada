"""The library's host code (scene validation, BVH builder, argument checks,
optimiser step, context creation without a device) under AddressSanitizer,
LeakSanitizer and UndefinedBehaviorSanitizer, on the CPU.  The host sources
are compiled with g++; kernels.hip with hipcc, sanitizers on its host part
only."""
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2211_17263_amd", "csrc")
ROCM = "/opt/rocm"

pytestmark = pytest.mark.skipif(shutil.which("hipcc") is None or shutil.which("g++") is None,
                                reason="needs hipcc and g++")


def test_host_code_under_sanitizers(tmp_path):
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC, "-I", os.path.join(ROCM, "include"),
           "-D__HIP_PLATFORM_AMD__"]
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer"]
    common = ["-O1", "-g", "-std=c++17", "-fPIC", "-w", "-ffp-contract=off", "-fno-fast-math"]
    objs = []
    for src in ("api.cpp", "bvh.cpp", "batch.cpp", "serve.cpp"):
        o = str(tmp_path / (src + ".o"))
        subprocess.run(["g++", "-c", *common, *san, *inc, os.path.join(CSRC, src), "-o", o],
                       check=True)
        objs.append(o)
    drv = str(tmp_path / "driver.o")
    subprocess.run(["g++", "-c", *common, *san, *inc,
                    os.path.join(ROOT, "tests", "host", "sanitize_driver.cpp"), "-o", drv], check=True)
    kern = str(tmp_path / "kernels.o")
    subprocess.run(["hipcc", "-c", *common, *inc, "--offload-arch=gfx950",
                    "-fhip-fp32-correctly-rounded-divide-sqrt", "-fno-gpu-flush-denormals-to-zero",
                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                    "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                    os.path.join(CSRC, "kernels.hip"), "-o", kern], check=True)
    exe = str(tmp_path / "driver")
    subprocess.run(["g++", *san, drv, *objs, kern, "-o", exe, "-L", os.path.join(ROCM, "lib"),
                    "-lamdhip64", "-lpthread", "-Wl,-rpath," + os.path.join(ROCM, "lib")],
                   check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", HIP_VISIBLE_DEVICES="")
    # the deep-stack scene of the GPU parity tests: its tree can drive a ray's
    # stack past the LDS entries, and stays within the private part's bound
    from paper_2211_17263_amd import scenes as S
    deep = S.deep_stack_scene()
    tri_file = tmp_path / "deep.f32"
    deep.arrays()["tris"].astype(np.float32).tofile(tri_file)
    r = subprocess.run([exe, str(tri_file)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-5000:]
    assert "host checks OK" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
    m = re.search(r"file depth4=(\d+) stack_bound=(\d+) lds_entries=(\d+)", r.stdout)
    depth, bound, lds = (int(g) for g in m.groups())
    assert lds < bound <= 3 * 13 + 1, r.stdout
    # one lane of the node loop replayed on the host (no distance culling,
    # random wave decisions): within the bound, and past the LDS part on the
    # deep-stack scene as on the GPU
    emu = [int(v) for v in re.findall(r"emulated deepest stack=(\d+)", r.stdout)]
    assert emu and max(emu) <= bound, r.stdout
    m = re.search(r"file emulated deepest stack=(\d+)", r.stdout)
    assert lds < int(m.group(1)) <= bound, r.stdout
