"""Build the HIP library libprdpt.so for gfx950 in-tree (hipcc, no JIT)."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OBJ = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libprdpt.so")
ARCH = os.environ.get("PRDPT_OFFLOAD_ARCH", "gfx950")

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", "-Wno-unused-value", "-Wno-unused-result",
          "-I", os.path.join(ROOT, "include"), "-I", CSRC,
          # binary32 results must follow the source's operation order
          "-ffp-contract=off", "-fno-fast-math"]
DEVICE = ["--offload-arch=" + ARCH, "-fhip-fp32-correctly-rounded-divide-sqrt",
          "-fno-gpu-flush-denormals-to-zero",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
SOURCES = [("kernels.hip", True), ("api.cpp", False), ("bvh.cpp", False),
           ("batch.cpp", False), ("serve.cpp", False)]


def _compile(src, device):
    path = os.path.join(CSRC, src)
    out = os.path.join(OBJ, src + ".o")
    cmd = ["hipcc", "-c", *COMMON]
    if device:
        cmd += DEVICE
    else:
        cmd += ["-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include"]
    cmd += [path, "-o", out]
    subprocess.run(cmd, check=True)
    return out


def build(verbose=False):
    os.makedirs(OBJ, exist_ok=True)
    srcs = [(s, dev) for s, dev in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with ThreadPoolExecutor(max_workers=4) as ex:
        objs = list(ex.map(lambda a: _compile(*a), srcs))
    cmd = ["hipcc", "-shared", "--offload-arch=" + ARCH, "-fPIC", *objs, "-o", LIB + ".tmp",
           "-lpthread"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
