"""Build librwmi.so (HIP for gfx950) in-tree with hipcc.

    python -m paper_2308_05007_amd.build

Translation units:
  k_fp64.hip  FP64 kernels and the precision-independent ones, with
              -ffp-contract=off so every double operation rounds once
  k_lowp.hip  FP32 / FP16 / BF16-storage kernels (contraction allowed)
  probe.hip   the bandwidth probe of the stream pattern (measurement only)
  capi.cpp    host side of the C ABI
All device code is built without packed FP32 instructions.
"""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librwmi.so")
BUILD = os.path.join(HERE, "_build")
ARCH = os.environ.get("RWMI_OFFLOAD_ARCH", "gfx950")

COMMON = ["-O3", "-std=c++17", "--offload-arch=" + ARCH, "-fPIC", "-Xclang", "-target-feature", "-Xclang",
          "-packed-fp32-ops", "-Wno-unused-result"]
UNITS = [
    ("k_fp64.hip", ["-ffp-contract=off"]),
    ("k_lowp.hip", ["-ffp-contract=fast"]),
    ("probe.hip", []),
    ("capi.cpp", ["-x", "hip", "-ffp-contract=off"]),
]


def hipcc():
    for c in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _compile(unit, extra):
    src = os.path.join(CSRC, unit)
    obj = os.path.join(BUILD, unit + ".o")
    cmd = [hipcc(), *COMMON, *extra, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s%s" % (" ".join(cmd), r.stdout, r.stderr))
    return obj


def build(verbose=True):
    """Compile every unit and link librwmi.so (always rebuilds)."""
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(UNITS)) as ex:
        objs = list(ex.map(lambda u: _compile(*u), UNITS))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s%s" % (" ".join(cmd), r.stdout, r.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
