"""Build libpmchwt.so (HIP, gfx950) in place.

    python paper_2008_04772_amd/build.py      # or __graft_entry__.build()

Compiles the device translation unit and the host sources with hipcc and
links them against rocSOLVER / rocBLAS.  Every call rebuilds.
"""

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libpmchwt.so")
BUILD = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# packed FP32 instructions are kept out of the device code
DEVICE_FLAGS = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17", "-munsafe-fp-atomics",
                "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# host sources reproduce plain IEEE evaluation order (no FMA contraction) for
# the geometric classification tables
HOST_FLAGS = ["-O2", "-fPIC", "-std=c++17", "-ffp-contract=off", "--offload-arch=gfx950"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("build step failed:\n" + " ".join(cmd) + "\n" + r.stdout)
    return r.stdout


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    jobs = [
        [HIPCC] + DEVICE_FLAGS + ["-c", os.path.join(CSRC, "kernels.hip"), "-o", os.path.join(BUILD, "kernels.o")],
        [HIPCC] + HOST_FLAGS + ["-x", "hip", "-c", os.path.join(CSRC, "api.cpp"), "-o", os.path.join(BUILD, "api.o")],
        [HIPCC] + HOST_FLAGS + ["-c", os.path.join(CSRC, "geometry.cpp"), "-o", os.path.join(BUILD, "geometry.o")],
    ]
    with ThreadPoolExecutor(3) as ex:
        outs = list(ex.map(_run, jobs))
    tmp = OUT + ".tmp"
    link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp,
            os.path.join(BUILD, "kernels.o"), os.path.join(BUILD, "api.o"), os.path.join(BUILD, "geometry.o"),
            "-L/opt/rocm/lib", "-lrocsolver", "-lrocblas", "-Wl,-rpath,/opt/rocm/lib"]
    outs.append(_run(link))
    os.replace(tmp, OUT)
    if verbose:
        for o in outs:
            if o.strip():
                print(o)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
