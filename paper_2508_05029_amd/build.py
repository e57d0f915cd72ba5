"""Build the native libraries in-tree.

  libtq.so      HIP kernels + C++ runtime + C ABI (hipcc, gfx950)
  libtqgen.so   seeded input generators (gcc, OpenMP)

Every hipcc line carries the packed-FP32 opt-out; nothing here uses fast-math
(the AVG division must round exactly).
"""
import glob
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-munsafe-fp-atomics",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-function", "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"build failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    if verbose and r.stderr.strip():
        print(r.stderr, flush=True)


def build_gen(verbose=False):
    src = os.path.join(HERE, "datagen", "datagen.c")
    out = os.path.join(HERE, "datagen", "libtqgen.so")
    _run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-Wall", src, "-o", out + ".tmp", "-lm"],
         verbose)
    os.replace(out + ".tmp", out)
    return out


def build_tq(verbose=False, jobs=8):
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))
    objs = []

    def compile_one(src):
        obj = os.path.join(BUILD, os.path.basename(src) + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        _run([HIPCC] + HIP_FLAGS + lang + ["-c", src, "-o", obj], verbose)
        return obj

    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(compile_one, srcs))
    out = os.path.join(HERE, "libtq.so")
    _run([HIPCC, "-shared", f"--offload-arch={ARCH}", "-fPIC"] + objs + ["-o", out + ".tmp", "-lpthread"],
         verbose)
    os.replace(out + ".tmp", out)
    return out


def build(verbose=False):
    build_gen(verbose)
    if glob.glob(os.path.join(CSRC, "*.hip")):
        build_tq(verbose)


if __name__ == "__main__":
    build(verbose=True)
