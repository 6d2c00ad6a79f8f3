"""Build libsem.so (HIP for gfx950) in-tree.

    python -m paper_1806_01422_amd.build        # or: python paper_1806_01422_amd/build.py

Every source under csrc/ is compiled with hipcc for gfx950 and linked into
paper_1806_01422_amd/libsem.so next to this file.  Objects go to paper_1806_01422_amd/_build/;
first, gen/fast_consts_gen.hip is built and run to write _build/gen/fast_consts.h (compile-time
coefficient constants from the library's own table routine).
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
GEN = os.path.join(OBJ, "gen")  # headers written by the build (fast_consts.h)
LIB = os.path.join(HERE, "libsem.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
    # packed FP32 instructions stay off (hipcc -O3 would otherwise form them from float code)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-I", GEN,
]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))


def _compile(src):
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    cmd = [HIPCC] + FLAGS + ["-c", src, "-o", obj]
    if src.endswith(".cpp"):
        cmd = [HIPCC, "-x", "hip"] + FLAGS + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def gen_headers():
    """Compile and run gen/fast_consts_gen.hip (host code, with the GLL routine it shares with the
    library) to write _build/gen/fast_consts.h."""
    os.makedirs(GEN, exist_ok=True)
    exe = os.path.join(GEN, "fast_consts_gen")
    cmd = [HIPCC, "-O2", "-std=c++17", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "--offload-arch=gfx950", "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-o", exe,
           os.path.join(HERE, "gen", "fast_consts_gen.hip"), "-x", "hip", os.path.join(CSRC, "gll.cpp")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"generator build failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    out = os.path.join(GEN, "fast_consts.h")
    r = subprocess.run([exe, out], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"generator failed: {r.stdout}\n{r.stderr}")


def build(verbose=False, jobs=None):
    os.makedirs(OBJ, exist_ok=True)
    gen_headers()
    srcs = sources()
    jobs = jobs or min(len(srcs), max(1, (os.cpu_count() or 4)))
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
