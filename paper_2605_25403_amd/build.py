"""Build libipcs.so (HIP kernels for gfx950 + host C++ + the C ABI) in-tree.

    python -m paper_2605_25403_amd.build        # or build() from Python

Objects go to paper_2605_25403_amd/_build/, the library to
paper_2605_25403_amd/lib/libipcs.so. Every call recompiles.
"""
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OBJ = os.path.join(PKG, "_build")
LIBDIR = os.path.join(PKG, "lib")
LIB = os.path.join(LIBDIR, "libipcs.so")

SOURCES = ["mesh.cpp", "parts.cpp", "run.cpp", "batch.cpp", "capi.cpp", "steady.cpp", "rules.cpp",
           "scratch.hip", "kernels_asm.hip", "kernels_krylov.hip", "kernels_fcg.hip",
           "kernels_fields.hip", "kernels_steady.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CXX = os.environ.get("IPCS_CXX", "/opt/rocm/llvm/bin/clang++")
ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          "-I", os.path.join(ROOT, "include"), "-I", CSRC]
# packed FP32 instructions are disabled for all device code
# code object v5 loads on every ROCm 6/7 runtime (torch may bring an older one)
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics", "-mcode-object-version=5"]
OPENMP = ["-fopenmp"]


def _compile(src):
    path = os.path.join(CSRC, src)
    out = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
    if src.endswith(".hip"):
        cmd = [HIPCC, "-x", "hip"] + DEVICE + COMMON + ["-c", path, "-o", out]
    else:
        # host-only translation units: plain C++ against the HIP runtime headers
        cmd = [CXX, "-x", "c++"] + COMMON + OPENMP + [
            "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include", "-c", path, "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return out, r.stderr


def build(verbose=False):
    os.makedirs(OBJ, exist_ok=True)
    os.makedirs(LIBDIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        results = list(ex.map(_compile, SOURCES))
    if verbose:
        for _, err in results:
            if err.strip():
                print(err, file=sys.stderr)
    objs = [o for o, _ in results]
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", f"--offload-arch={ARCH}", "-mcode-object-version=5", "-fopenmp",
           "-o", tmp] + objs + [
        "-Wl,-rpath,/opt/rocm/llvm/lib", "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    shutil.move(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
