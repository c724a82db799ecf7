"""The library's host code under AddressSanitizer, LeakSanitizer and
UndefinedBehaviorSanitizer, on the CPU.

1. The translation units that build meshes, DOF maps, patterns, SELL layouts,
   incidence and slot maps, Poisson row partitions and the tetrahedral rule
   (mesh.cpp, parts.cpp, rules.cpp), compiled with g++ (no device code) and
   driven by tests/host_sanitize.cpp over every mesh kind the library accepts,
   with consistency checks of every structure, and its error paths.
2. Every host translation unit of the library (the units above and run.cpp,
   batch.cpp, steady.cpp, capi.cpp), compiled with the ROCm clang++ and the
   sanitizers, linked with the library's own unsanitized kernel objects,
   driven through the C ABI's host-side calls by tests/host_sanitize_capi.cpp
   (no call reaches a device). The OpenMP runtime keeps one internal
   allocation until exit, which LeakSanitizer reports; that allocation is
   suppressed, nothing else.

Any sanitizer report fails the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2605_25403_amd", "csrc")
UNITS = ["mesh.cpp", "parts.cpp", "rules.cpp"]
HOST_UNITS = UNITS + ["run.cpp", "batch.cpp", "steady.cpp", "capi.cpp"]
KERNEL_OBJS = ["kernels_asm.o", "kernels_krylov.o", "kernels_fcg.o", "kernels_fields.o",
               "kernels_steady.o", "scratch.o"]
OBJ = os.path.join(ROOT, "paper_2605_25403_amd", "_build")
CLANG = "/opt/rocm/llvm/bin/clang++"
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_host_units_are_clean_under_address_and_ub_sanitizers(tmp_path):
    exe = str(tmp_path / "host_sanitize")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fopenmp",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I", os.path.join(ROOT, "include"),
           "-I", CSRC, os.path.join(ROOT, "tests", "host_sanitize.cpp")]
    cmd += [os.path.join(CSRC, u) for u in UNITS] + ["-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="4")
    run = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert run.returncode == 0, (run.stdout[-2000:], run.stderr[-6000:])
    assert "ok" in run.stdout and "runtime error" not in run.stderr, run.stderr[-4000:]


@pytest.mark.skipif(not os.path.exists(CLANG), reason="ROCm clang++ not available")
def test_c_abi_host_calls_are_clean_under_sanitizers(tmp_path):
    objs = [os.path.join(OBJ, o) for o in KERNEL_OBJS]
    if not all(os.path.exists(o) for o in objs):
        pytest.skip("kernel objects not built (run __graft_entry__.build())")
    flags = ["-x", "c++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fopenmp",
             "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I", os.path.join(ROOT, "include"),
             "-I", CSRC] + SAN
    srcs = [os.path.join(CSRC, u) for u in HOST_UNITS]
    srcs.append(os.path.join(ROOT, "tests", "host_sanitize_capi.cpp"))
    procs, outs = [], []
    for src in srcs:
        out = str(tmp_path / (os.path.basename(src) + ".o"))
        outs.append(out)
        procs.append(subprocess.Popen([CLANG] + flags + ["-c", src, "-o", out],
                                      stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True))
    for p in procs:
        _, err = p.communicate(timeout=600)
        assert p.returncode == 0, err[-4000:]
    exe = str(tmp_path / "host_sanitize_capi")
    r = subprocess.run([CLANG] + SAN + ["-fopenmp"] + outs + objs +
                       ["-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe],
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    supp = tmp_path / "lsan.supp"
    supp.write_text("leak:libomp.so\n")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
               LSAN_OPTIONS=f"suppressions={supp}", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="4")
    run = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert run.returncode == 0, (run.stdout[-2000:], run.stderr[-6000:])
    assert "ok" in run.stdout and "runtime error" not in run.stderr, run.stderr[-4000:]
