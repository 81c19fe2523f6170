"""Builds librcscm.so (HIP kernels for gfx950 + the C ABI) in-tree.

    python -m paper_1908_01964_amd.build [--jobs N] [--verbose] [--debug]

Every .hip and .cpp file under csrc/ is compiled with hipcc for
--offload-arch=gfx950 into _build/, then linked into
paper_1908_01964_amd/librcscm.so.  Packed-FP32 instructions are disabled
(-Xclang -target-feature -Xclang -packed-fp32-ops) for all device code.
Then the plain-C ABI client of the tests (tests/c/abi_run.c) is built
against the library.

--debug builds _build/debug/librcscm_debug.so instead, with -DRCSCM_DEBUG:
the kernels check their row, chunk and bin indexes against the extents of
the arrays they address (RCSCM_DASSERT) and stop with a message on the first
failed check.  Nothing loads it by default; the CPU tests only compile it.
"""
import argparse
import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "librcscm.so")
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-command-line-argument", f"-I{INCLUDE}", f"-I{CSRC}"]


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found (ROCm is required to build librcscm)")


DEBUG_BUILD = os.path.join(BUILD, "debug")
DEBUG_LIB = os.path.join(DEBUG_BUILD, "librcscm_debug.so")


def _compile(src, verbose, debug=False):
    obj = os.path.join(DEBUG_BUILD if debug else BUILD, os.path.basename(src) + ".o")
    cmd = [hipcc()] + COMMON + (["-DRCSCM_DEBUG"] if debug else []) + ["-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n{r.stdout}\n{r.stderr}")
    if verbose and r.stderr.strip():
        print(r.stderr, file=sys.stderr)
    return obj


def build(jobs=None, verbose=False, debug=False):
    os.makedirs(DEBUG_BUILD if debug else BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))
    jobs = jobs or min(8, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, debug), srcs))
    if debug:
        cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", DEBUG_LIB] + objs
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"link failed\n{r.stdout}\n{r.stderr}")
        return DEBUG_LIB
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    _build_c_client(verbose)
    return LIB


C_CLIENT_SRC = os.path.join(ROOT, "tests", "c", "abi_run.c")
C_CLIENT = os.path.join(ROOT, "tests", "c", "abi_run")


def _build_c_client(verbose):
    """The plain-C ABI client used by the tests (gcc, C99, linked against librcscm.so)."""
    cc = shutil.which("gcc") or shutil.which("cc")
    if not cc or not os.path.exists(C_CLIENT_SRC):
        return
    rocm = os.path.dirname(os.path.dirname(os.path.realpath(hipcc())))
    cmd = [cc, "-std=c99", "-O2", "-Wall", "-Wextra", "-D__HIP_PLATFORM_AMD__",
           f"-I{rocm}/include", f"-I{INCLUDE}", C_CLIENT_SRC, "-o", C_CLIENT, f"-L{PKG}",
           "-lrcscm", f"-L{rocm}/lib", "-lamdhip64",
           "-Wl,-rpath,$ORIGIN/../../paper_1908_01964_amd", f"-Wl,-rpath,{rocm}/lib"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"C client build failed\n{r.stdout}\n{r.stderr}")


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--debug", action="store_true", help="the bounds-checked build (-DRCSCM_DEBUG)")
    a = ap.parse_args()
    print(build(a.jobs, a.verbose, a.debug))
