"""A build of the library's host code with AddressSanitizer and UBSan, for CPU checks of the C ABI.

    python -m paper_1908_01964_amd.sanitize_build      # prints the path of the checker

The host-side logic of the library - argument validation, workspace sizing, the row, chunk and
class tables, error handling and clean-up (csrc/context.cpp) and the no-allocation entry point's
checks (csrc/noalloc.hip) - is compiled with the sanitizers on the host pass only, and linked with
the kernel objects of the regular build (python -m paper_1908_01964_amd.build, run first if they
are missing) and the plain-C client tests/c/abi_host.c into one executable, _build/san/abi_host.
Nothing in it needs a GPU: tests/test_sanitize_cpu.py runs it on the CPU.
"""
import os
import shutil
import subprocess
import sys

from .build import CSRC, INCLUDE, ROOT, hipcc

SAN = os.path.join(ROOT, "_build", "san")
CHECKER_SRC = os.path.join(ROOT, "tests", "c", "abi_host.c")
CHECKER = os.path.join(SAN, "abi_host")
# each sanitizer option applies to the host pass only
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined"]


def _rocm():
    return os.path.dirname(os.path.dirname(os.path.realpath(hipcc())))


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(" ".join(cmd) + "\n" + r.stdout + r.stderr)


# sources whose host code is checked; the other objects come from the regular build
SANITIZED = ("context.cpp", "noalloc.hip")


def build():
    from . import build as regular
    os.makedirs(SAN, exist_ok=True)
    srcs = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip") or f.endswith(".cpp"))
    if not all(os.path.exists(os.path.join(regular.BUILD, f + ".o")) for f in srcs):
        regular.build()
    objs = []
    for f in srcs:
        if f not in SANITIZED:
            objs.append(os.path.join(regular.BUILD, f + ".o"))
            continue
        obj = os.path.join(SAN, f + ".o")
        _run([hipcc(), "-O1", "-g", "-fno-omit-frame-pointer", "-std=c++17", "-fPIC",
              "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              f"-I{INCLUDE}", f"-I{CSRC}", "-Wno-unused-command-line-argument"] + HOST_SAN +
             ["-c", os.path.join(CSRC, f), "-o", obj])
        objs.append(obj)
    rocm = _rocm()
    clang = os.path.join(rocm, "llvm", "bin", "clang")
    cobj = os.path.join(SAN, "abi_host.o")
    _run([clang, "-std=c99", "-O1", "-g", "-Wall", "-Wextra", "-fsanitize=address,undefined",
          "-D__HIP_PLATFORM_AMD__", f"-I{rocm}/include", f"-I{INCLUDE}", "-c", CHECKER_SRC,
          "-o", cobj])
    _run([clang + "++", "-fsanitize=address,undefined", "-o", CHECKER, cobj] + objs +
         [f"-L{rocm}/lib", "-lamdhip64", f"-Wl,-rpath,{rocm}/lib"])
    return CHECKER


if __name__ == "__main__":
    if not shutil.which(hipcc()):
        sys.exit("hipcc not found")
    print(build())
