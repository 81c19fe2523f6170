"""The library's host code under AddressSanitizer and UBSan (no GPU needed).

paper_1908_01964_amd.sanitize_build compiles the host logic (context.cpp: validation, workspace
sizing, the row/chunk/class tables, error paths and clean-up; noalloc.hip: the checks of the
no-allocation entry point) with both sanitizers and links it with tests/c/abi_host.c, a C client
that drives every validation branch, builds the tables for ragged batches under every rule and
schedule, and takes the error paths that follow a failed device call.  Any sanitizer report, or
a wrong status, fails the test.
"""
import os
import subprocess

from paper_1908_01964_amd import sanitize_build


def test_host_code_under_asan_and_ubsan():
    exe = sanitize_build.build()
    obj = os.path.join(sanitize_build.SAN, "context.cpp.o")
    syms = subprocess.run(["nm", obj], capture_output=True, text=True).stdout
    assert "__asan_report" in syms and "__ubsan_handle" in syms  # the checks are compiled in
    env = dict(os.environ,
               ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    out = r.stdout + r.stderr
    print(out)
    assert "AddressSanitizer" not in out and "runtime error" not in out
    assert "LeakSanitizer" not in out
    assert r.returncode == 0 and "abi_host done" in r.stdout
