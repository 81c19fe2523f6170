"""The chunk order over the XCDs (csrc/xcd_order.h) is a permutation of [0, n) for every n:
each chunk of a launch is processed by exactly one workgroup. The device function has no
dependencies, so it is compiled here for the host with g++ and checked exhaustively for small n
and at the sizes of the bench workloads."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "paper_1908_01964_amd", "csrc", "xcd_order.h")

SRC = r"""
#include <cstdio>
#include <vector>
#define __device__
#define __forceinline__ inline
#include "xcd_order.h"
static bool check(int n) {
  std::vector<int> seen(n, 0);
  for (int w = 0; w < n; ++w) {
    const int c = rcscm::xcd_local_chunk(w, n);
    if (c < 0 || c >= n || seen[c]++) return false;
  }
  return true;
}
int main() {
  for (int n = 1; n <= 4096; ++n)
    if (!check(n)) { std::printf("fail %d\n", n); return 1; }
  const int big[] = {16400, 130193, 150001, 262144, 1000003};
  for (int n : big)
    if (!check(n)) { std::printf("fail %d\n", n); return 1; }
  std::printf("ok\n");
  return 0;
}
"""


def test_xcd_order_is_a_permutation(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    src = tmp_path / "xcd.cpp"
    src.write_text(SRC)
    exe = tmp_path / "xcd"
    subprocess.run([gxx, "-std=c++17", "-O2", f"-I{os.path.dirname(HDR)}", str(src), "-o", str(exe)],
                   check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout
