"""The bounds-checked debug build (-DRCSCM_DEBUG) compiles for gfx950 (no GPU needed).

In that build every kernel checks its row, chunk and bin indexes against the extents of the
arrays it addresses (RCSCM_DASSERT in rcscm_internal.h) and stops with a message on the first
failed check; the regular build has no such code.  The test builds it from source and checks
that the checks are in its device code and not in the regular library's.
"""
import os

from paper_1908_01964_amd import build as B

MSG = b"rcscm debug check failed"


def test_debug_build_compiles_with_device_checks():
    lib = B.build(debug=True)
    with open(lib, "rb") as f:
        assert f.read().count(MSG) > 0
    if os.path.exists(B.LIB):
        with open(B.LIB, "rb") as f:
            assert f.read().count(MSG) == 0
