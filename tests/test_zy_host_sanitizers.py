"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
on the GPU: tests/host_sanitizer_driver.cpp, built with every library source
by paper_1309_3848_amd/build.py (build_sanitized_driver; host code
instrumented, device code as in the library), calls every entry point of the
C ABI on small images and checks that the paths which must agree do agree.
A memory error, a leak from the library's own allocations or undefined
behaviour in host code ends it with a sanitizer report and a non-zero
status."""
import os
import subprocess
import sys

import pytest

from paper_1309_3848_amd import build as hipbuild

pytestmark = pytest.mark.gpu

# allocations made inside the ROCm runtime libraries on the library's behalf
# (their own caches and threads) are theirs to free, not the library's
LSAN_SUPPRESSIONS = """\
leak:libamdhip64
leak:libhsa-runtime64
leak:libamd_comgr
leak:librocprofiler
leak:libdrm
"""


def test_host_code_is_clean_under_sanitizers(tmp_path):
    exe = hipbuild.SAN_DRIVER
    if not os.path.exists(exe):
        pytest.fail("the sanitizer program is not built: run __graft_entry__.build()")
    supp = tmp_path / "lsan.supp"
    supp.write_text(LSAN_SUPPRESSIONS)
    env = dict(os.environ,
               ASAN_OPTIONS="detect_leaks=1:exitcode=23:protect_shadow_gap=0",
               LSAN_OPTIONS=f"suppressions={supp}:exitcode=23",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=24")
    print("[gpu-case] host sanitizer driver", flush=True)
    sys.stdout.flush()
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=900)
    out = r.stdout[-3000:] + r.stderr[-6000:]
    assert r.returncode == 0, out
    assert "host sanitizer runs: ok" in r.stdout, out
