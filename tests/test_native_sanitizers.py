"""Host code of the library under the compiler's sanitizers (CPU, no device).

Two harnesses in tests/native/ are compiled with the host compiler and run:
  * host_rules_harness.cpp with host_rules.cpp (the host-only entry points dacp_plan,
    dacp_accept_rule, dacp_spacing_ratios and the divide-and-conquer merge bookkeeping), under
    AddressSanitizer + UndefinedBehaviorSanitizer, on random and edge-case inputs;
  * block_cache_harness.cpp with block_cache.h (the stream-ordered device-block cache shared by the
    batched path's worker threads), on a recording stand-in for the runtime with 16 threads, under
    ThreadSanitizer and again under AddressSanitizer.  It checks that a reused block's wait captures
    exactly the event state recorded when the block was last freed, and that no event is recorded
    while a wait on it is being queued.
Each run must exit 0 with no sanitizer report.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2011_02107_amd", "csrc")
NATIVE = os.path.join(ROOT, "tests", "native")
CXX = shutil.which(os.environ.get("CXX", "g++"))

pytestmark = pytest.mark.skipif(CXX is None, reason="no host C++ compiler")


def build_and_run(tmp_path, name, sources, sanitize):
    exe = str(tmp_path / name)
    cmd = [CXX, "-std=c++17", "-O1", "-g", f"-fsanitize={sanitize}", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-I", CSRC, *sources, "-o", exe, "-lpthread"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", TSAN_OPTIONS="halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, f"{name} failed ({r.returncode}):\n{r.stdout}\n{r.stderr[-4000:]}"
    assert "Sanitizer" not in r.stderr, r.stderr[-4000:]
    return r.stdout


def test_host_rules_under_address_and_undefined_sanitizers(tmp_path):
    out = build_and_run(tmp_path, "host_rules_asan",
                        [os.path.join(NATIVE, "host_rules_harness.cpp"), os.path.join(CSRC, "host_rules.cpp")],
                        "address,undefined")
    assert "0 failures" in out


@pytest.mark.parametrize("sanitize", ["thread", "address,undefined"])
def test_block_cache_hand_off_under_sanitizers(tmp_path, sanitize):
    out = build_and_run(tmp_path, "block_cache_" + sanitize.split(",")[0],
                        [os.path.join(NATIVE, "block_cache_harness.cpp")], sanitize)
    assert "0 failures" in out
