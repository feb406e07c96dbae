"""The host library (lk_host.cpp, lk_serve.cpp) against a fake device of CPU-thread
workers that speak the same mailbox protocol (tests/fake/lk_backend_fake.cpp), built with
ThreadSanitizer and with AddressSanitizer + UBSan: exactly-once and FIFO under concurrent
clusters, ring-full, bad arguments, a hung worker (timeout, then recovery), disposed
state, cluster slicing, batches, serving with retained outputs, serving stopped by a hung
worker (posted tiles drained before it returns), the idle watchdog,
dispose with items in flight, dispose of a hung worker and the CU reservation.  No GPU involved."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2310_01212_amd", "csrc")
SOURCES = [os.path.join(ROOT, "tests", "fake", "fake_device_test.cpp"),
           os.path.join(ROOT, "tests", "fake", "lk_backend_fake.cpp"),
           os.path.join(CSRC, "lk_host.cpp"), os.path.join(CSRC, "lk_serve.cpp")]
SCENARIOS = ["single_worker_1000", "concurrent_clusters", "error_paths", "pinned_input", "cluster_split", "batch_tiles",
             "serving", "serving_error_drains", "idle_watchdog", "dispose_in_flight", "dispose_hung_worker", "cu_reservation", "xcd_mask"]


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
@pytest.mark.parametrize("sanitizer,env", [
    ("thread", {"TSAN_OPTIONS": "halt_on_error=1"}),
    ("address,undefined", {"ASAN_OPTIONS": "halt_on_error=1:detect_leaks=1",
                           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}),
])
def test_host_library_against_fake_device(tmp_path, sanitizer, env):
    exe = tmp_path / "fake_test"
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", f"-fsanitize={sanitizer}",
                    "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), "-I", CSRC, *SOURCES,
                    "-lpthread", "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=240, env={**os.environ, **env})
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "Sanitizer" not in out and "runtime error" not in out, out[-4000:]
    for name in SCENARIOS:
        assert f"OK {name}" in r.stdout
    assert "ALL OK" in r.stdout
