"""Host code of the library under AddressSanitizer and UBSan, without a GPU:
the size and argument checks of the entry points and the batch planner
(hl_batch_plan_bytes: per-instance layouts, update steps, per-XCD work
queues, Toeplitz records) on the 64-instance batched workload (beta in
{1/3, 1/2, 2/3, 1}, N in [32, 512], P from the condition estimate, seed 1810),
the N = 1024, P = 49152 shape and a mixed set of forms.  The driver is
tests/host_sanitize_driver.cpp; the build puts the sanitizers on the host code
only."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))

pytestmark = pytest.mark.slow


def shapes():
    from hankel_inputs import batch_configs
    lines = ["%d 8 %d 16 0" % (n, p) for (_b, n, p) in batch_configs()]
    lines += ["1024 16 49152 16 0", "256 8 8192 16 1", "40 6 1024 1 1", "64 32 2048 16 0", "33 1 256 1 0"]
    return "\n".join(lines) + "\n"


def test_planner_and_checks_clean_under_asan_ubsan(tmp_path):
    if not shutil.which("/opt/rocm/bin/hipcc") and not shutil.which("hipcc"):
        pytest.skip("no hipcc")
    from paper_1810_01478_amd.build import build_host_sanitized
    exe = build_host_sanitized(str(tmp_path / "san"), os.path.join(HERE, "host_sanitize_driver.cpp"))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], input=shapes(), capture_output=True, text=True, env=env, timeout=300)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert "69 instances, 0 failures" in out, out[-2000:]
