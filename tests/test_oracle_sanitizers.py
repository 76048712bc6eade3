"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (gcc,
-fno-sanitize-recover, leak detection on) runs every main path of its C API
-- all connection rules and models, per-neuron and drawn parameters, drawn
and listed weights, STDP, devices, recorded, replayed and sampled input,
refused calls -- without a report (oracle/sanitize_driver.c).  CPU only."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = tmp_path / "orc_sanitized"
    src = [os.path.join(ROOT, "oracle", f) for f in ("sanitize_driver.c", "snn_oracle.c")]
    subprocess.run(["gcc", "-std=c11", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-fno-omit-frame-pointer", "-ffp-contract=off", "-o", str(exe)] + src + ["-lm"], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "sanitized oracle run ok" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
