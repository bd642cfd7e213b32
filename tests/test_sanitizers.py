"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the host C code
used by the tests and the measurements (the oracle and the pruned CPU
baseline), run by a driver that calls every exported function on small
random and degenerate inputs."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no host C compiler")
def test_oracle_and_baseline_under_asan_ubsan(tmp_path):
    exe = tmp_path / "sanitized"
    srcs = [os.path.join(ROOT, "tests", "sanitize", "driver.c"),
            os.path.join(ROOT, "oracle", "bkm_oracle.c"),
            os.path.join(ROOT, "oracle", "graph_oracle.c"),
            os.path.join(ROOT, "baseline", "pruned_cpu.c")]
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fopenmp", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           "-o", str(exe), *srcs, "-lm"]
    subprocess.run(cmd, check=True)
    env = dict(os.environ, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "sanitized run ok" in r.stdout
