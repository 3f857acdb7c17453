"""The host C code -- the CPU oracle (oracle/lawler_pr.c) and the block-pair
workload builder (paper_2201_01556_amd/regions.c) -- built with gcc's
AddressSanitizer and UndefinedBehaviorSanitizer (host code only) and run on
seeded random inputs by tests/native/sanitize_driver.c; the run must end
cleanly."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_host_c_under_sanitizers():
    tmp = tempfile.mkdtemp()
    try:
        exe = os.path.join(tmp, "sanitize_driver")
        cmd = ["gcc", "-O1", "-g", "-std=gnu99", "-fopenmp",
               "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
               "-fno-omit-frame-pointer",
               os.path.join(HERE, "native", "sanitize_driver.c"),
               os.path.join(ROOT, "oracle", "lawler_pr.c"),
               os.path.join(ROOT, "paper_2201_01556_amd", "regions.c"),
               "-o", exe]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="2")
        r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
        assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
        assert "sanitized runs clean" in r.stdout
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
