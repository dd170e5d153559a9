"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer: the
driver oracle/sanitize_main.c compiles oracle.c into itself and runs every
entry point on small inputs (l up to 4, several primitives, argument errors),
in both the double and the long-double build.  Host code only."""
import os
import shutil
import subprocess

import pytest

ORACLE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle")


@pytest.mark.parametrize("kind", ["double", "long double"])
def test_oracle_asan_ubsan(tmp_path, kind):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_asan")
    cmd = ["gcc", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g",
           "-O1", "-fopenmp", "-std=gnu11", os.path.join(ORACLE, "sanitize_main.c"), "-lm", "-o", exe]
    if kind == "long double":
        cmd.insert(1, "-DORACLE_LD")
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "ok" in r.stdout
