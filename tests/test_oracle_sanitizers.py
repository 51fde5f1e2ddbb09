"""The FP64 oracle (test infrastructure) under the host address and
undefined-behaviour sanitizers, built with gcc from its C source together
with a small driver (tests/oracle_asan_driver.c).  CPU only; no GPU run
reads this file."""
import os
import shutil
import subprocess

import pytest


def test_oracle_under_host_sanitizers(oracle_lib, tmp_path):
    """The oracle built with the host address and undefined-behaviour
    sanitizers runs a walled channel with events, a periodic box whose sphere
    crosses a face, a demixed start and the adjoint without a report."""
    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    here = os.path.dirname(os.path.abspath(__file__))
    odir = os.path.dirname(oracle_lib.LIB_PATH)
    exe = tmp_path / "oracle_asan"
    flags = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all"]
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off"] + flags
                   + ["-I" + odir, "-o", str(exe), os.path.join(here, "oracle_asan_driver.c"),
                      os.path.join(odir, "lbm_oracle.c"), "-lm"], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr[-4000:]
    assert "Sanitizer" not in r.stderr, r.stderr[-4000:]
