"""The oracle and the library's host code under AddressSanitizer and
UndefinedBehaviorSanitizer, on the CPU.

The oracle's C sources and the library's hand-written units (host code
instrumented, device code compiled plainly, no kernel instantiations) are
built with clang's sanitizers into a temporary directory; the oracle pins
and the C-ABI tests then run in a child process with the shared sanitizer
runtime preloaded and ORACLE_LIB / QMC_LIB pointing at those builds.  Any
finding aborts the child and is written to the log this test prints.
"""
import glob
import os
import subprocess
import sys

import pytest

from oracle import oracle as O
from paper_1811_11722_amd import build_sanitized as BS

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(tmp_path, env_extra, files):
    env = dict(os.environ)
    env.update(env_extra)
    env["LD_PRELOAD"] = BS.runtime_path()
    env["ASAN_OPTIONS"] = f"detect_leaks=0:log_path={tmp_path}/asan"
    env["UBSAN_OPTIONS"] = f"print_stacktrace=1:log_path={tmp_path}/ubsan"
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-s", "-p", "no:cacheprovider", "-m", "not gpu", *files]
    res = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    reports = "".join(open(p).read() for p in glob.glob(f"{tmp_path}/asan*") + glob.glob(f"{tmp_path}/ubsan*"))
    assert res.returncode == 0 and not reports, (res.stdout[-3000:], res.stderr[-3000:], reports[:6000])


def test_oracle_sanitized(tmp_path):
    lib = O.build_sanitized(str(tmp_path / "liboracle_san.so"))
    _run(tmp_path, {"ORACLE_LIB": lib}, ["tests/test_oracle_pins.py", "tests/test_oracle_cvtrain_pins.py"])


def test_host_code_sanitized(tmp_path):
    lib = BS.build(str(tmp_path / "libqmc_san.so"))
    _run(tmp_path, {"QMC_LIB": lib}, ["tests/test_abi.py"])
