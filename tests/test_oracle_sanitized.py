"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host
only): its library is rebuilt with both, and the oracle's own pins run
against it in a child process, so an out-of-bounds access, a use after
free or undefined arithmetic anywhere they reach fails the run."""
import os
import subprocess
import sys

import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
MODULES = ["test_oracle_pass.py", "test_oracle_mlp.py", "test_oracle_learning.py", "test_oracle_tree.py",
           "test_oracle_cells_footprint.py", "test_oracle_cells5d.py"]


def _runtime(name):
    path = subprocess.run(["gcc", "-print-file-name=" + name], capture_output=True, text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_pins_under_asan_and_ubsan(tmp_path):
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("gcc has no AddressSanitizer runtime here")
    so = oracle.build(out=str(tmp_path / "liboracle_san.so"),
                      extra=("-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                             "-fno-sanitize-recover=undefined"))
    env = dict(os.environ, RLC_ORACLE_LIB=so, LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu"] +
                       [os.path.join(HERE, m) for m in MODULES], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=900)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert "passed" in r.stdout
