"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the host-side C
code, run on the CPU: the oracle (oracle/oracle.c) and the seeded input
generator (rmat.c), each under its own driver in tests/sanitize/. The two
are compiled separately and share nothing."""
import os
import shutil
import subprocess

import pytest

REPO = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(REPO, "tests", "sanitize")
FLAGS = ["-std=c99", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
         "-fno-sanitize-recover=all", "-Wall"]


def _run(tmp_path, name, sources, extra=()):
    if shutil.which("gcc") is None:
        pytest.skip("gcc is not installed")
    exe = str(tmp_path / name)
    subprocess.run(["gcc", *FLAGS, *extra, *sources, "-o", exe], check=True)
    # the environment is passed on unchanged; ASan is told not to insist on
    # being first in the library list
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ok" in r.stdout


def test_oracle_under_sanitizers(tmp_path):
    _run(tmp_path, "oracle_check", [os.path.join(HERE, "oracle_check.c"), os.path.join(REPO, "oracle", "oracle.c")])


def test_generator_under_sanitizers(tmp_path):
    _run(tmp_path, "rmat_check",
         [os.path.join(HERE, "rmat_check.c"), os.path.join(REPO, "paper_1208_5542_amd", "csrc", "rmat", "rmat.c")],
         extra=["-fopenmp"])
