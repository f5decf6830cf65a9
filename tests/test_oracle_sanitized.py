"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

``tests/csrc/oracle_check.c`` includes ``oracle/csrc/oracle.c`` and runs each
of its entry points (transforms and their round trips, automorphism, slot
encoding, plaintext lift, encryption, Galois and switching keys, phase,
rotation, plaintext product, cluster encoding from int8 and int16 rows,
scoring of a two-chunk ragged cluster) on the small-ring parameters.  The
sanitized build must run clean and write the same bytes as a plain -O2 build.
"""
import shutil
import subprocess
from pathlib import Path

import pytest

from oracle.bfv import Oracle
from oracle.params import preset

ROOT = Path(__file__).resolve().parents[1]
SRC = ROOT / "tests" / "csrc" / "oracle_check.c"


def _build(tmp, flags, name):
    gcc = shutil.which("gcc")
    if not gcc:
        pytest.skip("gcc not available")
    exe = tmp / name
    subprocess.run([gcc, "-std=c11", "-Wall", "-Wextra", "-Wno-unused-function", *flags, str(SRC), "-o", str(exe)],
                   check=True)
    return exe


@pytest.mark.parametrize("name", ["tiny"])
def test_oracle_runs_clean_under_sanitizers(tmp_path, name):
    o = Oracle(preset(name))
    params = tmp_path / "params.bin"
    params.write_bytes(bytes(o._s))
    san = _build(tmp_path, ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                            "-fno-omit-frame-pointer"], "oracle_san")
    plain = _build(tmp_path, ["-O2"], "oracle_plain")
    env = {"ASAN_OPTIONS": "detect_leaks=1", "UBSAN_OPTIONS": "print_stacktrace=1", "PATH": "/usr/bin:/bin"}
    r = subprocess.run([str(san), str(params), str(tmp_path / "san.out")], capture_output=True, text=True, env=env,
                       timeout=600)
    assert r.returncode == 0, r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    r = subprocess.run([str(plain), str(params), str(tmp_path / "plain.out")], capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0, r.stderr
    a, b = (tmp_path / "san.out").read_bytes(), (tmp_path / "plain.out").read_bytes()
    assert len(a) > 0 and a == b
