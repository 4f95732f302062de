"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

oracle/flash_oracle.c is built with -fsanitize=address,undefined (every
finding fatal) and the pins of tests/test_oracle_pins.py run against that
build in a child process with the ASan runtime preloaded, so an out-of-bounds
access, use after free or undefined arithmetic anywhere the pins reach ends
the run.  A copy with a planted heap overflow checks that the sanitizer is
really active.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "flash_oracle.c")
PINS = os.path.join(ROOT, "tests", "test_oracle_pins.py")
FLAGS = ["-O1", "-g", "-std=gnu99", "-fopenmp", "-fPIC", "-shared", "-fno-omit-frame-pointer",
         "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def _runtime():
    path = subprocess.run(["gcc", "-print-file-name=libasan.so"], stdout=subprocess.PIPE).stdout.decode().strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        pytest.skip("gcc has no AddressSanitizer runtime here")
    return path


def _build(src_text, out):
    csrc = out[:-3] + ".c"
    with open(csrc, "w") as f:
        f.write(src_text)
    subprocess.check_call(["gcc"] + FLAGS + [csrc, "-o", out])


def _pins(so, select=None):
    pre = os.environ.get("LD_PRELOAD", "")
    env = dict(os.environ, FLASH_ORACLE_LIB=so, OMP_NUM_THREADS="4",
               LD_PRELOAD=_runtime() + (":" + pre if pre else ""),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    # -s: a sanitizer report is written to the real stderr, not a capture file
    cmd = [sys.executable, "-m", "pytest", PINS, "-q", "-s", "-p", "no:cacheprovider"]
    if select:
        cmd += ["-k", select]
    r = subprocess.run(cmd, cwd=ROOT, env=env, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, timeout=900)
    return r.returncode, r.stdout.decode(errors="replace")


def test_pins_pass_under_address_and_undefined_sanitizers(tmp_path):
    so = str(tmp_path / "oracle_asan.so")
    _build(open(SRC).read(), so)
    rc, out = _pins(so)
    assert rc == 0 and "AddressSanitizer" not in out and "runtime error" not in out, out[-3000:]


def test_sanitizer_reports_a_planted_overflow(tmp_path):
    # a reservoir written one slot past R overruns the last bucket's array
    src = open(SRC).read()
    old = "for (i = g; i < e && i - g < R; i++)\n                tab["
    assert src.count(old) == 1
    so = str(tmp_path / "oracle_overflow.so")
    _build(src.replace(old, "for (i = g; i < e && i - g <= R; i++)\n                tab["), so)
    rc, out = _pins(so, select="tables_brute_force")
    assert rc != 0 and "AddressSanitizer" in out, out[-3000:]
