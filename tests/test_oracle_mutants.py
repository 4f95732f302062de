"""The oracle's pins catch plausible mistakes (CPU only).

Each case below plants one mistake in a copy of oracle/flash_oracle.c, builds
the copy into a temporary library and runs tests/test_oracle_pins.py against
it in a child process; at least one pin must fail.  The product library is
not involved: these tests show that the pins constrain the oracle, so that
the oracle can in turn stand in for the paper in the GPU parity tests.
"""
import concurrent.futures
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "flash_oracle.c")
PINS = os.path.join(ROOT, "tests", "test_oracle_pins.py")

# (name, [(text in the oracle, replacement), ...])
MUTANTS = [
    # Eq. 1: the bin keeps its largest permuted value instead of the smallest
    ("bin maximum", [("if (!occ[bin] || h < code[bin]) {", "if (!occ[bin] || h > code[bin]) {")]),
    # one-permutation bins are slices of the permuted range, not residues
    ("modulo bins", [("return (uint32_t)(((uint64_t)h * (uint64_t)n) >> 32);", "return h % n;")]),
    # Sec. 2.3 densification borrows from a bin densified earlier in the sweep
    ("chained densification",
     [("(uint32_t)B);\n            if (occ[p]) {\n                out[j] = code[p];",
       "(uint32_t)B);\n            if (occ[p] || p < (uint32_t)j) {\n                out[j] = occ[p] ? code[p] : out[p];")]),
    # the probe sequence depends on the row (its length), not only on the bin
    ("row-dependent probe", [("(((uint32_t)j << 16) | (uint32_t)a) ^ s_d)",
                              "(((uint32_t)j << 16) | (uint32_t)a) ^ s_d ^ (uint32_t)n)")]),
    # rotation densification to the left instead of the right
    ("rotation to the left", [("int p = (j + r) % B;", "int p = (j - r + B) % B;")]),
    # key fields in reverse order
    ("reversed key layout", [("key |= (codes[t * K + j] & mask) << (b * j);",
                              "key |= (codes[t * K + j] & mask) << (b * (K - 1 - j));")]),
    # a reservoir keeps one slot fewer than R
    ("reservoir one short", [("for (i = g; i < e && i - g < R; i++)\n                tab[",
                              "for (i = g; i < e && i - g < R - 1; i++)\n                tab[")]),
    # priorities without their random part: the R smallest ids are kept
    ("priority without randomness", [("return ((x >> 32) << 32) | (uint64_t)(uint32_t)id;",
                                      "return (x & 0) | (uint64_t)(uint32_t)id;")]),
    # run counting starts at one too many
    ("count off by one", [("kv[nkv].cnt = 0;", "kv[nkv].cnt = 1;")]),
    # ties broken by the larger id
    ("ties by larger id", [("return (x->id > y->id) - (x->id < y->id);",
                            "return (x->id < y->id) - (x->id > y->id);")]),
    # the query's own id is not left out
    ("self kept", [("if (self >= 0 && x == self) continue;", "if (self >= 0 && x == self - 1) continue;")]),
    # the shared pool rounded up to a power of two
    ("pool rounded", [("    return P < 1 ? 1 : P;\n}",
                       "    { uint64_t u = 1; while (u < P) u <<= 1; P = u; }\n    return P < 1 ? 1 : P;\n}")]),
]


def _mutant_source(edits):
    src = open(SRC).read()
    for old, new in edits:
        assert src.count(old) == 1, f"mutation anchor not found once: {old!r}"
        src = src.replace(old, new)
    return src


def _run(name, edits, tmpdir):
    tag = "".join(c if c.isalnum() else "_" for c in name)
    csrc = os.path.join(tmpdir, f"mut_{tag}.c")
    so = os.path.join(tmpdir, f"mut_{tag}.so")
    with open(csrc, "w") as f:
        f.write(_mutant_source(edits))
    subprocess.check_call(["gcc", "-O1", "-std=gnu99", "-fopenmp", "-fPIC", "-shared", "-w", csrc, "-o", so])
    env = dict(os.environ, FLASH_ORACLE_LIB=so, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", PINS, "-x", "-q", "-p", "no:cacheprovider"],
                       cwd=ROOT, env=env, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, timeout=600)
    return r.returncode, r.stdout.decode(errors="replace")


def test_unmutated_copy_passes_the_pins(tmp_path):
    rc, out = _run("none", [], str(tmp_path))
    assert rc == 0, out[-2000:]


def test_every_planted_mistake_fails_a_pin(tmp_path):
    with concurrent.futures.ThreadPoolExecutor(max_workers=4) as ex:
        futs = {name: ex.submit(_run, name, edits, str(tmp_path)) for name, edits in MUTANTS}
        results = {name: f.result() for name, f in futs.items()}
    survived = [name for name, (rc, _) in results.items() if rc == 0]
    broken = [name for name, (rc, _) in results.items() if rc not in (0, 1)]
    assert not survived, f"no pin fails for: {survived}"
    assert not broken, {n: results[n][1][-1500:] for n in broken}
