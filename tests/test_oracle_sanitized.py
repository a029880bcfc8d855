"""The FP64 oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The oracle's C source is compiled with gcc -fsanitize=address,undefined (errors fatal)
and driven from a child Python process that preloads the sanitizer runtimes.  The child
runs the oracle's condensed pins (test_oracle_mutations.py) on the sanitized build,
every planted mistake of the mutation harness (each built with the sanitizers too, so the
pins must reject them without a memory error), and calls over the edge shapes (batch 0
and 1, 1024-point axes, rectangles, per-array filter operators, one and many threads).
A control build with an out-of-bounds write planted must make the child fail with a
sanitizer report: that shows the sanitizers are really active.
"""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(ROOT, "oracle", "dct_oracle.c")

FLAGS = ["gcc", "-O1", "-g", "-std=c99", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
         "-fno-omit-frame-pointer", "-ffp-contract=off", "-fPIC", "-shared", "-pthread"]

CHILD = r"""
import sys
import numpy as np
sys.path.insert(0, sys.argv[1])
import oracle
from tests.test_oracle_mutations import _pins_pass
real = oracle.Oracle(sys.argv[2])
assert _pins_pass(real), "sanitized oracle failed its pins"
g = np.random.default_rng(3)
for shape in ((0, 8, 8), (1, 8, 8), (3, 8, 1024), (2, 1024, 8), (1, 384, 512), (4, 256, 256)):
    x = g.standard_normal(shape).astype(np.float32)
    for threads in (1, 8):
        y = real.forward(x, threads=threads)
        xi = real.inverse(y, threads=threads)
        rt = real.roundtrip(x, threads=threads)
        assert y.shape == x.shape and xi.shape == x.shape and rt.shape == x.shape
        if x.size:
            assert np.abs(rt - x).max() < 1e-12 * max(1.0, np.abs(x).max())
    if x.shape[0]:
        lam = g.uniform(-1, 1, x.shape)
        assert real.filter(x, lam).shape == x.shape
        assert real.filter(x, lam[0]).shape == x.shape
for n in (1, 8, 1024):
    q = real.qmatrix(n)
    assert abs(q[0, 0] - n ** -0.5) < 1e-15
for path in sys.argv[3:]:
    assert not _pins_pass(oracle.Oracle(path)), "pins missed the planted mistake in " + path
print("SANITIZED-OK", flush=True)
"""


def _build(src_text, path):
    src = path + ".c"
    with open(src, "w") as f:
        f.write(src_text)
    subprocess.run(FLAGS + [src, "-o", path, "-lm"], check=True)
    return path


def _child(libs, tmp_path):
    env = dict(os.environ)
    rt = [subprocess.run(["gcc", "-print-file-name=" + n], capture_output=True, text=True, check=True).stdout.strip()
          for n in ("libasan.so", "libubsan.so")]
    env["LD_PRELOAD"] = ":".join(rt)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1"
    return subprocess.run([sys.executable, "-c", CHILD, ROOT] + libs, capture_output=True, text=True, env=env,
                          cwd=str(tmp_path), timeout=600)


def test_sanitized_oracle_passes_pins_and_rejects_planted_mistakes(tmp_path):
    from tests.test_oracle_mutations import MUTATIONS
    src = open(SRC).read()
    real = _build(src, str(tmp_path / "liboracle_real.so"))
    mutants = []
    for name, (old, new) in sorted(MUTATIONS.items()):
        assert old in src, name
        mutants.append(_build(src.replace(old, new), str(tmp_path / ("liboracle_%s.so" % name))))
    r = _child([real] + mutants, tmp_path)
    assert r.returncode == 0 and "SANITIZED-OK" in r.stdout, r.stdout[-2000:] + r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]


def test_sanitizer_catches_a_planted_overflow(tmp_path):
    """Control: the per-array output pointer moved one element past its array makes the last
    array's final store land outside the output buffer; the sanitized child must abort."""
    src = open(SRC).read()
    old = "double* out = job->y + b * n;"
    if old not in src:
        pytest.fail("overflow anchor not found in the oracle source")
    bad = _build(src.replace(old, "double* out = job->y + b * n + 1;"),
                 str(tmp_path / "liboracle_overflow.so"))
    r = _child([bad], tmp_path)
    assert r.returncode != 0 and "AddressSanitizer" in r.stderr, r.stdout[-1000:] + r.stderr[-2000:]
