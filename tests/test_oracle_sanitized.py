"""The oracle's pins under AddressSanitizer and UndefinedBehaviorSanitizer.

The oracle is built a second time with gcc's -fsanitize=address,undefined
(host code only; every finding aborts) and the whole pin suite runs against
that build in a child process that preloads the sanitizer runtimes. Two
mistakes planted in copies of the oracle's source, a read past the end of
the density array and a signed integer overflow, show that the sanitizers
are live in that set-up: each run must abort with the sanitizer's report.
"""
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtimes():
    libs = []
    for name in ("libasan.so", "libubsan.so"):
        path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True,
                              text=True).stdout.strip()
        if not os.path.isabs(path) or not os.path.exists(path):
            pytest.skip(f"gcc has no {name}")
        libs.append(path)
    return ":".join(libs)


def _env(lib):
    env = dict(os.environ)
    env.update(LD_PRELOAD=_runtimes(), ASAN_OPTIONS="detect_leaks=0", MACLAB_ORACLE_LIB=lib,
               PYTHONPATH=ROOT)
    return env


def test_pins_pass_under_sanitizers():
    lib = oracle.build_sanitized()
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider"],
                       env=_env(lib), cwd=ROOT, capture_output=True, text=True, timeout=600)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0


PLANTED = {
    # the diagnostics loop runs one node too far
    "heap-buffer-overflow": ("for (int64_t x = 0; x < N; ++x) {\n    int finite",
                             "for (int64_t x = 0; x <= N; ++x) {\n    int finite"),
    # an int sum that overflows
    "signed integer overflow": ("  out7[6] = bad;", "  out7[6] = bad + (real)(INT32_MAX + (int)p->n[0]);"),
}

PROBE = """
import numpy as np, oracle
p = oracle.Problem(q=9, n=(6, 5, 1), dx=0.1, nu=0.01)
rho = np.ones(30); u = np.zeros((2, 30))
print(oracle.diagnostics(p, rho, u))
"""


@pytest.mark.parametrize("report", sorted(PLANTED))
def test_sanitizers_catch_a_planted_mistake(tmp_path, report):
    find, repl = PLANTED[report]
    src = open(oracle._SRC).read()
    assert src.count(find) == 1
    msrc = tmp_path / "maclab_oracle.c"
    msrc.write_text(src.replace(find, repl))
    lib = oracle.build(True, oracle.SANITIZE_FLAGS, str(tmp_path / "libplanted.so"), str(msrc))
    r = subprocess.run([sys.executable, "-c", PROBE], env=_env(lib), cwd=ROOT, capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert report in r.stderr
    # the same probe on the unplanted sanitized build runs clean
    ok = subprocess.run([sys.executable, "-c", PROBE], env=_env(oracle.build_sanitized()), cwd=ROOT,
                        capture_output=True, text=True, timeout=120)
    assert ok.returncode == 0, ok.stderr[-2000:]
