"""The oracle's C source built with AddressSanitizer and UndefinedBehaviorSanitizer (gcc, host code
only) and run over every entry point on small grids: both boundary kinds, the AMF and W = P schemes,
the Richardson pair and the combination over many threads.  The run must be free of sanitizer
reports, and its results must equal those of the ordinary build."""
import json
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "amfrw_oracle.c")

SCRIPT = r"""
import dataclasses, json
import numpy as np
import oracle
from paper_2408_00559_amd import inputs as I

out = {}
p = I.draw_instances(1, seed=11, d=3)[0]
for tag, q in (("neumann", p), ("dirichlet", dataclasses.replace(p, boundary=I.DIRICHLET))):
    levels = [2, 3, 1]
    Y = oracle.initial_data(q, levels)
    F = oracle.eval_F(q, levels, Y)
    acc = [float(np.sum(F))]
    for ax in range(3):
        acc.append(float(np.sum(oracle.solve_axis(q, levels, ax, 0.01, F))))
    acc.append(float(np.sum(oracle.solve_lower(q, levels, 0.01, F))))
    acc.append(oracle.interpolate(q, levels, oracle.solve_grid(q, levels, 3)))
    acc.append(oracle.price(q, I.combination(4, 1), 4, nthreads=4))
    acc.append(oracle.price(q, I.combination(3, 0), 2, richardson=True))
    acc.append(oracle.price(q, I.combination(3, 1), 2, scheme=oracle.scheme_theta_gs(0.5, 2)))
    d, m, a = oracle.coefficients(q, q.xeval)
    acc += [float(np.sum(d)), float(np.sum(m)), float(np.sum(a)), oracle.payoff(q, q.xeval)]
    out[tag] = acc
c = I.paper_caplet()
out["caplet"] = [oracle.price(c, I.combination(5, 1), 8, nthreads=2)]
out["grids"] = int(len(oracle.ct_grids(6, 6, 1)[1]))
print("RESULT " + json.dumps(out))
"""


def _run(env):
    r = subprocess.run([sys.executable, "-c", SCRIPT], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=600)
    return r


@pytest.mark.timeout(900)
def test_oracle_is_clean_under_asan_and_ubsan(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not found")
    asan = subprocess.run([gcc, "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("gcc has no AddressSanitizer runtime")
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.check_call([gcc, "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-fopenmp", "-fPIC", "-shared", "-std=c99", "-o", lib, SRC, "-lm"])
    base = dict(os.environ)
    base.pop("AMF_ORACLE_LIB", None)
    plain = _run(base)
    assert plain.returncode == 0, plain.stderr[-2000:]

    env = dict(base)
    env["AMF_ORACLE_LIB"] = lib
    env["LD_PRELOAD"] = asan
    # Python's own allocations are not the oracle's: leak checking is left out; every other
    # report aborts the run with a non-zero status.
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    san = _run(env)
    report = san.stderr[-4000:]
    assert san.returncode == 0, report
    assert "ERROR: AddressSanitizer" not in san.stderr, report
    assert "runtime error" not in san.stderr, report

    def parse(r):
        line = [l for l in r.stdout.splitlines() if l.startswith("RESULT ")][-1]
        return json.loads(line[len("RESULT "):])

    a, b = parse(plain), parse(san)
    assert a["grids"] == b["grids"]
    for key in ("neumann", "dirichlet", "caplet"):
        for x, y in zip(a[key], b[key]):
            assert abs(x - y) <= 1e-12 * max(1.0, abs(x)), (key, x, y)


@pytest.mark.timeout(300)
def test_sanitized_build_reports_a_planted_overflow(tmp_path):
    """The same build and run set-up catches a heap overflow planted in a copy of the oracle."""
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not found")
    asan = subprocess.run([gcc, "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("gcc has no AddressSanitizer runtime")
    src = tmp_path / "planted.c"
    src.write_text(open(SRC).read() + "\n#include <stdlib.h>\n"
                   "double orc_planted(long n) { double* v = malloc(n * sizeof(double));"
                   " double s = 0; for (long i = 0; i <= n; ++i) s += v[i] = (double)i;"
                   " free(v); return s; }\n")
    lib = str(tmp_path / "libplanted.so")
    subprocess.check_call([gcc, "-O1", "-g", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                           "-o", lib, str(src), "-lm"])
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0")
    code = ("import ctypes; L = ctypes.CDLL(%r); L.orc_planted.restype = ctypes.c_double; "
            "L.orc_planted.argtypes = [ctypes.c_long]; print(L.orc_planted(16))" % lib)
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                       timeout=120)
    assert r.returncode != 0
    assert "heap-buffer-overflow" in r.stderr
