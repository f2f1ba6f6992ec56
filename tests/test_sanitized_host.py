"""Host code under the sanitizers (CPU only, no GPU needed).

* The library's self-test of its internal checks (scratch capacity guard,
  byte cap, device status word).
* The library's host code built with AddressSanitizer and
  UndefinedBehaviorSanitizer (host-only objects, no device code) and run by a
  driver through every path that needs no GPU: self-test, coefficient
  derivation for every kernel, argument validation, context creation.
* The plain-C oracle (``oracle/csum.c``) built with the same sanitizers and run
  on a small case, its results equal to the numpy oracle's.
"""
import os
import subprocess

import numpy as np
import pytest

from oracle import interp
from oracle import kernels as K

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
OUT = os.path.join(ROOT, "_build", "sanitize")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def test_library_selftest():
    from paper_2107_01104_amd import ptk
    assert ptk.lib.ptk_selftest() == ptk.OK


def test_host_code_under_sanitizers():
    from paper_2107_01104_amd import build
    exe = build.build_host_sanitized(os.path.join(HERE, "host_driver.cpp"), OUT)
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all checks passed" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr


@pytest.mark.parametrize("fam,I,m", [(K.LAGRANGE, 4, 0), (K.SPLINE, 8, 2)])
def test_c_oracle_under_sanitizers(tmp_path, fam, I, m):
    os.makedirs(OUT, exist_ok=True)
    exe = os.path.join(OUT, "oracle_driver")
    subprocess.check_call(["gcc", "-O1", "-g", "-ffp-contract=off", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-o", exe,
                           os.path.join(HERE, "oracle_driver.c"), os.path.join(ROOT, "oracle", "csum.c"), "-lm"])
    N, n = 9, 500
    rng = np.random.default_rng(I)
    u = rng.standard_normal((N, N, N, 3))
    X = rng.uniform(-7.0, 13.0, (n, 3))
    X[:4] = [[0.0, 0.0, 0.0], [np.nextafter(2 * np.pi, 0), 0.0, -1e-300], [1e6, -1e6, 3.0], [-0.0, 6.0, 6.3]]
    coef = K.coeff_table_f64(fam, I, m)
    dcoef = np.zeros((I, I))
    dcoef[:, : I - 1] = K.coeff_table_f64(fam, I, m, deriv=True)[:, : I - 1]
    for name, arr in [("field", u), ("X", X), ("coef", coef), ("dcoef", dcoef)]:
        np.ascontiguousarray(arr, dtype=np.float64).tofile(str(tmp_path / f"{name}.bin"))
    ou, og = str(tmp_path / "u.bin"), str(tmp_path / "g.bin")
    r = subprocess.run([exe, str(tmp_path), str(N), str(n), str(I), ou, og], capture_output=True, text=True,
                       env=dict(ENV, OMP_NUM_THREADS="1"), timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    gu = np.fromfile(ou).reshape(n, 3)
    gg = np.fromfile(og).reshape(n, 3, 3)
    ru, rg = interp.interp_vec(u, X, fam, I, m, gradient=True)
    assert np.max(np.abs(gu - ru)) <= 1e-13 * np.sqrt(np.mean(ru ** 2))
    assert np.max(np.abs(gg - rg)) <= 1e-13 * np.sqrt(np.mean(rg ** 2))
