"""Host code under the address and undefined-behaviour sanitizers (CPU only).

Builds, with -fsanitize=address,undefined and no recovery:
  * tests/native/host_checks.cpp with the library's coefficient setup
    (qw_coeffs.cpp) and its host helpers from qw_kernels.h, compiled host-only:
    pass plans and tile index maps for every n, the fused schedule, the XCD
    tile order, Miller's Bessel values, Chebyshev and CF degrees;
  * tests/native/oracle_checks.c with the oracle's C loops (oracle/ref.c).
Both must run clean; the coefficient values they print are compared with the
oracle (Bessel values from mpmath, degrees from the truncation tail)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2608_12058_amd", "csrc")
NATIVE = os.path.join(ROOT, "tests", "native")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="2")


def _hipcc():
    for c in ("/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    pytest.skip("hipcc not available")


def _run(exe):
    p = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=300)
    assert p.returncode == 0, p.stderr[-4000:]
    assert "runtime error" not in p.stderr and "AddressSanitizer" not in p.stderr, p.stderr[-4000:]
    return p.stdout


@pytest.fixture(scope="module")
def host_checks_output(tmp_path_factory):
    d = tmp_path_factory.mktemp("san")
    exe = str(d / "host_checks")
    # host-only compilation: device code is parsed but not generated; each
    # sanitizer flag applies to the host side only
    cmd = [_hipcc(), "-x", "hip", "--offload-host-only", "-O1", "-g", "-std=c++17",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           os.path.join(NATIVE, "host_checks.cpp"), os.path.join(CSRC, "qw_coeffs.cpp"), "-o", exe]
    subprocess.check_call(cmd, stderr=subprocess.DEVNULL)
    return _run(exe)


def test_host_helpers_clean_under_sanitizers(host_checks_output):
    assert "PLANS OK" in host_checks_output


def test_sanitized_coefficients_match_oracle(host_checks_output, oracle_mod):
    coef = [ln.split() for ln in host_checks_output.splitlines() if ln.startswith("COEF")]
    bes = [ln.split() for ln in host_checks_output.splitlines() if ln.startswith("BESSEL")]
    assert len(coef) == 32 and len(bes) > 100
    for row in coef:
        method, a, tol, K = int(row[1]), float(row[2]), float(row[3]), int(row[4])
        alpha = np.array([float(x) for x in row[5:]])
        assert len(alpha) == K + 1
        if method == 0:
            ref = oracle_mod.cheb_alpha(a)
            assert K == oracle_mod.cheb_degree(ref, tol), (a, tol)
            assert np.max(np.abs(alpha - ref[:K + 1])) <= 1e-14, (a, tol)
        else:
            # CF: a degree no larger than the Chebyshev one, meeting the tolerance
            assert K <= oracle_mod.cheb_degree(oracle_mod.cheb_alpha(a), tol)
    for row in bes:
        a, m, val = float(row[1]), int(row[2]), float(row[3])
        ref = oracle_mod._bessel_table(a)
        want = ref[m] if m < len(ref) else 0.0
        assert abs(val - want) <= 1e-15, (a, m, val, want)


def test_oracle_loops_clean_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_checks")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c99", "-fopenmp", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                           os.path.join(ROOT, "oracle", "ref.c"), os.path.join(NATIVE, "oracle_checks.c"),
                           "-o", exe, "-lm"])
    assert "ORACLE LOOPS OK" in _run(exe)
