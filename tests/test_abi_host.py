"""The C-ABI library loads on a machine without a GPU, exports every symbol of
include/qwexp.h, and its host-only logic (Bessel values, coefficients, degree,
CF, tile index maps, argument validation) is correct.  No kernel is launched."""
import ctypes
import os
import re

import mpmath
import numpy as np
import pytest

import paper_2608_12058_amd as qw

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    src = open(os.path.join(ROOT, "include", "qwexp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(qw_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(qw.LIB_PATH)
    syms = header_symbols()
    assert "qw_expm_action_c64" in syms and "qw_cheb_coeffs" in syms
    for s in syms:
        assert hasattr(lib, s), s


def test_version_string():
    assert "gfx950" in qw.version()


@pytest.mark.parametrize("a", [0.5, 22.07, 99.0, 470.2, -31.3])
def test_miller_bessel_vs_mpmath(a):
    """Miller's backward recurrence (section II.B.1) in double precision against
    40-digit mpmath at every order."""
    M = int(abs(a) + 40)
    J = qw.bessel_j(a, M)
    with mpmath.workdps(40):
        ref = np.array([float(mpmath.besselj(m, a)) for m in range(M + 1)])
    assert np.max(np.abs(J - ref)) < 4e-16


def test_miller_bessel_at_large_argument():
    a = 1403.7
    J = qw.bessel_j(a, 1500)
    with mpmath.workdps(30):
        for m in (0, 1, 700, 1390, 1450, 1500):
            assert abs(J[m] - float(mpmath.besselj(m, a))) < 1e-15


@pytest.mark.parametrize("a,tol", [(22.07, 1e-12), (99.0, 2.0 ** -53), (300.0, 2.0 ** -23),
                                   (470.2, 2.0 ** -23), (470.2, 1e-12), (-55.0, 1e-9)])
def test_chebyshev_coefficients_match_oracle(oracle_mod, a, tol):
    al, err = qw.cheb_coeffs(a, tol)
    ref = oracle_mod.cheb_coeffs(a, tol)
    K = len(ref) - 1
    assert len(al) - 1 == K
    m = np.arange(K + 1)
    c = ((-1j) ** m) * al
    assert np.max(np.abs(c - ref)) < 1e-15
    assert err <= tol


def test_degree_pin_151():
    al, _ = qw.cheb_coeffs(99.0, 2.0 ** -53)
    assert abs(len(al) - 151) <= 1


@pytest.mark.parametrize("a,tol", [(22.07, 1e-12), (120.0, 2.0 ** -23), (470.2, 2.0 ** -23), (47.0, 1e-6),
                                   (1000.0, 2.0 ** -23), (2000.0, 1e-10)])
def test_cf_coefficients_match_oracle_and_tolerance(oracle_mod, a, tol):
    al, lam = qw.cheb_coeffs(a, tol, "cf")
    ref, lam_ref = oracle_mod.cf_coeffs(a, tol)
    assert len(al) == len(ref)
    c = ((-1j) ** np.arange(len(al))) * al
    assert np.max(np.abs(c - ref)) < 1e-13
    assert abs(lam - lam_ref) <= 1e-6 * lam_ref + 1e-18
    x = np.cos(np.linspace(0, np.pi, 50001))
    err = np.max(np.abs(oracle_mod.cheb_series_eval(c, x) - np.exp(-1j * a * x)))
    assert err <= tol * 1.05


@pytest.mark.parametrize("n", list(range(1, 25)))
def test_tile_index_maps(n):
    """Every pass of the plan is a bijection onto [0, 2^n) and flipped partners
    stay in the tile; the passes cover all n bits."""
    for prec in (64, 128):
        P = qw.debug_check_plan(n, prec)
        assert P >= 1, (n, prec, P)


def test_pass_counts():
    assert qw.debug_check_plan(13, 64) == 1
    assert qw.debug_check_plan(22, 64) == 2
    assert qw.debug_check_plan(28, 64) == 3
    # complex64 switches to 2^14-amplitude tiles where that saves a pass
    assert qw.debug_check_plan(23, 64) == 2
    assert qw.debug_check_plan(24, 64) == 2
    assert qw.debug_check_plan(25, 64) == 3
    assert qw.debug_check_plan(23, 128) == 3
    assert qw.debug_check_plan(12, 128) == 1
    assert qw.debug_check_plan(21, 128) == 2


def test_workspace_bytes():
    assert qw.workspace_bytes(28, 64) >= (8 + 8 + 4) * (1 << 28)
    assert qw.workspace_bytes(28, 128) >= (16 + 16 + 8) * (1 << 28)
    assert qw.workspace_bytes(32, 64, True) < (8 + 8 + 1) * (1 << 32)
    assert qw.workspace_bytes(0, 64) == 0 and qw.workspace_bytes(10, 32) == 0


def test_invalid_arguments_are_rejected_before_any_launch():
    lib = qw.lib()
    info = qw.QwInfo()
    h = np.zeros(3)
    J = np.zeros(3)
    hp = h.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    Jp = J.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    fake = ctypes.c_void_p(256)
    ws = ctypes.c_void_p(1 << 20)
    # n out of range, non-finite scalars, bad tol, missing buffers, unaligned workspace
    cases = [
        (0, 1.0, 1.0, 1e-6, fake, ws),
        (33, 1.0, 1.0, 1e-6, fake, ws),
        (3, float("nan"), 1.0, 1e-6, fake, ws),
        (3, 1.0, float("inf"), 1e-6, fake, ws),
        (3, 1.0, 1.0, 0.0, fake, ws),
        (3, 1.0, 1.0, -1.0, fake, ws),
        (3, 1.0, 1.0, 1e-6, None, ws),
        (3, 1.0, 1.0, 1e-6, fake, None),
        (3, 1.0, 1.0, 1e-6, fake, ctypes.c_void_p((1 << 20) + 8)),
    ]
    for n, g, t, tol, psi, w in cases:
        st = lib.qw_expm_action_c64(n, None, hp, Jp, g, t, psi, psi, tol, 0, w, 1 << 30, None, ctypes.byref(info))
        assert st == qw.QW_EINVAL, (n, g, t, tol)
        assert len(qw.lib().qw_last_error()) > 0
    # diag == NULL without couplings
    st = lib.qw_expm_action_c128(3, None, None, None, 1.0, 1.0, fake, fake, 1e-6, 0, ws, 1 << 30, None, None)
    assert st == qw.QW_EINVAL
    # NaN in the couplings
    hbad = np.array([0.0, np.nan, 0.0])
    st = lib.qw_expm_action_c64(3, None, hbad.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), Jp, 1.0, 1.0,
                                fake, fake, 1e-6, 0, ws, 1 << 30, None, None)
    assert st == qw.QW_EINVAL
    # workspace too small
    st = lib.qw_expm_action_c64(20, None, np.zeros(20).ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                np.zeros(190).ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 1.0, 1.0,
                                fake, fake, 1e-6, 0, ws, 1024, None, None)
    assert st == qw.QW_ENOMEM
    # unknown method
    st = lib.qw_expm_action_c64(3, None, hp, Jp, 1.0, 1.0, fake, fake, 1e-6, 7, ws, 1 << 30, None, None)
    assert st == qw.QW_EINVAL


def test_coefficient_errors():
    with pytest.raises(qw.QwError):
        qw.cheb_coeffs(1.0, 0.0)
    with pytest.raises(qw.QwError):
        qw.cheb_coeffs(float("nan"), 1e-6)
    with pytest.raises(qw.QwError):
        qw.cheb_coeffs(500.0, 1e-6, kmax=10)


@pytest.mark.parametrize("a,tol", [(8.0, 1e-6), (30.0, 2.0 ** -23), (90.0, 1e-10)])
def test_library_cf_against_remez(oracle_mod, a, tol):
    """The library's CF coefficients (qw_cheb_coeffs with QW_CF): the cos and
    sin parts of sum_m (-i)^m alpha_m T_m are within 0.1 % of the minimax error
    of their degree found by the oracle's Remez exchange, and the reported
    bound |lambda_c| + |lambda_s| equals the sum of the two minimax errors."""
    alpha, bound = qw.cheb_coeffs(a, tol, "cf")
    K = len(alpha) - 1
    m = np.arange(K + 1)
    cos_c = np.where(m % 2 == 0, alpha * (-1.0) ** (m // 2), 0.0)
    sin_c = np.where(m % 2 == 1, alpha * (-1.0) ** ((m - 1) // 2), 0.0)
    x = np.cos(np.linspace(0, np.pi, 40001))
    kc = K if K % 2 == 0 else K - 1
    ks = K if K % 2 == 1 else K - 1
    _, Ec = oracle_mod.remez_parity(lambda t: np.cos(a * t), 0, kc)
    _, Es = oracle_mod.remez_parity(lambda t: np.sin(a * t), 1, ks)
    ec = np.max(np.abs(np.polynomial.chebyshev.chebval(x, cos_c) - np.cos(a * x)))
    es = np.max(np.abs(np.polynomial.chebyshev.chebval(x, sin_c) - np.sin(a * x)))
    assert ec <= Ec * 1.001 + 1e-15 and es <= Es * 1.001 + 1e-15
    assert abs(bound / (Ec + Es) - 1) < 1e-3
    assert bound <= tol


def test_struct_layouts_match_the_header(tmp_path):
    """Every struct of include/qwexp.h has the size and field offsets the
    ctypes binding assumes (compiled with the host C compiler)."""
    import ctypes
    import subprocess
    import paper_2608_12058_amd as qw
    pairs = {"qw_info": qw.QwInfo, "qw_cfet_info": qw.CfetInfo, "qw_batch_item": qw.BatchItem,
             "qw_batch_info": qw.BatchInfo, "qw_batch_sched": qw.BatchSched, "qw_grad_info": qw.GradInfo}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "qwexp.h"', "int main(void) {"]
    for cname, cls in pairs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for field, _ in cls._fields_:
            if field == "reserved":
                continue
            lines.append(f'printf("{cname} {field} %zu\\n", offsetof({cname}, {field}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = str(tmp_path / "layout")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    subprocess.check_call(["gcc", "-I", os.path.join(root, "include"), str(src), "-o", exe])
    for line in subprocess.check_output([exe]).decode().splitlines():
        cname, field, val = line.split()
        cls = pairs[cname]
        got = ctypes.sizeof(cls) if field == "size" else getattr(cls, field).offset
        assert got == int(val), (cname, field, got, val)
