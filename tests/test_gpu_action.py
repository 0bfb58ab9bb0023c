"""GPU parity of qw_expm_action_{c64,c128} against the CPU oracle.

Element-by-element comparisons (relative L2 over the whole vector) at sizes the
oracle finishes in seconds, spanning the on-chip path (n <= 13) and every tile
shape of the multi-pass path: 2^12-amplitude tiles with 1024 threads (n <= 20 in
complex64, <= 21 in complex128), 2^13 tiles with 1024 threads (n = 21) and 512
threads (n = 22), 2^14 tiles (n = 23, 24), the split shape of three orientations
(n = 25..28: 2^12 tiles on the contiguous one); at the full 28-qubit
workload, properties that hold at any size, closed forms evaluated one
sampled amplitude at a time, and 4096 sampled amplitudes of the oracle's result
for the benchmark workload itself (tests/golden/action_n28_bench.json).  The
split shape is compared with the oracle over the whole vector at 25-27 qubits,
with negative gamma and negative t among the cases.

Tolerances: complex128 <= 1e-12 against the oracle run at the same truncation
tolerance (identical degree K), complex64 <= 1e-5 against the oracle at 1e-13.
"""
import json
import os

import numpy as np
import pytest

import synth
from device_energies import energies_torch

pytestmark = pytest.mark.gpu

C64_TOL = 1e-5
C128_TOL = 1e-12


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2608_12058_amd as qw
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    qw.lib()
    return torch, qw


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _run(env, n, psi_np, gamma, t, tol, prec, method="cheb", diag_np=None, h=None, J=None, inplace=False):
    torch, qw = env
    cdt = torch.complex64 if prec == 64 else torch.complex128
    rdt = torch.float32 if prec == 64 else torch.float64
    psi = torch.as_tensor(psi_np).to(cdt).cuda()
    diag = torch.as_tensor(diag_np).to(rdt).cuda() if diag_np is not None else None
    out = psi if inplace else None
    y, info = qw.expm_action(psi, gamma, t, diag=diag, h=h, J=J, tol=tol, method=method, out=out)
    torch.cuda.synchronize()
    return y.cpu().numpy().astype(np.complex128), info


def test_config1_plain_c128_vs_eigh(env, oracle_mod):
    """n = 10, complex128, SK seed 0, gamma = 1, t = 1, |+>, tol 1e-12."""
    n = 10
    h, J = synth.sk_instance(n, 0)
    E = oracle_mod.energies(n, h, J)
    psi = synth.plus_state(n)
    y0 = oracle_mod.expm_action_dense(n, E, 1.0, 1.0, psi)
    y1 = oracle_mod.expm_action(n, E, 1.0, 1.0, psi, 1e-12)
    for kw in (dict(h=h, J=J), dict(diag_np=E)):
        y, info = _run(env, n, psi, 1.0, 1.0, 1e-12, 128, **kw)
        assert info["K"] == 48
        assert rel(y, y0) <= C128_TOL
        assert rel(y, y1) <= C128_TOL


CASES = [
    # n, gamma, t, seed
    (1, 0.7, 2.0, 1),
    (2, 1.1, 1.5, 2),
    (5, 0.8, 3.0, 3),
    (12, 1.0, 1.0, 4),
    (13, 0.9, 1.3, 5),
    (14, 1.2, 0.8, 6),
    (17, 0.8, 1.0, 7),
    (20, 1.0, 0.5, 8),
    (21, 0.9, 0.5, 11),
    (22, 0.7, 0.4, 9),
    (23, 1.0, 0.3, 10),
    (24, 0.8, 0.2, 12),
    # negative gamma (complex64 rounds gamma/r towards zero by magnitude) and
    # negative t, on the one-workgroup, narrow and default shapes
    (11, -0.9, 1.2, 13),
    (19, 0.7, -0.9, 14),
    (22, -1.1, -0.3, 15),
]


@pytest.mark.parametrize("n,gamma,t,seed", CASES)
def test_parity_c128(env, oracle_mod, n, gamma, t, seed):
    h, J = synth.sk_instance(n, seed)
    E = oracle_mod.energies(n, h, J)
    psi = synth.random_state(n, seed + 100)
    ref = oracle_mod.expm_action(n, E, gamma, t, psi, 1e-12)
    y, info = _run(env, n, psi, gamma, t, 1e-12, 128, h=h, J=J)
    assert rel(y, ref) <= C128_TOL, info


@pytest.mark.parametrize("n,gamma,t,seed", CASES)
def test_parity_c64(env, oracle_mod, n, gamma, t, seed):
    h, J = synth.sk_instance(n, seed)
    E = oracle_mod.energies(n, h, J)
    psi = synth.random_state(n, seed + 200)
    ref = oracle_mod.expm_action(n, E, gamma, t, psi, 1e-13)
    y, info = _run(env, n, psi, gamma, t, 2.0 ** -23, 64, h=h, J=J)
    assert rel(y, ref) <= C64_TOL, info
    y2, _ = _run(env, n, psi, gamma, t, 2.0 ** -23, 64, diag_np=E)
    assert rel(y2, ref) <= C64_TOL


@pytest.mark.parametrize("prec", [64, 128])
def test_cf_method(env, oracle_mod, prec):
    n = 16
    h, J = synth.sk_instance(n, 31)
    E = oracle_mod.energies(n, h, J)
    psi = synth.plus_state(n)
    tol = 2.0 ** -23 if prec == 64 else 1e-11
    ref = oracle_mod.expm_action(n, E, 0.8, 4.0, psi, 1e-13)
    y, info = _run(env, n, psi, 0.8, 4.0, tol, prec, method="cf", h=h, J=J)
    assert info["method"] == 1
    assert rel(y, ref) <= (C64_TOL if prec == 64 else 2e-11)
    yo = oracle_mod.expm_action(n, E, 0.8, 4.0, psi, tol, method="cf")
    if prec == 128:
        assert rel(y, yo) <= C128_TOL


@pytest.mark.parametrize("prec", [64, 128])
@pytest.mark.parametrize("n", [11, 19])
def test_in_place(env, oracle_mod, prec, n):
    h, J = synth.sk_instance(n, 41)
    E = oracle_mod.energies(n, h, J)
    psi = synth.random_state(n, 41)
    ref = oracle_mod.expm_action(n, E, 1.0, 0.7, psi, 1e-13)
    y, _ = _run(env, n, psi, 1.0, 0.7, 1e-12 if prec == 128 else 2.0 ** -23, prec, h=h, J=J, inplace=True)
    assert rel(y, ref) <= (C64_TOL if prec == 64 else C128_TOL)


@pytest.mark.parametrize("prec,n", [(64, 16), (128, 16), (128, 22), (64, 25)])
@pytest.mark.parametrize("a", [1e-4, 1e-2, 0.3])
def test_low_degree_in_place(env, oracle_mod, prec, n, a):
    """Degrees 1..10, where every pass of the call belongs to the first term or
    two (whose b_{k+1} is psi scaled by c_K as the passes load it), with the
    output written over the input: two and three orientations."""
    torch, qw = env
    h, J = synth.sk_instance(n, 50 + n)
    E = oracle_mod.energies(n, h, J)
    _, r = oracle_mod.spectral_shift_radius(E, n, 0.8)
    psi = synth.random_state(n, 60 + n)
    tol = 1e-6 if prec == 64 else 1e-12
    y, info = _run(env, n, psi, 0.8, a / r, tol, prec, h=h, J=J, inplace=True)
    assert 1 <= info["K"] <= 10 and info["passes"] >= 2, info
    ref = oracle_mod.expm_action(n, E, 0.8, a / r, psi, 1e-13)
    assert rel(y, ref) <= (C64_TOL if prec == 64 else C128_TOL), info


@pytest.mark.parametrize("prec", [64, 128])
def test_closed_forms(env, oracle_mod, prec):
    tol = 2.0 ** -23 if prec == 64 else 1e-12
    bar = C64_TOL if prec == 64 else C128_TOL
    n = 18
    h, J = synth.sk_instance(n, 51)
    E = oracle_mod.energies(n, h, J)
    psi = synth.random_state(n, 51)
    y, _ = _run(env, n, psi, 0.0, 2.5, tol, prec, h=h, J=J)
    assert rel(y, oracle_mod.closed_form_gamma0(E, 2.5, psi)) <= bar
    z = np.zeros(n)
    zJ = np.zeros(n * (n - 1) // 2)
    y, _ = _run(env, n, psi, 1.3, 2.2, tol, prec, h=z, J=zJ)
    assert rel(y, oracle_mod.closed_form_hp0(n, 1.3, 2.2, psi)) <= bar


@pytest.mark.parametrize("prec", [64, 128])
def test_degenerate_cases(env, prec):
    n = 15
    psi = synth.random_state(n, 61)
    h, J = synth.sk_instance(n, 61)
    # t = 0: a = 0, K = 0, the identity
    y, info = _run(env, n, psi, 1.0, 0.0, 1e-10, prec, h=h, J=J)
    assert info["K"] == 0
    assert rel(y, psi) <= (1e-7 if prec == 64 else 1e-15)
    # H = 0 (no couplings, gamma = 0): zero bound, output = psi
    y, info = _run(env, n, psi, 0.0, 3.0, 1e-10, prec, h=np.zeros(n), J=np.zeros(n * (n - 1) // 2))
    assert info["radius_r"] == 0.0
    assert rel(y, psi) <= (1e-7 if prec == 64 else 1e-15)
    # constant diagonal only: a pure phase exp(-i t c)
    Ec = np.full(1 << n, 0.37)
    y, info = _run(env, n, psi, 0.0, 3.0, 1e-10, prec, diag_np=Ec)
    assert rel(y, np.exp(-1j * 3.0 * 0.37) * psi) <= (1e-6 if prec == 64 else 1e-14)


@pytest.mark.parametrize("prec", [64, 128])
@pytest.mark.parametrize("bad", [float("nan"), float("inf")])
def test_non_finite_diagonal_is_rejected(env, prec, bad):
    """A caller diagonal with one NaN or infinite energy (n = 16, on the
    multi-pass path) is refused with QW_EINVAL before any pass runs."""
    torch, qw = env
    n = 16
    E = np.linspace(-1.0, 1.0, 1 << n)
    E[12345] = bad
    with pytest.raises(qw.QwError) as ei:
        _run(env, n, synth.plus_state(n), 1.0, 1.0, 1e-8, prec, diag_np=E)
    assert ei.value.status == qw.QW_EINVAL


def test_spectral_bound_matches_oracle(env, oracle_mod):
    torch, qw = env
    n = 20
    h, J = synth.sk_instance(n, 71)
    E = oracle_mod.energies(n, h, J)
    c_ref, r_ref = oracle_mod.spectral_shift_radius(E, n, 0.9)
    c, r = qw.spectral_bound(n, 0.9, h=h, J=J, precision=128)
    assert abs(c - c_ref) < 1e-12 and abs(r - r_ref) < 1e-12
    c, r = qw.spectral_bound(n, 0.9, diag=torch.as_tensor(E).cuda(), precision=128)
    assert abs(c - c_ref) < 1e-12 and abs(r - r_ref) < 1e-12


def test_deterministic(env):
    n = 21
    h, J = synth.sk_instance(n, 81)
    psi = synth.plus_state(n)
    y1, _ = _run(env, n, psi, 1.0, 1.0, 2.0 ** -23, 64, h=h, J=J)
    y2, _ = _run(env, n, psi, 1.0, 1.0, 2.0 ** -23, 64, h=h, J=J)
    assert np.array_equal(y1, y2)


# ------------------------------------------------------------ full size (28 qubits)

N28 = 28


def test_n28_time_reversal_and_norm(env):
    """SK seed 0, gamma = 1, t = 5, |+> (the benchmark workload, same launch
    configuration): U(-t) U(t) psi = psi and the norm is conserved."""
    torch, qw = env
    h, J = synth.sk_instance(N28, 0)
    psi = synth.plus_state_torch(N28, "cuda", torch.complex64)
    y, info = qw.expm_action(psi, 1.0, 5.0, h=h, J=J, tol=2.0 ** -23)
    assert info["passes"] == 3
    nrm = torch.linalg.vector_norm(y.to(torch.complex128)).item()
    assert abs(nrm - 1.0) < 1e-5
    back, _ = qw.expm_action(y, 1.0, -5.0, h=h, J=J, tol=2.0 ** -23)
    err = (torch.linalg.vector_norm((back - psi).to(torch.complex128)) /
           torch.linalg.vector_norm(psi.to(torch.complex128))).item()
    assert err < 2 * C64_TOL
    del y, back
    torch.cuda.empty_cache()


def test_n28_c64_matches_c128(env):
    torch, qw = env
    h, J = synth.sk_instance(N28, 0)
    psi = synth.plus_state_torch(N28, "cuda", torch.complex128)
    y128, _ = qw.expm_action(psi, 1.0, 5.0, h=h, J=J, tol=1e-12)
    y64, _ = qw.expm_action(psi.to(torch.complex64), 1.0, 5.0, h=h, J=J, tol=2.0 ** -23)
    err = (torch.linalg.vector_norm(y64.to(torch.complex128) - y128) / torch.linalg.vector_norm(y128)).item()
    assert err < C64_TOL
    del y128, y64, psi
    torch.cuda.empty_cache()


@pytest.mark.parametrize("n", [25, 26, 27])
def test_split_shape_c64_matches_c128(env, n):
    """25-27 qubits run complex64 on the split tile shape (contiguous orientation
    on 2^12 tiles, 12 + groups of at most 8 bits) and complex128 on its default
    2^12 tiles (12 + groups of at most 9): a random state through both."""
    torch, qw = env
    h, J = synth.sk_instance(n, 300 + n)
    psi = torch.as_tensor(synth.random_state(n, 400 + n)).cuda()
    y128, i128 = qw.expm_action(psi, 0.9, 0.3, h=h, J=J, tol=1e-12)
    y64, i64 = qw.expm_action(psi.to(torch.complex64), 0.9, 0.3, h=h, J=J, tol=2.0 ** -23)
    assert i64["passes"] == 3
    err = (torch.linalg.vector_norm(y64.to(torch.complex128) - y128) / torch.linalg.vector_norm(y128)).item()
    assert err < C64_TOL
    del y128, y64, psi
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prec", [64, 128])
def test_n28_sampled_closed_forms(env, oracle_mod, prec):
    """H_P = 0 on a random product state, and gamma = 0 on |+>, checked at 4096
    sampled amplitudes computed one by one by the oracle."""
    torch, qw = env
    cdt = torch.complex64 if prec == 64 else torch.complex128
    tol = 2.0 ** -23 if prec == 64 else 1e-12
    rng = np.random.default_rng(5)
    idx = np.concatenate([[0, (1 << N28) - 1], rng.integers(0, 1 << N28, 4094)])
    f = synth.product_state_factors(N28, 17)
    psi = synth.product_state_torch(f, "cuda", cdt)
    zh, zJ = np.zeros(N28), np.zeros(N28 * (N28 - 1) // 2)
    y, _ = qw.expm_action(psi, 0.9, 2.0, h=zh, J=zJ, tol=tol)
    got = y[torch.as_tensor(idx, device="cuda")].cpu().numpy().astype(np.complex128)
    ref = oracle_mod.closed_form_hp0_product_amps(f, 0.9, 2.0, idx)
    assert rel(got, ref) <= (C64_TOL if prec == 64 else C128_TOL)
    del y, psi
    h, J = synth.sk_instance(N28, 0)
    psi = synth.plus_state_torch(N28, "cuda", cdt)
    y, _ = qw.expm_action(psi, 0.0, 5.0, h=h, J=J, tol=tol)
    got = y[torch.as_tensor(idx[:512], device="cuda")].cpu().numpy().astype(np.complex128)
    amp = np.full(512, 1.0 / np.sqrt(1 << N28), dtype=np.complex128)
    ref = oracle_mod.closed_form_gamma0_amps(N28, h, J, 5.0, amp, idx[:512])
    assert rel(got, ref) <= (C64_TOL if prec == 64 else C128_TOL)
    del y, psi
    torch.cuda.empty_cache()


# ------------------------------------------ split shape (25-28 qubits) vs the oracle

SPLIT_CASES = [
    # n, gamma, t, seed: K = 85, 70, 69, 75 at tol 1e-13
    (25, 0.9, 1.0, 525),
    (26, -0.7, 0.8, 526),
    (27, 1.1, -0.6, 527),
    (25, -1.2, -0.7, 535),
]


@pytest.mark.parametrize("n,gamma,t,seed", SPLIT_CASES)
def test_split_shape_vs_oracle(env, oracle_mod, n, gamma, t, seed):
    """The kernels of the benchmark's launch configuration (complex64: contiguous
    orientation on 2^12 tiles with 1024 threads, strided add passes on 2^13 tiles
    with 1024 threads, strided fused passes with 512; from 26 qubits the top
    orientation's fused pass rebuilds the diagonal from h and J) on a generic SK
    instance and a random state, compared over the whole vector with the oracle
    at tol 1e-13: complex64 from (h, J) and from a stored diagonal <= 1e-5;
    complex128 at the same tolerance (same degree) <= 1e-12."""
    torch, qw = env
    h, J = synth.sk_instance(n, seed)
    E = oracle_mod.energies(n, h, J)
    psi = synth.random_state(n, seed + 1000)
    oinfo = {}
    ref = oracle_mod.expm_action(n, E, gamma, t, psi, 1e-13, info=oinfo)
    assert oinfo["K"] >= 50
    y, info = _run(env, n, psi, gamma, t, 2.0 ** -23, 64, h=h, J=J)
    assert info["passes"] == 3
    e64 = rel(y, ref)
    y, _ = _run(env, n, psi, gamma, t, 2.0 ** -23, 64, diag_np=E)
    e64d = rel(y, ref)
    y, info128 = _run(env, n, psi, gamma, t, 1e-13, 128, h=h, J=J)
    e128 = rel(y, ref)
    print(f"n={n} gamma={gamma} t={t}: K {oinfo['K']} / c64 K {info['K']}: c64 (h, J) {e64:.2e}, "
          f"c64 diag {e64d:.2e}, c128 {e128:.2e}", flush=True)
    assert info128["K"] == oinfo["K"]
    assert e64 <= C64_TOL and e64d <= C64_TOL
    assert e128 <= C128_TOL
    del y
    torch.cuda.empty_cache()


GOLDEN28 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "action_n28_bench.json")


@pytest.mark.parametrize("prec", [64, 128])
def test_n28_bench_workload_vs_oracle_golden(env, prec):
    """The benchmark workload (SK seed 0, gamma = 1, t = 5, |+>, 28 qubits) in
    the benchmark's launch configuration (caller output and workspace) against
    4096 amplitudes and the norm of the oracle's result, written by
    tests/golden/make_bench_golden.py: complex64 at 2^-23 against the oracle at
    1e-13 (<= 1e-5 over the samples); complex128 at 1e-12 against the oracle at
    1e-12, same degree (<= 1e-12)."""
    torch, qw = env
    with open(GOLDEN28) as f:
        gold = json.load(f)
    n = gold["n"]
    assert (n, gold["gamma"], gold["t"], gold["seed"]) == (N28, 1.0, 5.0, 0)
    h, J = synth.sk_instance(n, 0)
    cdt = torch.complex64 if prec == 64 else torch.complex128
    tol = 2.0 ** -23 if prec == 64 else 1e-12
    run = gold["runs"]["1e-13" if prec == 64 else "1e-12"]
    psi = synth.plus_state_torch(n, "cuda", cdt)
    out = torch.empty_like(psi)
    ws = qw.Workspace.for_problem(n, prec)
    y, info = qw.expm_action(psi, 1.0, 5.0, h=h, J=J, tol=tol, out=out, workspace=ws)
    if prec == 128:
        assert info["K"] == run["K"]
    idx = torch.as_tensor(np.asarray(gold["idx"], dtype=np.int64), device="cuda")
    got = y[idx].cpu().numpy().astype(np.complex128)
    ref = np.asarray(run["re"]) + 1j * np.asarray(run["im"])
    err = rel(got, ref)
    nrm = torch.linalg.vector_norm(y.to(torch.complex128)).item()
    print(f"n28 bench workload c{prec}: K {info['K']} (oracle {run['K']}), sampled rel err {err:.2e}, "
          f"norm {nrm:.12f} (oracle {run['norm']:.12f})", flush=True)
    assert err <= (C64_TOL if prec == 64 else C128_TOL)
    assert abs(nrm - run["norm"]) <= (C64_TOL if prec == 64 else C128_TOL)
    del y, out, ws, psi
    torch.cuda.empty_cache()


# ---------------------------------------- complex64 at 29 and 30 qubits

@pytest.mark.parametrize("n,gamma,t,seed", [(29, 0.9, 0.4, 629), (30, -0.8, -0.3, 630)])
def test_n29_n30_c64_matches_c128(env, n, gamma, t, seed):
    """29 and 30 qubits, where the oracle is too slow for a test: complex64 with
    the contiguous 12 bits in the middle orientation and the diagonal rebuilt in
    both end passes (9 + 12 + 8 and 10 + 12 + 8 bits) against complex128 on 2^12
    tiles (12 + 9 + 8 and 12 + 9 + 9 bits, its end passes rebuilding the diagonal
    in double; the stored diagonal is checked against the rebuilt one by
    test_n29_caller_diagonal_c64_matches_tables), a
    generic SK instance and a seeded product state (not an eigenvector), over the
    whole vector on the GPU: <= 1e-5; both norms stay 1 (the 30-qubit case with
    negative gamma and t)."""
    torch, qw = env
    h, J = synth.sk_instance(n, seed)
    fac = synth.product_state_factors(n, seed)
    x = synth.product_state_torch(fac, "cuda", torch.complex128)
    y128, i128 = qw.expm_action(x, gamma, t, h=h, J=J, tol=1e-12, out=x)
    x = synth.product_state_torch(fac, "cuda", torch.complex64)
    y64, i64 = qw.expm_action(x, gamma, t, h=h, J=J, tol=2.0 ** -23, out=x)
    del x
    assert i64["passes"] == 3 and i128["passes"] == 3 and i64["otf_mask"] == 0b101
    n128 = torch.linalg.vector_norm(y128).item()
    n64 = torch.linalg.vector_norm(y64.to(torch.complex128)).item()
    d = y64.to(torch.complex128)
    d -= y128
    err = torch.linalg.vector_norm(d).item() / n128
    print(f"n={n} gamma={gamma} t={t}: K c64 {i64['K']} c128 {i128['K']}: c64 vs c128 {err:.2e}, "
          f"norms {n64:.9f} {n128:.13f}", flush=True)
    del d, y64, y128
    torch.cuda.empty_cache()
    assert err <= C64_TOL
    assert abs(n64 - 1.0) <= C64_TOL and abs(n128 - 1.0) <= 1e-11


def test_n29_caller_diagonal_c64_matches_tables(env):
    """29 qubits, complex64 with a caller diagonal (float32 energies formed on the
    device from their definition): the end passes read the stored normalised
    diagonal instead of rebuilding it from (h, J).  Against the call from (h, J)
    over the whole vector on a seeded product state: <= 1e-5."""
    torch, qw = env
    n = 29
    h, J = synth.sk_instance(n, 731)
    fac = synth.product_state_factors(n, 732)
    E = energies_torch(torch, n, h, J, torch.float32)
    x = synth.product_state_torch(fac, "cuda", torch.complex64)
    y_tab, i_tab = qw.expm_action(x, 0.7, 0.35, h=h, J=J)
    y_dia, i_dia = qw.expm_action(x, 0.7, 0.35, diag=E)
    del x, E
    assert i_tab["passes"] == 3 and i_dia["passes"] == 3
    assert i_tab["otf_mask"] == 0b101 and i_dia["otf_mask"] == 0
    d = y_tab.to(torch.complex128)
    ref = y_dia.to(torch.complex128)
    err = (torch.linalg.vector_norm(d - ref) / torch.linalg.vector_norm(ref)).item()
    print(f"n=29 caller diagonal vs (h, J): K {i_dia['K']} / {i_tab['K']}, {err:.2e}", flush=True)
    del d, ref, y_tab, y_dia
    torch.cuda.empty_cache()
    assert err <= C64_TOL
