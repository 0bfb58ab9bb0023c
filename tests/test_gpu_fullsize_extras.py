"""Full-size (28-qubit) checks of the caller-polynomial and anneal entry points,
in the launch configuration of the 28-qubit workload, on sampled amplitudes the
oracle computes one by one from closed forms:

* p(H~) psi with gamma = 0 is p(d~(z)) psi(z) (both bases);
* an anneal with A = 0 (all H(t) proportional to sum_j X_j, so they commute) is
  the product of single-qubit rotations by the angle integral of B;
* an anneal with B = 0 is exp(-i E(z) integral of A).
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

N28 = 28
C64_TOL = 1e-5


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2608_12058_amd as qw
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    qw.lib()
    return torch, qw


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _sample(seed, count=1024):
    rng = np.random.default_rng(seed)
    return np.concatenate([[0, (1 << N28) - 1], rng.integers(0, 1 << N28, count - 2)])


def _product_amps(factors, idx):
    amp = np.ones(len(idx), dtype=np.complex128)
    for j in range(factors.shape[0]):
        amp *= factors[j, (np.asarray(idx, dtype=np.int64) >> j) & 1]
    return amp


@pytest.mark.parametrize("basis", ["cheb", "mono"])
def test_poly_gamma0_sampled(env, oracle_mod, basis):
    torch, qw = env
    h, J = synth.sk_instance(N28, 0)
    f = synth.product_state_factors(N28, 61)
    psi = synth.product_state_torch(f, "cuda", torch.complex64)
    a = np.random.default_rng(62).standard_normal(24) * 0.75 ** np.arange(24)
    y, info = qw.poly_action(psi, a, 0.0, basis=basis, h=h, J=J)
    idx = _sample(63)
    got = y[torch.as_tensor(idx, device="cuda")].cpu().numpy().astype(np.complex128)
    d = (oracle_mod.energies_at(N28, h, J, idx) - info["shift_c"]) / info["radius_r"]
    ev = np.polynomial.polynomial.polyval if basis == "mono" else np.polynomial.chebyshev.chebval
    assert rel(got, ev(d, a) * _product_amps(f, idx)) <= C64_TOL
    del y, psi
    torch.cuda.empty_cache()


def test_anneal_driver_only_sampled(env, oracle_mod):
    """A = 0, B = 1 - s over T = 2: one exact step (the error term vanishes),
    rotation angle int B dt = 1."""
    torch, qw = env
    h, J = synth.sk_instance(N28, 0)
    f = synth.product_state_factors(N28, 64)
    psi = synth.product_state_torch(f, "cuda", torch.complex64)
    y, info, steps = qw.anneal_cfet4(psi, h, J, [0.0], [1.0, -1.0], 2.0, tol=1e-6)
    assert info["steps"] == 1
    idx = _sample(65)
    got = y[torch.as_tensor(idx, device="cuda")].cpu().numpy().astype(np.complex128)
    ref = oracle_mod.closed_form_hp0_product_amps(f, 1.0, 1.0, idx)
    assert rel(got, ref) <= C64_TOL
    del y, psi
    torch.cuda.empty_cache()


def test_anneal_problem_only_sampled(env, oracle_mod):
    """B = 0, A = s over T = 2 on |+>: exp(-i E(z) int A dt), int A dt = 1."""
    torch, qw = env
    h, J = synth.sk_instance(N28, 0)
    psi = synth.plus_state_torch(N28, "cuda", torch.complex64)
    y, info, steps = qw.anneal_cfet4(psi, h, J, [0.0, 1.0], [0.0], 2.0, tol=1e-6)
    assert info["steps"] == 1
    idx = _sample(66, 512)
    got = y[torch.as_tensor(idx, device="cuda")].cpu().numpy().astype(np.complex128)
    amp = np.full(len(idx), 2.0 ** (-N28 / 2), dtype=np.complex128)
    ref = oracle_mod.closed_form_gamma0_amps(N28, h, J, 1.0, amp, idx)
    assert rel(got, ref) <= C64_TOL
    del y, psi
    torch.cuda.empty_cache()
