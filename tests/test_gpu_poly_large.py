"""GPU parity at 29 to 32 qubits against the oracle itself, on sampled outputs:
a degree-4 caller polynomial p(H~) psi (Chebyshev basis by the Clenshaw
recurrence, monomial basis by Horner's rule) of a seeded product state, run
through the same per-orientation plans and pass kernels as exp(-itH) psi at
these sizes (complex64: contiguous bits in the middle add pass, the diagonal
rebuilt from (h, J) in both end passes; 31-32 qubits with no stored diagonal).
A degree-K polynomial reaches only the indices within Hamming distance K of an
output, so the oracle evaluates each sampled output on that ball
(``poly_amps_local``).  Shift and radius are given, the radius being the bound
sum |h| + sum |J| + |shift| + n |gamma|, so the spectrum of H~ lies in [-1, 1]."""
import numpy as np
import pytest

import synth

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


@pytest.mark.parametrize("n,prec,basis,gamma,seed", [(29, 64, "cheb", 0.8, 41), (30, 64, "mono", -0.6, 42),
                                                     (31, 64, "mono", 1.1, 43), (32, 64, "cheb", 0.9, 44),
                                                     (29, 128, "cheb", -0.7, 45)])
def test_degree4_sampled_outputs_vs_oracle(env, oracle_mod, n, prec, basis, gamma, seed):
    torch, qw = env
    h, J = synth.sk_instance(n, seed)
    fac = synth.product_state_factors(n, seed + 1000)
    rng = np.random.default_rng(seed)
    coef = rng.standard_normal(5) + 1j * rng.standard_normal(5)
    shift = 0.2
    radius = float(np.abs(h).sum() + np.abs(J).sum() + abs(shift) + n * abs(gamma))
    idx = np.concatenate([[0, (1 << n) - 1], rng.integers(0, 1 << n, 22)])
    print(f"n={n} prec={prec} basis={basis} gamma={gamma} seed={seed}", flush=True)
    cdt = torch.complex64 if prec == 64 else torch.complex128
    psi = synth.product_state_torch(fac, "cuda", cdt)
    torch.cuda.empty_cache()
    y, info = qw.poly_action(psi, coef, gamma, basis=basis, h=h, J=J, shift=shift, radius=radius, out=psi)
    got = y[torch.as_tensor(idx, device="cuda")].cpu().numpy().astype(np.complex128)
    del y, psi
    torch.cuda.empty_cache()
    assert info["passes"] == 3
    if prec == 64:
        assert info["otf_mask"] == 0b101
    ref = oracle_mod.poly_amps_local(n, h, J, gamma, shift, radius, coef, basis, fac, idx)
    err = rel(got, ref)
    print(f"  sampled relative error {err:.2e}", flush=True)
    assert err <= (C64_TOL if prec == 64 else C128_TOL)
