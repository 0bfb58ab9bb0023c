"""GPU parity of qw_anneal_cfet4_{c64,c128} (fourth-order commutator-free
Magnus anneal, sec. III.B) against the oracle's integrator run on the same
steps with the same per-exponential truncation tolerances, and the adaptive
step control against a DOP853 reference on small instances.

Tolerances: complex128 <= 1e-11 relative L2 (many exponentials, each at
<= 1e-12), complex64 <= 1e-5.  The adaptive runs must meet their own target
(measured error <= tol)."""
import numpy as np
import pytest

import synth
from device_energies import energies_torch
from test_oracle_cfet import exact

pytestmark = pytest.mark.gpu

C64_TOL = 1e-5
C128_TOL = 1e-11
LINEAR = ([0.0, 1.0], [1.0, -1.0])
QUARTIC = ([0.3, 1.0, 0.5, -0.8, 0.4], [1.0, -1.0, 0.0, 0.2])


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2608_12058_amd as qw
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    qw.lib()
    return torch, qw


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _tols(steps, T, tol, prec, adaptive):
    share = 0.25 if adaptive else 0.5
    floor = 2.0 ** -26 if prec == 64 else 1e-15
    return [max(floor, share * tol * hs / T) for hs in steps]


def _run(env, n, psi_np, h, J, sched, T, prec, steps, tol):
    torch, qw = env
    cdt = torch.complex64 if prec == 64 else torch.complex128
    psi = torch.as_tensor(psi_np).to(cdt).cuda()
    y, info, hs = qw.anneal_cfet4(psi, h, J, sched[0], sched[1], T, steps=steps, tol=tol)
    torch.cuda.synchronize()
    return y.cpu().numpy().astype(np.complex128), info, hs


@pytest.mark.parametrize("prec", [64, 128])
@pytest.mark.parametrize("n,seed,sched", [(6, 1, LINEAR), (16, 2, QUARTIC), (23, 3, LINEAR)])
def test_uniform_steps_vs_oracle(env, oracle_mod, n, seed, sched, prec):
    T, S = 2.0, 6
    h, J = synth.sk_instance(n, 1200 + seed)
    E = oracle_mod.energies(n, h, J)
    psi = synth.random_state(n, 1300 + seed)
    tol = 1e-12 if prec == 128 else 1e-7
    y, info, hs = _run(env, n, psi, h, J, sched, T, prec, S, tol)
    assert info["steps"] == S and info["exponentials"] == 2 * S and len(hs) == S
    assert abs(sum(hs) - T) < 1e-12
    ref = oracle_mod.anneal_cfet4(n, E, sched[0], sched[1], T, hs, psi, _tols(hs, T, 1e-12, 128, False))
    assert rel(y, ref) <= (C64_TOL if prec == 64 else C128_TOL), info


@pytest.mark.parametrize("sched", [LINEAR, QUARTIC])
def test_adaptive_steps_replayed_by_oracle(env, oracle_mod, sched):
    n, T, tol = 8, 3.0, 1e-6
    h, J = synth.sk_instance(n, 1400)
    E = oracle_mod.energies(n, h, J)
    psi = synth.plus_state(n)
    y, info, hs = _run(env, n, psi, h, J, sched, T, 128, 0, tol)
    assert info["steps"] == len(hs) > 1 and abs(sum(hs) - T) < 1e-9
    assert info["h_min"] == min(hs) and info["h_max"] == max(hs)
    ref = oracle_mod.anneal_cfet4(n, E, sched[0], sched[1], T, hs, psi, _tols(hs, T, tol, 128, True))
    assert rel(y, ref) <= C128_TOL


@pytest.mark.parametrize("tol", [1e-3, 1e-5, 1e-7])
def test_adaptive_meets_tolerance(env, oracle_mod, tol):
    """8-qubit SK, linear anneal over T = 3 (the setting of Fig. 6): the error
    against DOP853 at 1e-13 stays below the requested tolerance."""
    n, T = 8, 3.0
    h, J = synth.sk_instance(n, 1500)
    E = oracle_mod.energies(n, h, J)
    psi = synth.plus_state(n)
    ref = exact(n, E, LINEAR[0], LINEAR[1], T, 0.0, T, psi, oracle_mod)
    y, info, hs = _run(env, n, psi, h, J, LINEAR, T, 128, 0, tol)
    assert rel(y, ref) <= tol, (info, rel(y, ref))
    assert info["err_bound"] <= 0.5 * tol * (1 + 1e-9)


def test_constant_schedule_single_step(env, oracle_mod):
    """A constant schedule has a zero error term: one adaptive step, equal to
    the plain action exp(-iT (a H_P + b F)) within the requested tolerance (its
    two exponentials are each truncated at tol / 4)."""
    torch, qw = env
    n, T, tol = 18, 1.5, 1e-10
    h, J = synth.sk_instance(n, 1600)
    psi = synth.random_state(n, 1601)
    y, info, hs = _run(env, n, psi, h, J, ([0.6], [0.9]), T, 128, 0, tol)
    assert info["steps"] == 1 and hs[0] == T
    E = oracle_mod.energies(n, h, J)
    ref = oracle_mod.expm_action(n, 0.6 * E, 0.9, T, psi, 1e-13)
    assert rel(y, ref) <= tol


@pytest.mark.parametrize("n,prec", [(26, 64), (26, 128), (29, 64)])
def test_constant_schedule_large_n_vs_caller_diagonal(env, n, prec):
    """A constant schedule at sizes where the action rebuilds the diagonal from
    (h, J) in its end passes (26 qubits in both precisions, 29 in complex64): each
    of the anneal's exponentials scales the prepared energy tables by A, and the
    rebuilt diagonal must follow that scale.  One adaptive step, against one
    plain action with the caller diagonal a E (energies formed on the device from
    their definition; its passes read the stored diagonal), whole vector."""
    torch, qw = env
    T, a, b = 1.2, 0.6, 0.9
    h, J = synth.sk_instance(n, 1800 + n)
    fac = synth.product_state_factors(n, 1900 + n)
    cdt, rdt = (torch.complex64, torch.float32) if prec == 64 else (torch.complex128, torch.float64)
    tol = 1e-7 if prec == 64 else 1e-10
    psi = synth.product_state_torch(fac, "cuda", cdt)
    y, info, hs = qw.anneal_cfet4(psi, h, J, [a], [b], T, steps=0, tol=tol)
    assert info["steps"] == 1 and hs[0] == T
    E = energies_torch(torch, n, a * np.asarray(h), a * np.asarray(J), rdt)
    ref, iref = qw.expm_action(psi, b, T, diag=E, tol=2.0 ** -23 if prec == 64 else 1e-13)
    del psi, E
    assert iref["otf_mask"] == 0
    d = y.to(torch.complex128) - ref.to(torch.complex128)
    err = (torch.linalg.vector_norm(d) / torch.linalg.vector_norm(ref.to(torch.complex128))).item()
    print(f"n={n} c{prec}: anneal (rebuilt diagonal) vs caller diagonal {err:.2e}", flush=True)
    del d, y, ref
    torch.cuda.empty_cache()
    assert err <= (C64_TOL if prec == 64 else tol)


def test_c64_matches_c128_at_24_qubits(env):
    torch, qw = env
    n, T = 24, 2.0
    h, J = synth.sk_instance(n, 1700)
    psi = synth.plus_state_torch(n, "cuda", torch.complex128)
    y128, i128, h128 = qw.anneal_cfet4(psi, h, J, LINEAR[0], LINEAR[1], T, steps=8, tol=1e-7)
    y64, i64, h64 = qw.anneal_cfet4(psi.to(torch.complex64), h, J, LINEAR[0], LINEAR[1], T, steps=8, tol=1e-7)
    err = (torch.linalg.vector_norm(y64.to(torch.complex128) - y128) / torch.linalg.vector_norm(y128)).item()
    assert err < C64_TOL
    nrm = torch.linalg.vector_norm(y128).item()
    assert abs(nrm - 1.0) < 1e-7   # the requested truncation budget
    del y128, y64, psi
    torch.cuda.empty_cache()


def test_rejects_bad_arguments(env):
    torch, qw = env
    h, J = synth.sk_instance(6, 1)
    psi = torch.zeros(64, dtype=torch.complex128, device="cuda")
    psi[0] = 1
    with pytest.raises(qw.QwError):
        qw.anneal_cfet4(psi, h, J, [0.0, 1.0], [1.0, -1.0], -1.0)
    with pytest.raises(qw.QwError):
        qw.anneal_cfet4(psi, h, J, [0.0, 1.0], [1.0, -1.0], 1.0, tol=0.0)
    with pytest.raises(qw.QwError):
        qw.anneal_cfet4(psi, h, J, [0.0, 1.0], [1.0, -1.0], 1.0, steps=-3)
