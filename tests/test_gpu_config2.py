"""24-qubit SK workload (seed 0, gamma = 0.8, t = 10, |+>): Chebyshev and CF
coefficients in complex64 at 2^-23 and the complex128 recurrence at 1e-12,
compared at 4096 sampled amplitudes with the oracle's full-vector results
stored in tests/golden/action_n24.json (tests/golden/make_action_golden.py)."""
import json
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def gold():
    with open(os.path.join(HERE, "golden", "action_n24.json")) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2608_12058_amd as qw
    assert torch.cuda.is_available()
    qw.lib()
    return torch, qw


def sampled(env, gold, dtype, tol, method):
    torch, qw = env
    n = gold["n"]
    h, J = synth.sk_instance(n, gold["seed"])
    psi = synth.plus_state_torch(n, "cuda", dtype)
    y, info = qw.expm_action(psi, gold["gamma"], gold["t"], h=h, J=J, tol=tol, method=method)
    idx = torch.as_tensor(np.array(gold["idx"]), device="cuda")
    got = y[idx].cpu().numpy().astype(np.complex128)
    nrm = torch.linalg.vector_norm(y.to(torch.complex128)).item()
    del y, psi
    torch.cuda.empty_cache()
    return got, info, nrm


def ref(gold, key):
    run = gold["runs"][key]
    return np.array(run["re"]) + 1j * np.array(run["im"]), run


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_c128_at_1e12(env, gold):
    import torch
    r, run = ref(gold, "1e-12")
    got, info, nrm = sampled(env, gold, torch.complex128, 1e-12, "cheb")
    assert info["K"] == run["K"]
    assert rel(got, r) <= 1e-12
    assert abs(nrm - run["norm"]) < 1e-12


@pytest.mark.parametrize("method", ["cheb", "cf"])
def test_c64_at_2m23(env, gold, method):
    import torch
    r, run = ref(gold, "1e-13")
    got, info, nrm = sampled(env, gold, torch.complex64, 2.0 ** -23, method)
    assert rel(got, r) <= 1e-5, info
    assert abs(nrm - 1.0) < 1e-5
    if method == "cf":
        _, icheb, _ = sampled(env, gold, torch.complex64, 2.0 ** -23, "cheb")
        assert info["K"] <= icheb["K"]
