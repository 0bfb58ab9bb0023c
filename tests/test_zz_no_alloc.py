"""qw_expm_action_c64_noalloc (no workspace: the library's fixed device
scratch) against qw_expm_action_c64 with a caller workspace: identical results
on two calls in a row, the second on a smaller instance, both within the
complex64 bar of the oracle; sizes beyond the scratch are refused."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2608_12058_amd as qw
    assert torch.cuda.is_available()
    qw.lib()
    return torch, qw


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_noalloc_matches_workspace_entry(env, oracle_mod):
    torch, qw = env
    for n, gamma, t, seed, use_diag in ((20, 0.9, 0.8, 901, False), (16, -1.1, 1.3, 902, True)):
        h, J = synth.sk_instance(n, seed)
        psi_np = synth.random_state(n, seed + 1)
        psi = torch.as_tensor(psi_np).to(torch.complex64).cuda()
        diag = None
        if use_diag:
            diag = torch.as_tensor(oracle_mod.energies(n, h, J)).to(torch.float32).cuda()
        kw = dict(diag=diag) if use_diag else dict(h=h, J=J)
        ref, rinfo = qw.expm_action(psi, gamma, t, tol=2.0 ** -23, **kw)
        out = torch.empty_like(psi)
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        info = qw.expm_action_noalloc(psi, gamma, t, out, tol=2.0 ** -23, **kw)
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == before
        print(f"n={n}: K {info['K']} (workspace entry {rinfo['K']}), passes {info['passes']}", flush=True)
        assert info["K"] == rinfo["K"] and info["passes"] == rinfo["passes"]
        assert torch.equal(out, ref), n
        E = oracle_mod.energies(n, h, J)
        want = oracle_mod.expm_action(n, E, gamma, t, psi.cpu().numpy().astype(np.complex128), 1e-13)
        assert rel(out.cpu().numpy().astype(np.complex128), want) <= 1e-5


def test_noalloc_refuses_sizes_beyond_its_scratch(env):
    torch, qw = env
    n = 21
    h, J = synth.sk_instance(n, 3)
    psi = synth.plus_state_torch(n, "cuda", torch.complex64)
    out = torch.empty_like(psi)
    with pytest.raises(qw.QwError) as e:
        qw.expm_action_noalloc(psi, 1.0, 1.0, out, h=h, J=J)
    assert e.value.status == qw.QW_EINVAL and "1..20" in str(e.value)
