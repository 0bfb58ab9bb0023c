"""GPU parity of the batched form (qw_expm_action_batched_c64).

Every instance is compared with the CPU oracle (complex64 bar 1e-5, oracle at
1e-13) where the oracle is fast, and with the single-instance complex64 entry
point, which runs the same kernels with the same coefficients (agreement to
float rounding).  Schedules (one wave or several, graph or eager) must give
the same outputs; repeated calls with other work between them must agree.
"""
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


def mixed_instances():
    spec = [  # n, gamma, t, tol, seed
        (3, 0.7, 2.0, 1e-6, 1), (8, 1.3, 5.0, 1e-6, 2), (12, 0.4, 11.0, 1e-6, 3), (13, 1.9, 0.3, 1e-6, 4),
        (14, 0.9, 3.0, 1e-6, 5), (15, 1.1, 0.0, 1e-6, 6), (16, 0.2, 19.0, 1e-6, 7), (18, 1.6, 1.5, 2.0 ** -23, 8),
        (17, 0.0, 2.0, 1e-6, 9), (20, 0.5, 0.7, 1e-6, 10), (13, 1.0, 4.0, 1e-6, 11), (21, 1.0, 0.4, 1e-6, 12),
        # the widest high-bit group (22 qubits: 9 bits, 128-byte rows), 19 qubits,
        # negative gamma and negative t
        (22, 0.8, 0.5, 1e-6, 13), (19, 1.2, 0.9, 1e-6, 14), (16, -0.9, 1.5, 1e-6, 15), (18, 0.6, -1.1, 1e-6, 16),
    ]
    out = []
    for n, g, t, tol, seed in spec:
        h, J = synth.sk_instance(n, seed)
        out.append(dict(n=n, gamma=g, t=t, tol=tol, h=h, J=J, seed=seed))
    # an instance with H = 0 (zero bound)
    out.append(dict(n=14, gamma=0.0, t=1.0, tol=1e-6, h=np.zeros(14), J=np.zeros(91), seed=99))
    return out


def fill_states(torch, batch, insts):
    for i, ins in enumerate(insts):
        batch.state(i).copy_(torch.as_tensor(synth.random_state(ins["n"], 500 + i)).to(torch.complex64))


def test_batched_vs_oracle_and_single(env, oracle_mod):
    torch, qw = env
    insts = mixed_instances()
    b = qw.Batch(insts)
    fill_states(torch, b, insts)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        info = qw.expm_action_batched(b, stream=stream)
    stream.synchronize()
    assert info["count"] == len(insts)
    for i, ins in enumerate(insts):
        n = ins["n"]
        psi = b.state(i).cpu().numpy().astype(np.complex128)
        got = b.output(i).cpu().numpy().astype(np.complex128)
        E = oracle_mod.energies(n, ins["h"], ins["J"])
        ref = oracle_mod.expm_action(n, E, ins["gamma"], ins["t"], psi, 1e-13)
        assert rel(got, ref) <= 1e-5, (i, n)
        single, _ = qw.expm_action(b.state(i).clone(), ins["gamma"], ins["t"], h=ins["h"], J=ins["J"],
                                   tol=ins["tol"])
        single = single.cpu().numpy().astype(np.complex128)
        assert np.max(np.abs(single - got)) <= 1e-6, (i, n)


@pytest.mark.parametrize("wave,graph,conc", [(0, False, False), (64 << 20, True, False), (1 << 20, True, False),
                                             (1 << 20, False, False), (0, True, True), (1 << 20, False, True)])
def test_schedules_agree(env, wave, graph, conc):
    """Waves, graph or eager launches and the one-workgroup launch on a side
    stream change only the order of independent work: bit-identical outputs."""
    torch, qw = env
    insts = mixed_instances()
    b = qw.Batch(insts)
    fill_states(torch, b, insts)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        qw.expm_action_batched(b, stream=stream)
        ref = b.out_pool.clone()
        b.out_pool.zero_()
        info = qw.expm_action_batched(b, stream=stream, sched=dict(wave_bytes=wave, concurrent=conc),
                                      use_graph=graph)
    stream.synchronize()
    if wave == (1 << 20):
        assert info["waves"] > 1
    assert info["concurrent"] == int(conc)
    assert torch.equal(ref, b.out_pool)


@pytest.mark.parametrize("classes,onchip", [({n: 1 for n in range(14, 21)}, 13),
                                            ({n: 2 for n in range(14, 23)}, 13),
                                            ({13: 1, 14: 1, 15: 1, 16: 1, 21: 2, 22: 2}, 12)])
def test_tile_classes_vs_oracle(env, oracle_mod, classes, onchip):
    """Other tile classes (2^12 tiles for n <= 20, 2^13 tiles with 512 threads)
    and 13-qubit instances in the multi-pass path: every instance against the
    oracle (1e-5) and the default schedule (float rounding)."""
    torch, qw = env
    insts = mixed_instances()
    b = qw.Batch(insts)
    fill_states(torch, b, insts)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        qw.expm_action_batched(b, stream=stream)
        ref = b.out_pool.clone()
        info = qw.expm_action_batched(b, stream=stream, sched=dict(onchip_nmax=onchip, tile_class=classes))
    stream.synchronize()
    for n, c in classes.items():
        if n > onchip and any(ins["n"] == n for ins in insts):
            assert info["tile_class"][n] == c
    assert info["onchip_nmax"] == onchip
    assert torch.max(torch.abs(ref - b.out_pool)).item() <= 1e-6
    for i, ins in enumerate(insts):
        n = ins["n"]
        E = oracle_mod.energies(n, ins["h"], ins["J"])
        want = oracle_mod.expm_action(n, E, ins["gamma"], ins["t"], b.state(i).cpu().numpy().astype(np.complex128),
                                      1e-13)
        assert rel(b.output(i).cpu().numpy().astype(np.complex128), want) <= 1e-5, (i, n)


def test_invalid_tile_class_is_refused(env):
    torch, qw = env
    insts = mixed_instances()
    b = qw.Batch(insts)
    with pytest.raises(qw.QwError):
        qw.expm_action_batched(b, sched=dict(tile_class={22: 1}))   # 2^12 tiles cannot hold 22 qubits


def test_graph_is_reused(env):
    """A second call with the same launch sequence replays the instantiated
    graph (no capture) and gives the same output."""
    torch, qw = env
    insts = mixed_instances()
    b = qw.Batch(insts)
    fill_states(torch, b, insts)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        i1 = qw.expm_action_batched(b, stream=stream, sched=dict(wave_bytes=32 << 20))
        o1 = b.out_pool.clone()
        b.out_pool.zero_()
        i2 = qw.expm_action_batched(b, stream=stream, sched=dict(wave_bytes=32 << 20), timing=1)
    stream.synchronize()
    assert i1["graph_cached"] == 0 and i1["graph_ms"] > 0
    assert i2["graph_cached"] == 1 and i2["graph_ms"] == 0
    assert torch.equal(o1, b.out_pool)


def test_repeated_calls_with_work_between(env):
    """The first call captures the graph and the later ones replay it; eager
    torch work and synchronisations in between must not change any result."""
    torch, qw = env
    insts = mixed_instances()
    b = qw.Batch(insts)
    fill_states(torch, b, insts)
    stream = torch.cuda.Stream()
    outs = []
    for rep in range(3):
        with torch.cuda.stream(stream):
            junk = torch.randn(1 << 20, device="cuda").sum()
            qw.expm_action_batched(b, stream=stream)
            outs.append(b.out_pool.clone())
            b.out_pool.mul_(0.5)
            _ = (junk + 1).item()
        stream.synchronize()
    assert torch.equal(outs[0], outs[1]) and torch.equal(outs[0], outs[2])


def test_null_stream_runs_eagerly(env):
    torch, qw = env
    insts = mixed_instances()[:6]
    b = qw.Batch(insts)
    fill_states(torch, b, insts)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        qw.expm_action_batched(b, stream=stream)
    stream.synchronize()
    ref = b.out_pool.clone()
    b.out_pool.zero_()
    qw.expm_action_batched(b, stream=torch.cuda.default_stream())
    torch.cuda.synchronize()
    assert torch.equal(ref, b.out_pool)


def test_tune_cache_roundtrip(env, tmp_path):
    torch, qw = env
    insts = mixed_instances()
    b = qw.Batch(insts)
    fill_states(torch, b, insts)
    cache = str(tmp_path / "tune.txt")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        best = qw.batched_tune(b, cache, stream=stream)
        info = qw.expm_action_batched(b, tune_cache=cache, stream=stream)
    stream.synchronize()
    assert info["wave_bytes"] == best["wave_bytes"]
    assert info["onchip_nmax"] == best["onchip_nmax"] and info["concurrent"] == best["concurrent"]
    for n, c in best["tile_class"].items():
        if n > best["onchip_nmax"] and n in info["tile_class"]:
            assert info["tile_class"][n] == c
    fields = dict(f.split("=") for f in open(cache).read().split()[1:])
    assert int(fields["wave"]) == best["wave_bytes"] and int(fields["onchip"]) == best["onchip_nmax"]


def test_config3_batched_256(env, oracle_mod):
    """256 SK instances, n ~ U{12..22}, t ~ U(0.1, 20), gamma ~ U(0.2, 2),
    complex64, tol 1e-6: norms conserved, small instances, a sample of 14-16
    qubit ones and the two 22-qubit ones of shortest time against the oracle, a
    sample against the single-instance path."""
    torch, qw = env
    insts = synth.batch_instances(256, 0)
    for ins in insts:
        ins["tol"] = 1e-6
    b = qw.Batch(insts)
    for i, ins in enumerate(insts):
        b.state(i).fill_(1.0 / np.sqrt(1 << ins["n"]))
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        info = qw.expm_action_batched(b, stream=stream, timing=1)
    stream.synchronize()
    assert info["small_count"] + info["large_count"] == 256
    norms = [torch.linalg.vector_norm(b.output(i).to(torch.complex128)).item() for i in range(256)]
    assert max(abs(x - 1.0) for x in norms) < 1e-5
    rng = np.random.default_rng(3)
    small = [i for i, ins in enumerate(insts) if ins["n"] <= 13]
    large = [i for i, ins in enumerate(insts) if 14 <= ins["n"] <= 16]
    # 22-qubit instances (9-bit high group), the two with the shortest times
    top = sorted((i for i, ins in enumerate(insts) if ins["n"] == 22), key=lambda i: insts[i]["t"])[:2]
    check = small[:8] + list(rng.choice(large, 4, replace=False)) + top
    for i in check:
        ins = insts[i]
        n = ins["n"]
        E = oracle_mod.energies(n, ins["h"], ins["J"])
        ref = oracle_mod.expm_action(n, E, ins["gamma"], ins["t"], synth.plus_state(n), 1e-13)
        got = b.output(i).cpu().numpy().astype(np.complex128)
        assert rel(got, ref) <= 1e-5, (i, n, ins["t"], ins["gamma"])
    for i in rng.choice(256, 6, replace=False):
        ins = insts[i]
        single, _ = qw.expm_action(b.state(i).clone(), ins["gamma"], ins["t"], h=ins["h"], J=ins["J"], tol=1e-6)
        assert torch.max(torch.abs(single - b.output(i))).item() <= 1e-6
