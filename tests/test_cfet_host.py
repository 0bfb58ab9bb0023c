"""Host logic of the anneal integrator (no GPU): the library's bound on the
leading local-error operator E5 (sec. III.B) must bound its norm, computed
densely from H and its time derivatives, without being vacuous."""
import numpy as np
import pytest

import paper_2608_12058_amd as qw
import synth


def dense_F(n):
    X = np.array([[0.0, 1.0], [1.0, 0.0]])
    return sum(np.kron(np.kron(np.eye(1 << (n - 1 - j)), X), np.eye(1 << j)) for j in range(n))


def e5_dense(P, F, a, b, T, t):
    def dpoly(c, m):
        d = np.polynomial.polynomial.polyder(c, m) if m else np.asarray(c, dtype=float)
        return np.polynomial.polynomial.polyval(t / T, d) / T ** m

    H0, H1, H2, H3, H4 = [dpoly(a, m) * P + dpoly(b, m) * F for m in range(5)]

    def com(x, y):
        return x @ y - y @ x

    return (1j / 4320 * H4 - com(H0, H3) / 1080 - com(H1, H2) / 720 - 1j / 720 * com(H0, com(H0, H2))
            - 1j / 2160 * com(H1, com(H0, H1)) + com(H0, com(H0, com(H0, H1))) / 2880)


@pytest.mark.parametrize("n,seed", [(3, 1), (5, 2), (6, 3)])
@pytest.mark.parametrize("sched", ["linear", "quartic"])
def test_bound_dominates_e5(oracle_mod, n, seed, sched):
    h, J = synth.sk_instance(n, 40 + seed)
    E = oracle_mod.energies(n, h, J)
    P, F = np.diag(E), dense_F(n)
    if sched == "linear":
        a, b, T = [0.0, 1.0], [1.0, -1.0], 4.0
    else:
        a, b, T = [0.3, 1.0, 0.5, -0.8, 0.4], [1.0, -1.0, 0.0, 0.2], 2.0
    for t in np.linspace(0.0, T, 7):
        bound = qw.cfet4_step_bound(n, h, J, a, b, T, E.min(), E.max(), t)
        true = np.linalg.norm(e5_dense(P, F, a, b, T, t), 2)
        assert bound >= true * (1 - 1e-12), (t, bound, true)
        assert bound <= 1e3 * max(true, 1e-300), (t, bound, true)


def test_commutator_bound(oracle_mod):
    """||[H_P, F]|| <= sum_j 2(|h_j| + sum_k |J_jk|), the number the bound uses."""
    n = 6
    h, J = synth.sk_instance(n, 9)
    E = oracle_mod.energies(n, h, J)
    P, F = np.diag(E), dense_F(n)
    c = np.linalg.norm(P @ F - F @ P, 2)
    Jm = np.zeros((n, n))
    Jm[np.triu_indices(n, 1)] = J
    Jm = Jm + Jm.T
    assert c <= sum(2 * (abs(h[j]) + np.abs(Jm[j]).sum()) for j in range(n)) + 1e-12


def test_constant_schedule_has_zero_bound(oracle_mod):
    n = 4
    h, J = synth.sk_instance(n, 3)
    E = oracle_mod.energies(n, h, J)
    assert qw.cfet4_step_bound(n, h, J, [0.7], [0.4], 3.0, E.min(), E.max(), 1.0) == 0.0


def test_rejects_bad_schedule():
    h, J = synth.sk_instance(4, 3)
    with pytest.raises(qw.QwError):
        qw.cfet4_step_bound(4, h, J, [0.0, float("nan")], [1.0], 1.0, -1.0, 1.0, 0.5)
    with pytest.raises(qw.QwError):
        qw.cfet4_step_bound(4, h, J, [0.0] * 18, [1.0], 1.0, -1.0, 1.0, 0.5)
    with pytest.raises(qw.QwError):
        qw.cfet4_step_bound(4, h, J, [0.0], [1.0], 0.0, -1.0, 1.0, 0.5)
