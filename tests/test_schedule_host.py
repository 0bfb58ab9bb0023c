"""Host logic of the fused pass schedule (no GPU): the sequence returned by
qw_debug_schedule, executed with a numpy model of the three pass kinds on any
partition of the index bits into P groups, must give the Clenshaw result of
the oracle (Alg. 2 / Eq. recursion)."""
import ctypes

import numpy as np
import pytest

import paper_2608_12058_amd as qw
import synth


def schedule(K, P):
    lib = qw.lib()
    lib.qw_debug_schedule.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_int]
    cnt = lib.qw_debug_schedule(K, P, None, 0)
    buf = (ctypes.c_int * (4 * cnt))()
    assert lib.qw_debug_schedule(K, P, buf, cnt) == cnt
    return np.array(buf, dtype=np.int64).reshape(cnt, 4)


def simulate(sched, groups, c, d, g, v, phase):
    """START: dst = s(d b1 + g F b1) - acc + c_k v; ADD: dst = acc + s g F b1;
    FUSED: b_k = acc + s g F b1, b'_{k-1} = s'(d b_k + g F b_k) - b1 + c_{k-1} v."""
    idx = np.arange(len(v))

    def F(o, x):
        return sum(x[idx ^ (1 << j)] for j in groups[o])

    K, P = len(c) - 1, len(groups)
    X, Y, out = c[K] * v, None, None
    sc = lambda k: 1.0 if k == 0 else 2.0  # noqa: E731
    for mode, o, k, fin in sched:
        if mode == 0:
            acc = np.zeros_like(v) if k == K - 1 else Y
            r = sc(k) * (d * X + g * F(o, X)) - acc + c[k] * v
            if fin:
                out = phase * r
            elif P == 1:
                X, Y = r, X
            else:
                Y = r
        elif mode == 1:
            r = Y + sc(k) * g * F(o, X)
            if fin:
                out = phase * r
            else:
                Y = r
        else:
            bk = Y + sc(k) * g * F(o, X)
            X, Y = bk, sc(k - 1) * (d * bk + g * F(o, bk)) - X + c[k - 1] * v
    return out


GROUPS = {1: [list(range(7))], 2: [[0, 1, 2, 3], [4, 5, 6]], 3: [[0, 1, 2], [3, 4], [5, 6]],
          4: [[0, 1], [2, 3], [4, 5], [6]]}


@pytest.mark.parametrize("P", [1, 2, 3, 4])
@pytest.mark.parametrize("K", [1, 2, 3, 4, 7, 20])
def test_schedule_equals_clenshaw(oracle_mod, P, K):
    n = 7
    rng = np.random.default_rng(K * 10 + P)
    c = rng.standard_normal(K + 1) + 1j * rng.standard_normal(K + 1)
    d = rng.uniform(-0.5, 0.5, 1 << n)
    g = 0.5 / n
    v = synth.random_state(n, K)
    ref = oracle_mod.clenshaw(n, c, d, g, v)
    ph = np.exp(-0.3j)
    got = simulate(schedule(K, P), GROUPS[P], c, d, g, v, ph)
    assert np.allclose(got, ph * ref, atol=1e-12)


@pytest.mark.parametrize("P", [2, 3, 4])
def test_schedule_shape(P):
    K = 9
    S = schedule(K, P)
    assert S[0][0] == 0 and S[-1][0] == 1 and S[-1][3] == 1
    assert (S[:, 0] == 2).sum() == K - 1            # one fused pass between consecutive terms
    assert len(S) == 1 + (K - 1) * (P - 1) + (P - 1)  # passes per term drop from P to P - 1
    fused = S[S[:, 0] == 2]
    assert set(fused[:, 1]) <= {0, P - 1}           # fusion happens on the end orientations


@pytest.mark.parametrize("K", [1, 2, 3, 8, 31])
def test_batched_step_rule_matches_schedule(K):
    """The batched kernel derives each pass from (step j, K): j = 0 starts
    term K-1 in the low orientation, 1 <= j < K is a fused pass completing
    term K-j in orientation j mod 2, j = K is the final add; this must be the
    two-orientation schedule."""
    S = schedule(K, 2)
    assert len(S) == K + 1
    for j, (mode, o, k, fin) in enumerate(S):
        if j == 0:
            assert (mode, o, k) == (0, 0, K - 1)
        elif j == K:
            assert (mode, o, k, fin) == (1, j & 1, 0, 1)
        else:
            assert (mode, o, k, fin) == (2, j & 1, K - j, 0)
