"""Pins of the fourth-order commutator-free Magnus steps (sec. III.B): the
oracle's anneal integrator (O6) and the leading local-error term the library
uses to choose step sizes.

* The series derivation: expanding the two-exponential step and the exact
  propagator in h (noncommutative power series in H_P and F = sum_j X_j with
  A(t), B(t) Taylor-expanded) must agree through h^4, and the h^5 difference
  must be the six-term commutator expression E5 stated in the library's
  documentation.
* A constant schedule is integrated exactly in one step.
* Fourth-order convergence against scipy's DOP853 run at 1e-13.
* The local error of one step divided by h^5 tends to E5 psi.
"""
import numpy as np
import pytest
import scipy.integrate

import synth

R3 = np.sqrt(3.0)


def dense_F(n):
    X = np.array([[0.0, 1.0], [1.0, 0.0]])
    return sum(np.kron(np.kron(np.eye(1 << (n - 1 - j)), X), np.eye(1 << j)) for j in range(n))


def exact(n, E, a, b, T, t0, t1, psi, oracle_mod, tol=1e-13):
    F = dense_F(n)
    P = np.diag(E)

    def rhs(t, y):
        H = oracle_mod.schedule_value(a, T, t) * P + oracle_mod.schedule_value(b, T, t) * F
        return -1j * (H @ y)

    sol = scipy.integrate.solve_ivp(rhs, (t0, t1), np.asarray(psi, dtype=np.complex128), method="DOP853",
                                    rtol=tol, atol=tol)
    return sol.y[:, -1]


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_series_derivation_of_the_local_error():
    sp = pytest.importorskip("sympy")
    P, G = sp.symbols("P G", commutative=False)
    h = sp.symbols("h", positive=True)
    A = sp.symbols("A0:5")
    B = sp.symbols("B0:5")
    order = 5
    Hd = [A[j] * P + B[j] * G for j in range(5)]     # derivatives of H at the step start

    def trunc(x):
        x = sp.expand(x)
        return sum(x.coeff(h, k) * h ** k for k in range(order + 1))

    # exact propagator: power series of U' = -i H U
    U = [sp.Integer(1)]
    for k in range(order):
        U.append(sp.expand(-sp.I * sum(Hd[j] / sp.factorial(j) * U[k - j] for j in range(k + 1)) / (k + 1)))
    Uex = sum(U[k] * h ** k for k in range(order + 1))

    def Hat(tau):
        return sum(Hd[j] * tau ** j / sp.factorial(j) for j in range(5))

    c1, c2 = sp.Rational(1, 2) - sp.sqrt(3) / 6, sp.Rational(1, 2) + sp.sqrt(3) / 6
    w1, w2 = sp.Rational(1, 4) + sp.sqrt(3) / 6, sp.Rational(1, 4) - sp.sqrt(3) / 6

    def expo(X):
        out, term = sp.Integer(1), sp.Integer(1)
        for m in range(1, order + 1):
            term = trunc(term * X) / m
            out += term
        return trunc(out)

    first = trunc(-sp.I * h * (w1 * Hat(c1 * h) + w2 * Hat(c2 * h)))
    second = trunc(-sp.I * h * (w2 * Hat(c1 * h) + w1 * Hat(c2 * h)))
    D = sp.expand(trunc(expo(second) * expo(first)) - Uex)
    for k in range(1, 5):
        assert sp.simplify(D.coeff(h, k)) == 0, k

    def com(x, y):
        return x * y - y * x

    H0, H1, H2, H3, H4 = Hd
    E5 = (sp.I / 4320 * H4 - sp.Rational(1, 1080) * com(H0, H3) - sp.Rational(1, 720) * com(H1, H2)
          - sp.I / 720 * com(H0, com(H0, H2)) - sp.I / 2160 * com(H1, com(H0, H1))
          + sp.Rational(1, 2880) * com(H0, com(H0, com(H0, H1))))
    assert sp.simplify(sp.expand(D.coeff(h, 5) - E5)) == 0


def test_constant_schedule_is_one_exact_step(oracle_mod):
    n = 6
    h, J = synth.sk_instance(n, 21)
    E = oracle_mod.energies(n, h, J)
    psi = synth.random_state(n, 22)
    y = oracle_mod.anneal_cfet4(n, E, [0.7], [0.4], 2.0, [2.0], psi, [1e-14])
    ref = oracle_mod.expm_action_dense(n, 0.7 * E, 0.4, 2.0, psi)
    assert rel(y, ref) < 1e-12


def test_fourth_order_convergence_vs_dop853(oracle_mod):
    """Linear anneal A = s, B = 1 - s on 4 qubits: halving the step divides
    the error by about 2^4."""
    n, T = 4, 3.0
    h, J = synth.sk_instance(n, 23)
    E = oracle_mod.energies(n, h, J)
    psi = synth.plus_state(n)
    a, b = [0.0, 1.0], [1.0, -1.0]
    ref = exact(n, E, a, b, T, 0.0, T, psi, oracle_mod)
    errs = []
    for S in (6, 12, 24):
        y = oracle_mod.anneal_cfet4(n, E, a, b, T, [T / S] * S, psi, [1e-15] * S)
        errs.append(rel(y, ref))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 12.0 < r1 < 20.0 and 12.0 < r2 < 20.0, errs


def test_local_error_tends_to_e5(oracle_mod):
    """One step from t0 with a quartic schedule: (step - exact) psi / h^5 tends
    to E5 psi, E5 built from dense H and its time derivatives at t0."""
    n, T, t0 = 3, 2.0, 0.7
    h, J = synth.sk_instance(n, 24)
    E = oracle_mod.energies(n, h, J)
    a = np.array([0.3, 1.0, 0.5, -0.8, 0.4])
    b = np.array([1.0, -1.0, 0.0, 0.2])
    psi = synth.random_state(n, 25)
    P, F = np.diag(E), dense_F(n)

    def dpoly(c, m):
        d = np.polynomial.polynomial.polyder(c, m) if m else np.asarray(c)
        return np.polynomial.polynomial.polyval(t0 / T, d) / T ** m

    Hd = [dpoly(a, m) * P + dpoly(b, m) * F for m in range(5)]
    H0, H1, H2, H3, H4 = Hd

    def com(x, y):
        return x @ y - y @ x

    E5 = (1j / 4320 * H4 - com(H0, H3) / 1080 - com(H1, H2) / 720 - 1j / 720 * com(H0, com(H0, H2))
          - 1j / 2160 * com(H1, com(H0, H1)) + com(H0, com(H0, com(H0, H1))) / 2880)
    y0 = exact(n, E, a, b, T, 0.0, t0, psi, oracle_mod, tol=3e-14)
    ratios = []
    for hs in (0.04, 0.02):
        ex = exact(n, E, a, b, T, t0, t0 + hs, y0, oracle_mod, tol=3e-14)
        step = _one_step(oracle_mod, n, E, a, b, T, t0, hs, y0)
        ratios.append(np.linalg.norm((step - ex) / hs ** 5 - E5 @ y0) / np.linalg.norm(E5 @ y0))
    assert ratios[1] < 0.1 and ratios[1] < ratios[0], ratios


def _one_step(oracle_mod, n, E, a, b, T, t, hs, y):
    c1, c2 = 0.5 - R3 / 6, 0.5 + R3 / 6
    w1, w2 = 0.25 + R3 / 6, 0.25 - R3 / 6
    A1, A2 = oracle_mod.schedule_value(a, T, t + c1 * hs), oracle_mod.schedule_value(a, T, t + c2 * hs)
    B1, B2 = oracle_mod.schedule_value(b, T, t + c1 * hs), oracle_mod.schedule_value(b, T, t + c2 * hs)
    for alpha, beta in ((w1 * A1 + w2 * A2, w1 * B1 + w2 * B2), (w2 * A1 + w1 * A2, w2 * B1 + w1 * B2)):
        y = oracle_mod.expm_action_dense(n, alpha * E, beta, hs, y)
    return y


def test_pins_catch_swapped_exponentials(oracle_mod, monkeypatch):
    """Plant the two exponentials in the other order: the method drops to
    second order and the convergence pin fails."""
    def broken(n, E, a_coef, b_coef, T, step_sizes, psi, tols):
        c1, c2 = 0.5 - R3 / 6, 0.5 + R3 / 6
        w1, w2 = 0.25 + R3 / 6, 0.25 - R3 / 6
        y, t = np.asarray(psi, dtype=np.complex128), 0.0
        for hs, tol in zip(step_sizes, tols):
            A1, A2 = oracle_mod.schedule_value(a_coef, T, t + c1 * hs), oracle_mod.schedule_value(a_coef, T, t + c2 * hs)
            B1, B2 = oracle_mod.schedule_value(b_coef, T, t + c1 * hs), oracle_mod.schedule_value(b_coef, T, t + c2 * hs)
            for alpha, beta in ((w2 * A1 + w1 * A2, w2 * B1 + w1 * B2), (w1 * A1 + w2 * A2, w1 * B1 + w2 * B2)):
                y = oracle_mod.expm_action(n, alpha * np.asarray(E), beta, hs, y, tol)
            t += hs
        return y

    monkeypatch.setattr(oracle_mod, "anneal_cfet4", broken)
    n, T = 4, 3.0
    h, J = synth.sk_instance(n, 23)
    E = oracle_mod.energies(n, h, J)
    psi = synth.plus_state(n)
    ref = exact(n, E, [0.0, 1.0], [1.0, -1.0], T, 0.0, T, psi, oracle_mod)
    e1 = rel(oracle_mod.anneal_cfet4(n, E, [0.0, 1.0], [1.0, -1.0], T, [T / 12] * 12, psi, [1e-15] * 12), ref)
    e2 = rel(oracle_mod.anneal_cfet4(n, E, [0.0, 1.0], [1.0, -1.0], T, [T / 24] * 24, psi, [1e-15] * 24), ref)
    assert e1 / e2 < 8.0
