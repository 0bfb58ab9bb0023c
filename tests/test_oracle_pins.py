"""Pins of the CPU oracle to things other than itself (no GPU needed).

Each test names the passage of the paper (or the mathematical fact) it checks.
"""
import mpmath
import numpy as np
import pytest
import scipy.linalg
import scipy.sparse
import scipy.sparse.linalg

import synth

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# ---------------------------------------------------------------- operator

@pytest.mark.parametrize("n", [1, 2, 3, 5, 7])
def test_energies_match_pauli_z_kronecker(oracle_mod, n):
    """H_P = sum J_jk Z_j Z_k + sum h_j Z_j (SK form), built from Kronecker
    products of Z = diag(1, -1) with qubit j = bit j; its diagonal must equal the
    bit-loop energies."""
    h, J = synth.sk_instance(n, 11 + n)
    Z = np.array([1.0, -1.0])

    def zj(j):
        return np.kron(np.kron(np.ones(1 << (n - 1 - j)), Z), np.ones(1 << j))

    ref = np.zeros(1 << n)
    p = 0
    for j in range(n):
        ref += h[j] * zj(j)
        for k in range(j + 1, n):
            ref += J[p] * zj(j) * zj(k)
            p += 1
    assert np.allclose(oracle_mod.energies(n, h, J), ref, rtol=0, atol=1e-13)


def test_pair_index_layout():
    n = 6
    seen = [synth.pair_index(n, j, k) for j in range(n) for k in range(j + 1, n)]
    assert seen == list(range(synth.n_pairs(n)))


@pytest.mark.parametrize("n", [1, 4, 9])
def test_hmatvec_matches_dense_kronecker(oracle_mod, n):
    """Matrix-free H x (XOR loop) vs the dense H built from Kronecker products of
    Pauli X (section I definition of H_G)."""
    rng = np.random.default_rng(n)
    d = rng.standard_normal(1 << n)
    x = synth.random_state(n, 3)
    g = 0.37
    H = oracle_mod.hamiltonian_dense(n, d, g)
    assert np.allclose(oracle_mod.hmatvec(n, d, g, x), H @ x, rtol=0, atol=1e-13)


@pytest.mark.parametrize("n", [3, 8])
def test_hypercube_walsh_hadamard_form(oracle_mod, n):
    """sum_j X_j = W diag(n - 2 popcount(k)) W / N with W the (unnormalised)
    Sylvester-Hadamard matrix: X_j is diagonalised by the Hadamard on qubit j."""
    N = 1 << n
    W = scipy.linalg.hadamard(N).astype(np.float64)
    pop = np.array([bin(k).count("1") for k in range(N)])
    x = synth.random_state(n, 5)
    ref = W @ ((n - 2 * pop) * (W @ x)) / N
    got = oracle_mod.hmatvec(n, np.zeros(N), 1.0, x)
    assert np.allclose(got, ref, atol=1e-12)


def test_recursive_definition_of_hg(oracle_mod):
    """H_G(n) = I_2 (x) H_G(n-1) + H_G(1) (x) I_{2^{n-1}} (section II.D)."""
    X = np.array([[0.0, 1.0], [1.0, 0.0]])
    HG = X
    for n in range(2, 7):
        HG = np.kron(np.eye(2), HG) + np.kron(X, np.eye(1 << (n - 1)))
        N = 1 << n
        ref = oracle_mod.hamiltonian_dense(n, np.zeros(N), 1.0)
        assert np.array_equal(HG, ref)


def test_shift_and_bound(oracle_mod):
    """Shift makes max and min of the diagonal equal in magnitude; r is the
    induced 1-norm of the shifted H and bounds its spectral radius (sec. II.A)."""
    n = 7
    h, J = synth.sk_instance(n, 2)
    E = oracle_mod.energies(n, h, J)
    for gamma in (0.0, 0.8, -1.3):
        c, r = oracle_mod.spectral_shift_radius(E, n, gamma)
        assert np.isclose(np.max(E) - c, -(np.min(E) - c))
        H = oracle_mod.hamiltonian_dense(n, E - c, gamma)
        assert np.isclose(r, np.max(np.sum(np.abs(H), axis=0)), rtol=1e-14)
        assert np.max(np.abs(np.linalg.eigvalsh(H))) <= r * (1 + 1e-14)


# ---------------------------------------------------------------- coefficients

@pytest.mark.parametrize("a", [0.5, 7.25, 99.0, 470.2, 1403.7])
def test_bessel_values_vs_mpmath_50_digits(oracle_mod, a):
    """Oracle J_m(a) against 50-digit mpmath besselj at sampled orders (the
    oracle's own table is 30-digit mpmath up to a = 800, scipy above)."""
    Jm = oracle_mod._bessel_table(a)
    ms = sorted(set([0, 1, 2, 5] + list(np.linspace(0, len(Jm) - 1, 12).astype(int))))
    atol = 1e-16 if a <= 800 else 3e-14
    with mpmath.workdps(50):
        for m in ms:
            ref = float(mpmath.besselj(m, a))
            assert abs(Jm[m] - ref) <= atol * max(1.0, abs(ref)), (m, Jm[m], ref)


@pytest.mark.parametrize("a", [3.0, 150.0, 1400.0])
def test_bessel_three_term_recurrence(oracle_mod, a):
    """J_{m-1} + J_{m+1} = (2m/a) J_m holds across the whole table."""
    Jm = oracle_mod._bessel_table(a)
    m = np.arange(1, len(Jm) - 1)
    resid = Jm[m - 1] + Jm[m + 1] - (2 * m / a) * Jm[m]
    assert np.max(np.abs(resid)) < (1e-15 if a <= 800 else 5e-13) * max(1.0, 2 * len(Jm) / a)


def test_bessel_table_reaches_underflow(oracle_mod):
    for a in (0.3, 20.0, 470.0, 1400.0):
        Jm = oracle_mod._bessel_table(a)
        assert abs(Jm[-1]) < 1e-17 * np.max(np.abs(Jm))


@pytest.mark.parametrize("a", [1.0, 22.07, 300.0, 1400.0])
def test_bessel_sum_identities(oracle_mod, a):
    """J_0 + 2 sum J_2m = 1 and J_0^2 + 2 sum J_m^2 = 1 (generating function)."""
    Jm = oracle_mod._bessel_table(a)
    lim = 1e-14 if a <= 800 else 1e-12     # mpmath table below 800, scipy above
    assert abs(Jm[0] + 2 * np.sum(Jm[2::2]) - 1.0) < lim
    assert abs(Jm[0] ** 2 + 2 * np.sum(Jm[1:] ** 2) - 1.0) < lim


@pytest.mark.parametrize("a,tol", [(22.07, 1e-12), (300.0, 2.0 ** -23), (-47.5, 1e-10)])
def test_series_equals_exponential(oracle_mod, a, tol):
    """sum_m c_m T_m(x) = exp(-i a x) within the truncation tolerance on 10^4
    points of [-1, 1] (Eq. cheb with a -> -a; Eq. TruncError)."""
    c = oracle_mod.cheb_coeffs(a, tol)
    x = np.linspace(-1, 1, 10001)
    err = np.max(np.abs(oracle_mod.cheb_series_eval(c, x) - np.exp(-1j * a * x)))
    assert err <= tol * 1.01 + 1e-14


def test_higham_151_terms(oracle_mod):
    """Sec. II.B.2: on [-99, 99] the Chebyshev series needs 151 terms (degree 150)
    at double precision; soft pin +-1 (Higham's tolerance is a backward error)."""
    K = oracle_mod.cheb_degree(oracle_mod.cheb_alpha(99.0), 2.0 ** -53)
    assert abs((K + 1) - 151) <= 1


def test_degree_asymptote_r_plus_o_r(oracle_mod):
    """Sec. II.B.2 (Debye): the Chebyshev degree is r + o(r), far below e*r."""
    ratios = []
    for a in (100.0, 1000.0, 8000.0):
        K = oracle_mod.cheb_degree(oracle_mod.cheb_alpha(a), 1e-12)
        ratios.append(K / a)
    assert ratios[0] > ratios[1] > ratios[2] > 1.0
    assert ratios[2] < 1.06
    assert all(r < np.e for r in ratios)


def test_single_coefficient_returns_c0_psi(oracle_mod):
    """K = 0 must give c_0 psi (the printed listing would return H c_0 psi + c_0 psi)."""
    n = 4
    v = synth.random_state(n, 1)
    y = oracle_mod.clenshaw(n, np.array([0.3 - 0.2j]), np.ones(1 << n), 0.5, v)
    assert np.allclose(y, (0.3 - 0.2j) * v)


def test_clenshaw_equals_chebyshev_sum(oracle_mod):
    """Clenshaw result equals sum_k c_k T_k(H) v with T_k from the three-term
    recurrence T_{k+1} = 2 H T_k - T_{k-1} on the dense matrix."""
    n = 5
    rng = np.random.default_rng(0)
    d = rng.uniform(-0.5, 0.5, 1 << n)
    g = 0.5 / n
    c = rng.standard_normal(9) + 1j * rng.standard_normal(9)
    v = synth.random_state(n, 2)
    H = oracle_mod.hamiltonian_dense(n, d, g)
    Tm, T = np.eye(1 << n), H.copy()
    ref = c[0] * v + c[1] * (H @ v)
    for k in range(2, len(c)):
        Tm, T = T, 2 * H @ T - Tm
        ref = ref + c[k] * (T @ v)
    assert np.allclose(oracle_mod.clenshaw(n, c, d, g, v), ref, atol=1e-12)


# ---------------------------------------------------------------- the action

def test_config1_vs_dense_eigh(oracle_mod):
    """n = 10, SK seed 0, gamma = 1, t = 1, |+>, tol 1e-12: O1 vs O0 <= 1e-12."""
    n = 10
    h, J = synth.sk_instance(n, 0)
    E = oracle_mod.energies(n, h, J)
    psi = synth.plus_state(n)
    y = oracle_mod.expm_action(n, E, 1.0, 1.0, psi, 1e-12)
    y0 = oracle_mod.expm_action_dense(n, E, 1.0, 1.0, psi)
    assert rel(y, y0) <= 1e-12


@pytest.mark.parametrize("n,gamma,t,seed", [(3, 0.3, 4.0, 1), (6, 1.7, 2.5, 2), (8, -0.6, 7.0, 3),
                                            (9, 2.0, -3.0, 4)])
def test_random_cases_vs_dense_eigh(oracle_mod, n, gamma, t, seed):
    h, J = synth.sk_instance(n, seed)
    E = oracle_mod.energies(n, h, J)
    psi = synth.random_state(n, seed + 50)
    y = oracle_mod.expm_action(n, E, gamma, t, psi, 1e-13)
    y0 = oracle_mod.expm_action_dense(n, E, gamma, t, psi)
    assert rel(y, y0) <= 1e-12


def test_cf_action_vs_dense_eigh(oracle_mod):
    n = 8
    h, J = synth.sk_instance(n, 9)
    E = oracle_mod.energies(n, h, J)
    psi = synth.plus_state(n)
    y = oracle_mod.expm_action(n, E, 0.8, 10.0, psi, 1e-10, method="cf")
    y0 = oracle_mod.expm_action_dense(n, E, 0.8, 10.0, psi)
    assert rel(y, y0) <= 2e-10


def test_closed_form_gamma_zero(oracle_mod):
    n = 11
    h, J = synth.sk_instance(n, 4)
    E = oracle_mod.energies(n, h, J)
    psi = synth.random_state(n, 4)
    y = oracle_mod.expm_action(n, E, 0.0, 3.3, psi, 1e-13)
    assert rel(y, oracle_mod.closed_form_gamma0(E, 3.3, psi)) <= 1e-12
    # sampled form with energies summed per index in pure Python
    idx = np.array([0, 5, 777, (1 << n) - 1])
    amps = oracle_mod.closed_form_gamma0_amps(n, h, J, 3.3, psi[idx], idx)
    assert np.allclose(amps, y[idx], atol=1e-12)


def test_closed_form_hp_zero(oracle_mod):
    """H_P = 0: product of single-qubit rotations; random (non-eigen) state."""
    n = 10
    E = np.zeros(1 << n)
    psi = synth.random_state(n, 8)
    y = oracle_mod.expm_action(n, E, 1.3, 2.2, psi, 1e-13)
    assert rel(y, oracle_mod.closed_form_hp0(n, 1.3, 2.2, psi)) <= 1e-12
    f = synth.product_state_factors(n, 3)
    ps = synth.product_state(f)
    y2 = oracle_mod.expm_action(n, E, 0.7, 5.0, ps, 1e-13)
    idx = np.arange(1 << n)
    assert np.allclose(oracle_mod.closed_form_hp0_product_amps(f, 0.7, 5.0, idx), y2, atol=1e-12)


def test_vs_scipy_expm_multiply(oracle_mod):
    """Independent library check: scipy.sparse.linalg.expm_multiply at n = 13."""
    n = 13
    h, J = synth.sk_instance(n, 21)
    E = oracle_mod.energies(n, h, J)
    N = 1 << n
    rows, cols = [np.arange(N)], [np.arange(N)]
    vals = [E]
    for j in range(n):
        rows.append(np.arange(N))
        cols.append(np.arange(N) ^ (1 << j))
        vals.append(np.full(N, 0.9))
    Hs = scipy.sparse.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                                 shape=(N, N))
    psi = synth.plus_state(n)
    ref = scipy.sparse.linalg.expm_multiply(-1j * 2.0 * Hs, psi)
    y = oracle_mod.expm_action(n, E, 0.9, 2.0, psi, 1e-13)
    assert rel(y, ref) <= 1e-11


def test_invariants(oracle_mod):
    """Unitarity, energy conservation, time reversal and the group property."""
    n = 12
    h, J = synth.sk_instance(n, 6)
    E = oracle_mod.energies(n, h, J)
    psi = synth.random_state(n, 6)
    g = 0.9
    y = oracle_mod.expm_action(n, E, g, 2.5, psi, 1e-13)
    assert abs(np.linalg.norm(y) - 1.0) < 1e-12

    def energy(v):
        return np.real(np.vdot(v, oracle_mod.hmatvec(n, E, g, v)))

    assert abs(energy(y) - energy(psi)) < 1e-11
    back = oracle_mod.expm_action(n, E, g, -2.5, y, 1e-13)
    assert rel(back, psi) < 1e-12
    two = oracle_mod.expm_action(n, E, g, 1.0, oracle_mod.expm_action(n, E, g, 1.5, psi, 1e-13), 1e-13)
    assert rel(two, y) < 1e-12


def test_error_within_paper_bound(oracle_mod):
    """Measured error vs O0 is below truncation tol + coefficient error K u +
    the evaluation bound of sec. II.B.3 computed from the recurrence's norms."""
    n = 9
    h, J = synth.sk_instance(n, 7)
    E = oracle_mod.energies(n, h, J)
    psi = synth.plus_state(n)
    for tol in (1e-6, 1e-12):
        info = {}
        y = oracle_mod.expm_action(n, E, 1.1, 4.0, psi, tol, info=info)
        y0 = oracle_mod.expm_action_dense(n, E, 1.1, 4.0, psi)
        err = np.linalg.norm(y - y0)
        bound = tol + info["K"] * 2.0 ** -53 + info["eval_bound"]
        assert err <= bound
        assert info["eval_bound"] < 1e-12



# Hand-worked value of the evaluation-error bound of sec. II.B.3,
#   sum_k u ||b_k|| + u ||c_k v - b_{k+2}|| + sqrt(d) gamma_d ||b_{k+1}||,
# for n = 1 (d = n + 1 = 2 non-zeros per column of H), u = 2^-10 and the
# three steps (1, 1, 0), (2, 3, 1), (0.5, 4, 2):
#   gamma_2 = 2u / (1 - 2u) = (2/1024) / (1022/1024) = 1/511,
#   u-terms = (1 + 1 + 2 + 3 + 0.5 + 4) / 1024 = 11.5 / 1024 = 23/2048,
#   matvec terms = sqrt(2) * (1/511) * (0 + 1 + 2) = 3 sqrt(2) / 511,
#   bound = 23/2048 + 3 sqrt(2)/511 = 0.019533...
_BOUND_STEPS = [(1.0, 1.0, 0.0), (2.0, 3.0, 1.0), (0.5, 4.0, 2.0)]
_BOUND_HAND = 23.0 / 2048.0 + 3.0 * np.sqrt(2.0) / 511.0


def _bound_pin_holds(fn):
    return abs(fn(_BOUND_STEPS, 1, 2.0 ** -10) - _BOUND_HAND) <= 1e-15


def test_evaluation_bound_hand_value(oracle_mod):
    """sec. II.B.3: the bound's value on a case worked by hand (above)."""
    assert abs(_BOUND_HAND - 0.0195330918) < 1e-9
    assert _bound_pin_holds(oracle_mod.evaluation_error_bound)


def test_evaluation_bound_pin_catches_planted_mistakes():
    """Plausible mistakes in the bound -- d = n instead of n + 1, a dropped
    sqrt(d), u in place of gamma_d, a dropped u ||b_k|| term -- each miss the
    hand-worked value."""
    def d_is_n(norms, n, u):
        g = n * u / (1.0 - n * u)
        return sum(u * a + u * b + np.sqrt(n) * g * c for a, b, c in norms)

    def no_sqrt(norms, n, u):
        d = n + 1
        g = d * u / (1.0 - d * u)
        return sum(u * a + u * b + g * c for a, b, c in norms)

    def u_for_gamma(norms, n, u):
        d = n + 1
        return sum(u * a + u * b + np.sqrt(d) * u * c for a, b, c in norms)

    def no_bk(norms, n, u):
        d = n + 1
        g = d * u / (1.0 - d * u)
        return sum(u * b + np.sqrt(d) * g * c for a, b, c in norms)

    for broken in (d_is_n, no_sqrt, u_for_gamma, no_bk):
        assert not _bound_pin_holds(broken), broken.__name__


def test_evaluation_bound_norms_worked_by_hand(oracle_mod):
    """The per-step norms the Clenshaw recurrence collects for the bound
    (sec. II.B.3, Eq. recursion) on a 2 x 2 case worked by hand: d = (1/2, -1/2),
    g = 1/4, v = (1, 0), c = (1, 1, 1).
      b_2 = c_2 v = (1, 0);  b_1 = 2 H b_2 + c_1 v = 2 (1/2, 1/4) + (1, 0) = (2, 1/2);
      y = H b_1 - b_2 + c_0 v = (1 + 1/8, 1/2 - 1/4) - (1, 0) + (1, 0) = (9/8, 1/4).
    Steps k = 2, 1, 0: (||b_2||, ||c_2 v||, 0) = (1, 1, 0);
    (||b_1||, ||c_1 v - b_3||, ||b_2||) = (sqrt(17)/2, 1, 1);
    (||y||, ||c_0 v - b_2||, ||b_1||) = (sqrt(85)/8, 0, sqrt(17)/2)."""
    d = np.array([0.5, -0.5])
    v = np.array([1.0, 0.0], dtype=np.complex128)
    c = np.array([1.0, 1.0, 1.0], dtype=np.complex128)
    norms = []
    y = oracle_mod.clenshaw(1, c, d, 0.25, v, norms)
    assert np.allclose(y, [9.0 / 8.0, 0.25], atol=1e-15)
    want = [(1.0, 1.0, 0.0), (np.sqrt(17.0) / 2, 1.0, 1.0), (np.sqrt(85.0) / 8, 0.0, np.sqrt(17.0) / 2)]
    assert len(norms) == len(want)
    for got, exp in zip(norms, want):
        assert np.allclose(got, exp, atol=1e-15), (got, exp)


# ---------------------------------------------------------------- CF

def _err_curve(p, f, x):
    return f(x) - np.polynomial.chebyshev.chebval(x, p)


def _alternations(e, level):
    """Number of sign-alternating extrema of e with |e| >= level."""
    count, last = 0, 0
    i = 0
    while i < len(e):
        if abs(e[i]) >= level:
            s = 1 if e[i] > 0 else -1
            if s != last:
                count += 1
                last = s
        i += 1
    return count


@pytest.mark.parametrize("a,kind,m", [(10.0, "cos", 9), (30.0, "cos", 27), (30.0, "sin", 26),
                                       (50.0, "sin", 42), (20.0, "sin", 16)])
def test_cf_equioscillation_and_lambda(oracle_mod, a, kind, m):
    """Sec. II.C: the minimax error equioscillates at >= k+2 points, and the CF
    eigenvalue estimates it; CF <= Chebyshev <= (Lambda + 1) CF with
    Lambda + 1 = (2/pi) ln(k+1) + 2."""
    Jm = oracle_mod._bessel_table(a)
    M = len(Jm) - 1
    mm = np.arange(M + 1)
    if kind == "cos":
        coef = np.where(mm % 2 == 0, 2.0 * (-1.0) ** (mm // 2) * Jm, 0.0)
        coef[0] = Jm[0]

        def f(x):
            return np.cos(a * x)
    else:
        coef = np.where(mm % 2 == 1, 2.0 * (-1.0) ** ((mm - 1) // 2) * Jm, 0.0)

        def f(x):
            return np.sin(a * x)
    p, lam = oracle_mod.cf_real(coef, m)
    x = np.cos(np.linspace(0, np.pi, 200001))
    e = _err_curve(p, f, x)
    emax = np.max(np.abs(e))
    assert abs(emax - abs(lam)) <= 0.02 * abs(lam)
    assert _alternations(e, 0.98 * emax) >= m + 2
    ec = np.max(np.abs(_err_curve(coef[:m + 1], f, x)))
    assert emax <= ec
    assert ec <= ((2 / np.pi) * np.log(m + 1) + 2) * emax


@pytest.mark.parametrize("a,tol", [(22.07, 1e-12), (120.0, 2.0 ** -23), (470.0, 2.0 ** -23)])
def test_cf_coefficients_meet_tolerance(oracle_mod, a, tol):
    c_cf, lam = oracle_mod.cf_coeffs(a, tol)
    c_ch = oracle_mod.cheb_coeffs(a, tol)
    assert len(c_cf) <= len(c_ch)
    x = np.cos(np.linspace(0, np.pi, 100001))
    err = np.max(np.abs(oracle_mod.cheb_series_eval(c_cf, x) - np.exp(-1j * a * x)))
    assert err <= lam * 1.05 + 1e-15
    assert err <= tol * 1.05


# ---------------------------------------------------------------- gradient

def test_gradient_vs_daleckii_krein(oracle_mod):
    n = 5
    h, J = synth.sk_instance(n, 13)
    gam = np.array([1.5, 0.9, 0.2])
    ts = np.array([0.5, 0.7, 0.4])
    psi0 = synth.plus_state(n)
    E1, g1 = oracle_mod.anneal_energy_grad(n, h, J, gam, ts, psi0, 1e-14)
    E2, g2 = oracle_mod.anneal_grad_daleckii_krein(n, h, J, gam, ts, psi0)
    assert abs(E1 - E2) < 1e-12
    for key in ("gamma", "t", "h", "J"):
        assert rel(g1[key], g2[key]) < 1e-9, key


def test_gradient_vs_finite_differences(oracle_mod):
    n = 6
    h, J = synth.sk_instance(n, 14)
    gam = np.array([1.8, 1.0, 0.3, 0.05])
    ts = np.array([0.5, 0.5, 0.5, 0.5])
    psi0 = synth.plus_state(n)
    tol = 1e-13
    _, g = oracle_mod.anneal_energy_grad(n, h, J, gam, ts, psi0, tol)
    step = 1e-3

    def energy(h_, J_, gam_, ts_):
        return oracle_mod.anneal_forward(n, h_, J_, gam_, ts_, psi0, tol)[0]

    def fd(vec, which):
        out = np.zeros_like(vec)
        for i in range(len(vec)):
            vp, vm = vec.copy(), vec.copy()
            vp[i] += step
            vm[i] -= step
            args_p = dict(h_=h, J_=J, gam_=gam, ts_=ts)
            args_m = dict(h_=h, J_=J, gam_=gam, ts_=ts)
            args_p[which], args_m[which] = vp, vm
            out[i] = (energy(**args_p) - energy(**args_m)) / (2 * step)
        return out

    # central differences carry an O(step^2) error of about 1e-5 here; the
    # Daleckii-Krein test above is the tight pin of the adjoint
    assert rel(g["gamma"], fd(gam, "gam_")) < 5e-5
    assert rel(g["t"], fd(ts, "ts_")) < 5e-5
    assert rel(g["h"], fd(h, "h_")) < 5e-5
    assert rel(g["J"], fd(J, "J_")) < 5e-5


# ---------------------------------------------------------------- planted mistakes

def test_pins_catch_a_dropped_factor_two(oracle_mod, monkeypatch):
    """Plant a mistake in the oracle (alpha_m = J_m instead of 2 J_m): the
    eigendecomposition pin must fail."""
    real = oracle_mod.cheb_alpha

    def broken(a):
        al = real(a)
        al[1:] *= 0.5
        return al

    monkeypatch.setattr(oracle_mod, "cheb_alpha", broken)
    n = 6
    h, J = synth.sk_instance(n, 1)
    E = oracle_mod.energies(n, h, J)
    psi = synth.plus_state(n)
    y = oracle_mod.expm_action(n, E, 1.0, 1.0, psi, 1e-12)
    assert rel(y, oracle_mod.expm_action_dense(n, E, 1.0, 1.0, psi)) > 1e-3


def test_pins_catch_a_wrong_time_sign(oracle_mod, monkeypatch):
    """Plant c_m = i^m alpha_m (the sign of Eq. cheb without a -> -a)."""
    def broken(a, tol):
        al = oracle_mod.cheb_alpha(a)
        K = oracle_mod.cheb_degree(al, tol)
        return (1j ** np.arange(K + 1)) * al[:K + 1]

    monkeypatch.setattr(oracle_mod, "cheb_coeffs", broken)
    n = 6
    h, J = synth.sk_instance(n, 1)
    E = oracle_mod.energies(n, h, J)
    psi = synth.plus_state(n)
    y = oracle_mod.expm_action(n, E, 1.0, 1.0, psi, 1e-12)
    assert rel(y, oracle_mod.expm_action_dense(n, E, 1.0, 1.0, psi)) > 1e-3


# ---------------------------------------------------------------- O5: caller polynomials, Horner (Alg. 1)

def test_horner_vs_dense_matrix_powers(oracle_mod):
    """Horner's rule against sum_m a_m H^m v with H the dense Kronecker-built
    Hamiltonian and numpy matrix powers."""
    n = 4
    rng = np.random.default_rng(11)
    d = rng.uniform(-1, 1, 1 << n)
    a = rng.standard_normal(7) + 1j * rng.standard_normal(7)
    v = synth.random_state(n, 12)
    H = oracle_mod.hamiltonian_dense(n, d, 0.21)
    ref = sum(a[m] * (np.linalg.matrix_power(H, m) @ v) for m in range(len(a)))
    assert rel(oracle_mod.horner(n, a, d, 0.21, v), ref) < 1e-13


def test_horner_gamma_zero_is_elementwise_polyval(oracle_mod):
    """gamma = 0: p(H) v = p(d) .* v (numpy polyval)."""
    n = 7
    rng = np.random.default_rng(13)
    d = rng.uniform(-1, 1, 1 << n)
    a = rng.standard_normal(12)
    v = synth.random_state(n, 14)
    ref = np.polynomial.polynomial.polyval(d, a) * v
    assert rel(oracle_mod.horner(n, a, d, 0.0, v), ref) < 1e-14


def test_horner_matches_clenshaw_after_basis_change(oracle_mod):
    """A degree-20 monomial polynomial (the Fig. 4 workload, smaller degree)
    evaluated by Horner's rule and, converted to the Chebyshev basis with
    numpy's poly2cheb, by the Clenshaw recurrence: two algorithms, one result."""
    n = 6
    h, J = synth.sk_instance(n, 15)
    E = oracle_mod.energies(n, h, J)
    c, r = oracle_mod.spectral_shift_radius(E, n, 0.7)
    d = (E - c) / r
    g = 0.7 / r
    a = np.random.default_rng(16).standard_normal(21)
    v = synth.random_state(n, 17)
    yh = oracle_mod.horner(n, a, d, g, v)
    yc = oracle_mod.clenshaw(n, np.polynomial.chebyshev.poly2cheb(a).astype(np.complex128), d, g, v)
    assert rel(yh, yc) < 1e-12


@pytest.mark.parametrize("s", [0.5, 3.0, 12.0])
def test_sincos_taylor_coefficients(oracle_mod, s):
    K = int(3 * s + 40)
    x = np.linspace(-1, 1, 201)
    p = np.polynomial.polynomial.polyval(x, oracle_mod.sincos_taylor_coeffs(s, K))
    assert np.max(np.abs(p - (np.sin(s * x) + np.cos(s * x)))) < 1e-12 * max(1.0, np.exp(s) / 1e3)


@pytest.mark.parametrize("s", [0.5, 3.0, 30.0, 120.0])
def test_sincos_chebyshev_coefficients(oracle_mod, s):
    K = int(s + 12 * s ** (1 / 3) + 30)
    x = np.linspace(-1, 1, 401)
    p = np.polynomial.chebyshev.chebval(x, oracle_mod.sincos_cheb_coeffs(s, K))
    assert np.max(np.abs(p - (np.sin(s * x) + np.cos(s * x)))) < 1e-13


@pytest.mark.parametrize("basis", ["cheb", "mono"])
def test_poly_amps_local_vs_dense_eigendecomposition(oracle_mod, basis):
    """The sampled-output evaluation against the spectral definition p(H~) psi =
    V p(Lambda) V^H psi, with H~ the dense Kronecker-built Hamiltonian (numpy
    eigh) and p evaluated at the eigenvalues by numpy's chebval / polyval; every
    output of a 9-qubit instance, degree 5, gamma != 0, a shift and a radius that
    is not the spectral bound."""
    n = 9
    h, J = synth.sk_instance(n, 31)
    fac = synth.product_state_factors(n, 32)
    psi = synth.product_state(fac)
    E = oracle_mod.energies(n, h, J)
    gamma, c, r = 0.7, 0.3, 9.5
    rng = np.random.default_rng(33)
    coef = rng.standard_normal(6) + 1j * rng.standard_normal(6)
    Ht = (oracle_mod.hamiltonian_dense(n, E, gamma) - c * np.eye(1 << n)) / r
    w, V = np.linalg.eigh(Ht)
    ev = np.polynomial.chebyshev.chebval if basis == "cheb" else np.polynomial.polynomial.polyval
    ref = V @ (ev(w, coef) * (V.conj().T @ psi))
    got = oracle_mod.poly_amps_local(n, h, J, gamma, c, r, coef, basis, fac, np.arange(1 << n))
    assert rel(got, ref) < 1e-13


def test_poly_amps_local_gamma_zero_is_chebval(oracle_mod):
    """gamma = 0 at 30 qubits: p(H~) psi at z is chebval(d~(z)) psi(z) with
    d~(z) = (E(z) - c) / r and E(z) summed by its definition per sampled index."""
    n = 30
    h, J = synth.sk_instance(n, 34)
    fac = synth.product_state_factors(n, 35)
    idx = np.random.default_rng(36).integers(0, 1 << n, 6)
    coef = np.array([0.5, -0.25 + 0.1j, 0.3, 0.2j])
    c, r = -0.4, 60.0
    amp = np.ones(len(idx), dtype=np.complex128)
    for j in range(n):
        amp *= fac[j, (idx >> j) & 1]
    ref = np.polynomial.chebyshev.chebval((oracle_mod.energies_at(n, h, J, idx) - c) / r, coef) * amp
    got = oracle_mod.poly_amps_local(n, h, J, 0.0, c, r, coef, "cheb", fac, idx)
    assert rel(got, ref) < 1e-14


@pytest.mark.parametrize("basis", ["cheb", "mono"])
def test_poly_amps_local_matches_full_vector_recurrences(oracle_mod, basis):
    """At 14 qubits: sampled outputs against the full-vector clenshaw / horner
    (Alg. 2 / Alg. 1) on the same normalised diagonal, degree 6."""
    n = 14
    h, J = synth.sk_instance(n, 37)
    fac = synth.product_state_factors(n, 38)
    psi = synth.product_state(fac)
    E = oracle_mod.energies(n, h, J)
    gamma, c, r = -0.6, 0.2, 25.0
    rng = np.random.default_rng(39)
    coef = rng.standard_normal(7) + 1j * rng.standard_normal(7)
    d, g = (E - c) / r, gamma / r
    full = oracle_mod.clenshaw(n, coef, d, g, psi) if basis == "cheb" else oracle_mod.horner(n, coef, d, g, psi)
    idx = np.concatenate([[0, (1 << n) - 1], rng.integers(0, 1 << n, 30)])
    got = oracle_mod.poly_amps_local(n, h, J, gamma, c, r, coef, basis, fac, idx)
    assert rel(got, full[idx]) < 1e-13


def test_pins_catch_a_shifted_horner_coefficient(oracle_mod, monkeypatch):
    """Plant y <- H y + a_{k+1} v (an off-by-one in Alg. 1): the dense pin fails."""
    def broken(n, a, d, g, v):
        a = np.asarray(a, dtype=np.complex128)
        y = a[-1] * v
        for k in range(len(a) - 2, -1, -1):
            y = oracle_mod.hmatvec(n, d, g, y) + a[k + 1] * v
        return y

    monkeypatch.setattr(oracle_mod, "horner", broken)
    n = 4
    rng = np.random.default_rng(11)
    d = rng.uniform(-1, 1, 1 << n)
    a = rng.standard_normal(7) + 1j * rng.standard_normal(7)
    v = synth.random_state(n, 12)
    H = oracle_mod.hamiltonian_dense(n, d, 0.21)
    ref = sum(a[m] * (np.linalg.matrix_power(H, m) @ v) for m in range(len(a)))
    assert rel(oracle_mod.horner(n, a, d, 0.21, v), ref) > 1e-3


# ---------------------------------------------------------------- O7: Remez exchange, minimax check of CF

@pytest.mark.parametrize("m", [1, 3, 6, 10])
def test_remez_closed_forms(oracle_mod, m):
    """The best approximation of x^(n) by polynomials of degree n - 2 (same
    parity) on [-1, 1] has error 2^(1-n) (x^n - T_n / 2^(n-1))."""
    _, E = oracle_mod.remez_parity(lambda x: x ** (2 * m + 2), 0, 2 * m)
    assert abs(E / 2.0 ** -(2 * m + 1) - 1) < 1e-6
    _, E = oracle_mod.remez_parity(lambda x: x ** (2 * m + 3), 1, 2 * m + 1)
    assert abs(E / 2.0 ** -(2 * m + 2) - 1) < 1e-6


@pytest.mark.parametrize("parity,deg,a", [(0, 12, 9.0), (1, 15, 13.0)])
def test_remez_equioscillates(oracle_mod, parity, deg, a):
    """The error of the Remez result takes +-E alternately at m + 2 points of
    [0, 1] (the alternation theorem for the parity-restricted system)."""
    f = (lambda x: np.cos(a * x)) if parity == 0 else (lambda x: np.sin(a * x))
    c, E = oracle_mod.remez_parity(f, parity, deg)
    x = 0.5 * (1 - np.cos(np.pi * np.arange(200001) / 200000))
    e = f(x) - np.polynomial.chebyshev.chebval(x, c)
    assert np.max(np.abs(e)) <= E * (1 + 1e-6)
    m = (deg - parity) // 2
    assert _alternations(e, E * (1 - 1e-5)) >= m + 2


CF_CASES = [(5.0, 4), (5.0, 10), (20.0, 20), (20.0, 26), (60.0, 60), (60.0, 66)]


def _parts(oracle_mod, a):
    Jm = oracle_mod._bessel_table(a)
    mm = np.arange(len(Jm))
    ac = np.where(mm % 2 == 0, 2.0 * (-1.0) ** (mm // 2) * Jm, 0.0)
    ac[0] = Jm[0]
    as_ = np.where(mm % 2 == 1, 2.0 * (-1.0) ** ((mm - 1) // 2) * Jm, 0.0)
    return ac, as_


@pytest.mark.parametrize("a,deg", CF_CASES)
def test_cf_is_minimax_by_remez(oracle_mod, a, deg):
    """The CF estimate |lambda| and the sampled error of the CF polynomial both
    equal the minimax error found by the Remez exchange (sec. II.C: CF is close
    to the best approximation at a fraction of the cost)."""
    ac, as_ = _parts(oracle_mod, a)
    x = np.cos(np.linspace(0, np.pi, 40001))
    for parity, coefs, f, d in ((0, ac, np.cos, deg), (1, as_, np.sin, deg + 1)):
        p, lam = oracle_mod.cf_real(coefs, d + 1)
        _, Estar = oracle_mod.remez_parity(lambda t: f(a * t), parity, d)
        err = np.max(np.abs(np.polynomial.chebyshev.chebval(x, p) - f(a * x)))
        assert abs(abs(lam) / Estar - 1) < 1e-4
        assert Estar * (1 - 1e-6) <= err <= Estar * (1 + 1e-4)


def test_energies_at_matches_full_vector(oracle_mod):
    n = 9
    h, J = synth.sk_instance(n, 31)
    idx = np.arange(1 << n)
    assert np.allclose(oracle_mod.energies_at(n, h, J, idx), oracle_mod.energies(n, h, J), rtol=0, atol=1e-12)
