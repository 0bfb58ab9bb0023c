"""CPU oracle for psi(t) = exp(-itH) psi with H = H_P + gamma * sum_j X_j.

TEST INFRASTRUCTURE ONLY.  Only tests/, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no code
with the HIP library (no kernels, headers, tables or helpers); the only common
dependency is ``synth``, which draws the seeded random inputs.

Everything is float64 / complex128.  The element loops that cost O(N) per call
are plain C in ``ref.c`` (built into ``libqworacle.so`` with gcc + OpenMP); the
steps of the method are written here, in the order and notation of
Hopkins & Kendon, "Numerical methods for the simulation of quantum walks and
quantum annealing":

  O0 ``expm_action_dense``   exact result by dense eigendecomposition (sec. II.A).
  O1 ``expm_action``         Chebyshev-Bessel series (Eq. cheb), degree chosen by
                             the truncation tail (Eq. TruncError), spectral shift
                             and induced 1-norm bound (sec. II.A), matrix Clenshaw
                             recurrence (Alg. 2 / Eq. recursion), global phase
                             restored.
  O2 ``cf_real`` / ``cf_coeffs``  Caratheodory-Fejer correction (sec. II.C,
                             Eq. iter) applied to the cos and sin parts.
  O3 ``closed_form_*``       the gamma = 0 and H_P = 0 closed forms.
  O6 ``anneal_cfet4``        fourth-order commutator-free Magnus steps for a
                             time-dependent anneal (sec. III.B), each exponential
                             by O1.
  O7 ``remez_parity``        best approximation by the Remez exchange, the
                             independent check of the CF coefficients (sec. II.C).
  O5 ``horner``              Horner's rule for a polynomial in the monomial basis
                             (Alg. 1), with ``clenshaw`` the evaluation of a
                             caller's Chebyshev series; ``sincos_*_coeffs`` give
                             the sin + cos test function of Figs. 1 and 3 in both
                             bases; ``poly_amps_local`` either basis at sampled
                             outputs, for sizes where no vector fits the host.
  O4 ``anneal_energy_grad``  energy of a piecewise-constant anneal and its
                             gradient by the adjoint of the Clenshaw recurrence
                             (not in the paper; derived from Eq. recursion).

Pins (tests/test_oracle_pins.py) tie each of these to something other than
itself; functions without such a pin say "parity unpinned" in their docstring.
"""
from __future__ import annotations

import ctypes
import functools
import os
import subprocess

import mpmath
import numpy as np
import scipy.special

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ref.c")
_SO = os.path.join(_HERE, "libqworacle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)


def build(force: bool = True) -> str:
    """Compile ref.c into libqworacle.so (gcc, OpenMP)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        lib = ctypes.CDLL(_SO)
        for name in ("orc_energies",):
            getattr(lib, name).restype = None
        lib.orc_energies.argtypes = [ctypes.c_int, _dp, _dp, _dp]
        lib.orc_hmatvec.argtypes = [ctypes.c_int, _dp, ctypes.c_double, _dp, _dp]
        lib.orc_hmatvec.restype = None
        for name in ("orc_clenshaw_step", "orc_clenshaw_final"):
            f = getattr(lib, name)
            f.argtypes = [ctypes.c_int, _dp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                          _dp, _dp, _dp, _dp]
            f.restype = None
        lib.orc_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    assert a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def num_threads() -> int:
    return int(_load().orc_num_threads())


# --------------------------------------------------------------------------
# Operator: H_P diagonal, spectral shift and bound (sec. I, sec. II.A)
# --------------------------------------------------------------------------

def energies(n: int, h: np.ndarray, J: np.ndarray) -> np.ndarray:
    """E(z) = sum_{j<k} J_jk s_j s_k + sum_j h_j s_j, s_j = 1 - 2 bit_j(z).

    Pinned against the diagonal of sum J_jk Z_j Z_k + sum h_j Z_j built from
    Kronecker products of Pauli Z."""
    h = np.ascontiguousarray(h, dtype=np.float64)
    J = np.ascontiguousarray(J, dtype=np.float64)
    assert h.shape == (n,) and J.shape == (n * (n - 1) // 2,)
    E = np.empty(1 << n, dtype=np.float64)
    _load().orc_energies(n, _p(h), _p(J), _p(E))
    return E


def spectral_shift_radius(E: np.ndarray, n: int, gamma: float) -> tuple[float, float]:
    """Shift c and bound r (sec. II.A).

    The diagonal is shifted by c so that its largest and smallest entries have
    equal magnitude; r is the induced 1-norm (largest column sum of |H - cI|).
    Every column of gamma*sum_j X_j holds n entries of magnitude |gamma|, so
    r = max_z |E(z) - c| + n |gamma| = (max E - min E)/2 + n |gamma|."""
    emax = float(np.max(E))
    emin = float(np.min(E))
    c = 0.5 * (emax + emin)
    r = 0.5 * (emax - emin) + n * abs(gamma)
    return c, r


def hmatvec(n: int, d: np.ndarray, g: float, x: np.ndarray) -> np.ndarray:
    """y = d .* x + g * sum_j X_j x (the matrix-free product, sec. II.D)."""
    d = np.ascontiguousarray(d, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.complex128)
    y = np.empty_like(x)
    _load().orc_hmatvec(n, _p(d), float(g), _p(x), _p(y))
    return y


def hamiltonian_dense(n: int, E: np.ndarray, gamma: float) -> np.ndarray:
    """Dense H = diag(E) + gamma * sum_j X_j, with X_j = I (x) .. X .. (x) I built
    by Kronecker products (qubit j = bit j of the index)."""
    N = 1 << n
    X = np.array([[0.0, 1.0], [1.0, 0.0]])
    H = np.diag(np.asarray(E, dtype=np.float64)).copy()
    for j in range(n):
        H += gamma * np.kron(np.kron(np.eye(1 << (n - 1 - j)), X), np.eye(1 << j))
    assert H.shape == (N, N)
    return H


# --------------------------------------------------------------------------
# Coefficients: Chebyshev-Bessel series (Eq. cheb) and degree (Eq. TruncError)
# --------------------------------------------------------------------------

@functools.lru_cache(maxsize=256)
def _bessel_table_abs(x: float, M: int) -> np.ndarray:
    if x == 0.0:
        return (np.arange(M + 1) == 0).astype(np.float64)
    if x <= _MP_LIMIT:
        with mpmath.workdps(30):
            return np.array([float(mpmath.besselj(m, x)) for m in range(M + 1)])
    return scipy.special.jv(np.arange(M + 1, dtype=np.float64), x)


_MP_LIMIT = 800.0


def _bessel_table(a: float, extra: int = 0) -> np.ndarray:
    """J_m(|a|) for m = 0..M, M = |a| + 12|a|^(1/3) + 40 (+extra), past the Airy
    transition where J_m has decayed below 1e-17 of its peak.

    Sec. II.B.1 asks for coefficients correct to about u, so the values come from
    mpmath at 30 digits for |a| <= 800.  Above that scipy.special.jv is used
    (summed absolute error about 5e-12 at |a| = 1400, measured against mpmath),
    which is only needed by the single-precision batched workloads."""
    x = abs(float(a))
    M = int(x + 12.0 * max(x, 1.0) ** (1.0 / 3.0) + 40) + extra
    return _bessel_table_abs(x, M).copy()


def cheb_alpha(a: float) -> np.ndarray:
    """Real series weights alpha_m with exp(-i a x) = sum_m (-i)^m alpha_m T_m(x).

    Eq. cheb gives exp(i a x) = J_0(a) + 2 sum_m i^m J_m(a) T_m(x); replacing a
    by -a (the propagator is exp(-itH)) and J_m(-a) = (-1)^m J_m(a) gives
    alpha_0 = J_0(a), alpha_m = 2 J_m(a)."""
    Jm = _bessel_table(a)
    alpha = 2.0 * Jm
    alpha[0] = Jm[0]
    if a < 0:
        alpha = alpha * (-1.0) ** np.arange(len(alpha))
    return alpha


def cheb_degree(alpha: np.ndarray, tol: float) -> int:
    """Smallest K with sum_{m>K} |alpha_m| <= tol (Eq. TruncError with
    |T_m(x)| <= 1 on [-1, 1])."""
    tail = np.cumsum(np.abs(alpha)[::-1])[::-1]  # tail[m] = sum_{j>=m} |alpha_j|
    for K in range(len(alpha)):
        rest = tail[K + 1] if K + 1 < len(alpha) else 0.0
        if rest <= tol:
            return K
    raise RuntimeError("Bessel table too short for the requested tolerance")


def cheb_coeffs(a: float, tol: float) -> np.ndarray:
    """Complex Chebyshev coefficients c_m = (-i)^m alpha_m, m = 0..K."""
    alpha = cheb_alpha(a)
    K = cheb_degree(alpha, tol)
    m = np.arange(K + 1)
    return ((-1j) ** m) * alpha[:K + 1]


def cheb_series_eval(c: np.ndarray, x: np.ndarray) -> np.ndarray:
    """sum_m c_m T_m(x) for scalar points x (numpy's Chebyshev evaluator)."""
    return np.polynomial.chebyshev.chebval(x, c.real) + 1j * np.polynomial.chebyshev.chebval(x, c.imag)


# --------------------------------------------------------------------------
# Matrix Clenshaw recurrence (Alg. 2, Eq. recursion) and the action itself
# --------------------------------------------------------------------------

def clenshaw(n: int, c: np.ndarray, d: np.ndarray, g: float, v: np.ndarray,
             norms: list | None = None) -> np.ndarray:
    """y = sum_k c_k T_k(H) v for H = diag(d) + g sum_j X_j.

    b_{K+1} = 0, b_K = c_K v, b_k = 2 H b_{k+1} - b_{k+2} + c_k v,
    y = H b_1 - b_2 + c_0 v.  K = 0 returns c_0 v (the printed listing would
    return H c_0 v + c_0 v for a single coefficient).  The update of b_{k+2}
    into b_k is done in place, as in sec. II.D.

    If ``norms`` is a list, (||b_k||, ||c_k v - b_{k+2}||, ||b_{k+1}||) is
    appended for every step k = K, K-1, .., 0, the quantities of the
    evaluation-error bound (sec. II.B.3); the step k = 0 forms the result y, so
    its first entry is ||y||."""
    d = np.ascontiguousarray(d, dtype=np.float64)
    v = np.ascontiguousarray(v, dtype=np.complex128)
    K = len(c) - 1
    if K == 0:
        return c[0] * v
    lib = _load()
    b1 = (c[K] * v).astype(np.complex128)   # b_K
    b2 = np.zeros_like(v)                    # b_{K+1}
    if norms is not None:
        norms.append((np.linalg.norm(b1), np.linalg.norm(b1), 0.0))
    for k in range(K - 1, 0, -1):
        if norms is not None:
            ck_v_minus_b2 = np.linalg.norm(c[k] * v - b2)
            nb1 = np.linalg.norm(b1)
        lib.orc_clenshaw_step(n, _p(d), float(g), float(c[k].real), float(c[k].imag),
                              _p(v), _p(b1), _p(b2), _p(b2))
        b1, b2 = b2, b1                      # b1 <- b_k, b2 <- b_{k+1}
        if norms is not None:
            norms.append((np.linalg.norm(b1), ck_v_minus_b2, nb1))
    y = np.empty_like(v)
    if norms is not None:
        final = (np.linalg.norm(c[0] * v - b2), np.linalg.norm(b1))
    lib.orc_clenshaw_final(n, _p(d), float(g), float(c[0].real), float(c[0].imag),
                           _p(v), _p(b1), _p(b2), _p(y))
    if norms is not None:
        # the last step forms y = p(H) v in the place of b_0, so its rounding
        # term is u ||y||
        norms.append((np.linalg.norm(y), final[0], final[1]))
    return y


def horner(n: int, a: np.ndarray, d: np.ndarray, g: float, v: np.ndarray) -> np.ndarray:
    """y = sum_k a_k H^k v for H = diag(d) + g sum_j X_j by Horner's rule (Alg. 1):
    start from a_K v, then K times y <- H y + a_k v for k = K-1 .. 0."""
    a = np.asarray(a, dtype=np.complex128)
    v = np.ascontiguousarray(v, dtype=np.complex128)
    K = len(a) - 1
    y = a[K] * v
    for k in range(K - 1, -1, -1):
        y = hmatvec(n, d, g, y) + a[k] * v
    return y


def _ball_masks(n: int, R: int):
    """Every n-bit mask of at most R set bits, ordered by bit count (so the masks
    of at most r bits are a prefix, of length sizes[r]), and the table
    nb[i, j] = position of masks[i] ^ 2^j (-1 if that has more than R bits)."""
    import itertools
    masks, sizes = [], []
    for r in range(R + 1):
        for bits in itertools.combinations(range(n), r):
            masks.append(sum(1 << j for j in bits))
        sizes.append(len(masks))
    masks = np.array(masks, dtype=np.int64)
    order = np.argsort(masks)
    sm = masks[order]
    nb = np.full((len(masks), n), -1, dtype=np.int64)
    for j in range(n):
        m = masks ^ (1 << j)
        pos = np.minimum(np.searchsorted(sm, m), len(sm) - 1)
        hit = sm[pos] == m
        nb[hit, j] = order[pos[hit]]
    return masks, sizes, nb


def poly_amps_local(n: int, h: np.ndarray, J: np.ndarray, gamma: float, shift: float,
                    radius: float, coef: np.ndarray, basis: str, factors: np.ndarray,
                    idx: np.ndarray) -> np.ndarray:
    """[p(H~) psi](z) at sampled basis indices z, for H~ = (H - shift) / radius,
    H = diag(E) + gamma sum_j X_j and the product state psi(x) = prod_j
    factors[j, bit_j(x)] (O5 at sizes where no full vector fits the host).

    p = sum_k coef_k T_k (basis "cheb") or sum_k coef_k x^k ("mono").  A degree-K
    polynomial in H~ reaches only the indices within Hamming distance K of z, so
    u_k = T_k(H~) psi (three-term recurrence T_{k+1} = 2 x T_k - T_{k-1},
    sec. II.B) or H~^k psi is formed on the ball of radius K - k around z, where
    every flip partner it needs is defined: (H~ u)(x) = ((E(x) - shift) u(x) +
    gamma sum_j u(x ^ 2^j)) / radius.  E(x) is the SK energy summed by its
    definition (one matrix product over the ball's spins)."""
    coef = np.asarray(coef, dtype=np.complex128)
    K = len(coef) - 1
    masks, sizes, nb = _ball_masks(n, K)
    h = np.asarray(h, dtype=np.float64)
    Jm = np.zeros((n, n))
    Jm[np.triu_indices(n, 1)] = np.asarray(J, dtype=np.float64)
    out = np.empty(len(idx), dtype=np.complex128)
    for q, z in enumerate(np.asarray(idx, dtype=np.int64)):
        x = int(z) ^ masks
        bits = (x[:, None] >> np.arange(n)[None, :]) & 1
        amp = np.prod(np.asarray(factors)[np.arange(n)[None, :], bits], axis=1)
        s = 1.0 - 2.0 * bits
        E = s @ h + np.einsum("pj,jk,pk->p", s, Jm, s)
        dt = (E - shift) / radius
        g = gamma / radius

        def hop(u, m):
            # (H~ u) on the first m ball points; u is defined on a larger prefix
            return dt[:m] * u[:m] + g * u[nb[:m]].sum(axis=1)

        prev, cur = None, amp
        acc = coef[0] * cur[0]
        for k in range(1, K + 1):
            m = sizes[K - k]
            if basis == "cheb":
                nxt = hop(cur, m) if k == 1 else 2.0 * hop(cur, m) - prev[:m]
            else:
                nxt = hop(cur, m)
            prev, cur = cur, nxt
            acc += coef[k] * cur[0]
        out[q] = acc
    return out


def sincos_taylor_coeffs(s: float, K: int) -> np.ndarray:
    """Maclaurin coefficients of sin(s x) + cos(s x) up to x^K (the test function
    of Fig. 1 and Fig. 3): a_m = s^m / m! with sign + for m = 0, 1 (mod 4) and
    - for m = 2, 3 (mod 4)."""
    out = np.empty(K + 1)
    term = 1.0
    for m in range(K + 1):
        if m > 0:
            term *= s / m
        out[m] = term if (m % 4) in (0, 1) else -term
    return out


def sincos_cheb_coeffs(s: float, K: int) -> np.ndarray:
    """Chebyshev coefficients of sin(s x) + cos(s x) on [-1, 1] up to T_K, from the
    Jacobi-Anger expansions (sec. II.B.1): cos(s x) = J_0(s) + 2 sum_{q>=1}
    (-1)^q J_2q(s) T_2q(x) and sin(s x) = 2 sum_{q>=0} (-1)^q J_2q+1(s) T_2q+1(x)."""
    Jm = _bessel_table(float(s), extra=K + 1)[:K + 1]
    out = np.empty(K + 1)
    for m in range(K + 1):
        q = m // 2
        out[m] = (1.0 if m == 0 else 2.0) * (-1.0) ** q * Jm[m]
    return out


def schedule_value(coef, T: float, t: float) -> float:
    """A(t) for a schedule given by monomial coefficients in s = t / T."""
    return float(np.polynomial.polynomial.polyval(t / T, np.asarray(coef, dtype=np.float64)))


def anneal_cfet4(n: int, E: np.ndarray, a_coef, b_coef, T: float, step_sizes, psi: np.ndarray,
                 tols) -> np.ndarray:
    """U(T, 0) psi for H(t) = A(t) diag(E) + B(t) sum_j X_j by the fourth-order
    commutator-free Magnus steps of sec. III.B: a step of length h from t uses
    the two Gauss-Legendre nodes t + (1/2 -+ sqrt(3)/6) h and applies
    exp(-i h (w1 H(t1) + w2 H(t2))) and then exp(-i h (w2 H(t1) + w1 H(t2))),
    w_{1,2} = 1/4 +- sqrt(3)/6; every exponential of alpha diag(E) + beta sum X_j
    is ``expm_action`` (O1) with the energies scaled by alpha.  ``step_sizes``
    lists h for every step, ``tols`` the truncation tolerance of every step's
    two exponentials."""
    r3 = np.sqrt(3.0)
    c1, c2 = 0.5 - r3 / 6.0, 0.5 + r3 / 6.0
    w1, w2 = 0.25 + r3 / 6.0, 0.25 - r3 / 6.0
    E = np.asarray(E, dtype=np.float64)
    y = np.asarray(psi, dtype=np.complex128).copy()
    t = 0.0
    for hs, tol in zip(step_sizes, tols):
        A1, A2 = schedule_value(a_coef, T, t + c1 * hs), schedule_value(a_coef, T, t + c2 * hs)
        B1, B2 = schedule_value(b_coef, T, t + c1 * hs), schedule_value(b_coef, T, t + c2 * hs)
        for alpha, beta in ((w1 * A1 + w2 * A2, w1 * B1 + w2 * B2), (w2 * A1 + w1 * A2, w2 * B1 + w1 * B2)):
            y = expm_action(n, alpha * E, beta, hs, y, tol)
        t += hs
    return y


def evaluation_error_bound(norms: list, n: int, u: float) -> float:
    """Sum over steps of u||b_k|| + u||c_k v - b_{k+2}|| + sqrt(d) gamma_d ||b_{k+1}||
    with d = n + 1 non-zeros per column and gamma_d = d u / (1 - d u)
    (sec. II.B.3, after normalising ||H||_2 <= 1)."""
    dnz = n + 1
    gam = dnz * u / (1.0 - dnz * u)
    return float(sum(u * a + u * b + np.sqrt(dnz) * gam * c for a, b, c in norms))


def expm_action(n: int, E: np.ndarray, gamma: float, t: float, psi: np.ndarray,
                tol: float, method: str = "cheb", info: dict | None = None) -> np.ndarray:
    """psi(t) = exp(-i t H) psi for H = diag(E) + gamma sum_j X_j (O1).

    Steps: shift c and bound r; if r == 0 return exp(-itc) psi; normalised
    d = (E - c)/r, g = gamma/r; a = t r; coefficients of exp(-i a x) chosen for
    truncation error <= tol (Chebyshev, or CF with method="cf"); Clenshaw;
    multiply by the global phase exp(-itc) removed by the shift."""
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    c, r = spectral_shift_radius(E, n, gamma)
    if info is not None:
        info.update(shift_c=c, radius_r=r)
    if r == 0.0:
        return np.exp(-1j * t * c) * psi
    d = (np.asarray(E, dtype=np.float64) - c) / r
    g = gamma / r
    a = t * r
    if method == "cheb":
        coef = cheb_coeffs(a, tol)
    elif method == "cf":
        coef, lam = cf_coeffs(a, tol)
        if info is not None:
            info["cf_lambda"] = lam
    else:
        raise ValueError(method)
    norms = [] if info is not None else None
    y = clenshaw(n, coef, d, g, psi, norms)
    if info is not None:
        info.update(K=len(coef) - 1, a=a, coeffs=coef,
                    eval_bound=evaluation_error_bound(norms, n, 2.0 ** -53))
    return np.exp(-1j * t * c) * y


def expm_action_dense(n: int, E: np.ndarray, gamma: float, t: float, psi: np.ndarray) -> np.ndarray:
    """O0: exp(-itH) psi = Q exp(-it Lambda) Q^T psi from numpy.linalg.eigh (sec. II.A)."""
    H = hamiltonian_dense(n, E, gamma)
    lam, Q = np.linalg.eigh(H)
    return Q @ (np.exp(-1j * t * lam) * (Q.T @ np.asarray(psi, dtype=np.complex128)))


# --------------------------------------------------------------------------
# Closed forms (O3)
# --------------------------------------------------------------------------

def closed_form_gamma0(E: np.ndarray, t: float, psi: np.ndarray) -> np.ndarray:
    """gamma = 0: H is diagonal, psi(t)[z] = exp(-i t E(z)) psi[z]."""
    return np.exp(-1j * t * np.asarray(E)) * psi


def closed_form_hp0(n: int, gamma: float, t: float, psi: np.ndarray) -> np.ndarray:
    """H_P = 0: the X_j commute, so exp(-i t gamma sum X_j) is the product over
    qubits of cos(gamma t) I - i sin(gamma t) X_j, applied one qubit at a time."""
    co, si = np.cos(gamma * t), np.sin(gamma * t)
    M = np.array([[co, -1j * si], [-1j * si, co]])
    T = np.asarray(psi, dtype=np.complex128).reshape((2,) * n)
    for j in range(n):
        ax = n - 1 - j            # C-order axis holding bit j
        T = np.moveaxis(np.tensordot(M, T, axes=([1], [ax])), 0, ax)
    return T.reshape(-1)


def closed_form_hp0_product_amps(factors: np.ndarray, gamma: float, t: float,
                                 idx: np.ndarray) -> np.ndarray:
    """H_P = 0 applied to a product state prod_j phi_j: the output is the product
    state prod_j (cos(gamma t) phi_j - i sin(gamma t) X phi_j); returns its
    amplitudes at the basis indices idx (one O(n) product per index)."""
    co, si = np.cos(gamma * t), np.sin(gamma * t)
    M = np.array([[co, -1j * si], [-1j * si, co]])
    out_f = factors @ M.T                      # row j = M phi_j
    idx = np.asarray(idx, dtype=np.int64)
    amp = np.ones(idx.shape, dtype=np.complex128)
    for j in range(factors.shape[0]):
        amp *= out_f[j, (idx >> j) & 1]
    return amp


def energies_at(n: int, h: np.ndarray, J: np.ndarray, idx: np.ndarray) -> np.ndarray:
    """E(z) = sum_{j<k} J_jk s_j s_k + sum_j h_j s_j at sampled indices z, summed
    by the definition (pure Python loops; small samples only)."""
    out = np.empty(len(idx))
    for q, z in enumerate(np.asarray(idx, dtype=np.int64)):
        z = int(z)
        s = [1.0 - 2.0 * ((z >> j) & 1) for j in range(n)]
        e = sum(h[j] * s[j] for j in range(n))
        p = 0
        for j in range(n):
            for k in range(j + 1, n):
                e += J[p] * s[j] * s[k]
                p += 1
        out[q] = e
    return out


def closed_form_gamma0_amps(n: int, h: np.ndarray, J: np.ndarray, t: float,
                            psi_amps: np.ndarray, idx: np.ndarray) -> np.ndarray:
    """gamma = 0 at sampled indices: exp(-i t E(z)) psi[z], E(z) summed by its
    definition for each sampled z."""
    return np.exp(-1j * t * energies_at(n, h, J, idx)) * np.asarray(psi_amps)


# --------------------------------------------------------------------------
# Caratheodory-Fejer (sec. II.C, Eq. iter)  -- O2
# --------------------------------------------------------------------------

def cf_real(acoef: np.ndarray, m: int) -> tuple[np.ndarray, float]:
    """CF correction of the degree-m truncation of f = sum_j a_j T_j (a_0 not halved).

    Hankel matrix of the tail a_{m+1..M}; eigenpair (lam, u) of largest |lam|;
    Laurent coefficients b_j = a_j for j > m, extended downwards for
    j = m, ..., -m by b_j = -(b_{j+1} u_2 + ... + b_{j+K-1} u_K)/u_1 (u 1-indexed,
    K = M - m); corrected coefficients p_0 = a_0 - b_0, p_j = a_j - b_j - b_{-j}.
    Returns (p[0..m], lam); lam estimates the minimax error."""
    a = np.asarray(acoef, dtype=np.float64)
    M = len(a) - 1
    K = M - m
    if K <= 0:
        p = np.zeros(m + 1)
        p[:M + 1] = a
        return p, 0.0
    Hk = np.zeros((K, K))
    for i in range(K):
        for j in range(K):
            if m + 1 + i + j <= M:
                Hk[i, j] = a[m + 1 + i + j]
    w, V = np.linalg.eigh(Hk)
    sel = int(np.argmax(np.abs(w)))
    lam = float(w[sel])
    u = V[:, sel]
    if abs(u[0]) < 1e-300:
        raise ZeroDivisionError("leading eigenvector entry vanishes")
    # b is stored with offset m: b[j + m] holds b_j for j = -m .. M + K
    b = np.zeros(2 * m + M + K + 2)
    for j in range(m + 1, M + 1):
        b[j + m] = a[j]
    for j in range(m, -m - 1, -1):
        s = 0.0
        for i in range(1, K):
            s += b[j + i + m] * u[i]
        b[j + m] = -s / u[0]
    p = np.empty(m + 1)
    p[0] = a[0] - b[m]
    for j in range(1, m + 1):
        p[j] = a[j] - b[j + m] - b[-j + m]
    return p, lam


def _cf_parts(a: float, K: int, tail_cut: float = 1e-17):
    """CF polynomials of cos(a x) and sin(a x) whose combined degree is at most K.

    cos(ax) has only even Chebyshev coefficients 2(-1)^q J_2q(a) (J_0 for q=0),
    sin(ax) only odd ones 2(-1)^q J_{2q+1}(a).  Their CF problems are set up at
    an odd nominal degree for cos and an even one for sin, so each Hankel matrix
    splits into two blocks instead of having +-lambda pairs."""
    Jm = _bessel_table(a)
    M = len(Jm) - 1
    big = np.max(np.abs(Jm))
    while M > 0 and abs(Jm[M]) < tail_cut * big:
        M -= 1
    mm = np.arange(M + 1)
    ac = np.where(mm % 2 == 0, 2.0 * (-1.0) ** (mm // 2) * Jm[:M + 1], 0.0)
    ac[0] = Jm[0]
    as_ = np.where(mm % 2 == 1, 2.0 * (-1.0) ** ((mm - 1) // 2) * Jm[:M + 1], 0.0)
    if a < 0:
        as_ = -as_
    Kc = K if K % 2 == 0 else K - 1       # even effective degree for cos
    Ks = K if K % 2 == 1 else K - 1       # odd effective degree for sin
    pc, lc = cf_real(ac, Kc + 1)
    if Ks >= 0:
        ps, ls = cf_real(as_, Ks + 1)
    else:
        ps, ls = np.zeros(1), float(np.sum(np.abs(as_)))
    coef = np.zeros(K + 1, dtype=np.complex128)
    coef += pc[:K + 1] if len(pc) >= K + 1 else np.pad(pc, (0, K + 1 - len(pc)))
    coef -= 1j * (ps[:K + 1] if len(ps) >= K + 1 else np.pad(ps, (0, K + 1 - len(ps))))
    return coef, abs(lc) + abs(ls)


def remez_parity(f, parity: int, deg: int, grid: int = 40001, iters: int = 60,
                 rtol: float = 1e-9) -> tuple[np.ndarray, float]:
    """Best (minimax) approximation on [-1, 1] of an even (parity 0) or odd
    (parity 1) function f by polynomials of the same parity and degree <= deg,
    by the Remez exchange (the reference the paper contrasts CF with, sec. II.C).

    By symmetry the problem lives on [0, 1] with the basis T_{2j} (even) or
    T_{2j+1} (odd), j = 0..m, which is a Haar system there (polynomials in x^2,
    times x for odd).  Each step solves sum_j c_j phi_j(x_i) + (-1)^i E = f(x_i)
    on m + 2 reference points, then moves the reference to alternating extrema
    of the error on a fine grid (multi-point exchange), until the largest error
    equals |E| to rtol.  Returns (Chebyshev coefficients of T_0..T_deg, |E|)."""
    m = (deg - parity) // 2
    if m < 0:
        raise ValueError("degree below the parity")
    orders = 2 * np.arange(m + 1) + parity

    def basis(x):
        return np.cos(np.outer(np.arccos(np.clip(x, -1.0, 1.0)), orders))

    # fine grid on [0, 1], denser near the ends; x = 0 is dropped for odd f
    xs = np.sort(0.5 * (1.0 - np.cos(np.pi * np.arange(grid) / (grid - 1))))
    if parity == 1:
        xs = xs[1:]
    fx = f(xs)
    Bx = basis(xs)
    y = 0.5 * (1.0 + np.cos(np.pi * np.arange(m + 2)[::-1] / (m + 1)))
    ref = np.sqrt(y)
    if parity == 1:
        ref[0] = max(ref[0], xs[0])
    E = 0.0
    c = np.zeros(m + 1)
    for _ in range(iters):
        A = np.hstack([basis(ref), ((-1.0) ** np.arange(m + 2))[:, None]])
        sol = np.linalg.solve(A, f(ref))
        c, E = sol[:-1], sol[-1]
        err = fx - Bx @ c
        # local extrema of the error (ends included), then alternating maxima
        idx = [0] + [i for i in range(1, len(xs) - 1)
                     if (err[i] - err[i - 1]) * (err[i + 1] - err[i]) <= 0] + [len(xs) - 1]
        cand = []
        for i in idx:
            if cand and np.sign(err[i]) == np.sign(err[cand[-1]]):
                if abs(err[i]) > abs(err[cand[-1]]):
                    cand[-1] = i
            else:
                cand.append(i)
        while len(cand) > m + 2:   # drop the smaller end
            if abs(err[cand[0]]) < abs(err[cand[-1]]):
                cand.pop(0)
            else:
                cand.pop()
        emax = float(np.max(np.abs(err)))
        if len(cand) == m + 2:
            ref = xs[cand]
        if emax - abs(E) <= rtol * emax:
            break
    out = np.zeros(deg + 1)
    out[orders] = c
    return out, float(abs(E))


def cf_coeffs(a: float, tol: float) -> tuple[np.ndarray, float]:
    """Complex coefficients c_0..c_K of a CF approximation to exp(-i a x) on
    [-1, 1] with |lam_cos| + |lam_sin| <= tol and K as small as possible,
    starting from the Chebyshev degree and lowering it while the estimate holds."""
    Kc = cheb_degree(cheb_alpha(a), tol)
    best = None
    K = Kc
    while K >= 0:
        coef, lam = _cf_parts(a, K)
        if lam > tol:
            break
        best = (coef, lam)
        K -= 1
    if best is None:
        return cheb_coeffs(a, tol), float("nan")
    return best


# --------------------------------------------------------------------------
# Anneal energy and its gradient (O4; not in the paper)
# --------------------------------------------------------------------------

def _segment_setup(n, E, gamma, t, tol):
    c, r = spectral_shift_radius(E, n, gamma)
    d = (E - c) / r
    g = gamma / r
    a = t * r
    alpha = cheb_alpha(a)
    K = cheb_degree(alpha, tol)
    m = np.arange(K + 1)
    coef = ((-1j) ** m) * alpha[:K + 1]
    return dict(c=c, r=r, d=d, g=g, a=a, K=K, coef=coef)


def anneal_forward(n, h, J, gammas, ts, psi0, tol):
    """States psi_s = exp(-i t_s (H_P + gamma_s sum X_j)) psi_{s-1} by O1 and the
    energy E = <psi_S|H_P|psi_S>."""
    E_diag = energies(n, h, J)
    psi = np.ascontiguousarray(psi0, dtype=np.complex128)
    states = [psi]
    for gam, t in zip(gammas, ts):
        psi = expm_action(n, E_diag, float(gam), float(t), psi, tol)
        states.append(psi)
    energy = float(np.real(np.vdot(psi, E_diag * psi)))
    return energy, states, E_diag


def anneal_energy_grad(n, h, J, gammas, ts, psi0, tol):
    """E and dE/d(gamma_s, t_s, h_j, J_jk) by reverse mode through each segment's
    Clenshaw recurrence, with the shift c_s, bound r_s and degree K_s held fixed.

    Per segment, with v = psi_{s-1}, w = p(H~)v, psi_s = phi w, phi = exp(-i t c):
      beta_0 = conj(phi) ybar, beta_1 = H~ beta_0, beta_{k+1} = 2 H~ beta_k - beta_{k-1};
      vbar = sum_k conj(c_k) beta_k (the adjoint passed to segment s-1);
      dL/dd~_i = sum_{k<K} w_k Re(conj(beta_k,i) b_{k+1,i}),
      dL/dg~   = sum_{k<K} w_k Re<beta_k, F b_{k+1}>, w_0 = 1, w_k = 2;
      dL/dc_k  -> Re(dc_k <beta_k, v>), dc_k/dt = r (-i)^k alpha_k'(a),
                  alpha_0' = -J_1, alpha_k' = J_{k-1} - J_{k+1};
      phase:     Re(-i c <ybar, psi_s>).
    Chain rule: dE/dgamma_s = (1/r_s) dL/dg~_s; G_i = sum_s (1/r_s) dL/dd~_{s,i}
    + |psi_S,i|^2; dE/dh_j = sum_i G_i s_j(i); dE/dJ_jk = sum_i G_i s_j(i) s_k(i).
    Loss seed ybar_S = 2 H_P psi_S."""
    lib = _load()
    E_diag = energies(n, h, J)
    S = len(gammas)
    psi = np.ascontiguousarray(psi0, dtype=np.complex128)
    states = [psi]
    segs = []
    for s in range(S):
        sg = _segment_setup(n, E_diag, float(gammas[s]), float(ts[s]), tol)
        segs.append(sg)
        y = clenshaw(n, sg["coef"], sg["d"], sg["g"], psi)
        psi = np.exp(-1j * ts[s] * sg["c"]) * y
        states.append(psi)
    psiT = states[-1]
    energy = float(np.real(np.vdot(psiT, E_diag * psiT)))

    ybar = 2.0 * E_diag * psiT
    G = np.abs(psiT) ** 2
    dgam = np.zeros(S)
    dt = np.zeros(S)
    zero_d = np.zeros(1 << n)
    for s in range(S - 1, -1, -1):
        sg = segs[s]
        v = states[s]
        K, coef, d, g, r, c = sg["K"], sg["coef"], sg["d"], sg["g"], sg["r"], sg["c"]
        phi = np.exp(-1j * ts[s] * c)
        dt[s] += float(np.real(-1j * c * np.vdot(ybar, states[s + 1])))
        # forward b_k of this segment, all stored (b[k] for k = 1..K+1)
        b = [None] * (K + 2)
        b[K + 1] = np.zeros_like(v)
        b[K] = coef[K] * v
        for k in range(K - 1, 0, -1):
            out = np.empty_like(v)
            lib.orc_clenshaw_step(n, _p(d), float(g), float(coef[k].real), float(coef[k].imag),
                                  _p(v), _p(b[k + 1]), _p(b[k + 2]), _p(out))
            b[k] = out
        # ascending adjoint sweep
        Jm = _bessel_table(sg["a"], extra=2)
        sgn = -1.0 if sg["a"] < 0 else 1.0
        beta_prev = None
        beta = np.conj(phi) * ybar
        vbar = np.zeros_like(v)
        dd = np.zeros(1 << n)
        dg = 0.0
        for k in range(0, K + 1):
            vbar += np.conj(coef[k]) * beta
            bv = np.vdot(beta, v)
            if k == 0:
                dalpha = -Jm[1]
            else:
                dalpha = Jm[k - 1] - Jm[k + 1]
            dalpha *= sgn ** (k + 1) if sg["a"] < 0 else 1.0
            dt[s] += float(np.real(r * ((-1j) ** k) * dalpha * bv))
            if k < K:
                wk = 1.0 if k == 0 else 2.0
                dd += wk * np.real(np.conj(beta) * b[k + 1])
                Fb = hmatvec(n, zero_d, 1.0, b[k + 1])
                dg += wk * float(np.real(np.vdot(beta, Fb)))
                Hb = hmatvec(n, d, g, beta)
                nxt = Hb if k == 0 else 2.0 * Hb - beta_prev
                beta_prev, beta = beta, nxt
        dgam[s] = dg / r
        G += dd / r
        ybar = vbar
    zs = np.arange(1 << n, dtype=np.int64)
    spins = 1.0 - 2.0 * ((zs[None, :] >> np.arange(n)[:, None]) & 1)   # (n, N)
    dh = spins @ G
    dJ = np.empty(n * (n - 1) // 2)
    p = 0
    for j in range(n):
        for k in range(j + 1, n):
            dJ[p] = np.dot(G, spins[j] * spins[k])
            p += 1
    return energy, dict(gamma=dgam, t=dt, h=dh, J=dJ)


def anneal_grad_daleckii_krein(n, h, J, gammas, ts, psi0):
    """Exact gradient by dense eigendecomposition (n <= 8): the Frechet derivative
    of exp(-itH) in direction dH is Q (Phi o (Q^T dH Q)) Q^T with
    Phi_ij = (e^{-it l_i} - e^{-it l_j})/(l_i - l_j), Phi_ii = -it e^{-it l_i}.
    Pins O4 independently of the Clenshaw adjoint."""
    E_diag = energies(n, h, J)
    N = 1 << n
    S = len(gammas)
    Us, eig = [], []
    for s in range(S):
        H = hamiltonian_dense(n, E_diag, float(gammas[s]))
        lam, Q = np.linalg.eigh(H)
        Us.append(Q @ np.diag(np.exp(-1j * ts[s] * lam)) @ Q.T)
        eig.append((lam, Q, H))
    states = [np.asarray(psi0, dtype=np.complex128)]
    for s in range(S):
        states.append(Us[s] @ states[-1])
    psiT = states[-1]
    energy = float(np.real(np.vdot(psiT, E_diag * psiT)))
    # adjoint states phi_s = (U_S ... U_{s+1})^dagger H_P psi_T
    phis = [None] * S
    acc = E_diag * psiT
    for s in range(S - 1, -1, -1):
        phis[s] = acc
        acc = Us[s].conj().T @ acc

    def frechet(s, dH):
        lam, Q, _ = eig[s]
        t = ts[s]
        el = np.exp(-1j * t * lam)
        diff = lam[:, None] - lam[None, :]
        with np.errstate(divide="ignore", invalid="ignore"):
            Phi = (el[:, None] - el[None, :]) / diff
        close = np.abs(diff) < 1e-12
        Phi[close] = (-1j * t * el[:, None] * np.ones((1, N)))[close]
        return Q @ (Phi * (Q.T @ dH @ Q)) @ Q.T

    X = np.array([[0.0, 1.0], [1.0, 0.0]])
    F = np.zeros((N, N))
    for j in range(n):
        F += np.kron(np.kron(np.eye(1 << (n - 1 - j)), X), np.eye(1 << j))
    zs = np.arange(N)
    spins = 1.0 - 2.0 * ((zs[None, :] >> np.arange(n)[:, None]) & 1)

    def dE(dHs, dHP):
        tot = float(np.real(np.vdot(psiT, dHP * psiT))) if dHP is not None else 0.0
        for s in range(S):
            if dHs[s] is None:
                continue
            tot += 2.0 * float(np.real(np.vdot(phis[s], frechet(s, dHs[s]) @ states[s])))
        return tot

    dgam = np.array([dE([F if q == s else None for q in range(S)], None) for s in range(S)])
    dt = np.array([2.0 * float(np.real(np.vdot(phis[s], -1j * eig[s][2] @ states[s + 1])))
                   for s in range(S)])
    dh = np.array([dE([np.diag(spins[j])] * S, spins[j]) for j in range(n)])
    dJ = []
    for j in range(n):
        for k in range(j + 1, n):
            w = spins[j] * spins[k]
            dJ.append(dE([np.diag(w)] * S, w))
    return energy, dict(gamma=dgam, t=dt, h=dh, J=np.array(dJ))


def time_clenshaw_terms(n: int, coef: np.ndarray, d: np.ndarray, g: float, v: np.ndarray,
                        terms: int) -> float:
    """Wall-clock seconds of `terms` plain Clenshaw steps (the recurrence loop of
    ``clenshaw``, in place, complex128) starting from b_K = c_K v, b_{K+1} = 0.
    Used only for the CPU baseline of the benchmark."""
    import time
    lib = _load()
    d = np.ascontiguousarray(d, dtype=np.float64)
    K = len(coef) - 1
    terms = min(terms, K - 1)
    b1 = (coef[K] * v).astype(np.complex128)
    b2 = np.zeros_like(b1)
    t0 = time.perf_counter()
    for k in range(K - 1, K - 1 - terms, -1):
        lib.orc_clenshaw_step(n, _p(d), float(g), float(coef[k].real), float(coef[k].imag),
                              _p(v), _p(b1), _p(b2), _p(b2))
        b1, b2 = b2, b1
    return time.perf_counter() - t0
