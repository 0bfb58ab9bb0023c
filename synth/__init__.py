"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only draws random numbers and lays them out; it holds none of the
method's arithmetic (no energies, no spectral bound, no coefficients).  Both the
CPU oracle and the HIP path receive what it returns as plain data.

Workload recipe (Sherrington-Kirkpatrick spin glass, as in the paper's SK test
sets, section II.A, Figs. 3-4):
  * couplings J_jk ~ N(0, 1/n) for j < k, stored as the packed upper triangle in
    row-major order (j outer, k inner);
  * fields h_j ~ N(0, 1);
  * one ``numpy.random.default_rng(seed)`` stream draws J first, then h.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "n_pairs", "pair_index", "sk_instance", "plus_state", "random_state",
    "product_state_factors", "product_state", "basis_state",
    "batch_instances", "anneal_schedule", "product_state_torch", "plus_state_torch",
]


def n_pairs(n: int) -> int:
    """Number of couplings j < k for n spins."""
    return n * (n - 1) // 2


def pair_index(n: int, j: int, k: int) -> int:
    """Offset of J_jk (j < k) in the packed row-major upper triangle."""
    assert 0 <= j < k < n
    return j * n - j * (j + 1) // 2 + (k - j - 1)


def sk_instance(n: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Return (h, J): float64 arrays of length n and n(n-1)/2."""
    rng = np.random.default_rng(seed)
    J = rng.standard_normal(n_pairs(n)) / np.sqrt(n)
    h = rng.standard_normal(n)
    return np.ascontiguousarray(h, dtype=np.float64), np.ascontiguousarray(J, dtype=np.float64)


def plus_state(n: int, dtype=np.complex128) -> np.ndarray:
    """|+>^n: every amplitude 1/sqrt(N)."""
    N = 1 << n
    return np.full(N, 1.0 / np.sqrt(N), dtype=dtype)


def basis_state(n: int, z: int = 0, dtype=np.complex128) -> np.ndarray:
    psi = np.zeros(1 << n, dtype=dtype)
    psi[z] = 1.0
    return psi


def random_state(n: int, seed: int, dtype=np.complex128) -> np.ndarray:
    """Unit-norm state with i.i.d. complex Gaussian amplitudes."""
    rng = np.random.default_rng(seed)
    N = 1 << n
    v = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    v /= np.linalg.norm(v)
    return v.astype(dtype)


def product_state_factors(n: int, seed: int) -> np.ndarray:
    """n random unit 2-vectors phi_j (complex128, shape (n, 2)); qubit j = bit j."""
    rng = np.random.default_rng(seed)
    f = rng.standard_normal((n, 2)) + 1j * rng.standard_normal((n, 2))
    f /= np.linalg.norm(f, axis=1, keepdims=True)
    return f


def product_state(factors: np.ndarray, dtype=np.complex128) -> np.ndarray:
    """Amplitude of z is prod_j factors[j, bit_j(z)] (laid out with bit j = qubit j)."""
    psi = np.ones(1, dtype=np.complex128)
    for j in range(factors.shape[0]):
        # qubit j becomes the new most significant bit of the index
        psi = np.concatenate([psi * factors[j, 0], psi * factors[j, 1]])
    return psi.astype(dtype)


def batch_instances(count: int, seed: int, n_lo: int = 12, n_hi: int = 22,
                    t_lo: float = 0.1, t_hi: float = 20.0,
                    g_lo: float = 0.2, g_hi: float = 2.0):
    """Independent SK instances of uneven size.

    Returns a list of dicts {n, gamma, t, h, J, seed}; n ~ U{n_lo..n_hi},
    t ~ U(t_lo, t_hi), gamma ~ U(g_lo, g_hi); instance i uses SK seed seed*100003+i.
    """
    rng = np.random.default_rng(seed)
    ns = rng.integers(n_lo, n_hi + 1, size=count)
    ts = rng.uniform(t_lo, t_hi, size=count)
    gs = rng.uniform(g_lo, g_hi, size=count)
    out = []
    for i in range(count):
        s = seed * 100003 + i
        h, J = sk_instance(int(ns[i]), s)
        out.append(dict(n=int(ns[i]), gamma=float(gs[i]), t=float(ts[i]), h=h, J=J, seed=s))
    return out


def anneal_schedule(S: int = 16, g_start: float = 2.0, g_end: float = 0.05,
                    t_seg: float = 0.5) -> tuple[np.ndarray, np.ndarray]:
    """Piecewise-constant schedule: gamma_s linear from g_start to g_end, t_s fixed."""
    gam = np.linspace(g_start, g_end, S)
    ts = np.full(S, t_seg)
    return gam.astype(np.float64), ts.astype(np.float64)


def product_state_torch(factors: np.ndarray, device, dtype):
    """Device copy of product_state(factors): the Kronecker product built on the
    GPU one qubit at a time (qubit j = bit j), for sizes too large for the host."""
    import torch
    f = torch.as_tensor(np.asarray(factors), dtype=torch.complex128, device=device)
    psi = f[0].clone()
    for j in range(1, f.shape[0]):
        psi = torch.kron(f[j], psi)     # new qubit becomes the most significant bit
    return psi.to(dtype).contiguous()


def plus_state_torch(n: int, device, dtype):
    import torch
    N = 1 << n
    return torch.full((N,), 1.0 / np.sqrt(N), dtype=dtype, device=device)
