"""SK energies of every basis state formed on the GPU by torch from their
definition, for tests that hand the library a caller diagonal at sizes where
the host cannot hold one."""


def energies_torch(torch, n, h, J, dtype):
    """E(z) = sum_{j<k} J_jk s_j s_k + sum_j h_j s_j, s_j = 1 - 2 bit_j(z), for
    every z: float64 matrix products over chunks of indices on the device,
    rounded once to dtype."""
    dev = "cuda"
    hv = torch.as_tensor(h, dtype=torch.float64, device=dev)
    Jm = torch.zeros((n, n), dtype=torch.float64, device=dev)
    iu = torch.triu_indices(n, n, 1, device=dev)
    Jm[iu[0], iu[1]] = torch.as_tensor(J, dtype=torch.float64, device=dev)
    E = torch.empty(1 << n, dtype=dtype, device=dev)
    ar = torch.arange(n, device=dev)
    chunk = min(1 << n, 1 << 22)
    for lo in range(0, 1 << n, chunk):
        z = torch.arange(lo, lo + chunk, device=dev, dtype=torch.int64)
        s = 1.0 - 2.0 * ((z[:, None] >> ar[None, :]) & 1).to(torch.float64)
        E[lo:lo + chunk] = (s @ hv + ((s @ Jm) * s).sum(dim=1)).to(dtype)
    return E
