"""Write tests/golden/action_n28_bench.json: 4096 sampled amplitudes and the
norm of the oracle's exp(-itH)psi for the 28-qubit benchmark workload (SK seed
0, gamma = 1, t = 5, psi0 = |+>), at truncation tolerance 1e-13 (the reference
for complex64 at 2^-23) and at 1e-12 (the complex128 setting, same degree K).
Calls only oracle/ and synth/.  Needs about 30 GB of host memory and a few
minutes per tolerance on 8 cores."""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402


def main():
    n, gamma, t = 28, 1.0, 5.0
    h, J = synth.sk_instance(n, 0)
    E = oracle.energies(n, h, J)
    psi = synth.plus_state(n)
    rng = np.random.default_rng(28)
    idx = np.unique(np.concatenate([[0, 1, (1 << n) - 1], rng.integers(0, 1 << n, 4093)]))
    out = {"n": n, "gamma": gamma, "t": t, "seed": 0, "psi0": "plus", "idx": idx.tolist(), "runs": {}}
    for tol in (1e-13, 1e-12):
        c, r = oracle.spectral_shift_radius(E, n, gamma)
        K = len(oracle.cheb_coeffs(t * r, tol)) - 1
        t0 = time.time()
        y = oracle.expm_action(n, E, gamma, t, psi, tol)
        print(f"tol {tol}: K = {K}, {time.time() - t0:.1f} s", flush=True)
        out["runs"][repr(tol)] = {"K": K, "norm": float(np.linalg.norm(y)),
                                  "re": y[idx].real.tolist(), "im": y[idx].imag.tolist()}
        del y
    with open(os.path.join(HERE, "action_n28_bench.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
