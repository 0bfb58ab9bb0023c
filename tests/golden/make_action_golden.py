"""Write tests/golden/action_n24.json: sampled amplitudes of the oracle's
exp(-itH)psi for the 24-qubit SK workload (seed 0, gamma = 0.8, t = 10,
psi0 = |+>) at truncation tolerance 1e-13 and at 1e-12 (the complex128 GPU
setting, same degree K), with the norm of the full result.  Calls only oracle/
and synth/.  Takes a few minutes on 8 cores."""
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
    n, gamma, t = 24, 0.8, 10.0
    h, J = synth.sk_instance(n, 0)
    E = oracle.energies(n, h, J)
    psi = synth.plus_state(n)
    rng = np.random.default_rng(24)
    idx = np.unique(np.concatenate([[0, 1, (1 << n) - 1], rng.integers(0, 1 << n, 4093)]))
    out = {"n": n, "gamma": gamma, "t": t, "seed": 0, "psi0": "plus", "idx": idx.tolist(), "runs": {}}
    for tol in (1e-13, 1e-12):
        info = {}
        t0 = time.time()
        y = oracle.expm_action(n, E, gamma, t, psi, tol, info=info)
        print(f"tol {tol}: K = {info['K']}, {time.time() - t0:.1f} s", flush=True)
        out["runs"][repr(tol)] = {"K": info["K"], "norm": float(np.linalg.norm(y)),
                                  "re": y[idx].real.tolist(), "im": y[idx].imag.tolist()}
        del y
    with open(os.path.join(HERE, "action_n24.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
