"""Write tests/golden/grad_n20_s16.json: the FP64 oracle's anneal energy and
gradient for the 20-qubit, 16-segment schedule (SK seed 0, gamma linear 2 ->
0.05, t_s = 0.5, psi0 = |+>), plus central finite differences (step 1e-3) of the
oracle's forward for a subset of parameters.  Calls only oracle/ and synth/."""
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
    n, S, tol = 20, 16, 1e-12
    h, J = synth.sk_instance(n, 0)
    gam, ts = synth.anneal_schedule(S)
    psi0 = synth.plus_state(n)
    t0 = time.time()
    E, g = oracle.anneal_energy_grad(n, h, J, gam, ts, psi0, tol)
    print(f"oracle adjoint: {time.time() - t0:.1f} s, E = {E}", flush=True)
    step = 1e-3
    subset = {"gamma": [0, 7, 15], "t": [0, 9], "h": [3], "J": [0, 100]}
    fd = {}
    for key, idxs in subset.items():
        for i in idxs:
            vals = []
            for sgn in (+1, -1):
                hh, JJ, gg, tt = h.copy(), J.copy(), gam.copy(), ts.copy()
                {"gamma": gg, "t": tt, "h": hh, "J": JJ}[key][i] += sgn * step
                vals.append(oracle.anneal_forward(n, hh, JJ, gg, tt, psi0, tol)[0])
            fd[f"{key}[{i}]"] = (vals[0] - vals[1]) / (2 * step)
            print(f"fd {key}[{i}] = {fd[f'{key}[{i}]']:.10g}  adjoint {g[key][i]:.10g}", flush=True)
    out = {"n": n, "S": S, "seed": 0, "tol": tol, "schedule": {"gamma": gam.tolist(), "t": ts.tolist()},
           "E": E, "grad": {k: np.asarray(v).tolist() for k, v in g.items()}, "fd_step": step, "fd": fd}
    with open(os.path.join(HERE, "grad_n20_s16.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
