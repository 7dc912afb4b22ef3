"""Write oracle reference values for end-to-end parity tests.

Calls only oracle/ and synth_inputs/ (seeded synthetic inputs).  Usage:
    python tests/golden/make_golden.py o4v12
writes tests/golden/<name>.json with energies, zeta, gradients of every
state and the requested couplings (both orders) at x = 0.
"""
import json
import os
import sys
import time

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import scc  # noqa: E402
from synth_inputs import make_system  # noqa: E402


def main(name):
    torch.set_num_threads(max(1, len(os.sched_getaffinity(0))))
    S = make_system(name)
    t0 = time.time()
    sol = scc.solve_system(S)
    print(f"solve {time.time() - t0:.1f}s E0 {sol.E0} E {sol.E} zeta {sol.zeta}", flush=True)
    targets = [("grad", k) for k in range(S.nstates)]
    for (m, n) in S.nacs:
        targets += [("nac", m, n), ("nac", n, m)]
    out = dict(system=name, seed=S.seed, reading=S.reading, o=S.o, v=S.v, nj=S.nj,
               nstates=S.nstates, ncoord=S.ncoord, E0=sol.E0, E=list(map(float, sol.E)),
               zeta=list(map(float, sol.zeta)), grad={}, nac={})
    for tg in targets:
        t1 = time.time()
        r = scc.gradient_and_nacs(S, sol, [tg])[tg]
        print(f"{tg} {time.time() - t1:.1f}s {r['value']}", flush=True)
        if tg[0] == "grad":
            out["grad"][str(tg[1])] = list(map(float, r["value"]))
        else:
            out["nac"][f"{tg[1]},{tg[2]}"] = list(map(float, r["value"]))
    with open(os.path.join(HERE, f"{name}.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main(sys.argv[1])
