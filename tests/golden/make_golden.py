"""Write oracle reference values for end-to-end parity tests.

Calls only oracle/ and synth_inputs/ (seeded synthetic inputs).  Usage:
    python tests/golden/make_golden.py o4v12            (every coupling in both orders)
    python tests/golden/make_golden.py o4v12s3 --one-order
writes tests/golden/<name>.json with energies, zeta, gradients of every
state and the requested couplings at x = 0.  It also records the oracle's
own wall time for the whole geometry and for its CCSD ground-state solve
alone (the ratio is the oracle's cost per geometry in units of its own
ground-state solve, which the benchmark's CPU baseline uses).
"""
import json
import os
import sys
import time

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import cc, scc  # noqa: E402
from synth_inputs import make_system  # noqa: E402


def ground_seconds(S):
    """Wall time of the oracle's CCSD ground-state solve at x = 0 (the
    sample the benchmark times at its own workload)."""
    h, L = S.at(np.zeros(S.ncoord))
    ht, gt = torch.as_tensor(h), cc.chol_to_g(torch.as_tensor(L))
    eps = np.diag(cc.fock(ht, gt, S.o).numpy()).copy()
    c0 = time.perf_counter()
    scc.solve_ground(ht, gt, S.o, eps)
    return time.perf_counter() - c0


def main(name, both_orders=True):
    threads = max(1, len(os.sched_getaffinity(0)))
    torch.set_num_threads(threads)
    S = make_system(name)
    t0 = time.time()
    sol = scc.solve_system(S)
    t_solve = time.time() - t0
    print(f"solve {t_solve:.1f}s E0 {sol.E0} E {sol.E} zeta {sol.zeta}", flush=True)
    targets = [("grad", k) for k in range(S.nstates)]
    for (m, n) in S.nacs:
        targets += [("nac", m, n)] + ([("nac", n, m)] if both_orders else [])
    out = dict(system=name, seed=S.seed, reading=S.reading, o=S.o, v=S.v, nj=S.nj,
               nstates=S.nstates, ncoord=S.ncoord, E0=sol.E0, E=list(map(float, sol.E)),
               zeta=list(map(float, sol.zeta)), grad={}, nac={})
    t_targets = 0.0
    for tg in targets:
        t1 = time.time()
        r = scc.gradient_and_nacs(S, sol, [tg])[tg]
        t_targets += time.time() - t1
        print(f"{tg} {time.time() - t1:.1f}s {r['value']}", flush=True)
        if tg[0] == "grad":
            out["grad"][str(tg[1])] = list(map(float, r["value"]))
        else:
            out["nac"][f"{tg[1]},{tg[2]}"] = list(map(float, r["value"]))
    out["oracle_timing"] = dict(threads=threads, solve_seconds=t_solve, targets_seconds=t_targets,
                                ground_seconds=ground_seconds(S),
                                targets=[list(map(str, t)) for t in targets])
    with open(os.path.join(HERE, f"{name}.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main(sys.argv[1], both_orders="--one-order" not in sys.argv[2:])
