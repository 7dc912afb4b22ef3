"""Time the oracle's CCSD ground-state iteration (residual with full N^4
integrals plus its DIIS step) for a stored golden system and record it next
to the whole-geometry time in tests/golden/<name>.json ("oracle_timing").

Calls only oracle/ and synth_inputs/.  Run it with the thread count of the
golden run (make_golden.py records it), e.g.
    taskset -c 4-7 python tests/golden/time_oracle.py o4v12s3
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


def main(name, iterations=25):
    path = os.path.join(HERE, f"{name}.json")
    rec = json.load(open(path))
    threads = rec["oracle_timing"]["threads"]
    torch.set_num_threads(threads)
    S = make_system(name)
    h, L = S.at(np.zeros(S.ncoord))
    ht, gt = torch.as_tensor(h), cc.chol_to_g(torch.as_tensor(L))
    eps = np.diag(cc.fock(ht, gt, S.o).numpy()).copy()
    c0 = time.perf_counter()
    try:
        scc.solve_ground(ht, gt, S.o, eps, tol=0.0, maxiter=iterations)
    except RuntimeError:
        pass  # tol = 0: stops at the step limit
    best = (time.perf_counter() - c0) / iterations
    rec["oracle_timing"]["ground_iteration_seconds"] = best
    with open(path, "w") as f:
        json.dump(rec, f, indent=1)
    print(f"{name}: {best:.4f} s per ground-state step on {threads} threads")


if __name__ == "__main__":
    main(sys.argv[1])
