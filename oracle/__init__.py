"""Plain FP64 CPU oracle for the SCCSD gradient / coupling path.

TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py may import this package.  It shares no code with
the HIP library (paper_2403_01007_amd/): the two meet only through the seeded
input generator in synth_inputs/ (random draws, no method arithmetic).

  fockspace.py  determinant-space definitions (brute force, tiny systems)
  cc.py         factorised closed-shell SCCSD functions (torch CPU, FP64)
  scc.py        solvers, Lagrange multipliers, gradients and couplings
"""
