"""End-to-end GPU parity through the C ABI: energies, zeta, gradients of every
state and couplings (both orders) against the FP64 oracle.

Tolerances are those the method is held to: 1e-10 Eh in energies and 1e-8 in
gradients and couplings (absolute, in Hartree per unit coordinate).
"""
import json
import os

import numpy as np
import pytest

from synth_inputs import make_system

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
E_TOL, G_TOL = 1e-10, 1e-8


def _run_gpu(S, scc=True, tol=1e-11):
    from paper_2403_01007_amd import Context
    h, L = S.at(np.zeros(S.ncoord))
    ctx = Context(S.o, S.v, S.nj, S.nstates, tol=tol, tol_overlap=1e-12, scc=scc)
    ctx.set_hamiltonian(h, L)
    E, z, _ = ctx.excited()
    e0 = float(ctx.get(3).cpu()[0])
    grads = {k: ctx.gradient(k, S.dh, S.dL)[0] for k in range(S.nstates)}
    nacs = {}
    for (m, n) in S.nacs:
        nacs[(m, n)] = ctx.nac(m, n, S.dh, S.dL)[0]
        nacs[(n, m)] = ctx.nac(n, m, S.dh, S.dL)[0]
    return ctx, e0, E, z, grads, nacs


def _compare(S, gpu, E0, E, zeta, grads, nacs, ztol=1e-7):
    _, e0, Eg, zg, gg, ng = gpu
    assert abs(e0 - E0) < E_TOL
    assert np.abs(np.asarray(Eg) - np.asarray(E)).max() < E_TOL
    if len(zeta):
        assert np.abs(np.asarray(zg) - np.asarray(zeta)).max() < ztol
    for k, ref in grads.items():
        err = np.abs(gg[k] - np.asarray(ref)).max()
        print(f"  grad {k} max err {err:.2e}", flush=True)
        assert err < G_TOL
    for key, ref in nacs.items():
        err = np.abs(ng[key] - np.asarray(ref)).max()
        print(f"  nac {key} max err {err:.2e}", flush=True)
        assert err < G_TOL


@pytest.mark.parametrize("scc", [True, False], ids=["sccsd", "ccsd"])
def test_o2v4_against_live_oracle(scc):
    from oracle import scc as oscc
    S = make_system("o2v4")
    print(f"[o2v4 scc={scc}]", flush=True)
    gpu = _run_gpu(S, scc=scc)
    sol = oscc.solve_system(S, scc=scc)
    targets = [("grad", k) for k in range(S.nstates)]
    for (m, n) in S.nacs:
        targets += [("nac", m, n), ("nac", n, m)]
    ref = oscc.gradient_and_nacs(S, sol, targets)
    grads = {k: ref[("grad", k)]["value"] for k in range(S.nstates)}
    nacs = {}
    for (m, n) in S.nacs:
        nacs[(m, n)] = ref[("nac", m, n)]["value"]
        nacs[(n, m)] = ref[("nac", n, m)]["value"]
    zeta = np.asarray(sol.zeta) if scc else []
    if not scc:
        assert np.all(gpu[3] == 0.0)
    _compare(S, gpu, sol.E0, sol.E, zeta, grads, nacs)


def test_single_state_has_no_constraint():
    """One excited state: no pair, so no zeta and no orthogonality condition;
    the SCCSD state is the EOM-CCSD state.  Energy and gradient of the state
    through the lockstep path (one target, no couplings) against the live
    oracle."""
    from oracle import scc as oscc
    from paper_2403_01007_amd import Context
    S = make_system("o2v4", nstates=1, nacs=[])
    print("[o2v4 one state]", flush=True)
    h, L = S.at(np.zeros(S.ncoord))
    ctx = Context(S.o, S.v, S.nj, S.nstates, tol=1e-11, tol_overlap=1e-12)
    ctx.set_hamiltonian(h, L)
    E, _, _ = ctx.excited()
    e0 = float(ctx.get(3).cpu()[0])
    g, d, _ = ctx.gradients_and_couplings([0], [], S.dh, S.dL)
    sol = oscc.solve_system(S)
    ref = oscc.gradient_and_nacs(S, sol, [("grad", 0)])[("grad", 0)]["value"]
    assert abs(e0 - sol.E0) < E_TOL
    assert abs(E[0] - sol.E[0]) < E_TOL
    err = np.abs(g[0] - np.asarray(ref)).max()
    print(f"  grad max err {err:.2e}", flush=True)
    assert err < G_TOL


def test_o4v12_against_stored_oracle():
    """o4v12 (two states, SCC active) against values written by
    tests/golden/make_golden.py, which calls only the oracle."""
    with open(os.path.join(HERE, "golden", "o4v12.json")) as f:
        ref = json.load(f)
    S = make_system("o4v12")
    assert (S.seed, S.reading, S.o, S.v, S.nj) == (ref["seed"], ref["reading"], ref["o"], ref["v"], ref["nj"])
    print("[o4v12 golden]", flush=True)
    gpu = _run_gpu(S)
    grads = {int(k): v for k, v in ref["grad"].items()}
    nacs = {tuple(int(x) for x in k.split(",")): v for k, v in ref["nac"].items()}
    _compare(S, gpu, ref["E0"], ref["E"], ref["zeta"], grads, nacs)


def test_two_electron_exact():
    """Two electrons: CCSD is exact, SCC is inactive (no triples), so the
    energies are singlet FCI eigenvalues, the gradients Hellmann-Feynman
    expectation values and the couplings <m|H1|n>/(E_n - E_m)."""
    from oracle.fockspace import FockSpace, singlet_fci
    S = make_system("o1v5")
    print("[o1v5]", flush=True)
    h, L = S.at(np.zeros(S.ncoord))
    g = np.einsum("Jpq,Jrs->pqrs", L, L)
    fs = FockSpace(S.o + S.v, S.o)
    w, U = singlet_fci(fs, fs.hamiltonian(h, g), 1 + S.nstates)
    ctx, e0, E, z, grads, nacs = _run_gpu(S)
    assert abs(e0 - w[0]) < E_TOL
    assert np.abs(np.asarray(E) - w[1:1 + S.nstates]).max() < E_TOL
    # phase-match each FCI vector to the library's state exp(T)(R0 + R1 + R2)|HF>
    nov = S.o * S.v
    tv = ctx.get(0).cpu().numpy()
    T = fs.expm(fs.cluster_op(tv[:nov].reshape(S.v, S.o), tv[nov:].reshape(S.v, S.o, S.v, S.o)))
    vecs = []
    for k in range(S.nstates):
        r = ctx.get(1, k).cpu().numpy()
        psi = T @ fs.vector(float(r[0]), r[1:1 + nov].reshape(S.v, S.o), r[1 + nov:].reshape(S.v, S.o, S.v, S.o))
        u = U[:, 1 + k] * np.sign(U[:, 1 + k] @ psi)
        assert abs(abs(u @ psi) - 1.0) < 1e-9     # O_kk = 1 is the FCI norm for two electrons
        vecs.append(u)
    for c in range(S.ncoord):
        g1 = np.einsum("Jpq,Jrs->pqrs", S.dL[c], L) + np.einsum("Jpq,Jrs->pqrs", L, S.dL[c])
        H1 = fs.hamiltonian(S.dh[c], g1)
        for k in range(S.nstates):
            ref = vecs[k] @ H1 @ vecs[k]
            assert abs(grads[k][c] - ref) < G_TOL
        for (m, n) in S.nacs:
            for a, b in [(m, n), (n, m)]:
                ref = vecs[a] @ H1 @ vecs[b] / (w[1 + b] - w[1 + a])
                assert abs(nacs[(a, b)][c] - ref) < G_TOL
            assert abs(nacs[(m, n)][c] + nacs[(n, m)][c]) < G_TOL


def test_call_order_and_input_errors():
    from paper_2403_01007_amd import Context
    from paper_2403_01007_amd.binding import SccError
    S = make_system("o2v4")
    print("[errors]", flush=True)
    h, L = S.at(np.zeros(S.ncoord))
    ctx = Context(S.o, S.v, S.nj, S.nstates)
    with pytest.raises(SccError) as e:
        ctx.excited()
    assert e.value.code == -2  # SCC_ESTATE: no Hamiltonian yet
    # a non-Hartree-Fock basis (rotated orbitals) is rejected
    rng = np.random.default_rng(0)
    X = rng.normal(size=(S.o + S.v, S.o + S.v)) * 0.05
    U = np.linalg.qr(np.eye(S.o + S.v) + X - X.T)[0]
    with pytest.raises(SccError) as e:
        ctx.set_hamiltonian(U.T @ h @ U, np.einsum("pr,Jrs,sq->Jpq", U.T, L, U))
    assert e.value.code == -1  # SCC_EINVAL
    ctx.set_hamiltonian(h, L)
    with pytest.raises(SccError) as e:
        ctx.gradient(0, S.dh, S.dL)
    assert e.value.code == -2  # gradient before the excited states
    ctx.excited()
    with pytest.raises(SccError) as e:
        ctx.gradient(S.nstates, S.dh, S.dL)
    assert e.value.code == -1


def test_deterministic():
    """Two runs on the same inputs give bitwise identical results."""
    S = make_system("o2v4")
    print("[determinism]", flush=True)
    a = _run_gpu(S)
    b = _run_gpu(S)
    assert a[1] == b[1]
    assert np.array_equal(a[2], b[2]) and np.array_equal(a[3], b[3])
    for k in a[4]:
        assert np.array_equal(a[4][k], b[4][k])
    for k in a[5]:
        assert np.array_equal(a[5][k], b[5][k])


def test_fp32_product_residual_is_close():
    """Reduced-precision pass: FP32 products with FP32 accumulation in the
    dense contractions keep the residual within single-precision error of
    the FP64 oracle."""
    import torch
    from oracle import cc
    from paper_2403_01007_amd import Context
    from synth_inputs import random_amplitudes
    S = make_system("o5v19", seed=7)
    print("[fp32 residual o5v19]", flush=True)
    h, L = S.at(np.zeros(S.ncoord))
    ctx = Context(S.o, S.v, S.nj, S.nstates, precision="fp32")
    ctx.set_hamiltonian(h, L)
    t1, t2 = random_amplitudes(S.o, S.v, seed=5, scale=0.05)
    out = ctx.eval_residual(np.concatenate([t1.ravel(), t2.ravel()])).cpu().numpy()
    T = lambda a: torch.as_tensor(np.asarray(a), dtype=torch.float64)
    g = np.einsum("Jpq,Jrs->pqrs", L, L)
    E, s, d = cc.residual(T(h), T(g), T(t1), T(t2), S.o)
    ref = np.concatenate([[float(E)], s.numpy().ravel(), d.numpy().ravel()])
    err = np.abs(out - ref).max() / np.abs(ref).max()
    print(f"  relative max error {err:.2e}", flush=True)
    assert 1e-12 < err < 1e-5   # FP32 rounding is visible, and bounded


@pytest.mark.parametrize("name", ["o2v4", "o4v12"])
def test_fp32_then_fp64_refinement_matches_fp64(name):
    """precision=1: the FP32-product pass followed by FP64 refinement reaches
    the FP64 results to the FP64 tolerances."""
    from paper_2403_01007_amd import Context
    S = make_system(name)
    print(f"[mixed {name}]", flush=True)
    ref = _run_gpu(S)
    h, L = S.at(np.zeros(S.ncoord))
    ctx = Context(S.o, S.v, S.nj, S.nstates, tol=1e-11, tol_overlap=1e-12, precision="fp32")
    ctx.set_hamiltonian(h, L)
    E, z, _ = ctx.excited()
    assert np.abs(E - ref[2]).max() < E_TOL
    for k in range(S.nstates):
        assert np.abs(ctx.gradient(k, S.dh, S.dL)[0] - ref[4][k]).max() < G_TOL
    for (m, n) in S.nacs:
        assert np.abs(ctx.nac(m, n, S.dh, S.dL)[0] - ref[5][(m, n)]).max() < G_TOL


def test_fixed_basis_displaced_geometry():
    """Hamiltonian given in the fixed basis at a displaced geometry: RHF on
    the device, then energies, gradients and couplings (derivative integrals
    in the fixed basis) against the oracle's RHF + SCCSD at the same x."""
    import torch
    from oracle import scc as oscc
    from paper_2403_01007_amd import Context
    S = make_system("o2v4")
    x = 0.05 * np.random.default_rng(3).normal(size=S.ncoord)
    print("[fixed basis o2v4, displaced]", flush=True)
    h, L = S.at(x)
    ctx = Context(S.o, S.v, S.nj, S.nstates, tol=1e-11, tol_overlap=1e-12)
    C, info = ctx.set_hamiltonian_fixed_basis(h, L)
    E, z, _ = ctx.excited()
    sol = oscc.solve_system(S, x=x)
    assert np.abs(C.cpu().numpy() - np.asarray(sol.C)).max() < 1e-9
    assert np.abs(E - np.asarray(sol.E)).max() < E_TOL
    targets = [("grad", k) for k in range(S.nstates)]
    for (m, n) in S.nacs:
        targets += [("nac", m, n), ("nac", n, m)]
    ref = oscc.gradient_and_nacs(S, sol, targets)
    for k in range(S.nstates):
        err = np.abs(ctx.gradient(k, S.dh, S.dL)[0] - ref[("grad", k)]["value"]).max()
        print(f"  grad {k} max err {err:.2e}", flush=True)
        assert err < G_TOL
    for (m, n) in S.nacs:
        for a, b in [(m, n), (n, m)]:
            err = np.abs(ctx.nac(a, b, S.dh, S.dL)[0] - ref[("nac", a, b)]["value"]).max()
            print(f"  nac {(a, b)} max err {err:.2e}", flush=True)
            assert err < G_TOL
    # densities come back in the fixed basis
    d1, z3, kb = ctx.densities(1, S.nacs[0][1], S.nacs[0][0])
    d1_ref = ref[("nac", S.nacs[0][1], S.nacs[0][0])]["D1"]
    assert np.abs(d1.cpu().numpy() - d1_ref).max() < 1e-9 * max(1.0, np.abs(d1_ref).max())


def test_graph_replays_match_eager_launches():
    """Programs captured as HIP graphs and replayed many times (with other
    programs and host synchronisations in between) give bitwise the results
    of launching every kernel eagerly."""
    from paper_2403_01007_amd import Context
    from synth_inputs import random_amplitudes
    S = make_system("o2v4")
    print("[graphs vs eager o2v4]", flush=True)
    h, L = S.at(np.zeros(S.ncoord))
    t1, t2 = random_amplitudes(S.o, S.v, seed=5, scale=0.05)
    t = np.concatenate([t1.ravel(), t2.ravel()])
    r1, r2 = random_amplitudes(S.o, S.v, seed=6, scale=0.3)
    vec = np.concatenate([[0.3], r1.ravel(), r2.ravel()])
    outs = []
    for eager in (True, False):
        ctx = Context(S.o, S.v, S.nj, S.nstates, eager=eager)
        ctx.set_hamiltonian(h, L)
        reps = []
        for _ in range(4):
            reps.append(ctx.eval_residual(t).cpu().numpy())
            reps.append(ctx.eval_sigma(vec).cpu().numpy())
            reps.append(ctx.eval_left(vec).cpu().numpy())
        outs.append(reps)
        E, z, _ = ctx.excited()
        outs[-1].append(E)
        outs[-1].append(ctx.gradient(0, S.dh, S.dL)[0])
        outs[-1].append(ctx.nac(0, 1, S.dh, S.dL)[0])
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a, b)
    for k in range(3, 12):
        assert np.array_equal(outs[1][k], outs[1][k % 3])


def test_batched_targets_match_single_target_solves():
    """scc_gradients_and_couplings (all targets in lockstep) reproduces the
    one-target-at-a-time results."""
    S = make_system("o5v19", seed=7)
    print("[batched targets o5v19]", flush=True)
    ctx, e0, E, z, grads, nacs = _run_gpu(S)
    pairs = list(S.nacs) + [(n, m) for (m, n) in S.nacs]
    g, d, info = ctx.gradients_and_couplings(list(range(S.nstates)), pairs, S.dh, S.dL)
    for k in range(S.nstates):
        assert np.abs(g[k] - grads[k]).max() < 1e-9
    for i, p in enumerate(pairs):
        assert np.abs(d[i] - nacs[p]).max() < 1e-9


def test_consecutive_geometries_on_one_context():
    """Three displaced geometries solved one after another on one context
    (gradients and couplings of every target in lockstep) give the results of
    a fresh context per geometry: no state leaks from one geometry into the
    next, and every call releases the solver memory it used (a call that did
    not is reported as an error by the library)."""
    from paper_2403_01007_amd import Context
    from synth_inputs import family_geometries
    S = make_system("o5v19", seed=7)
    print("[three geometries on one context o5v19]", flush=True)
    pairs = list(S.nacs) + [(n, m) for (m, n) in S.nacs]
    states = list(range(S.nstates))

    def solve(ctx, x):
        h, L = S.at(x)
        ctx.set_hamiltonian_fixed_basis(h, L)
        E, z, _ = ctx.excited()
        g, d, _ = ctx.gradients_and_couplings(states, pairs, S.dh, S.dL)
        return E, z, g, d

    shared = Context(S.o, S.v, S.nj, S.nstates, tol=1e-11, tol_overlap=1e-12)
    for i, x in enumerate(family_geometries(S.ncoord, range(20000, 20003))):
        a = solve(shared, x)
        fresh = Context(S.o, S.v, S.nj, S.nstates, tol=1e-11, tol_overlap=1e-12)
        b = solve(fresh, x)
        fresh.close()
        print(f"  geometry {i}: E {a[0]}", flush=True)
        assert np.abs(a[0] - b[0]).max() < E_TOL
        assert np.abs(a[1] - b[1]).max() < 1e-9
        assert np.abs(a[2] - b[2]).max() < G_TOL
        assert np.abs(a[3] - b[3]).max() < G_TOL


def test_failure_paths():
    """Error semantics of the boundary, forced from the host: an iteration
    limit (SCC_ENOCONV), a workspace below the required size (SCC_ENOMEM),
    and guesses that are not finite (rejected by their residual, with the
    plain start used instead)."""
    import ctypes

    import torch
    from paper_2403_01007_amd import Context, binding
    from paper_2403_01007_amd.binding import SccError
    S = make_system("o2v4")
    print("[failure paths o2v4]", flush=True)
    h, L = S.at(np.zeros(S.ncoord))
    # iteration limit
    ctx = Context(S.o, S.v, S.nj, S.nstates, max_iter=2)
    ctx.set_hamiltonian(h, L)
    with pytest.raises(SccError) as e:
        ctx.ground()
    assert e.value.code == -3
    with pytest.raises(SccError) as e:
        ctx.excited()
    assert e.value.code == -3
    ctx.close()
    # workspace one byte short of the required size
    lib = binding.load_library()
    dims = binding.Dims(S.o, S.v, S.nj, S.nstates)
    opts = binding.Options(1e-10, 1e-11, 200, 1, 0, 0, 0)
    need = binding.workspace_bytes(S.o, S.v, S.nj, S.nstates, opts)
    ws = torch.empty(need + 256, dtype=torch.uint8, device="cuda:0")
    base = (ws.data_ptr() + 255) // 256 * 256
    handle = ctypes.c_void_p()
    rc = lib.scc_create(ctypes.byref(dims), ctypes.byref(opts), ctypes.c_void_p(base), need - 1, None,
                        ctypes.byref(handle))
    assert rc == -7 and not handle.value
    # non-finite guesses: the plain start is used and the solution is unchanged
    ref = Context(S.o, S.v, S.nj, S.nstates, tol=1e-11, tol_overlap=1e-12)
    ref.set_hamiltonian(h, L)
    e_ref, _ = ref.ground()
    E_ref, z_ref, _ = ref.excited()
    ctx = Context(S.o, S.v, S.nj, S.nstates, tol=1e-11, tol_overlap=1e-12)
    ctx.set_hamiltonian(h, L)
    nov = S.o * S.v
    bad_t = np.full(nov + nov * nov, np.nan)
    e0, info = ctx.ground(bad_t)
    assert info.fallback_used == 1 and info.converged == 1
    assert abs(e0 - e_ref) < E_TOL
    nst = 1 + nov + nov * nov
    npair = S.nstates * (S.nstates - 1) // 2
    bad_r = np.full(S.nstates * nst + npair, np.nan)
    E, z, info = ctx.excited(bad_r)
    assert info.fallback_used == 1 and info.converged == 1
    assert np.abs(E - E_ref).max() < E_TOL
    assert np.abs(z - z_ref).max() < 1e-9
    # a bad target and a bad coordinate count are rejected before any work
    with pytest.raises(SccError) as e:
        ctx.densities(1, 0, 0)
    assert e.value.code == -1


@pytest.mark.parametrize("name", ["o4v12s3", "o6v26"])
def test_three_state_batched_targets_against_stored_oracle(name):
    """Three states, their three gradients and the three couplings (0,1),
    (0,2), (1,2) over six coordinates, all targets solved in lockstep by
    scc_gradients_and_couplings (the path the benchmark times), against
    values written by tests/golden/make_golden.py, which calls only the
    oracle (dense EOM at o4v12s3, Davidson at o6v26)."""
    path = os.path.join(HERE, "golden", f"{name}.json")
    if not os.path.exists(path):
        pytest.skip(f"tests/golden/{name}.json not written (the oracle's complete o6v26 run takes hours)")
    with open(path) as f:
        ref = json.load(f)
    from paper_2403_01007_amd import Context
    S = make_system(name)
    assert (S.seed, S.reading, S.o, S.v, S.nj) == (ref["seed"], ref["reading"], ref["o"], ref["v"], ref["nj"])
    print(f"[{name} golden, batched targets]", flush=True)
    h, L = S.at(np.zeros(S.ncoord))
    ctx = Context(S.o, S.v, S.nj, S.nstates, tol=1e-11, tol_overlap=1e-12)
    ctx.set_hamiltonian(h, L)
    E, z, _ = ctx.excited()
    e0 = float(ctx.get(3).cpu()[0])
    print(f"  E0 err {abs(e0 - ref['E0']):.2e}, E err {np.abs(E - np.asarray(ref['E'])).max():.2e}, "
          f"zeta err {np.abs(z - np.asarray(ref['zeta'])).max():.2e}", flush=True)
    assert abs(e0 - ref["E0"]) < E_TOL
    assert np.abs(E - np.asarray(ref["E"])).max() < E_TOL
    assert np.abs(z - np.asarray(ref["zeta"])).max() < 1e-7
    states = list(range(S.nstates))
    g, d, _ = ctx.gradients_and_couplings(states, list(S.nacs), S.dh, S.dL)
    for k in states:
        err = np.abs(g[k] - np.asarray(ref["grad"][str(k)])).max()
        print(f"  grad {k} max err {err:.2e}", flush=True)
        assert err < G_TOL
    for i, (m, n) in enumerate(S.nacs):
        err = np.abs(d[i] - np.asarray(ref["nac"][f"{m},{n}"])).max()
        print(f"  nac {(m, n)} max err {err:.2e}", flush=True)
        assert err < G_TOL


def test_multiplier_guesses():
    """Starting multipliers for the lockstep gradient/coupling solve: the
    converged multipliers of a solve restart it in a few Krylov steps with
    the same results; a perturbed guess takes fewer steps than the zero
    start; a guess that is not finite is dropped (fallback_used) and changes
    nothing."""
    import torch
    S = make_system("o5v19", seed=7)
    print("[multiplier guesses o5v19]", flush=True)
    ctx, e0, E, z, grads, nacs = _run_gpu(S)
    pairs = list(S.nacs) + [(n, m) for (m, n) in S.nacs]
    states = list(range(S.nstates))
    g0, d0, info0, M = ctx.gradients_and_couplings(states, pairs, S.dh, S.dL, multipliers=True)
    assert M.shape == (len(states) + len(pairs), ctx.multiplier_length())
    g1, d1, info1 = ctx.gradients_and_couplings(states, pairs, S.dh, S.dL, guess=M)
    print(f"  zero start {info0.iterations} iterations, converged guess {info1.iterations}", flush=True)
    assert info1.fallback_used == 0 and info1.iterations < info0.iterations
    assert np.abs(g1 - g0).max() < G_TOL and np.abs(d1 - d0).max() < G_TOL
    noise = torch.as_tensor(np.random.default_rng(3).normal(size=tuple(M.shape)), device=M.device)
    Mp = M + 1e-4 * M.abs().max() * noise
    g2, d2, info2 = ctx.gradients_and_couplings(states, pairs, S.dh, S.dL, guess=Mp)
    print(f"  perturbed guess {info2.iterations} iterations", flush=True)
    assert info2.fallback_used == 0 and info2.iterations < info0.iterations
    assert np.abs(g2 - g0).max() < G_TOL and np.abs(d2 - d0).max() < G_TOL
    bad = torch.full_like(M, float("nan"))
    g3, d3, info3 = ctx.gradients_and_couplings(states, pairs, S.dh, S.dL, guess=bad)
    assert info3.fallback_used == 1
    assert np.abs(g3 - g0).max() < G_TOL and np.abs(d3 - d0).max() < G_TOL
    # one target through scc_multipliers (the gradient of state 0, the first
    # lockstep target): the same multipliers, restarted from the lockstep
    # ones in fewer steps, and a guess that is not finite dropped
    ctx.excited()  # the same states again; the single-target Krylov space starts empty
    i_zero, x0 = ctx.multipliers(0, 0, 0, out=True)
    rel = float(torch.abs(x0 - M[0]).max() / torch.abs(M[0]).max())
    print(f"  single target: {i_zero.iterations} iterations from zero, max relative difference from the "
          f"lockstep multipliers {rel:.1e}", flush=True)
    assert rel < 1e-6
    i_warm = ctx.multipliers(0, 0, 0, guess=M[0])
    print(f"  single target from the lockstep multipliers: {i_warm.iterations} iterations", flush=True)
    assert i_warm.fallback_used == 0 and i_warm.iterations < i_zero.iterations
    i_bad, x_bad = ctx.multipliers(0, 0, 0, guess=torch.full_like(M[0], float("nan")), out=True)
    assert i_bad.fallback_used == 1
    assert float(torch.abs(x_bad - x0).max() / torch.abs(x0).max()) < 1e-6
