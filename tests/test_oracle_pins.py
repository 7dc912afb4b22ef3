"""The FP64 oracle pinned to things other than itself.

* determinant-space definitions (oracle/fockspace.py) of the residual, the
  right transformation with the SCC triple excitation, and the overlap O_ab;
* two-electron exact limits: CCSD/EOM-CCSD energies equal full CI, gradients
  equal Hellmann-Feynman FCI values, couplings equal
  <psi_m|H^(1)|psi_n>/(E_n - E_m);
* SCCSD gradients equal 5-point central differences of the SCCSD energies;
* SCCSD couplings equal 5-point central differences of the bra-frozen
  overlap built in the determinant space, with the orbitals at the displaced
  geometry reached by the exact orbital rotation (no multipliers involved);
* closed forms of the Lagrangian (K-vectors and Lbar_0, gradient/coupling
  stationarity sections).
"""
import numpy as np
import pytest
import torch

from oracle import cc, scc
from oracle.fockspace import (FockSpace, ground_projections, sigma_right,
                              scc_overlap, singlet_fci, x3_operator)
from synth_inputs import make_system, random_amplitudes

T = lambda a: torch.as_tensor(np.asarray(a), dtype=torch.float64)


def _ham(name, seed=7):
    S = make_system(name, seed=seed)
    h, L = S.at(np.zeros(S.ncoord))
    g = np.einsum("Jpq,Jrs->pqrs", L, L)
    return S, h, g


@pytest.mark.parametrize("name", ["o1v5", "o2v3", "o2v4"])
def test_residual_matches_definition(name):
    S, h, g = _ham(name)
    fs = FockSpace(S.n, S.o)
    H = fs.hamiltonian(h, g)
    t1, t2 = random_amplitudes(S.o, S.v, seed=5, scale=0.1)
    e0, c1, c2 = ground_projections(fs, H, t1, t2)
    E, s, d = cc.residual(T(h), T(g), T(t1), T(t2), S.o)
    assert abs(e0 - float(E)) < 1e-12
    assert np.abs(c1 - s.numpy()).max() < 1e-12
    assert np.abs(c2 - d.numpy()).max() < 1e-12


def _three_states(o, v):
    (a1, a2), (b1, b2), (c1, c2) = random_amplitudes(o, v, seed=9, scale=0.3, nvec=3)
    return (0.3, a1, a2), (-0.2, b1, b2), (0.7, c1, c2)


@pytest.mark.parametrize("name", ["o2v3", "o2v4"])
def test_scc_terms_match_definition(name):
    """Residual and right transformation with zeta X3 in the cluster operator."""
    S, h, g = _ham(name)
    fs = FockSpace(S.n, S.o)
    H = fs.hamiltonian(h, g)
    t1, t2 = random_amplitudes(S.o, S.v, seed=5, scale=0.1)
    ra, rb, rc = _three_states(S.o, S.v)
    zeta = 0.37
    x3 = zeta * x3_operator(fs, ra, rb)
    rs = [tuple(T(x) for x in ra), tuple(T(x) for x in rb)]
    e0, c1, c2 = ground_projections(fs, H, t1, t2, x3)
    E, s, d = cc.residual(T(h), T(g), T(t1), T(t2), S.o, T([zeta]), rs)
    assert abs(e0 - float(E)) < 1e-12
    assert np.abs(c1 - s.numpy()).max() < 1e-12
    assert np.abs(c2 - d.numpy()).max() < 1e-12
    c0, c1, c2 = sigma_right(fs, H, t1, t2, *rc, x3=x3)
    s0, s1, s2 = cc.sigma(T(h), T(g), T(t1), T(t2), S.o, T(rc[0]), T(rc[1]), T(rc[2]), T([zeta]), rs)
    assert abs(c0 - float(s0)) < 1e-12
    assert np.abs(c1 - s1.numpy()).max() < 1e-12
    assert np.abs(c2 - s2.numpy()).max() < 1e-12


@pytest.mark.parametrize("name", ["o2v3", "o2v4"])
def test_overlap_matches_definition(name):
    S, h, g = _ham(name)
    fs = FockSpace(S.n, S.o)
    t1, t2 = random_amplitudes(S.o, S.v, seed=5, scale=0.1)
    ra, rb, _ = _three_states(S.o, S.v)
    ref = scc_overlap(fs, t1, t2, ra, rb)
    val = cc.overlap(T(t1), T(t2), tuple(T(x) for x in ra), tuple(T(x) for x in rb))
    assert abs(ref - float(val)) < 1e-12


def test_two_electron_limit_energies():
    """Two electrons: CCSD and EOM-CCSD are exact (T1 + T2 span every
    excitation), so energies equal the singlet full-CI eigenvalues."""
    S, h, g = _ham("o1v5")
    fs = FockSpace(S.n, S.o)
    w, _ = singlet_fci(fs, fs.hamiltonian(h, g), 3)
    sol = scc.solve_system(S, nstates=2)
    assert not sol.scc            # no triples for two electrons: plain CCSD
    assert abs(sol.E0 - w[0]) < 1e-11
    assert np.abs(sol.E - w[1:3]).max() < 1e-10


def _fci_state_vector(fs, sol, k):
    r0, r1, r2 = (np.asarray(x) for x in sol.R[k])
    T1 = fs.cluster_op(sol.t1.numpy(), sol.t2.numpy())
    return fs.expm(T1) @ fs.vector(float(r0), r1, r2)


def test_two_electron_limit_gradients_and_couplings():
    """Two electrons: g_n = <psi_n|H^(1)|psi_n> (FCI is variational and
    orbital invariant); d_mn = <psi_m|H^(1)|psi_n> / (E_n - E_m) for the
    normalised, phase-matched FCI vectors (the derivative acts on the ket)."""
    S, h, g = _ham("o1v5")
    fs = FockSpace(S.n, S.o)
    H = fs.hamiltonian(h, g)
    w, U = singlet_fci(fs, H, 3)
    sol = scc.solve_system(S, nstates=2)
    targets = [("grad", 0), ("grad", 1), ("nac", 0, 1), ("nac", 1, 0)]
    res = scc.gradient_and_nacs(S, sol, targets)
    vecs = []
    for k in range(2):
        psi = _fci_state_vector(fs, sol, k)
        u = U[:, k + 1] * np.sign(U[:, k + 1] @ psi)
        assert abs(abs(u @ psi) - 1.0) < 1e-9        # O_kk = 1 is the FCI norm here
        vecs.append(u)
    for c in range(S.ncoord):
        L0 = S.L0
        g1 = np.einsum("Jpq,Jrs->pqrs", S.dL[c], L0) + np.einsum("Jpq,Jrs->pqrs", L0, S.dL[c])
        H1 = fs.hamiltonian(S.dh[c], g1)
        for n in range(2):
            hf = vecs[n] @ H1 @ vecs[n]
            assert abs(res[("grad", n)]["value"][c] - hf) < 1e-9
        for (m, n) in [(0, 1), (1, 0)]:
            exact = (vecs[m] @ H1 @ vecs[n]) / (w[n + 1] - w[m + 1])
            assert abs(res[("nac", m, n)]["value"][c] - exact) < 1e-8


@pytest.fixture(scope="module")
def o2v4_solution():
    S = make_system("o2v4")
    sol = scc.solve_system(S)
    assert sol.scc and abs(float(sol.zeta[0])) > 1e-3
    targets = [("grad", 0), ("grad", 1), ("nac", 0, 1), ("nac", 1, 0)]
    return S, sol, scc.gradient_and_nacs(S, sol, targets)


def test_scc_orthogonality_holds(o2v4_solution):
    S, sol, _ = o2v4_solution
    O = cc.overlap(sol.t1, sol.t2, sol.R[0], sol.R[1])
    assert abs(float(O)) < 1e-11
    for k in range(2):
        assert abs(float(cc.overlap(sol.t1, sol.t2, sol.R[k], sol.R[k])) - 1.0) < 1e-12


def test_scc_gradient_matches_finite_differences(o2v4_solution):
    """5-point central differences, h = 1e-3, RHF and SCC re-solved at every
    displacement (continued from the reference solution)."""
    S, sol, res = o2v4_solution
    step = 1e-3
    for c in range(S.ncoord):
        E = {}
        for st in (-2, -1, 1, 2):
            x = np.zeros(S.ncoord)
            x[c] = st * step
            E[st] = scc.solve_system(S, x=x, start=sol).E
        fd = (E[-2] - 8 * E[-1] + 8 * E[1] - E[2]) / (12 * step)
        for n in range(2):
            assert abs(fd[n] - res[("grad", n)]["value"][c]) < 1e-8


def test_scc_coupling_matches_finite_differences(o2v4_solution):
    """d_mn[c] = dO_mn/dx_c at x0 with O_mn(x) = <calL_m(x0)| exp(-T0)
    exp(-kappa(x)) exp(T(x)) |calR_n(x)> (derivative on the ket,
    coupling section), evaluated from definitions in the determinant space:
    the displaced solution (RHF and SCC re-solved, continued from x0) is
    mapped to the x0 orbitals by the Fock-space rotation exp(sum_pq A_pq E_pq),
    A = log of the orbital rotation C(x0)^T C(x) (C(x0) = 1 here), then
    exp(-T0) and the projection onto the excitation space are applied and the
    x0 left vector is contracted.  5-point differences, h = 1e-3."""
    import scipy.linalg as sla
    S, sol, res = o2v4_solution
    m, n = 0, 1
    lag = scc.Lagrangian(sol)
    fs = FockSpace(S.o + S.v, S.o)
    back = sla.expm(-fs.cluster_op(sol.t1.numpy(), sol.t2.numpy()))

    def overlap(x):
        sx = scc.solve_system(S, x=x, start=sol)
        A = np.real(sla.logm(np.asarray(sx.C)))
        rot = sla.expm(np.einsum("pq,pqIJ->IJ", A, fs.E))
        r = sx.R[n]
        ket = sla.expm(fs.cluster_op(sx.t1.numpy(), sx.t2.numpy())) @ fs.vector(
            float(r[0]), np.asarray(r[1]), np.asarray(r[2]))
        c0, c1, c2 = fs.coefficients(back @ rot @ ket)
        return float(lag.Lam[m] @ torch.cat([T([c0]), lag.P.pack(T(c1), T(c2))]))

    assert abs(overlap(np.zeros(S.ncoord))) < 1e-10  # <calL_m|calR_n> = 0
    step = 1e-3
    for c in range(S.ncoord):
        O = {}
        for st in (-2, -1, 1, 2):
            x = np.zeros(S.ncoord)
            x[c] = st * step
            O[st] = overlap(x)
        fd = (O[-2] - 8 * O[-1] + 8 * O[1] - O[2]) / (12 * step)
        assert abs(fd - res[("nac", m, n)]["value"][c]) < 1e-8


def test_lagrangian_closed_forms(o2v4_solution):
    """<Lbar_k|R_k> = delta_kn for gradients and 0 for couplings (the
    K-vectors of the gradient and coupling expressions), and
    Lbar_0^m = sum gamma_bar (1/omega_m) dO/dR_0^m."""
    S, sol, res = o2v4_solution
    lag = scc.Lagrangian(sol)
    na = lag.na
    for key, r in res.items():
        mult = r["mult"]
        n = key[-1]
        off = na
        gam = mult[-lag.np_:]
        for k in range(lag.ns):
            lbar = mult[off:off + na + 1]
            rk = scc.packed_from_state(lag.P, sol.R[k]).numpy()
            expect = (1.0 if k == n else 0.0) if key[0] == "grad" else 0.0
            assert abs(lbar @ rk - expect) < 1e-10
            # dO_01/dR_0^k from the overlap's explicit R0 dependence
            st = [tuple(torch.as_tensor(x, dtype=torch.float64) for x in s_) for s_ in sol.R]
            r0 = torch.tensor(float(st[k][0]), dtype=torch.float64, requires_grad=True)
            st[k] = (r0, st[k][1], st[k][2])
            O = cc.overlap(sol.t1, sol.t2, st[0], st[1])
            (dO,) = torch.autograd.grad(O, r0)
            om = sol.E[k] - sol.E0
            assert abs(lbar[0] - gam[0] * float(dO) / om) < 1e-10
            off += na + 2


def _packed_scale(P):
    """Packed doubles coordinate of a basis vector E_ai E_bj |HF>: 1 for
    (ai) < (bj), 2 for (ai) = (bj) (the packed coordinate x stands for
    1/2 x E_ai E_ai there)."""
    o, v = P.o, P.v
    nov = o * v
    iu0, iu1 = P.iu[0].numpy(), P.iu[1].numpy()
    return np.concatenate([[1.0], np.ones(nov), np.where(iu0 == iu1, 2.0, 1.0)])


@pytest.mark.parametrize("name", ["o2v3", "o2v4"])
def test_eom_matrix_matches_determinant_space(name):
    """The oracle's assembled calHbar (reference row and column, the
    Jacobian of the residual, the E0 diagonal and the {R1, Omega1} doubles
    term, plus the SCC term with X3) equals the matrix of the projected
    determinant-space operator P_E exp(-T) H exp(T) P_E, element by element,
    at random amplitudes with zeta X3 in the cluster operator."""
    S, h, g = _ham(name)
    fs = FockSpace(S.n, S.o)
    H = fs.hamiltonian(h, g)
    t1, t2 = random_amplitudes(S.o, S.v, seed=5, scale=0.1)
    ra, rb, _ = _three_states(S.o, S.v)
    zeta = 0.37
    x3 = zeta * x3_operator(fs, ra, rb)
    rs = [tuple(T(x) for x in ra), tuple(T(x) for x in rb)]
    M = scc.eom_matrix(T(h), T(g), S.o, T(t1), T(t2), T([zeta]), rs).numpy()
    from oracle.fockspace import hbar
    Hb = hbar(fs, H, t1, t2, x3)
    B = fs.basis
    Mfs = np.linalg.solve(fs.gram, B.T @ Hb @ B)     # columns: coefficients of Hbar |nu>
    P = scc.Packer(S.o, S.v)
    d = _packed_scale(P)
    ref = d[:, None] * Mfs / d[None, :]
    assert np.abs(M - ref).max() < 1e-11 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("name", ["o2v3", "o2v4"])
def test_davidson_states_match_dense_eigenvectors(name):
    """The iterative EOM path (Davidson on the excited block, left vectors
    from the transposed map, R0 from the reference row) reproduces the
    eigenvectors of the dense calHbar: energies, zeta and normalised right
    and left vectors of the SCCSD solution."""
    S = make_system(name)
    a = scc.solve_system(S, eom_method="dense")
    b = scc.solve_system(S, eom_method="davidson")
    assert np.abs(a.E - b.E).max() < 1e-12
    assert abs(a.E0 - b.E0) < 1e-12
    assert np.abs((a.zeta - b.zeta).numpy()).max() < 1e-7
    for k in range(S.nstates):
        for i in range(3):
            assert float(torch.abs(torch.as_tensor(a.R[k][i]) - torch.as_tensor(b.R[k][i])).max()) < 1e-10
            assert float(torch.abs(torch.as_tensor(a.Lv[k][i]) - torch.as_tensor(b.Lv[k][i])).max()) < 1e-10


def test_canonical_phase_is_a_symmetry(o2v4_solution):
    """Reading of the phase: each converged right vector has its
    largest-magnitude R1 element positive.  Flipping a state together with
    zeta of its pairs is an exact symmetry of the SCC equations (X3^{kl} is
    bilinear in R_k and R_l, so zeta_kl X3^{kl} is unchanged): the residual
    is the same to rounding, and the canonical phase maps the flipped
    solution back onto the converged one."""
    S, sol, _ = o2v4_solution
    P = scc.Packer(S.o, S.v)
    for k in range(S.nstates):
        r1 = scc.packed_from_state(P, sol.R[k]).numpy()[1:1 + P.nov]
        assert r1[np.argmax(np.abs(r1))] > 0
    flip = lambda st: scc.state_from_packed(P, -scc.packed_from_state(P, st))
    R2 = [flip(sol.R[0]), sol.R[1]]
    L2 = [flip(sol.Lv[0]), sol.Lv[1]]
    z2 = -sol.zeta
    a = cc.residual(sol.h, sol.g, sol.t1, sol.t2, S.o, sol.zeta, sol.R)
    b = cc.residual(sol.h, sol.g, sol.t1, sol.t2, S.o, z2, R2)
    for x, y in zip(a, b):
        assert float(torch.abs(torch.as_tensor(x) - torch.as_tensor(y)).max()) < 1e-14
    # flipping only the state (zeta kept) changes the residual at first order
    c = cc.residual(sol.h, sol.g, sol.t1, sol.t2, S.o, sol.zeta, R2)
    assert float(torch.abs(torch.as_tensor(c[2]) - torch.as_tensor(a[2])).max()) > 1e-6
    R3, L3, z3 = scc.canonical_phase(P, R2, L2, z2, cc.pair_list(S.nstates))
    assert float(torch.abs(z3 - sol.zeta).max()) == 0.0
    for k in range(S.nstates):
        for i in range(3):
            assert float(torch.abs(torch.as_tensor(R3[k][i]) - torch.as_tensor(sol.R[k][i])).max()) == 0.0
            assert float(torch.abs(torch.as_tensor(L3[k][i]) - torch.as_tensor(sol.Lv[k][i])).max()) == 0.0
