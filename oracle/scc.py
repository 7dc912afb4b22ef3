"""Plain FP64 SCCSD(E) solution, Lagrange multipliers, gradients and NACs.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Steps, in the paper's order:
  1. RHF in the fixed orthonormal basis, MO integrals (orbital-explicit
     Hbar section: kappa = 0 are the HF orbitals at the geometry);
  2. ground state Omega(t) = 0 (CC theory section);
  3. EOM right/left eigenvectors of calHbar (EOM section): from the dense
     matrix for small systems, else by a plain nonsymmetric Davidson
     iteration on the excited-excited block with the reference row and
     column from the block structure (R0 = eta.R / omega, L0 = 0);
  4. SCC: zeta_kl with O_kl = <psi_k|P|psi_l> = 0, solved together with the
     ground and excited states (SCC theory section; natural projection);
  5. Lagrangian of the gradient / coupling: the multipliers solve the
     stationarity conditions dL/dlambda = 0 (Lagrangian section).  The
     multipliers of the amplitude, excited-state and orthogonality
     constraints are found first; the orbital multipliers kappa-bar after,
     because the HF condition does not depend on the CC parameters;
  6. g_n = dL_n/dx and d_mn = dL_mn/dx, contracted with the derivative
     integrals (gradient and coupling expressions).

Parameter layout of the Lagrangian (packed vectors, one independent
coefficient per singles (ai) and per doubles pair (ai) <= (bj)):
  lambda = [t | zeta_kl (k<l) | for each state k: r0_k, r_k, E_k]
  e(lambda) = [Omega | for each k: (calHbar - E_k) calR_k, 1 - Lam_k.calR_k
               | O_kl (k<l)],
  with Lam_k = calL_k at the solution (a fixed vector).  The partial
  derivatives that make up the paper's stationarity equations (A, Fbar(R),
  Y, Z, z, eta, grad O ...) are taken by reverse-mode differentiation of
  these explicit constraint functions.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla
import torch

from . import cc

f64 = torch.float64


def tt(a):
    return torch.as_tensor(np.asarray(a), dtype=f64)


# ---------------------------------------------------------------------------
# packed <-> full amplitude layouts
# ---------------------------------------------------------------------------
class Packer:
    def __init__(self, o, v):
        self.o, self.v = o, v
        nov = o * v
        iu = np.triu_indices(nov)
        self.iu = (torch.as_tensor(iu[0]), torch.as_tensor(iu[1]))
        self.nov = nov
        self.n2 = len(iu[0])
        self.namp = nov + self.n2

    def pack(self, x1, x2):
        m = x2.reshape(self.nov, self.nov)
        return torch.cat([x1.reshape(-1), m[self.iu[0], self.iu[1]]])

    def unpack(self, vec):
        nov = self.nov
        x1 = vec[:nov].reshape(self.v, self.o)
        m = torch.zeros((nov, nov), dtype=vec.dtype)
        m = m.index_put((self.iu[0], self.iu[1]), vec[nov:])
        m = m + m.T - torch.diag(torch.diagonal(m))
        return x1, m.reshape(self.v, self.o, self.v, self.o)

    def denominators(self, eps):
        o = self.o
        eo, ev = eps[:o], eps[o:]
        d1 = ev[:, None] - eo[None, :]
        d2 = d1.reshape(-1)[:, None] + d1.reshape(-1)[None, :]
        return np.concatenate([d1.reshape(-1), d2[self.iu[0].numpy(), self.iu[1].numpy()]])


# ---------------------------------------------------------------------------
# RHF in the fixed basis
# ---------------------------------------------------------------------------
def rhf(h, L, o, C0=None, tol=1e-13, maxiter=500):
    """Roothaan iterations with Pulay's DIIS extrapolation of the Fock matrix
    (error vectors F D - D F, orthonormal basis, last 8 iterations); returns
    canonical MO coefficients whose columns are phase-aligned with C0
    (default identity).  Plain Roothaan steps oscillate for some of the
    synthetic systems; the converged orbitals are the same."""
    n = h.shape[0]
    C = np.eye(n) if C0 is None else C0.copy()
    Fs, Es = [], []
    for it in range(maxiter):
        Co = C[:, :o]
        D = Co @ Co.T
        Jm = np.einsum("Jpq,Jrs,rs->pq", L, L, D)
        K = np.einsum("Jps,Jsq->pq", np.einsum("Jpr,rs->Jps", L, D), L)
        F = h + 2 * Jm - K
        err = F @ D - D @ F
        if np.abs(err).max() < tol:
            w, C = np.linalg.eigh(F)
            break
        Fs, Es = (Fs + [F])[-8:], (Es + [err])[-8:]
        m = len(Fs)
        B = -np.ones((m + 1, m + 1))
        B[m, m] = 0.0
        for i in range(m):
            for j in range(m):
                B[i, j] = np.sum(Es[i] * Es[j])
        rhs = np.zeros(m + 1)
        rhs[m] = -1.0
        c = np.linalg.lstsq(B, rhs, rcond=None)[0][:m]
        w, C = np.linalg.eigh(sum(ci * Fi for ci, Fi in zip(c, Fs)))
    else:
        raise RuntimeError("RHF did not converge")
    ref = np.eye(n) if C0 is None else C0
    s = np.sign(np.einsum("pk,pk->k", ref, C))
    s[s == 0] = 1
    return C * s, w


def mo_integrals(h, L, C):
    return C.T @ h @ C, np.einsum("Pp,JPQ,Qq->Jpq", C, L, C)


# ---------------------------------------------------------------------------
# state container
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class Solution:
    o: int
    v: int
    h: torch.Tensor          # MO one-electron integrals
    L: torch.Tensor          # MO Cholesky vectors
    g: torch.Tensor
    eps: np.ndarray          # diagonal of the MO Fock matrix
    t1: torch.Tensor
    t2: torch.Tensor
    E0: float
    zeta: torch.Tensor       # (npairs,)
    R: list                  # [(r0, r1, r2)] per state
    Lv: list                 # [(l0, l1, l2)] per state (packed pairing)
    E: np.ndarray            # excited-state energies
    scc: bool
    iters: dict


def residual_norm(res):
    return max(float(torch.abs(res[1]).max()), float(torch.abs(res[2]).max()))


def solve_ground(h, g, o, eps, t1=None, t2=None, zeta=None, rstates=None,
                 tol=1e-12, maxiter=200):
    """Jacobi steps with the orbital-energy preconditioner plus DIIS."""
    n = h.shape[0]
    v = n - o
    P = Packer(o, v)
    D = tt(P.denominators(eps))
    if t1 is None:
        t1 = torch.zeros((v, o), dtype=f64)
        govov = g[:o, o:, :o, o:]
        d1 = tt(eps[o:, None] - eps[None, :o])
        t2 = -govov.permute(1, 0, 3, 2) / (d1[:, :, None, None] + d1[None, None, :, :])
    x = P.pack(t1, t2)
    hist, errs = [], []
    for it in range(maxiter):
        a, b = P.unpack(x)
        E0, s, d = cc.residual(h, g, a, b, o, zeta, rstates)
        r = P.pack(s, d)
        if float(torch.abs(r).max()) < tol:
            return a, b, float(E0), it
        xn = x - r / D
        hist.append(xn); errs.append(r / D)
        hist, errs = hist[-8:], errs[-8:]
        m = len(hist)
        B = -np.ones((m + 1, m + 1)); B[m, m] = 0
        for i in range(m):
            for j in range(m):
                B[i, j] = float(errs[i] @ errs[j])
        rhs = np.zeros(m + 1); rhs[m] = -1
        c = np.linalg.lstsq(B, rhs, rcond=None)[0][:m]
        x = sum(float(ci) * hi for ci, hi in zip(c, hist))
    raise RuntimeError("ground state did not converge")


def eom_matrix(h, g, o, t1, t2, zeta=None, rstates=None):
    """Full calHbar in packed coordinates (index 0 is the reference).  The
    SCC term depends on t only through T1 (the T1-transformed Hamiltonian),
    so its Jacobian is taken along the singles directions alone."""
    n = h.shape[0]
    v = n - o
    P = Packer(o, v)

    def f(x):
        a, b = P.unpack(x)
        E0, s, d = cc.residual(h, g, a, b, o)
        return torch.cat([E0.reshape(1), P.pack(s, d)])

    hh, gg = cc.t1_transform(h, g, t1)

    def f2(x2):      # t2 directions: the T1-transformed Hamiltonian is fixed
        _, b = P.unpack(torch.cat([torch.zeros(P.nov, dtype=f64), x2]))
        E0, s, d = cc.omega_gen(hh, gg, b, o)
        return torch.cat([E0.reshape(1), P.pack(s, d)])

    def f1(a):       # t1 directions
        E0, s, d = cc.residual(h, g, a, t2, o)
        return torch.cat([E0.reshape(1), P.pack(s, d)])

    x0 = P.pack(t1, t2)
    Jm = torch.cat([torch.func.jacfwd(f1)(t1).reshape(P.namp + 1, P.nov),
                    torch.func.jacfwd(f2)(x0[P.nov:])], dim=1)   # d(E0, Omega)/dt
    val = f(x0)
    if zeta is not None and rstates is not None:
        def fs(a):
            _, s, d = cc.residual(h, g, a, t2, o, zeta, rstates)
            _, s0, d0 = cc.residual(h, g, a, t2, o)
            return P.pack(s - s0, d - d0)
        Js = torch.func.jacfwd(fs)(t1).reshape(P.namp, P.nov)
        Jm[1:, :P.nov] += Js
        val[1:] += fs(t1)
    E0, Om = val[0], val[1:]
    na = P.namp
    M = torch.zeros((na + 1, na + 1), dtype=f64)
    M[0, 0] = E0
    M[0, 1:] = Jm[0]
    M[1:, 0] = Om
    M[1:, 1:] = Jm[1:] + E0 * torch.eye(na, dtype=f64)
    # {R1, Omega1} term: doubles component gains r_ai O_bj + O_ai r_bj
    O1, _ = P.unpack(Om)
    eye = torch.eye(P.nov, dtype=f64).reshape(P.nov, v, o)
    z2 = torch.einsum("nai,bj->naibj", eye, O1) + torch.einsum("ai,nbj->naibj", O1, eye)
    z2 = z2.reshape(P.nov, P.nov, P.nov)[:, P.iu[0], P.iu[1]]
    M[1 + P.nov:, 1:1 + P.nov] += z2.T
    return M


def state_from_packed(P, vec):
    r1, r2 = P.unpack(vec[1:])
    return (vec[0], r1, r2)


def packed_from_state(P, st):
    return torch.cat([torch.as_tensor(st[0], dtype=f64).reshape(1), P.pack(st[1], st[2])])


DENSE_EOM_LIMIT = 3000   # packed amplitudes above which the EOM states come from Davidson


def davidson(apply, diag, nroots, guesses, tol, maxit=400, maxsub=None, nbuf=2):
    """Plain nonsymmetric Davidson iteration for the eigenvalues of lowest
    real part of the linear map `apply`: orthonormal search space V, images
    W = A V, subspace matrix V^T W, preconditioned residuals (diag - theta)^-1 r
    added after two passes of Gram-Schmidt.  Returns (theta [nwork], X [n,
    nwork]) with the first nroots converged to ||A x - theta x|| < tol.
    Complex Ritz pairs contribute their real and imaginary parts to the
    search space; a wanted root that converges complex is an error."""
    n = diag.size
    nwork = nroots + nbuf
    maxsub = maxsub or max(40, 32 * nwork)
    V, W = [], []

    def add(vec):
        n0 = np.linalg.norm(vec)
        if not n0 > 0:
            return False
        vec = vec / n0
        for _ in range(2):
            for u in V:
                vec = vec - (u @ vec) * u
        nv = np.linalg.norm(vec)
        if nv < 1e-10:      # (numerically) inside the search space already
            return False
        V.append(vec / nv)
        W.append(apply(V[-1]))
        return True

    for gv in guesses:
        add(np.array(gv, dtype=np.float64))
    for k in np.argsort(diag):
        if len(V) >= nwork + 1:
            break
        e = np.zeros(n)
        e[k] = 1.0
        add(e)
    for it in range(maxit):
        Vm, Wm = np.array(V).T, np.array(W).T
        w, Y = np.linalg.eig(Vm.T @ Wm)
        order = np.argsort(w.real)[:nwork]
        X, AX, th, cplx, res = [], [], [], [], []
        for k in order:
            y = Y[:, k]
            y = y / np.linalg.norm(y)
            x, ax = Vm @ y, Wm @ y
            r = ax - w[k] * x
            X.append(x)
            AX.append(ax)
            th.append(w[k])
            cplx.append(abs(w[k].imag) > 1e-10 * max(1.0, abs(w[k].real)))
            res.append(np.linalg.norm(r))
        for k in range(nroots):
            if cplx[k] and res[k] < tol:
                raise RuntimeError("complex excited-state energy")
        if all(res[k] < tol and not cplx[k] for k in range(nroots)):
            return np.array([t.real for t in th]), np.array([x.real for x in X]).T
        new = []
        for k in range(nwork):
            if res[k] < tol and not cplx[k]:
                continue
            r = AX[k] - th[k] * X[k]
            den = diag - th[k].real
            den = np.where(np.abs(den) < 0.05, np.where(den < 0, -0.05, 0.05), den)
            new.append((r.real / den, r.imag / den if cplx[k] else None))
        if len(V) + 2 * len(new) > maxsub:
            # thick restart on the real and imaginary parts of the Ritz vectors
            keep = [x.real for x in X] + [x.imag for x, c in zip(X, cplx) if c]
            V, W = [], []
            for x in keep:
                add(x)
        for a, b in new:
            add(a)
            if b is not None:
                add(b)
    raise RuntimeError("Davidson iterations did not converge")


def eom_states_davidson(h, g, o, t1, t2, nstates, eps, zeta=None, rstates=None, prev=None, tol=1e-11):
    """As eom_states, from Davidson iterations on the excited-excited block of
    calHbar in packed coordinates (R0 = 0 there): right vectors from the map
    x -> pack(sigma(unpack(x))), left vectors from its transpose (the
    reverse-mode derivative of the same map).  R0 = eta.R / omega from the
    reference row; L0 = 0."""
    n = h.shape[0]
    P = Packer(o, n - o)
    E0 = float(cc.residual(h, g, t1, t2, o, zeta, rstates)[0])

    def right(x):
        r1, r2 = P.unpack(tt(x))
        _, s1, s2 = cc.sigma(h, g, t1, t2, o, 0.0, r1, r2, zeta, rstates)
        return P.pack(s1, s2).numpy()

    def left(y):
        x = torch.zeros(P.namp, dtype=f64, requires_grad=True)
        r1, r2 = P.unpack(x)
        _, s1, s2 = cc.sigma(h, g, t1, t2, o, 0.0, r1, r2, zeta, rstates)
        (gx,) = torch.autograd.grad(P.pack(s1, s2), x, tt(y))
        return gx.numpy()

    def eta_dot(x):
        r1, r2 = P.unpack(tt(x))
        return float(cc.sigma(h, g, t1, t2, o, 0.0, r1, r2, zeta, rstates)[0])

    diag = E0 + P.denominators(eps)
    nbuf = 2
    if prev is None:
        gr, gl = [], []
    else:
        gr = [packed_from_state(P, Rp).numpy()[1:] for (Lp, Rp) in prev]
        gl = [packed_from_state(P, Lp).numpy()[1:] for (Lp, Rp) in prev]
    nroots = nstates
    while True:
        wr, XR = davidson(right, diag, nroots, gr, tol, nbuf=nbuf)
        if prev is None:
            pick = list(range(nstates))
        else:
            pick = []
            for (Lp, Rp) in prev:
                lp = packed_from_state(P, Lp).numpy()[1:]
                ov = [abs(lp @ XR[:, k]) / np.linalg.norm(XR[:, k]) for k in range(XR.shape[1])]
                pick.append(int(np.argmax(ov)))
        if max(pick) < nroots:      # every picked root is a converged one
            break
        nroots = max(pick) + 1
    # left vectors: the same lowest roots of the transpose, paired by energy
    wl, XL = davidson(left, diag, nroots, [XR[:, k] for k in range(nroots)] + gl, tol, nbuf=nbuf)
    Rs, Ls, Es = [], [], []
    for s_, k in enumerate(pick):
        Ek = wr[k]
        re = XR[:, k]
        rv = np.concatenate([[eta_dot(re) / (Ek - E0)], re])
        st = state_from_packed(P, tt(rv))
        rv = rv / np.sqrt(float(cc.overlap(t1, t2, st, st)))
        if prev is None:
            r1 = rv[1:1 + P.nov]
            if r1[np.argmax(np.abs(r1))] < 0:
                rv = -rv
        else:
            lp = packed_from_state(P, prev[s_][0]).numpy()
            if lp @ rv < 0:
                rv = -rv
        kl = int(np.argmin(np.abs(wl[:nroots] - Ek)))
        if abs(wl[kl] - Ek) > 1e-8 * max(1.0, abs(Ek)):
            raise RuntimeError("left and right excitation energies differ")
        lv = np.concatenate([[0.0], XL[:, kl]])
        lv = lv / (lv @ rv)
        Rs.append(state_from_packed(P, tt(rv)))
        Ls.append(state_from_packed(P, tt(lv)))
        Es.append(Ek)
    return Rs, Ls, np.array(Es), None


def eom_states(h, g, o, t1, t2, nstates, zeta=None, rstates=None, prev=None, method=None, tol=1e-11):
    """Lowest excited right/left eigenvectors, normalised O_kk = 1 and
    calL_k . calR_k = 1; phase: largest |R1| positive (or positive overlap
    with the previous left vector); order: ascending energy (or maximum
    overlap with the previous states).  method: "dense" (eigenvectors of the
    whole calHbar), "davidson" (eom_states_davidson, residual norm < tol) or
    None (dense up to DENSE_EOM_LIMIT packed amplitudes)."""
    n = h.shape[0]
    P = Packer(o, n - o)
    if method == "davidson" or (method is None and P.namp > DENSE_EOM_LIMIT):
        eps = np.diag(cc.fock(h, g, o).numpy()).copy()
        return eom_states_davidson(h, g, o, t1, t2, nstates, eps, zeta, rstates, prev, tol=tol)
    M = eom_matrix(h, g, o, t1, t2, zeta, rstates).numpy()
    w, VL, VR = sla.eig(M, left=True, right=True)
    E0 = M[0, 0]
    order = np.argsort(w.real)
    cand = [k for k in order if abs(VR[0, k]) < 0.999 or abs(w[k] - E0) > 1e-8]
    cand = [k for k in cand if abs(w[k].real - E0) > 1e-6]
    if prev is None:
        pick = cand[:nstates]
    else:
        pick = []
        for (Lp, Rp) in prev:
            lp = packed_from_state(P, Lp).numpy()
            ov = [abs(lp @ VR[:, k].real) / np.linalg.norm(VR[:, k]) for k in cand]
            pick.append(cand[int(np.argmax(ov))])
    Rs, Ls, Es = [], [], []
    for s_, k in enumerate(pick):
        if abs(w[k].imag) > 1e-10:
            raise RuntimeError("complex excited-state energy")
        rv = VR[:, k].real
        lv = VL[:, k].real
        st = state_from_packed(P, tt(rv))
        nrm = float(cc.overlap(t1, t2, st, st))
        rv = rv / np.sqrt(nrm)
        if prev is None:
            r1 = rv[1:1 + P.nov]
            if r1[np.argmax(np.abs(r1))] < 0:
                rv = -rv
        else:
            lp = packed_from_state(P, prev[s_][0]).numpy()
            if lp @ rv < 0:
                rv = -rv
        lv = lv / (lv @ rv)
        lv[0] = 0.0 if abs(lv[0]) < 1e-12 else lv[0]
        Rs.append(state_from_packed(P, tt(rv)))
        Ls.append(state_from_packed(P, tt(lv)))
        Es.append(w[k].real)
    return Rs, Ls, np.array(Es), M


def canonical_phase(P, R, Lv, zeta, pairs):
    """Phase of the converged states fixed by the solution alone: the
    largest-magnitude R1 element of every right vector positive (reading of
    the phase, which the paper leaves open).  A flipped R_k flips L_k and,
    for every pair (k, l), O_kl and X3^{kl}; zeta_kl flips with them, so that
    zeta_kl X3^{kl} (and with it the ground-state amplitudes) is unchanged."""
    sign = []
    R, Lv = list(R), list(Lv)
    for k in range(len(R)):
        rv = packed_from_state(P, R[k]).numpy()
        r1 = rv[1:1 + P.nov]
        s_ = -1.0 if r1[np.argmax(np.abs(r1))] < 0 else 1.0
        sign.append(s_)
        if s_ < 0:
            R[k] = state_from_packed(P, tt(-rv))
            Lv[k] = state_from_packed(P, -packed_from_state(P, Lv[k]))
    zeta = zeta.clone()
    for p, (k, l) in enumerate(pairs):
        zeta[p] = zeta[p] * sign[k] * sign[l]
    return R, Lv, zeta


def scc_solve(h, g, o, eps, nstates, scc=True, tol=1e-12, maxiter=60,
              start=None, eom_method=None):
    """Ground + excited states with the orthogonality constraints O_kl = 0
    solved simultaneously; zeta by Newton steps with a finite-difference
    Jacobian (the root reached from zeta = 0, or continued from `start`).
    Iterative EOM vectors (eom_method "davidson", or None above the dense
    limit) are converged to a residual norm of 1e-11; the SCC loop then
    stops at |O_kl| below that level and successive right vectors within 10
    times it (the eigenvector noise of the iteration)."""
    pairs = cc.pair_list(nstates)
    use_scc = scc and o >= 2 and len(pairs) > 0
    namp = Packer(o, h.shape[0] - o).namp
    iterative = eom_method == "davidson" or (eom_method is None and namp > DENSE_EOM_LIMIT)
    tol_eom = 1e-11
    tol_dr = max(tol, 10 * tol_eom) if iterative else tol
    tol_o = max(tol, tol_eom) if iterative else tol

    def eom(*a, **k):
        return eom_states(*a, method=eom_method, tol=tol_eom, **k)
    if start is None:
        t1, t2, E0, _ = solve_ground(h, g, o, eps, tol=tol)
        R, Lv, E, _ = eom(h, g, o, t1, t2, nstates)
        zeta = torch.zeros(len(pairs), dtype=f64)
    else:
        t1, t2, zeta, R, Lv = start.t1, start.t2, start.zeta.clone(), start.R, start.Lv
        t1, t2, E0, _ = solve_ground(h, g, o, eps, t1, t2, zeta if use_scc else None,
                                     R if use_scc else None, tol=tol)
        R, Lv, E, _ = eom(h, g, o, t1, t2, nstates, zeta if use_scc else None,
                                 R if use_scc else None, prev=list(zip(Lv, R)))
    it = 0
    if use_scc:
        def overlaps(t1_, t2_, R_):
            return torch.stack([cc.overlap(t1_, t2_, R_[k], R_[l]) for (k, l) in pairs])

        def solve_at(z, Rfix, tstart, prev):
            a, b, e0, _ = solve_ground(h, g, o, eps, tstart[0], tstart[1], z, Rfix, tol=tol)
            Rn, Ln, En, _ = eom(h, g, o, a, b, nstates, z, Rfix, prev=prev)
            return a, b, e0, Rn, Ln, En

        Jz = None
        for it in range(maxiter):
            Rfix = R
            t1, t2, E0, Rn, Ln, En = solve_at(zeta, Rfix, (t1, t2), list(zip(Lv, R)))
            Ov = overlaps(t1, t2, Rn)
            dR = max(float(torch.abs(packed_from_state(Packer(o, h.shape[0] - o), a)
                                     - packed_from_state(Packer(o, h.shape[0] - o), b)).max())
                     for a, b in zip(Rn, R))
            R, Lv, E = Rn, Ln, En
            if float(torch.abs(Ov).max()) < tol_o and dR < tol_dr:
                break
            if Jz is None:
                Jz = torch.zeros((len(pairs), len(pairs)), dtype=f64)
                dz = 1e-5
                for p in range(len(pairs)):
                    zp = zeta.clone(); zp[p] += dz
                    a, b, _, Rp, _, _ = solve_at(zp, Rfix, (t1, t2), list(zip(Lv, R)))
                    Jz[:, p] = (overlaps(a, b, Rp) - Ov) / dz
            step = -torch.linalg.solve(Jz, Ov)
            zeta = zeta + step
        else:
            raise RuntimeError("SCC iterations did not converge")
    R, Lv, zeta = canonical_phase(Packer(o, h.shape[0] - o), R, Lv, zeta, pairs if use_scc else [])
    return Solution(o=o, v=h.shape[0] - o, h=h, L=None, g=g, eps=eps, t1=t1, t2=t2,
                    E0=E0, zeta=zeta, R=R, Lv=Lv, E=np.array(E), scc=use_scc,
                    iters=dict(scc=it))


# ---------------------------------------------------------------------------
# Lagrangian
# ---------------------------------------------------------------------------
def gmres(A, Minv, b, tol, maxiter, log=None):
    """Right-preconditioned GMRES without restarts (Arnoldi with two passes of
    modified Gram-Schmidt, Givens rotations for the least-squares problem)."""
    n = b.size
    bn = np.linalg.norm(b)
    if bn == 0:
        return np.zeros(n), 0
    V = [b / bn]
    Z = []
    H = np.zeros((maxiter + 1, maxiter))
    cs, sn = np.zeros(maxiter), np.zeros(maxiter)
    g = np.zeros(maxiter + 1)
    g[0] = bn
    k = 0
    for j in range(maxiter):
        z = Minv(V[j])
        w = A(z)
        Z.append(z)
        for _ in range(2):
            for i in range(j + 1):
                hij = V[i] @ w
                H[i, j] += hij
                w = w - hij * V[i]
        H[j + 1, j] = np.linalg.norm(w)
        V.append(w / H[j + 1, j] if H[j + 1, j] > 0 else w)
        for i in range(j):
            a, c_ = H[i, j], H[i + 1, j]
            H[i, j], H[i + 1, j] = cs[i] * a + sn[i] * c_, -sn[i] * a + cs[i] * c_
        r = np.hypot(H[j, j], H[j + 1, j])
        cs[j], sn[j] = H[j, j] / r, H[j + 1, j] / r
        H[j, j], H[j + 1, j] = r, 0.0
        g[j + 1], g[j] = -sn[j] * g[j], cs[j] * g[j]
        k = j + 1
        if log is not None and j % 20 == 0:
            log(f"    gmres {j} rel. residual {abs(g[j + 1]) / bn:.3e}")
        if abs(g[j + 1]) / bn < tol:
            break
    y = np.linalg.solve(np.triu(H[:k, :k]), g[:k])
    x = sum(yi * zi for yi, zi in zip(y, Z))
    return x, k


class Lagrangian:
    """Constraint functions e(lambda; kappa, h, g) of the gradient/coupling
    Lagrangians (eq. Lagrangian_gradient / Lagrangian_coupling)."""

    def __init__(self, sol: Solution):
        self.sol = sol
        o, v = sol.o, sol.v
        self.P = Packer(o, v)
        self.ns = len(sol.R)
        self.pairs = cc.pair_list(self.ns) if sol.scc else []
        self.na = self.P.namp
        self.np_ = len(self.pairs)
        self.Lam = [packed_from_state(self.P, l) for l in sol.Lv]
        self.dense_limit = 1500
        self._jac = None

    # parameter vector -------------------------------------------------------
    def lam0(self):
        s = self.sol
        parts = [self.P.pack(s.t1, s.t2), s.zeta[:self.np_]]
        for k in range(self.ns):
            parts += [packed_from_state(self.P, s.R[k]), torch.tensor([s.E[k]], dtype=f64)]
        return torch.cat(parts)

    def split(self, lam):
        na, P = self.na, self.P
        t = lam[:na]
        off = na
        zeta = lam[off:off + self.np_]; off += self.np_
        states, energies = [], []
        for k in range(self.ns):
            rv = lam[off:off + na + 1]; off += na + 1
            energies.append(lam[off]); off += 1
            states.append(state_from_packed(P, rv))
        return t, zeta, states, energies

    def constraints(self, lam, kappa, h, g):
        o = self.sol.o
        P = self.P
        t, zeta, states, energies = self.split(lam)
        t1, t2 = P.unpack(t)
        hk, gk = cc.rotate(h, g, kappa)
        z = zeta if self.np_ else None
        rs = states if self.np_ else None
        _, s, d = cc.residual(hk, gk, t1, t2, o, z, rs)
        out = [P.pack(s, d)]
        for k in range(self.ns):
            r0, r1, r2 = states[k]
            s0, s1, s2 = cc.sigma(hk, gk, t1, t2, o, r0, r1, r2, z, rs)
            vec = torch.cat([s0.reshape(1), P.pack(s1, s2)]) \
                - energies[k] * torch.cat([torch.as_tensor(r0).reshape(1), P.pack(r1, r2)])
            out.append(vec)
            out.append((1.0 - self.Lam[k] @ torch.cat([torch.as_tensor(r0).reshape(1),
                                                       P.pack(r1, r2)])).reshape(1))
        for (k, l) in self.pairs:
            out.append(cc.overlap(t1, t2, states[k], states[l]).reshape(1))
        return torch.cat(out)

    def fock_ov(self, kappa, h, g):
        o = self.sol.o
        hk, gk = cc.rotate(h, g, kappa)
        return cc.fock(hk, gk, o)[o:, :o].reshape(-1)

    # targets ---------------------------------------------------------------
    def target(self, kind, m, n, lam, kappa):
        t, zeta, states, energies = self.split(lam)
        if kind == "grad":
            return energies[n]
        # bra-frozen overlap O_mn = <calL_m| exp(-T0) exp(-kappa) exp(T) |calR_n>
        s = self.sol
        P = self.P
        t1, t2 = P.unpack(t)
        c = cc.project_exp_t(t1 - s.t1, t2 - s.t2, states[n])
        lm = self.Lam[m]
        val = lm @ torch.cat([torch.as_tensor(c[0]).reshape(1), P.pack(c[1], c[2])])
        # orbital part: -<calL_m| exp(-T) kappa exp(T) |calR_n> at fixed T, R
        nn = s.h.shape[0]
        K = cc.vo_matrix(kappa, nn)
        hkap = K - K.T
        gz = torch.zeros_like(s.g)
        r0, r1, r2 = s.R[n]
        zz = s.zeta[:self.np_] if self.np_ else None
        rs = s.R if self.np_ else None
        s0, s1, s2 = cc.sigma(hkap, gz, s.t1, s.t2, s.o, torch.as_tensor(r0), r1, r2, zz, rs)
        val = val - lm @ torch.cat([s0.reshape(1), P.pack(s1, s2)])
        return val

    # multipliers -------------------------------------------------------------
    def solve_multipliers(self, kind, m, n, tol=1e-12, maxiter=1500):
        s = self.sol
        lam = self.lam0().requires_grad_(True)
        kap = torch.zeros((s.v, s.o), dtype=f64, requires_grad=True)
        h, g = s.h, s.g
        e = self.constraints(lam, kap, h, g)
        tg = self.target(kind, m, n, lam, kap)
        c_lam, c_kap = torch.autograd.grad(tg, (lam, kap), allow_unused=True)
        c_lam = torch.zeros_like(lam) if c_lam is None else c_lam
        c_kap = torch.zeros_like(kap) if c_kap is None else c_kap
        nl = lam.numel()

        def jt(vec):
            u = torch.as_tensor(vec, dtype=f64)
            (gl,) = torch.autograd.grad(e, lam, u, retain_graph=True)
            return gl.numpy()

        # preconditioner: maps a parameter-space residual to the constraint
        # space of the multipliers, pairing t <-> Omega, (r0, R)_k <-> the
        # eigenvalue rows of state k, E_k <-> its normalisation, zeta <-> O,
        # scaled by orbital-energy differences (shifted by omega_k)
        dvec = self.P.denominators(s.eps)
        na, np_ = self.na, self.np_
        scale = np.ones(nl)
        src = np.arange(nl)
        scale[:na] = 1.0 / dvec
        for k in range(self.ns):
            om = s.E[k] - s.E0
            dk = np.concatenate([[-om], dvec - om])
            dk = np.where(np.abs(dk) < 0.05, np.sign(dk + 1e-300) * 0.05, dk)
            cs, ps = na + k * (na + 2), na + np_ + k * (na + 2)
            scale[cs:cs + na + 1] = 1.0 / dk
            src[cs:cs + na + 2] = np.arange(ps, ps + na + 2)
        co = na + self.ns * (na + 2)
        src[co:co + np_] = np.arange(na, na + np_)

        def prec(vec):
            return scale * vec[src]
        b = -c_lam.detach().numpy()
        if nl <= self.dense_limit:
            # small systems: the whole Jacobian, one row per constraint
            if self._jac is None:
                f = lambda l: self.constraints(l, kap.detach(), h, g)
                self._jac = torch.func.jacrev(f, chunk_size=64)(lam.detach()).numpy()
            x = np.linalg.solve(self._jac.T, b)
            info = "dense"
        else:
            x, info = gmres(jt, prec, b, tol, maxiter)
        res = np.abs(jt(x) - b).max()
        if res > 1e3 * tol * max(1.0, np.abs(b).max()):
            raise RuntimeError(f"multiplier solve failed: residual {res:.2e}")
        mult = torch.as_tensor(x, dtype=f64)
        # orbital multipliers: A_HF^T kappa_bar = -(c_kap + (d e/d kappa)^T mult)
        (gk,) = torch.autograd.grad(e, kap, mult, retain_graph=True)
        eta = (c_kap + gk).reshape(-1)
        Ahf = torch.func.jacrev(lambda kk: self.fock_ov(kk, h, g))(
            torch.zeros((s.v, s.o), dtype=f64)).reshape(s.v * s.o, s.v * s.o)
        kbar = torch.linalg.solve(Ahf.T, -eta)
        return mult, kbar.reshape(s.v, s.o), dict(gmres_info=info, residual=res)

    def integral_derivatives(self, kind, m, n, mult, kbar):
        """dL/dh and dL/dL^J at the solution (kappa = 0)."""
        s = self.sol
        h = s.h.clone().requires_grad_(True)
        L = s.L.clone().requires_grad_(True)
        g = cc.chol_to_g(L)
        lam = self.lam0()
        kap = torch.zeros((s.v, s.o), dtype=f64)
        tot = self.target(kind, m, n, lam, kap) + mult @ self.constraints(lam, kap, h, g) \
            + kbar.reshape(-1) @ self.fock_ov(kap, h, g)
        dh, dL = torch.autograd.grad(tot, (h, L), allow_unused=True)
        return dh, dL


# ---------------------------------------------------------------------------
# top-level drivers
# ---------------------------------------------------------------------------
def solve_system(system, x=None, nstates=None, scc=True, start=None, C0=None, tol=1e-12, eom_method=None):
    """RHF + SCCSD solution of a synth_inputs.System at coordinates x."""
    o = system.o
    xv = np.zeros(system.ncoord) if x is None else np.asarray(x, dtype=np.float64)
    hf, Lf = system.at(xv)
    if C0 is None and not np.any(xv):
        C = np.eye(system.n)
        epsd = system.eps.copy()
    else:
        C, epsd = rhf(hf, Lf, o, C0)
    hm, Lm = mo_integrals(hf, Lf, C)
    h, L = tt(hm), tt(Lm)
    g = cc.chol_to_g(L)
    F = cc.fock(h, g, o).numpy()
    eps = np.diag(F).copy()
    ns = system.nstates if nstates is None else nstates
    sol = scc_solve(h, g, o, eps, ns, scc=scc, start=start, tol=tol, eom_method=eom_method)
    sol.L = L
    sol.C = C
    return sol


def gradient_and_nacs(system, sol, targets, coords=None):
    """targets: list of ("grad", n) or ("nac", m, n).  Returns dict of arrays
    over coordinates; also the effective densities dL/dh, dL/dL in the fixed
    basis."""
    lag = Lagrangian(sol)
    C = tt(sol.C)
    out = {}
    ks = range(system.ncoord) if coords is None else coords
    for tg in targets:
        if tg[0] == "grad":
            kind, m, n = "grad", None, tg[1]
        else:
            kind, m, n = "nac", tg[1], tg[2]
        mult, kbar, info = lag.solve_multipliers(kind, m, n)
        dh, dL = lag.integral_derivatives(kind, m, n, mult, kbar)
        D1 = C @ dh @ C.T
        Z = torch.einsum("pP,JPQ,qQ->Jpq", C, dL, C)
        vals = np.array([float(torch.sum(tt(system.dh[k]) * D1) + torch.sum(tt(system.dL[k]) * Z))
                         for k in ks])
        out[tg] = dict(value=vals, D1=D1.detach().numpy(), Z=Z.detach().numpy(),
                       mult=mult.numpy(), kbar=kbar.numpy(), info=info)
    return out
