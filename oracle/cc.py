"""Factorised closed-shell SCCSD functions in plain FP64 (CPU PyTorch).

TEST INFRASTRUCTURE ONLY: used by tests/, by the smoke check and by the
benchmark's CPU-baseline leg; never by the product path.

Conventions (shared with the determinant-space definitions in fockspace.py):
* orbitals: occupied first (0..o-1), virtual after (o..N-1);
* H = sum h_pq E_pq + 1/2 sum g_pqrs e_pqrs, e_pqrs = E_pq E_rs - d_qr E_ps;
* T1 = sum t_ai E_ai, T2 = 1/2 sum_aibj t_aibj E_ai E_bj with t2[a,i,b,j]
  symmetric under (ai) <-> (bj); every "doubles" array uses that layout;
* a projection onto the excitation space E = {HF, singles, doubles} returns
  the coefficients of the orthogonal projection in that same layout.

Everything is built from one function, `omega_gen(h, g, X)`: the projections
<mu| exp(-X) H exp(X) |HF> for a doubles operator X and a general two-body
operator H (no Hermiticity; only g_pqrs = g_rspq).  These are the spin-adapted
T1-transformed CCSD expressions (A1..D1, A2..E2 terms) of the integral-direct
CCSD literature the paper builds on, evaluated with T1 = 0; the singles
amplitudes enter through the T1-transformed Hamiltonian exp(-T1) H exp(T1)
(SCCSD implementation section).  fockspace.py pins every output of this module
to the determinant-space definitions.
"""
from __future__ import annotations

import torch

einsum = torch.einsum
f64 = torch.float64


# ---------------------------------------------------------------------------
# Hamiltonian transformations
# ---------------------------------------------------------------------------
def vo_matrix(x1, n):
    """N x N matrix with the [v,o] array x1 in its virtual-occupied block."""
    v, o = x1.shape
    M = torch.zeros((n, n), dtype=x1.dtype)
    M[o:, :o] = x1
    return M


def t1_transform(h, g, t1):
    """exp(-T1) H exp(T1): h -> (1 - T) h (1 + T) on each index pair."""
    n = h.shape[0]
    T = vo_matrix(t1, n)
    X = torch.eye(n, dtype=T.dtype) - T
    Y = torch.eye(n, dtype=T.dtype) + T
    hh = X @ h @ Y
    gg = einsum("pP,PQRS->pQRS", X, g)
    gg = einsum("PQRS,Qq->PqRS", gg, Y)
    gg = einsum("rR,PqRS->PqrS", X, gg)
    gg = einsum("PqrS,Ss->Pqrs", gg, Y)
    return hh, gg


def commutator_singles(h, g, r1):
    """[H, R1] for R1 = sum r_ai E_ai as a two-body operator (h', g')."""
    n = h.shape[0]
    R = vo_matrix(r1, n)
    hh = h @ R - R @ h
    gg = (einsum("ptrs,tq->pqrs", g, R) - einsum("pt,tqrs->pqrs", R, g)
          + einsum("pqrt,ts->pqrs", g, R) - einsum("rt,pqts->pqrs", R, g))
    return hh, gg


def rotate(h, g, kappa):
    """exp(kappa) H exp(-kappa) to first order in kappa = sum k_ai E^-_ai:
    every orbital index is transformed with U = 1 + K, K_ai = k_ai,
    K_ia = -k_ai.  First order suffices for derivatives at kappa = 0."""
    n = h.shape[0]
    K = vo_matrix(kappa, n)
    U = torch.eye(n, dtype=h.dtype) + K - K.T
    hh = U @ h @ U.T
    gg = einsum("pP,PQRS,qQ,rR,sS->pqrs", U, g, U, U, U)
    return hh, gg


def fock(h, g, o):
    return h + 2.0 * einsum("pqkk->pq", g[:, :, :o, :o]) - einsum("pkkq->pq", g[:, :o, :o, :])


def chol_to_g(L):
    return einsum("Jpq,Jrs->pqrs", L, L)


# ---------------------------------------------------------------------------
# <mu| exp(-X) H exp(X) |HF> for a doubles operator X
# ---------------------------------------------------------------------------
def omega_gen(h, g, X, o):
    """Returns (e, s[a,i], d[a,i,b,j]): reference, singles and doubles
    projections of exp(-X) H exp(X) |HF>."""
    O, V = slice(0, o), slice(o, h.shape[0])
    F = fock(h, g, o)
    u = 2.0 * X - X.permute(0, 3, 2, 1)
    # energy
    e = 2.0 * torch.trace(h[O, O]) + 2.0 * einsum("iijj->", g[O, O, O, O]) \
        - einsum("ijji->", g[O, O, O, O])
    govov = g[O, V, O, V]
    e = e + einsum("aibj,iajb->", X, 2.0 * govov - govov.permute(0, 3, 2, 1))
    # singles
    s = F[V, O].clone()
    s = s + einsum("ckdi,adkc->ai", u, g[V, V, O, V])
    s = s - einsum("akcl,kilc->ai", u, g[O, O, O, V])
    s = s + einsum("aick,kc->ai", u, F[O, V])
    # doubles
    gvovo = g[V, O, V, O]
    A2 = gvovo + einsum("cidj,acbd->aibj", X, g[V, V, V, V])
    chi = g[O, O, O, O] + einsum("cidj,kcld->kilj", X, govov)
    B2 = einsum("akbl,kilj->aibj", X, chi)
    W = g[O, O, V, V] - 0.5 * einsum("dial,kdlc->kiac", X, govov)   # [k,i,a,c]
    C2 = -0.5 * einsum("bkcj,kiac->aibj", X, W) - einsum("bkci,kjac->aibj", X, W)
    Lvoov = 2.0 * g[V, O, O, V] - g[V, V, O, O].permute(0, 3, 2, 1)  # L_aikc = 2g_aikc - g_acki
    Lovov = 2.0 * govov - govov.permute(0, 3, 2, 1)                  # L_ldkc = 2g_ldkc - g_lckd
    Q = Lvoov + 0.5 * einsum("aidl,ldkc->aikc", u, Lovov)
    D2 = 0.5 * einsum("bjck,aikc->aibj", u, Q)
    Fvv = F[V, V] - einsum("bkdl,ldkc->bc", u, govov)
    Foo = F[O, O] + einsum("cldj,kdlc->kj", u, govov)
    E2 = einsum("aicj,bc->aibj", X, Fvv) - einsum("aibk,kj->aibj", X, Foo)
    P = C2 + D2 + E2
    d = A2 + B2 + P + P.permute(2, 3, 0, 1)
    return e, s, d


def omega_linear(h, g, X, o):
    """<mu|[H, X]|HF> (the part of omega_gen linear in X)."""
    ep, sp, dp = omega_gen(h, g, X, o)
    em, sm, dm = omega_gen(h, g, -X, o)
    return 0.5 * (ep - em), 0.5 * (sp - sm), 0.5 * (dp - dm)


def sym_product(p, q):
    """Doubles layout of the product of two singles operators P1 Q1."""
    return einsum("ai,bj->aibj", p, q) + einsum("ai,bj->aibj", q, p)


def triple_projection(h, g, p1, q2, o):
    """<mu| H P1 Q2 |HF> (singles, doubles) for singles P1 and doubles Q2,
    from H P Q = [[H,P],Q] + Q[H,P] + P[H,Q] + P Q H on |HF>: the last term
    leaves the excitation space, [H,P]|HF> contributes only its reference
    component and [H,Q]|HF> only its reference and singles components."""
    ht, gt = commutator_singles(h, g, p1)
    _, s_a, d_a = omega_linear(ht, gt, q2, o)                 # [[H,P],Q]
    c0 = omega_gen(ht, gt, torch.zeros_like(q2), o)[0]        # <HF|[H,P]|HF>
    e_q, s_q, _ = omega_linear(h, g, q2, o)                   # [H,Q]|HF>, ranks 0, 1
    s = s_a + e_q * p1
    d = d_a + c0 * q2 + sym_product(p1, s_q)
    return s, d


# ---------------------------------------------------------------------------
# SCCSD residual, right transformation, orthogonality overlap
# ---------------------------------------------------------------------------
def pair_list(nstates):
    return [(k, l) for k in range(nstates) for l in range(k + 1, nstates)]


def residual(h, g, t1, t2, o, zeta=None, rstates=None):
    """(E0, Omega1, Omega2) of SCCSD with T = T1 + T2 + sum_{k<l} zeta_kl X3^kl,
    X3^kl = R1^k R2^l - R1^l R2^k.  Higher commutators of X3 vanish in these
    projections, so only zeta [H^, X3] enters (SCCSD implementation section)."""
    hh, gg = t1_transform(h, g, t1)
    e, s, d = omega_gen(hh, gg, t2, o)
    if zeta is not None and rstates is not None:
        for p, (k, l) in enumerate(pair_list(len(rstates))):
            rk, rl = rstates[k], rstates[l]
            s1, d1 = triple_projection(hh, gg, rk[1], rl[2], o)
            s2, d2 = triple_projection(hh, gg, rl[1], rk[2], o)
            s = s + zeta[p] * (s1 - s2)
            d = d + zeta[p] * (d1 - d2)
    return e, s, d


def sigma(h, g, t1, t2, o, r0, r1, r2, zeta=None, rstates=None):
    """Coefficients of P_E Hbar |R>, |R> = (r0 + R1 + R2)|HF>:
    <HF|Hbar|R> = E0 r0 + eta.R, <mu|Hbar|R> = Omega r0 + (A R) + E0 R
    + [doubles] {R1, Omega1}; A R and eta.R are directional derivatives of
    the residual and the energy along (r1, r2), taken by the complex step
    (exact here: the residual is a polynomial in t, so the step 1e-30 leaves
    no truncation error above rounding)."""
    E0, O1, O2 = residual(h, g, t1, t2, o, zeta, rstates)
    dE, dO1, dO2 = directional(h, g, t1, t2, o, r1, r2, zeta, rstates)
    s0 = E0 * r0 + dE
    s1 = O1 * r0 + dO1 + E0 * r1
    s2 = O2 * r0 + dO2 + E0 * r2 + sym_product(r1, O1)
    return s0, s1, s2


STEP = 1e-30


def directional(h, g, t1, t2, o, r1, r2, zeta=None, rstates=None):
    """d/de residual(t + e r) at e = 0 by the complex step."""
    c = torch.complex128
    hc, gc = h.to(c), g.to(c)
    a = t1.to(c) + 1j * STEP * r1.to(c)
    b = t2.to(c) + 1j * STEP * r2.to(c)
    zc = None if zeta is None else zeta.to(c)
    rc = None if rstates is None else [tuple(torch.as_tensor(x).to(c) for x in r) for r in rstates]
    E, s, d = residual(hc, gc, a, b, o, zc, rc)
    return E.imag / STEP, s.imag / STEP, d.imag / STEP


def metric_dot(a, b):
    """Physical inner product of two excitation-space coefficient triples."""
    return a[0] * b[0] + 2.0 * torch.sum(a[1] * b[1]) \
        + torch.sum(a[2] * (2.0 * b[2] - b[2].permute(0, 3, 2, 1)))


def project_exp_t(t1, t2, r):
    """Coefficients of P_E exp(T1 + T2) |R>."""
    r0, r1, r2 = r
    c1 = r1 + r0 * t1
    c2 = r2 + sym_product(t1, r1) + r0 * (t2 + einsum("ai,bj->aibj", t1, t1))
    return r0, c1, c2


def overlap(t1, t2, ra, rb):
    """O_ab = <psi_a| P |psi_b> with the natural projection (SCCSD(E))."""
    return metric_dot(project_exp_t(t1, t2, ra), project_exp_t(t1, t2, rb))


def hf_energy(h, g, o):
    return 2.0 * torch.trace(h[:o, :o]) + 2.0 * einsum("iijj->", g[:o, :o, :o, :o]) \
        - einsum("ijji->", g[:o, :o, :o, :o])
