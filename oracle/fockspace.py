"""Determinant-space (full CI space) definitions of the method's quantities.

TEST INFRASTRUCTURE ONLY: imported by tests/ and by the oracle's own checks,
never by the product path.

Every quantity here is evaluated straight from its definition on a closed-shell
system small enough that the whole N-electron space (fixed numbers of alpha and
beta electrons) fits in a dense matrix.  Nothing is factorised:

* E_pq = sum_sigma a+_{p sigma} a_{q sigma} is built as a dense matrix;
* H = sum h_pq E_pq + 1/2 sum g_pqrs (E_pq E_rs - d_qr E_ps) (the second
  quantised Hamiltonian of the paper's density-matrix section);
* cluster operators T1 = sum t_ai E_ai, T2 = 1/2 sum t_aibj E_ai E_bj and the
  triple excitation X3 = R1^k R2^l - R1^l R2^k (SCCSD method section) are
  matrix products of those E_pq, and exp(+-T) is the matrix exponential;
* "projection onto the excitation space" is the orthogonal projection of a
  vector onto span{|HF>, E_ai|HF>, E_ai E_bj|HF>}; the coefficients of that
  projection are returned in the amplitude layout used everywhere else:
  singles [a,i] and a full (ai)<->(bj) symmetric doubles array d such that
  the doubles part equals 1/2 sum_aibj d_aibj E_ai E_bj |HF>.
"""
from __future__ import annotations

from itertools import combinations

import numpy as np
import scipy.linalg as sla


class FockSpace:
    """Dense closed-shell N-electron space for `nmo` orbitals, `nocc` pairs."""

    def __init__(self, nmo: int, nocc: int):
        self.n, self.o, self.v = nmo, nocc, nmo - nocc
        strings = [sum(1 << p for p in c) for c in combinations(range(nmo), nocc)]
        index = {s: i for i, s in enumerate(strings)}
        ns = len(strings)
        es = np.zeros((nmo, nmo, ns, ns))
        for col, s in enumerate(strings):
            for q in range(nmo):
                if not (s >> q) & 1:
                    continue
                s1 = s & ~(1 << q)
                sg1 = -1 if bin(s & ((1 << q) - 1)).count("1") % 2 else 1
                for p in range(nmo):
                    if (s1 >> p) & 1:
                        continue
                    s2 = s1 | (1 << p)
                    sg2 = -1 if bin(s1 & ((1 << p) - 1)).count("1") % 2 else 1
                    es[p, q, index[s2], col] += sg1 * sg2
        eye = np.eye(ns)
        # alpha string is the slow index; a beta excitation passes the same
        # number of alpha operators twice, so no extra sign appears.
        self.E = (np.einsum("pqAB,ab->pqAaBb", es, eye)
                  + np.einsum("pqab,AB->pqAaBb", es, eye)).reshape(nmo, nmo, ns * ns, ns * ns)
        self.dim = ns * ns
        hf = index[(1 << nocc) - 1]
        self.hf = np.zeros(self.dim)
        self.hf[hf * ns + hf] = 1.0
        o, v = self.o, self.v
        self.pairs = [(a, i, b, j) for a in range(v) for i in range(o)
                      for b in range(v) for j in range(o) if a * o + i <= b * o + j]
        cols = [self.hf]
        cols += [self.E[o + a, i] @ self.hf for a in range(v) for i in range(o)]
        cols += [self.E[o + a, i] @ (self.E[o + b, j] @ self.hf)
                 for (a, i, b, j) in self.pairs]
        self.basis = np.array(cols).T
        self.gram = self.basis.T @ self.basis

    # ---- operators -------------------------------------------------------
    def hamiltonian(self, h, g, hnuc=0.0):
        n = self.n
        E = self.E
        H = np.einsum("pq,pqIJ->IJ", h, E)
        M = np.einsum("pqrs,pqIJ->rsIJ", g, E).reshape(n * n, self.dim, self.dim)
        Er = E.reshape(n * n, self.dim, self.dim)
        H += 0.5 * np.einsum("xIK,xKJ->IJ", M, Er)
        H -= 0.5 * np.einsum("pqqs,psIJ->IJ", g, E)
        return H + hnuc * np.eye(self.dim)

    def singles_op(self, t1):
        o = self.o
        return np.einsum("ai,aiIJ->IJ", t1, self.E[o:, :o])

    def doubles_op(self, t2):
        o = self.o
        Ev = self.E[o:, :o].reshape(-1, self.dim, self.dim)
        M = np.einsum("xy,yIJ->xIJ", t2.reshape(Ev.shape[0], -1), Ev)
        return 0.5 * np.einsum("xIK,xKJ->IJ", Ev, M)

    def cluster_op(self, t1, t2):
        return self.singles_op(t1) + self.doubles_op(t2)

    def excitation_vector_op(self, r0, r1, r2):
        return r0 * np.eye(self.dim) + self.cluster_op(r1, r2)

    def rotation_op(self, kappa):
        """kappa = sum kappa_ai (E_ai - E_ia), kappa given as [v,o]."""
        o = self.o
        return (np.einsum("ai,aiIJ->IJ", kappa, self.E[o:, :o])
                - np.einsum("ai,iaIJ->IJ", kappa, self.E[:o, o:]))

    @staticmethod
    def expm(A):
        return sla.expm(A)

    # ---- projection onto the excitation space ------------------------------
    def coefficients(self, vec):
        """Coefficients (c0, c1[a,i], c2[a,i,b,j] symmetric) of the orthogonal
        projection of `vec` onto span{HF, singles, doubles}."""
        c = np.linalg.solve(self.gram, self.basis.T @ vec)
        o, v = self.o, self.v
        c0 = c[0]
        c1 = c[1:1 + o * v].reshape(v, o)
        c2 = np.zeros((v, o, v, o))
        for k, (a, i, b, j) in enumerate(self.pairs):
            val = c[1 + o * v + k]
            if (a, i) == (b, j):
                c2[a, i, a, i] = 2.0 * val
            else:
                c2[a, i, b, j] = val
                c2[b, j, a, i] = val
        return c0, c1, c2

    def vector(self, c0, c1, c2):
        """|vec> = (c0 + sum c1 E_ai + 1/2 sum c2 E_ai E_bj)|HF>."""
        return self.excitation_vector_op(c0, c1, c2) @ self.hf

    def projector(self):
        """Orthogonal projector onto span{HF, singles, doubles}."""
        B = self.basis
        return B @ np.linalg.solve(self.gram, B.T)


# ---- definitions of the method's quantities --------------------------------
def hbar(fs: FockSpace, H, t1, t2, x3=None):
    """exp(-T) H exp(T); T = T1 + T2 (+ x3, a given Fock-space operator)."""
    T = fs.cluster_op(t1, t2)
    if x3 is not None:
        T = T + x3
    return fs.expm(-T) @ H @ fs.expm(T)


def ground_projections(fs, H, t1, t2, x3=None):
    """(E0, Omega1, Omega2): coefficients of P_E Hbar |HF>."""
    return fs.coefficients(hbar(fs, H, t1, t2, x3) @ fs.hf)


def sigma_right(fs, H, t1, t2, r0, r1, r2, x3=None):
    """Coefficients of P_E Hbar |R> with |R> = (r0 + R1 + R2)|HF>."""
    return fs.coefficients(hbar(fs, H, t1, t2, x3) @ fs.vector(r0, r1, r2))


def x3_operator(fs, rk, rl):
    """X3 = R1^k R2^l - R1^l R2^k for state vectors rk = (r0, r1, r2)."""
    return (fs.singles_op(rk[1]) @ fs.doubles_op(rl[2])
            - fs.singles_op(rl[1]) @ fs.doubles_op(rk[2]))


def inner(fs, a, b):
    """Physical inner product of two excitation-space coefficient triples."""
    return float(fs.vector(*a) @ fs.vector(*b))


def scc_overlap(fs, t1, t2, ra, rb):
    """O_ab = < P exp(T) R_a | P exp(T) R_b >  (natural projection)."""
    T = fs.expm(fs.cluster_op(t1, t2))
    P = fs.projector()
    va = P @ (T @ fs.vector(*ra))
    vb = P @ (T @ fs.vector(*rb))
    return float(va @ vb)


def hf_energy_and_fock(h, g, o):
    F = h + 2.0 * np.einsum("pqkk->pq", g[:, :, :o, :o]) - np.einsum("pkkq->pq", g[:, :o, :o, :])
    e = 2.0 * np.trace(h[:o, :o]) + 2.0 * np.einsum("iijj->", g[:o, :o, :o, :o]) \
        - np.einsum("ijji->", g[:o, :o, :o, :o])
    return e, F


def singlet_fci(fs: FockSpace, H, nroots):
    """Lowest `nroots` singlet eigenpairs of H (spin-adapted via S^2 filter)."""
    w, U = np.linalg.eigh(H)
    S2 = spin_squared(fs)
    out_w, out_v = [], []
    for k in range(len(w)):
        s2 = U[:, k] @ S2 @ U[:, k]
        if abs(s2) < 1e-6:
            out_w.append(w[k])
            out_v.append(U[:, k])
        if len(out_w) == nroots:
            break
    return np.array(out_w), np.array(out_v).T


def spin_squared(fs: FockSpace):
    """S^2 on the Ms = 0 space from the singlet excitation operators:
    for Ne electrons in n spatial orbitals,
        sum_pq E_pq E_qp = Ne (n + 2) - Ne^2 / 2 - 2 S^2,
    so S^2 = (Ne (n + 2) - Ne^2 / 2) / 2 - (1/2) sum_pq E_pq E_qp."""
    n = fs.n
    Ne = 2 * fs.o
    EEt = np.einsum("pqIK,qpKJ->IJ", fs.E, fs.E)
    return 0.5 * (Ne * (n + 2) - 0.5 * Ne * Ne) * np.eye(fs.dim) - 0.5 * EEt
