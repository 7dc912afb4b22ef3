"""Seeded synthetic Cholesky-factored Hamiltonians (input data only).

This module is shared by the test suite, the benchmark and the oracle as a
source of *inputs*.  It contains none of the SCCSD method: it draws orbital
energies, Cholesky vectors and per-coordinate derivative integrals, and builds
the one-electron operator so that the fixed orthonormal basis is the canonical
restricted Hartree-Fock basis at the reference geometry x0 = 0.

Hamiltonian (second quantisation, spin-free, closed shell):

    H(x) = sum_pq h_pq(x) E_pq + 1/2 sum_pqrs g_pqrs(x) (E_pq E_rs - d_qr E_ps)

with g_pqrs(x) = sum_J L^J_pq(x) L^J_rs(x) and, for the coordinates x_k,

    h(x) = h0 + sum_k x_k dh_k,      L(x) = L0 + sum_k x_k dL_k.

Draw recipe (PCG64, one generator per system):
  1. occupied orbital energies ~ U[-1.5, -0.3], sorted;
  2. virtual orbital energies  ~ U[0.2, 3.0], sorted;
  3. L0^J_pq (p <= q) ~ N(0, (0.05 s)^2), mirrored to q < p;
  4. per coordinate k: a symmetric derivative Fock matrix F_k ~ N(0, sf^2) and
     symmetric dL_k ~ N(0, (sl s)^2);
  5. h0 = diag(eps) - sum_i [2 g_pqii - g_piiq]   (so F(x0) = diag(eps)),
     dh_k = F_k - sum_i [2 g1_pqii - g1_piiq] with g1 = dL_k L0^T + L0 dL_k^T
     (so dF/dx_k at x0, frozen orbitals, equals F_k).

"s" is the Cholesky scale.  The literal reading s = 1 gives unphysical,
Hartree-Fock-unstable systems once the Cholesky rank exceeds a few dozen
(sum_J L_ai^2 grows like N_J); the default reading keeps the two-electron
integral magnitudes of the rank-48 system: s = sqrt(48 / N_J).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Workload shapes.  o: occupied, v: virtual spatial orbitals, nj: Cholesky
# rank, nstates: excited states in the constrained set, ncoord: perturbation
# coordinates, nacs: state pairs (m, n) whose couplings are requested.
CONFIGS = {
    # rank-48 system with two excited states and one coordinate
    "o4v12": dict(o=4, v=12, nj=48, nstates=2, ncoord=1, nacs=[(0, 1)],
                  sf=0.01 * 0.05, sl=0.01 * 0.05),
    # rank-300 system shaped like a small organic molecule in a TZ basis
    "o10v90": dict(o=10, v=90, nj=300, nstates=3, ncoord=36,
                   nacs=[(0, 1), (0, 2), (1, 2)], sf=0.01, sl=0.01),
    "o20v180": dict(o=20, v=180, nj=600, nstates=3, ncoord=60,
                    nacs=[(0, 1), (0, 2), (1, 2)], sf=0.01, sl=0.01),
    "o30v270": dict(o=30, v=270, nj=900, nstates=4, ncoord=90,
                    nacs=[(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)],
                    sf=0.01, sl=0.01),
    # trajectory family H(x) = H0 + sum_k x_k H_k of the learned guess, at
    # the o4v12 size with 36 coordinates and N(0, 0.01) perturbations
    "o4v12x36": dict(o=4, v=12, nj=48, nstates=2, ncoord=36, nacs=[(0, 1)],
                     sf=0.01, sl=0.01),
    # small ragged systems for parity tests (several GEMM tiles + tails)
    "o5v19": dict(o=5, v=19, nj=40, nstates=2, ncoord=3, nacs=[(0, 1)],
                  sf=0.002, sl=0.002),
    # three states with all three pairwise couplings, as in o10v90, at a size
    # the oracle solves completely
    "o6v26": dict(o=6, v=26, nj=70, nstates=3, ncoord=6,
                  nacs=[(0, 1), (0, 2), (1, 2)], sf=0.01, sl=0.01),
    # three states with all three pairwise couplings at the o4v12 size: the
    # oracle's complete run (energies, three gradients, three couplings)
    # takes minutes
    "o4v12s3": dict(o=4, v=12, nj=48, nstates=3, ncoord=6,
                    nacs=[(0, 1), (0, 2), (1, 2)], sf=0.01, sl=0.01),
    # tiny systems for determinant-space checks
    "o1v5": dict(o=1, v=5, nj=12, nstates=2, ncoord=2, nacs=[(0, 1)],
                 sf=0.01, sl=0.01),
    "o2v3": dict(o=2, v=3, nj=10, nstates=2, ncoord=2, nacs=[(0, 1)],
                 sf=0.01, sl=0.01),
    "o2v4": dict(o=2, v=4, nj=12, nstates=2, ncoord=2, nacs=[(0, 1)],
                 sf=0.01, sl=0.01),
}

CONFIG_SEEDS = {"o4v12": 1001, "o10v90": 1002, "o20v180": 1003,
                "o4v12x36": 1004, "o30v270": 1005, "o4v12s3": 1006}


@dataclass
class System:
    name: str
    o: int
    v: int
    nj: int
    nstates: int
    ncoord: int
    nacs: list
    eps: np.ndarray          # (N,)
    h0: np.ndarray           # (N, N)
    L0: np.ndarray           # (nj, N, N), symmetric in the last two indices
    dF: np.ndarray           # (ncoord, N, N)
    dh: np.ndarray           # (ncoord, N, N)
    dL: np.ndarray           # (ncoord, nj, N, N)
    scale: float
    seed: int
    reading: str
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.o + self.v

    def at(self, x) -> tuple[np.ndarray, np.ndarray]:
        """(h(x), L(x)) in the fixed basis for coordinate vector x."""
        x = np.asarray(x, dtype=np.float64)
        h = self.h0 + np.einsum("k,kpq->pq", x, self.dh)
        L = self.L0 + np.einsum("k,kJpq->Jpq", x, self.dL)
        return h, L


def _sym_normal(rng, shape_lead, n, std):
    a = rng.normal(0.0, std, size=tuple(shape_lead) + (n, n))
    iu = np.triu_indices(n)
    out = np.zeros_like(a)
    out[..., iu[0], iu[1]] = a[..., iu[0], iu[1]]
    out = out + np.swapaxes(out, -1, -2)
    d = np.arange(n)
    out[..., d, d] *= 0.5
    return out


def _mean_field_part(La, Lb, o):
    """sum_i [2 (ab-pair term)_pqii - exchange_piiq] for g = La Lb^T."""
    J = np.einsum("Jpq,Jii->pq", La, Lb[:, :o, :o])
    K = np.einsum("Jpi,Jiq->pq", La[:, :, :o], Lb[:, :o, :])
    return 2.0 * J - K


def make_system(name: str, seed: int | None = None, reading: str = "rescaled",
                o=None, v=None, nj=None, nstates=None, ncoord=None,
                nacs=None, sf=None, sl=None, dtype=np.float64) -> System:
    """Draw the synthetic system `name` (a key of CONFIGS, or 'custom')."""
    if name in CONFIGS:
        c = dict(CONFIGS[name])
    else:
        c = dict(o=o, v=v, nj=nj, nstates=nstates, ncoord=ncoord, nacs=nacs,
                 sf=sf, sl=sl)
    for key, val in dict(o=o, v=v, nj=nj, nstates=nstates, ncoord=ncoord,
                         nacs=nacs, sf=sf, sl=sl).items():
        if val is not None:
            c[key] = val
    if seed is None:
        seed = CONFIG_SEEDS.get(name, 1000)
    o_, v_, nj_ = c["o"], c["v"], c["nj"]
    n = o_ + v_
    if reading == "literal":
        s = 1.0
    elif reading == "rescaled":
        s = math.sqrt(48.0 / nj_) if nj_ > 48 else 1.0
    else:
        raise ValueError("reading must be 'literal' or 'rescaled'")
    rng = np.random.Generator(np.random.PCG64(seed))
    eo = np.sort(rng.uniform(-1.5, -0.3, size=o_))
    ev = np.sort(rng.uniform(0.2, 3.0, size=v_))
    eps = np.concatenate([eo, ev])
    L0 = _sym_normal(rng, (nj_,), n, 0.05 * s)
    dF = _sym_normal(rng, (c["ncoord"],), n, c["sf"])
    dL = _sym_normal(rng, (c["ncoord"], nj_), n, c["sl"] * s)
    h0 = np.diag(eps) - _mean_field_part(L0, L0, o_)
    dh = np.empty_like(dF)
    for k in range(c["ncoord"]):
        g1 = _mean_field_part(dL[k], L0, o_) + _mean_field_part(L0, dL[k], o_)
        dh[k] = dF[k] - g1
    return System(name=name, o=o_, v=v_, nj=nj_, nstates=c["nstates"],
                  ncoord=c["ncoord"], nacs=list(c["nacs"]), eps=eps,
                  h0=h0.astype(dtype), L0=L0.astype(dtype),
                  dF=dF.astype(dtype), dh=dh.astype(dtype),
                  dL=dL.astype(dtype), scale=s, seed=seed, reading=reading)


def random_amplitudes(o, v, seed, scale=0.05, nvec=1):
    """Seeded random singles [v,o] and symmetric doubles [v,o,v,o] arrays."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(nvec):
        t1 = rng.normal(0, scale, size=(v, o))
        t2 = rng.normal(0, scale, size=(v, o, v, o))
        t2 = 0.5 * (t2 + t2.transpose(2, 3, 0, 1))
        out.append((t1, t2))
    return out if nvec > 1 else out[0]


def trajectory(ncoord, ngeom, seed):
    """Smooth synthetic trajectory x_k(n) = A_k sin(2 pi f_k n / 100 + phi_k)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    A = rng.normal(0, 0.05, size=ncoord)
    f = rng.uniform(0.5, 2.0, size=ncoord)
    ph = rng.uniform(0, 2 * np.pi, size=ncoord)
    nn = np.arange(ngeom)[:, None]
    return A * np.sin(2 * np.pi * f * nn / 100.0 + ph)


def family_geometries(ncoord, seeds, std=0.05):
    """Geometries x ~ N(0, std^2) i.i.d. per coordinate, one seed each
    (training seeds 10000.., held-out seeds 20000..)."""
    return np.stack([np.random.Generator(np.random.PCG64(sd)).normal(0, std, size=ncoord) for sd in seeds])
