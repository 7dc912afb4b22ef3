"""Host logic of the device programs, run on the CPU: the programs are
dumped (tests/native/graph_dump.cpp, built against libscc.so) with the
storage plan the device uses, and interpreted with numpy in one flat arena
laid out as on the device, so that temporaries share memory exactly as
there.

- The residual program (after the setup program) matches the oracle's
  SCCSD residual, with X3 terms (Theory / CC and SCCSD sections); the
  right transformation matches the oracle's sigma, and the left
  transformation the oracle's reverse-mode derivative of <l, sigma(r)>.
- Every program gives the same outputs with and without the fusion of sums
  of products into multi-product contractions, on the same random inputs.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest
import torch

from oracle import cc
from synth_inputs import make_system, random_amplitudes

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
PKG = os.path.join(ROOT, "paper_2403_01007_amd")


@pytest.fixture(scope="module")
def dumper(tmp_path_factory):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not os.path.exists(os.path.join(PKG, "libscc.so")):
        pytest.skip("libscc.so not built")
    if not shutil.which(hipcc) and not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("graph")
    exe = str(d / "graph_dump")
    subprocess.run([hipcc, "-O1", "-std=c++17", os.path.join(HERE, "native", "graph_dump.cpp"), "-L", PKG, "-lscc",
                    f"-Wl,-rpath,{PKG}", "-o", exe], check=True, capture_output=True, timeout=600)

    def dump(o, v, nj, ns, fuse):
        out = str(d / f"g_{o}_{v}_{nj}_{ns}_{int(fuse)}.txt")
        subprocess.run([exe, str(o), str(v), str(nj), str(ns), "1" if fuse else "0", out], check=True,
                       capture_output=True, timeout=600)
        return Graph(out)
    return dump


class Graph:
    """The dump: tensors (zero / unused flags, dims, arena offset), ops,
    programs, host tensors and named keys."""

    def __init__(self, path):
        self.t, self.ops, self.progs, self.keys = {}, [], [], {}
        for line in open(path):
            w = line.split()
            tag = w[0]
            if tag == "A":
                self.arena = int(w[1])
            elif tag == "T":
                i, z, u, nd = int(w[1]), int(w[2]), int(w[3]), int(w[4])
                self.t[i] = dict(zero=bool(z), unused=bool(u), dims=tuple(int(x) for x in w[5:5 + nd]),
                                 off=int(w[5 + nd]))
            elif tag == "C":
                lab = lambda s: "" if s == "_" else s
                out, a, b, c0 = map(int, w[1:5])
                prods = [(a, b, lab(w[7]), lab(w[8]), float(w[5]))]
                nseg = int(w[10])
                for q in range(nseg):
                    x = w[11 + 5 * q:16 + 5 * q]
                    prods.append((int(x[0]), int(x[1]), lab(x[2]), lab(x[3]), float(x[4])))
                self.ops.append(("C", out, prods, c0, float(w[6]), lab(w[9])))
            elif tag == "L":
                out, lo, n = int(w[1]), w[2].replace("_", ""), int(w[3])
                terms = [(int(w[4 + 3 * q]), float(w[5 + 3 * q]), w[6 + 3 * q].replace("_", "")) for q in range(n)]
                self.ops.append(("L", out, lo, terms))
            elif tag in ("SL", "EM"):
                out, a, nd = int(w[1]), int(w[2]), int(w[3])
                self.ops.append((tag, out, a, [int(x) for x in w[4:4 + nd]]))
            elif tag == "N":
                self.ops.append(("N",))
            elif tag == "P":
                self.progs.append([int(x) for x in w[3:]])
            elif tag == "H":
                self.pinned = [int(x) for x in w[2:]]
            elif tag == "K":
                self.keys[w[1]] = [int(x) for x in w[2:]]
            elif tag == "B":
                self.batched = getattr(self, "batched", {})
                self.batched[int(w[1])] = int(w[2])

    def produced(self, prog):
        return {self.ops[k][1] for k in prog if self.ops[k][0] != "N"}

    def read(self, prog):
        ids = set()
        for k in prog:
            op = self.ops[k]
            if op[0] == "C":
                for a, b, *_ in op[2]:
                    ids |= {a, b}
                if op[3] >= 0:
                    ids.add(op[3])
            elif op[0] == "L":
                ids |= {i for i, _, _ in op[3]}
            elif op[0] in ("SL", "EM"):
                ids.add(op[2])
        return ids


class Arena:
    """Tensors at their device offsets in one flat FP64 array."""

    def __init__(self, g):
        self.g = g
        self.mem = np.full(g.arena, np.nan)

    def view(self, i):
        d = self.g.t[i]
        if d["zero"]:
            return np.zeros(d["dims"])
        n = int(np.prod(d["dims"], dtype=np.int64))
        assert d["off"] >= 0 and not d["unused"], f"tensor {i} has no storage"
        return self.mem[d["off"]:d["off"] + n].reshape(d["dims"])

    def set(self, i, val):
        self.view(i)[...] = val

    def run(self, prog):
        for k in prog:
            op = self.g.ops[k]
            kind = op[0]
            if kind == "N":
                continue
            if kind == "C":
                _, out, prods, c0, beta, lo = op
                acc = sum(alpha * np.einsum(f"{la},{lb}->{lo}", self.view(a), self.view(b))
                          for a, b, la, lb, alpha in prods)
                if c0 >= 0:
                    acc = acc + beta * self.view(c0)
                self.set(out, acc)
            elif kind == "L":
                _, out, lo, terms = op
                self.set(out, sum(c * np.einsum(f"{li}->{lo}", self.view(i)) for i, c, li in terms))
            elif kind == "SL":
                _, out, a, off = op
                src = self.view(a)
                sl = tuple(slice(o, o + n) for o, n in zip(off, self.g.t[out]["dims"]))
                self.set(out, src[sl])
            else:  # EM
                _, out, a, off = op
                dst = np.zeros(self.g.t[out]["dims"])
                sl = tuple(slice(o, o + n) for o, n in zip(off, self.g.t[a]["dims"]))
                dst[sl] = self.view(a)
                self.set(out, dst)


def _flat(x):
    return np.asarray(x, dtype=np.float64)


@pytest.mark.parametrize("name,ns", [("o2v3", 2), ("custom-o3v6-3", 3)])
def test_residual_and_transformations_match_oracle(dumper, name, ns):
    if name.startswith("custom"):
        S = make_system("custom", seed=17, o=3, v=6, nj=14, nstates=ns, ncoord=1, nacs=[(0, 1)], sf=0.01, sl=0.01)
    else:
        S = make_system(name, seed=7)
    g = dumper(S.o, S.v, S.nj, ns, True)
    h, L = S.at(np.zeros(S.ncoord))
    N = S.o + S.v
    t1, t2 = random_amplitudes(S.o, S.v, seed=5, scale=0.05)
    amps = random_amplitudes(S.o, S.v, seed=9, scale=0.3, nvec=ns)
    states = [(0.3 - 0.2 * k, amps[k][0], amps[k][1]) for k in range(ns)]
    npair = ns * (ns - 1) // 2
    zeta = 0.37 + 0.1 * np.arange(npair)
    A = Arena(g)
    K = g.keys
    A.set(K["In"][0], np.eye(N))
    A.set(K["Io"][0], np.eye(S.o))
    A.set(K["one"][0], 1.0)
    if not g.t[K["z2"][0]]["zero"]:
        A.set(K["z2"][0], 0.0)
    A.set(K["h"][0], h)
    A.set(K["L"][0], L)
    A.set(K["kappa"][0], 0.0)
    A.run(g.progs[0])  # setup: integrals at kappa = 0
    A.set(K["t1"][0], t1)
    A.set(K["t2"][0], t2)
    for p in range(npair):
        A.set(K[f"zeta{p}"][0], zeta[p])
    for k in range(ns):
        r0, r1, r2 = K[f"xs{k}"]
        for i, val in ((r0, states[k][0]), (r1, states[k][1]), (r2, states[k][2])):
            if not g.t[i]["zero"]:
                A.set(i, val)
    A.run(g.progs[1])  # residual
    T = lambda a: torch.as_tensor(_flat(a))
    gg = np.einsum("Jpq,Jrs->pqrs", L, L)
    rs = [tuple(T(x) for x in r) for r in states]
    E, s, d = cc.residual(T(h), T(gg), T(t1), T(t2), S.o, T(zeta), rs)
    assert abs(float(A.view(K["E"][0])) - float(E)) < 1e-11
    np.testing.assert_allclose(A.view(K["O1"][0]), s.numpy(), rtol=0, atol=1e-12)
    np.testing.assert_allclose(A.view(K["O2"][0]), d.numpy(), rtol=0, atol=1e-12)

    # right transformation of one vector (the programs' symmetric doubles)
    v1, v2 = random_amplitudes(S.o, S.v, seed=31, scale=0.3)
    vec = (0.7, v1, v2)
    A.run(g.progs[2])  # sigma: amplitude-only part
    for i, val in zip(K["vin"], vec):
        A.set(i, val)
    A.run(g.progs[3])
    s0, s1, s2 = cc.sigma(T(h), T(gg), T(t1), T(t2), S.o, T(vec[0]), T(vec[1]), T(vec[2]), T(zeta), rs)
    out = [A.view(i) for i in K["sig"]]
    assert abs(float(out[0]) - float(s0)) < 1e-11
    np.testing.assert_allclose(out[1], s1.numpy(), rtol=0, atol=1e-12)
    np.testing.assert_allclose(out[2], s2.numpy(), rtol=0, atol=1e-12)

    # left transformation: gradient of <l, sigma(r)> with respect to r,
    # restricted to symmetric doubles
    l1, l2 = random_amplitudes(S.o, S.v, seed=21, scale=0.3)
    lvec = (0.4, l1, l2)
    for i, val in zip(K["lin"], lvec):
        A.set(i, val)
    A.run(g.progs[4])
    r0, r1, r2 = (T(x).requires_grad_(True) for x in vec)
    q0, q1, q2 = cc.sigma(T(h), T(gg), T(t1), T(t2), S.o, r0, r1, r2, T(zeta), rs)
    val = T(lvec[0]) * q0 + torch.sum(T(l1) * q1) + torch.sum(T(l2) * q2)
    g0, g1, g2 = torch.autograd.grad(val, (r0, r1, r2))
    g2 = 0.5 * (g2 + g2.permute(2, 3, 0, 1))
    out = [A.view(i) for i in K["lout"]]
    o2 = 0.5 * (out[2] + out[2].transpose(2, 3, 0, 1))
    assert abs(float(out[0]) - float(g0)) < 1e-11
    np.testing.assert_allclose(out[1], g1.numpy(), rtol=0, atol=1e-12)
    np.testing.assert_allclose(o2, g2.numpy(), rtol=0, atol=1e-12)


def test_batched_transformations_match_single(dumper):
    """Every slot of the batched right and left transformations (leading
    batch index Z) equals the single-vector program on that slot's vector."""
    S = make_system("custom", seed=17, o=3, v=6, nj=14, nstates=2, ncoord=1, nacs=[(0, 1)], sf=0.01, sl=0.01)
    ns = 2
    g = dumper(S.o, S.v, S.nj, ns, True)
    K = g.keys
    h, L = S.at(np.zeros(S.ncoord))
    N = S.o + S.v
    A = Arena(g)
    A.set(K["In"][0], np.eye(N))
    A.set(K["Io"][0], np.eye(S.o))
    A.set(K["one"][0], 1.0)
    if not g.t[K["z2"][0]]["zero"]:
        A.set(K["z2"][0], 0.0)
    A.set(K["h"][0], h)
    A.set(K["L"][0], L)
    A.set(K["kappa"][0], 0.0)
    A.run(g.progs[0])
    t1, t2 = random_amplitudes(S.o, S.v, seed=5, scale=0.05)
    A.set(K["t1"][0], t1)
    A.set(K["t2"][0], t2)
    amps = random_amplitudes(S.o, S.v, seed=9, scale=0.3, nvec=ns)
    A.set(K["zeta0"][0], 0.41)
    for k in range(ns):
        for i, val in zip(K[f"xs{k}"], (0.3 - 0.2 * k, amps[k][0], amps[k][1])):
            if not g.t[i]["zero"]:
                A.set(i, val)
    A.run(g.progs[1])
    A.run(g.progs[2])
    nb = g.t[K["vinB"][0]]["dims"][0]
    vecs = random_amplitudes(S.o, S.v, seed=44, scale=0.3, nvec=nb)
    r0s = 0.1 + 0.2 * np.arange(nb)
    for single, batched, prog, progB, outs, outsB in (("vin", "vinB", 3, 12, "sig", "sigB"),
                                                      ("lin", "linB", 4, 13, "lout", "loutB")):
        for i, val in zip(K[batched], (r0s, np.stack([x[0] for x in vecs]), np.stack([x[1] for x in vecs]))):
            A.set(i, val)
        A.run(g.progs[progB])
        got = [A.view(i).copy() for i in K[outsB]]
        for j in range(nb):
            for i, val in zip(K[single], (r0s[j], vecs[j][0], vecs[j][1])):
                A.set(i, val)
            A.run(g.progs[prog])
            for q, i in enumerate(K[outs]):
                ref = A.view(i)
                np.testing.assert_allclose(got[q][j], ref, rtol=0, atol=1e-12 * max(1.0, float(np.abs(ref).max())))


def test_batched_lagrangian_matches_single(dumper):
    """Every slot of the batched Lagrangian product (all multiplier targets
    in lockstep) equals the single-target program on that slot's inputs."""
    g = dumper(3, 8, 16, 3, True)
    P_LAG_PRE, P_LAG, P_LAGB = 7, 8, 17
    pre, lag, lagB = g.progs[P_LAG_PRE], g.progs[P_LAG], g.progs[P_LAGB]
    A = Arena(g)
    rng = np.random.default_rng(77)
    produced = g.produced(pre) | g.produced(lag) | g.produced(lagB)
    shared = sorted((g.read(pre) | g.read(lag) | g.read(lagB)) - produced)
    bmap = g.batched
    batched_in = {b for s, b in bmap.items() if b in g.read(lagB) and b not in g.produced(lagB)}
    for i in shared:
        if g.t[i]["zero"] or i in batched_in:
            continue
        A.set(i, 0.3 * rng.normal(size=g.t[i]["dims"]))
    A.run(pre)
    ins = {s: b for s, b in bmap.items() if b in batched_in}
    outs = {s: b for s, b in bmap.items() if b in g.produced(lagB)}
    assert ins and outs
    for s, b in ins.items():
        A.set(b, 0.3 * rng.normal(size=g.t[b]["dims"]))
    A.run(lagB)
    got = {s: A.view(b).copy() for s, b in outs.items()}
    nb = next(iter(got.values())).shape[0]
    for j in range(nb):
        for s, b in ins.items():
            A.set(s, A.view(b)[j])
        A.run(lag)
        for s in outs:
            ref = A.view(s)
            scale = max(1.0, float(np.abs(ref).max()))
            assert np.abs(got[s][j] - ref).max() <= 1e-11 * scale, (j, s)


def test_fused_programs_match_unfused(dumper):
    o, v, nj, ns = 3, 8, 16, 3
    gf, gu = dumper(o, v, nj, ns, True), dumper(o, v, nj, ns, False)
    assert len(gf.progs) == len(gu.progs)
    nfused = sum(1 for op in gf.ops if op[0] == "C" and len(op[2]) > 1)
    assert nfused > 0, "no sums of products were fused at this size"
    # outputs of a program: host tensors, and tensors read by another
    # program that does not compute them itself
    readers = {}
    for p, prog in enumerate(gu.progs):
        for i in gu.read(prog) - gu.produced(prog):
            readers.setdefault(i, set()).add(p)
    pinned = set(gu.pinned)
    checked = 0
    for p, (pf, pu) in enumerate(zip(gf.progs, gu.progs)):
        ins = sorted(gu.read(pu) - gu.produced(pu))
        outs = sorted(i for i in gu.produced(pu) if i in pinned or readers.get(i, set()) - {p})
        rng = np.random.default_rng(1000 + p)
        vals = {i: rng.normal(size=gu.t[i]["dims"]) for i in ins if not gu.t[i]["zero"]}
        res = []
        for g, prog in ((gf, pf), (gu, pu)):
            A = Arena(g)
            for i, x in vals.items():
                A.set(i, x)
            A.run(prog)
            res.append({i: A.view(i).copy() for i in outs})
        for i in outs:
            a, b = res[0][i], res[1][i]
            scale = max(1.0, float(np.abs(b).max()))
            assert np.abs(a - b).max() <= 1e-11 * scale, (p, i, float(np.abs(a - b).max()), scale)
            checked += 1
    assert checked > 0
