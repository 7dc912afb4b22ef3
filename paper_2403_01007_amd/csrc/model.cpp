// SCCSD(E) programs: CCSD residual (Cholesky form), SCC triple-excitation
// terms, right/left transformations, the orthogonality overlap, and the
// gradient / coupling Lagrangian with its derivative programs.
#include "model.hpp"

#include <stdexcept>

namespace scc {

namespace {

int at(const std::vector<int>& v, int id) { return (id >= 0 && id < (int)v.size()) ? v[id] : -1; }

// exp(-T1) H exp(T1) applied to the rotated integrals (hk, Lk): the
// T1-transformed one-electron integrals, Cholesky vectors, Fock matrix,
// reference energy and the dressed two-electron blocks the CCSD terms use.
struct Dressed {
  int hh, LL, Loo, Lov, Lvo, Lvv, F, Foo, Fov, Fvo, Fvv;
  int govov, goooo, gooov, goovv, gvoov, gvovo, Lovov, Lvoov, e_ref;
};

Dressed build_dressed(Model& m, int t1) {
  Graph& g = m.g;
  const Dims& d = m.d;
  const int64_t o = d.o, v = d.v, n = d.n, J = d.nj;
  Dressed D;
  int Tm = g.embed(t1, {o, 0}, {n, n});
  int X = g.lincomb("pq", {{1.0, m.In, "pq"}, {-1.0, Tm, "pq"}});
  int Y = g.lincomb("pq", {{1.0, m.In, "pq"}, {1.0, Tm, "pq"}});
  D.hh = g.contract("pr,rq->pq", g.contract("pr,rq->pq", X, m.hk), Y);
  D.LL = g.contract("Jpr,rq->Jpq", g.contract("pr,Jrq->Jpq", X, m.Lk), Y);
  D.Loo = g.slice(D.LL, {0, 0, 0}, {J, o, o});
  D.Lov = g.slice(D.LL, {0, 0, o}, {J, o, v});
  D.Lvo = g.slice(D.LL, {0, o, 0}, {J, v, o});
  D.Lvv = g.slice(D.LL, {0, o, o}, {J, v, v});
  int LNo = g.slice(D.LL, {0, 0, 0}, {J, n, o});
  int LoN = g.slice(D.LL, {0, 0, 0}, {J, o, n});
  int hoo = g.slice(D.hh, {0, 0}, {o, o});
  int dJ = g.contract("Jkl,kl->J", D.Loo, m.Io);
  D.F = g.contract("Jpk,Jkq->pq", LNo, LoN, -1.0, g.contract("Jpq,J->pq", D.LL, dJ, 2.0, D.hh));
  D.Foo = g.slice(D.F, {0, 0}, {o, o});
  D.Fov = g.slice(D.F, {0, o}, {o, v});
  D.Fvo = g.slice(D.F, {o, 0}, {v, o});
  D.Fvv = g.slice(D.F, {o, o}, {v, v});
  D.govov = g.contract("Jia,Jjb->iajb", D.Lov, D.Lov);
  D.goooo = g.contract("Jij,Jkl->ijkl", D.Loo, D.Loo);
  D.gooov = g.contract("Jki,Jlc->kilc", D.Loo, D.Lov);
  D.goovv = g.contract("Jki,Jac->kiac", D.Loo, D.Lvv);
  D.gvoov = g.contract("Jai,Jkc->aikc", D.Lvo, D.Lov);
  D.gvovo = g.contract("Jai,Jbj->aibj", D.Lvo, D.Lvo);
  D.Lovov = g.lincomb("iajb", {{2.0, D.govov, "iajb"}, {-1.0, D.govov, "ibja"}});
  D.Lvoov = g.lincomb("aikc", {{2.0, D.gvoov, "aikc"}, {-1.0, D.goovv, "kiac"}});
  int e = g.contract("ij,ij->", hoo, m.Io, 2.0);
  e = g.contract("J,J->", dJ, dJ, 2.0, e);
  D.e_ref = g.contract("Jij,Jji->", D.Loo, D.Loo, -1.0, e);
  return D;
}

// Closed-shell CCSD projections <HF|Hbar|HF>, <mu_1|Hbar|HF>, <mu_2|Hbar|HF>
// of the T1-transformed Hamiltonian for the doubles operator X (T1-transformed
// spin-adapted formulation).  linear = true keeps only the terms linear in X,
// i.e. <mu|[H^, X]|HF>.  The vvvv ladder uses the bare block G_acbd with the
// exact T1 dependence of the dressed integrals written out through the ovvv
// and ovov blocks, so no T1-dressed v^4 tensor is ever formed.
CCOut build_terms(Model& m, const Dressed& D, int t1, int t2, bool linear) {
  Graph& g = m.g;
  int E = g.contract("aibj,iajb->", t2, D.Lovov, 1.0, linear ? -1 : D.e_ref);
  int u = g.lincomb("aibj", {{2.0, t2, "aibj"}, {-1.0, t2, "ajbi"}});
  // singles
  int Y1 = g.contract("ckdi,Jkc->Jdi", u, D.Lov);
  int s = g.contract("Jad,Jdi->ai", D.Lvv, Y1, 1.0, linear ? -1 : D.Fvo);
  s = g.contract("akcl,kilc->ai", u, D.gooov, -1.0, s);
  int O1 = g.contract("aick,kc->ai", u, D.Fov, 1.0, s);
  // doubles: particle-particle ladder
  int lad = g.contract("abcd,cidj->aibj", m.G, t2);
  int W = g.contract("kcbd,cidj->kibj", m.Govvv, t2);
  int tw = g.contract("ak,kibj->aibj", t1, W);
  int V = g.contract("kcld,cidj->kilj", m.Govov, t2);
  int ttv = g.contract("bl,ailj->aibj", t1, g.contract("ak,kilj->ailj", t1, V));
  std::vector<Graph::Term> a2 = {{1.0, lad, "aibj"}, {-1.0, tw, "aibj"}, {-1.0, tw, "bjai"}, {1.0, ttv, "aibj"}};
  if (!linear) a2.push_back({1.0, D.gvovo, "aibj"});
  int A2 = g.lincomb("aibj", a2);
  // hole-hole ladder
  int chi = linear ? D.goooo : g.contract("cidj,kcld->kilj", t2, D.govov, 1.0, D.goooo);
  int B2 = g.contract("akbl,kilj->aibj", t2, chi);
  // ring terms
  int Wc = linear ? D.goovv : g.contract("dial,kdlc->kiac", t2, D.govov, -0.5, D.goovv);
  int C2 = g.contract("bkci,kjac->aibj", t2, Wc, -1.0, g.contract("bkcj,kiac->aibj", t2, Wc, -0.5));
  int Q = linear ? D.Lvoov : g.contract("aidl,ldkc->aikc", u, D.Lovov, 0.5, D.Lvoov);
  int D2 = g.contract("bjck,aikc->aibj", u, Q, 0.5);
  // Fock-dressed terms
  int Fvv2 = linear ? D.Fvv : g.contract("bkdl,ldkc->bc", u, D.govov, -1.0, D.Fvv);
  int Foo2 = linear ? D.Foo : g.contract("cldj,kdlc->kj", u, D.govov, 1.0, D.Foo);
  int E2 = g.contract("aibk,kj->aibj", t2, Foo2, -1.0, g.contract("aicj,bc->aibj", t2, Fvv2));
  int P = g.lincomb("aibj", {{1.0, C2, "aibj"}, {1.0, D2, "aibj"}, {1.0, E2, "aibj"}});
  int O2 = g.lincomb("aibj", {{1.0, A2, "aibj"}, {1.0, B2, "aibj"}, {1.0, P, "aibj"}, {1.0, P, "bjai"}});
  return {E, O1, O2};
}

int or_zeros(Graph& g, int id, const std::vector<int64_t>& dims) { return id >= 0 ? id : g.zeros(dims); }

// SCCSD residual: CCSD projections plus sum_{k<l} zeta_kl <mu|[H^, X3^kl]|HF>,
// X3^kl = R1^k R2^l - R1^l R2^k (higher commutators vanish in these
// projections).  For singles P1 and doubles Q2, with S = e P1 + d Q2,
// H^ exp(S)|HF> = exp(S) Hbar_S|HF>, Hbar_S having CC projections (E, O1, O2)
// at amplitudes (t1 + e P1, d Q2); the e d coefficient gives
//   <mu_1|H^ P1 Q2|HF> = O1_ed + P1 E_d
//   <mu_2|H^ P1 Q2|HF> = O2_ed + {P1, O1_d} + Q2 E_e
// where the d-derivatives are the terms linear in Q2 and the e-derivatives
// are directional derivatives along t1 -> P1.  Since this is linear in Q2,
// the pairs sharing R1^k are summed first: Q2^k = sum_l (+-) zeta_kl R2^l.
CCOut build_residual(Model& m, int t1, int t2, const std::vector<int>& zeta, const std::vector<StateT>& xs) {
  Graph& g = m.g;
  const int64_t o = m.d.o, v = m.d.v;
  int db = (int)g.ops.size();
  Dressed D = build_dressed(m, t1);
  int de = (int)g.ops.size();
  CCOut c = build_terms(m, D, t1, t2, false);
  int O1 = c.O1, O2 = c.O2;
  const int ns = (int)xs.size();
  if (ns < 2) return c;
  for (int k = 0; k < ns; ++k) {
    // Q2^k = sum_{l>k} zeta_kl R2^l - sum_{l<k} zeta_lk R2^l
    int Q2 = g.zeros({v, o, v, o});
    for (int l = 0; l < ns; ++l) {
      if (l == k) continue;
      int a = std::min(k, l), b = std::max(k, l);
      int p = a * ns - a * (a + 1) / 2 + (b - a - 1);
      Q2 = g.contract(",aibj->aibj", zeta[p], xs[l].r2, k < l ? 1.0 : -1.0, Q2);
    }
    const int P1 = xs[k].r1;
    // e-derivatives of the dressed integrals along t1 -> P1
    auto td = g.jvp(db, de, {{t1, P1}});
    std::map<int, int> seeds = {{t1, P1}};
    for (int id = 0; id < (int)td.size(); ++id)
      if (td[id] >= 0) seeds[id] = td[id];
    int lb = (int)g.ops.size();
    CCOut lin = build_terms(m, D, t1, Q2, true);
    int le = (int)g.ops.size();
    auto ta = g.jvp(lb, le, seeds);
    int E_e = at(td, D.e_ref);
    int O1_ed = at(ta, lin.O1), O2_ed = at(ta, lin.O2);
    int s = or_zeros(g, O1_ed, {v, o});
    s = g.contract(",ai->ai", lin.E, P1, 1.0, s);
    int dd = or_zeros(g, O2_ed, {v, o, v, o});
    if (E_e >= 0) dd = g.contract(",aibj->aibj", E_e, Q2, 1.0, dd);
    int x = g.contract("ai,bj->aibj", P1, lin.O1);
    dd = g.lincomb("aibj", {{1.0, dd, "aibj"}, {1.0, x, "aibj"}, {1.0, x, "bjai"}});
    O1 = g.lincomb("ai", {{1.0, O1, "ai"}, {1.0, s, "ai"}});
    O2 = g.lincomb("aibj", {{1.0, O2, "aibj"}, {1.0, dd, "aibj"}});
  }
  return {c.E, O1, O2};
}

// calHbar calR for calR = (r0, r1, r2), from the residual program ops[b, e):
//   <HF|Hbar|R> = E0 r0 + eta.R,  <mu|Hbar|R> = Omega r0 + A R + E0 R + {R1, Omega1}
// with A R and eta.R the directional derivatives of (Omega, E0) along R.
SigmaOut build_sigma(Model& m, int b, int e, const CCOut& r, int t1, int t2, const StateT& v) {
  Graph& g = m.g;
  const int64_t o = m.d.o, vv = m.d.v;
  auto tg = g.jvp(b, e, {{t1, v.r1}, {t2, v.r2}});
  int dE = at(tg, r.E), dO1 = at(tg, r.O1), dO2 = at(tg, r.O2);
  int s0 = g.contract(",->", r.E, v.r0, 1.0, dE);
  int s1 = g.contract(",ai->ai", v.r0, r.O1, 1.0, or_zeros(g, dO1, {vv, o}));
  s1 = g.contract(",ai->ai", r.E, v.r1, 1.0, s1);
  int s2 = g.contract(",aibj->aibj", v.r0, r.O2, 1.0, or_zeros(g, dO2, {vv, o, vv, o}));
  s2 = g.contract(",aibj->aibj", r.E, v.r2, 1.0, s2);
  int x = g.contract("ai,bj->aibj", v.r1, r.O1);
  s2 = g.lincomb("aibj", {{1.0, s2, "aibj"}, {1.0, x, "aibj"}, {1.0, x, "bjai"}});
  return {s0, s1, s2};
}

// coefficients of P_E exp(T1 + T2) |R>
StateT project_exp_t(Model& m, int t1, int t2, const StateT& r) {
  Graph& g = m.g;
  int c1 = g.contract(",ai->ai", r.r0, t1, 1.0, r.r1);
  int tr = g.contract("ai,bj->aibj", t1, r.r1);
  int tt = g.contract("ai,bj->aibj", t1, t1);
  int t2t = g.lincomb("aibj", {{1.0, t2, "aibj"}, {1.0, tt, "aibj"}});
  int c2 = g.lincomb("aibj", {{1.0, r.r2, "aibj"}, {1.0, tr, "aibj"}, {1.0, tr, "bjai"}});
  c2 = g.contract(",aibj->aibj", r.r0, t2t, 1.0, c2);
  return {r.r0, c1, c2};
}

// O_ab = <P exp(T) R_a | P exp(T) R_b>: physical metric of the spin-adapted
// excitation space, <X|Y> = X0 Y0 + 2 X1.Y1 + X2.(2 Y2 - Y2^(aj,bi)).
int build_overlap(Model& m, int t1, int t2, const StateT& a, const StateT& b) {
  Graph& g = m.g;
  StateT ca = project_exp_t(m, t1, t2, a);
  StateT cb = project_exp_t(m, t1, t2, b);
  int x = g.contract(",->", ca.r0, cb.r0);
  x = g.contract("ai,ai->", ca.r1, cb.r1, 2.0, x);
  int m2 = g.lincomb("aibj", {{2.0, cb.r2, "aibj"}, {-1.0, cb.r2, "ajbi"}});
  return g.contract("aibj,aibj->", ca.r2, m2, 1.0, x);
}

int full_dot(Graph& g, const StateT& a, const StateT& b) {
  int x = g.contract(",->", a.r0, b.r0);
  x = g.contract("ai,ai->", a.r1, b.r1, 1.0, x);
  return g.contract("aibj,aibj->", a.r2, b.r2, 1.0, x);
}

StateT new_state(Graph& g, const Dims& d, const char* name) {
  const int64_t o = d.o, v = d.v;
  std::string s(name);
  return {g.tensor({}, s + ".r0"), g.tensor({v, o}, s + ".r1"), g.tensor({v, o, v, o}, s + ".r2")};
}

int fock_full(Model& m, int hk, int Lk) {
  Graph& g = m.g;
  const int64_t o = m.d.o, n = m.d.n, J = m.d.nj;
  int Loo = g.slice(Lk, {0, 0, 0}, {J, o, o});
  int dJ = g.contract("Jkl,kl->J", Loo, m.Io);
  int LNo = g.slice(Lk, {0, 0, 0}, {J, n, o});
  int LoN = g.slice(Lk, {0, 0, 0}, {J, o, n});
  return g.contract("Jpk,Jkq->pq", LNo, LoN, -1.0, g.contract("Jpq,J->pq", Lk, dJ, 2.0, hk));
}

int fock_vo(Model& m, int F) {
  const int64_t o = m.d.o, v = m.d.v;
  return m.g.slice(F, {o, 0}, {v, o});
}

std::vector<int> minus(const std::vector<int>& a, const std::vector<int>& b) {
  std::set<int> sb(b.begin(), b.end());
  std::vector<int> r;
  for (int x : a)
    if (!sb.count(x)) r.push_back(x);
  return r;
}

std::set<int> outputs_of(const Graph& g, const std::vector<int>& list) {
  std::set<int> s;
  for (int k : list) s.insert(g.ops[k].out);
  return s;
}

}  // namespace

void build_model(Model& m, const Dims& d, int nb, int nbt) {
  m.d = d;
  m.nb = nb;
  m.nbt = nbt;
  Graph& g = m.g;
  const int64_t o = d.o, v = d.v, n = d.n, J = d.nj;
  const int ns = d.ns, np = d.npairs();
  // constants and inputs
  m.In = g.tensor({n, n}, "I_N");
  m.Io = g.tensor({o, o}, "I_o");
  m.one = g.tensor({}, "one");
  m.z2 = g.tensor({v, o, v, o}, "zero_t2");
  m.h = g.tensor({n, n}, "h");
  m.L = g.tensor({J, n, n}, "L");
  m.kappa = g.tensor({v, o}, "kappa");
  // orbital rotation exp(kappa) H exp(-kappa) to first order, U = 1 + K - K^T
  int K = g.embed(m.kappa, {o, 0}, {n, n});
  int U = g.lincomb("pq", {{1.0, m.In, "pq"}, {1.0, K, "pq"}, {-1.0, K, "qp"}});
  m.hk = g.contract("ps,qs->pq", g.contract("pr,rs->ps", U, m.h), U);
  m.Lk = g.contract("Jps,qs->Jpq", g.contract("pr,Jrs->Jps", U, m.L), U);
  int Lkvv = g.slice(m.Lk, {0, o, o}, {J, v, v});
  int Lkov = g.slice(m.Lk, {0, 0, o}, {J, o, v});
  m.G = g.contract("Jac,Jbd->abcd", Lkvv, Lkvv);
  m.Govvv = g.contract("Jkc,Jbd->kcbd", Lkov, Lkvv);
  m.Govov = g.contract("Jkc,Jld->kcld", Lkov, Lkov);
  m.fock = fock_full(m, m.hk, m.Lk);
  m.p_setup = g.needed_ops({m.hk, m.Lk, m.G, m.Govvv, m.Govov, m.fock});
  std::set<int> have = outputs_of(g, m.p_setup);

  // ---- ground-state residual
  m.t1 = g.tensor({v, o}, "t1");
  m.t2 = g.tensor({v, o, v, o}, "t2");
  for (int p = 0; p < np; ++p) m.zeta.push_back(g.tensor({}, "zeta"));
  for (int k = 0; k < ns; ++k) m.xs.push_back(new_state(g, d, "xs"));
  m.res_begin = (int)g.ops.size();
  m.res = build_residual(m, m.t1, m.t2, m.zeta, m.xs);
  m.res_end = (int)g.ops.size();
  m.p_res = g.needed_ops({m.res.E, m.res.O1, m.res.O2}, have);

  // ---- right transformation
  m.vin = new_state(g, d, "vin");
  m.sig = build_sigma(m, m.res_begin, m.res_end, m.res, m.t1, m.t2, m.vin);
  int sig_end = (int)g.ops.size();
  m.sig_end = sig_end;
  {
    auto all = g.needed_ops({m.sig.s0, m.sig.s1, m.sig.s2}, have);
    m.p_sig = g.dependent_ops(all, {m.vin.r0, m.vin.r1, m.vin.r2});
    m.p_sig_pre = minus(all, m.p_sig);
  }
  // ---- left transformation (adjoint of sigma with respect to calR)
  m.lin = new_state(g, d, "lin");
  {
    auto adj = g.vjp(m.res_begin, sig_end, {{m.sig.s0, m.lin.r0}, {m.sig.s1, m.lin.r1}, {m.sig.s2, m.lin.r2}},
                     {m.vin.r0, m.vin.r1, m.vin.r2, m.hk});
    m.lout = {or_zeros(g, adj[m.vin.r0], {}), or_zeros(g, adj[m.vin.r1], {v, o}),
              or_zeros(g, adj[m.vin.r2], {v, o, v, o})};
    m.dens_hk = or_zeros(g, adj[m.hk], {n, n});
    auto all = g.needed_ops({m.lout.r0, m.lout.r1, m.lout.r2}, have);
    m.p_left = g.dependent_ops(all, {m.lin.r0, m.lin.r1, m.lin.r2});
    auto alld = g.needed_ops({m.dens_hk}, have);
    m.p_dens = g.dependent_ops(alld, {m.lin.r0, m.lin.r1, m.lin.r2, m.vin.r0, m.vin.r1, m.vin.r2});
  }
  // ---- batched right and left transformations
  if (nb > 1) {
    std::map<int, int> mp;
    m.p_sigB = g.batchify(m.p_sig, {m.vin.r0, m.vin.r1, m.vin.r2}, nb, mp);
    m.vinB = {mp.at(m.vin.r0), mp.at(m.vin.r1), mp.at(m.vin.r2)};
    m.sigB = {mp.at(m.sig.s0), mp.at(m.sig.s1), mp.at(m.sig.s2)};
    std::map<int, int> ml;
    m.p_leftB = g.batchify(m.p_left, {m.lin.r0, m.lin.r1, m.lin.r2}, nb, ml);
    m.linB = {ml.at(m.lin.r0), ml.at(m.lin.r1), ml.at(m.lin.r2)};
    m.loutB = {ml.at(m.lout.r0), ml.at(m.lout.r1), ml.at(m.lout.r2)};
  }
  // ---- overlap of two states
  m.oa = new_state(g, d, "oa");
  m.ob = new_state(g, d, "ob");
  m.ovl = build_overlap(m, m.t1, m.t2, m.oa, m.ob);
  m.p_ovl = g.needed_ops({m.ovl}, have);

  // ---- Lagrangian
  m.pt1 = g.tensor({v, o}, "pt1");
  m.pt2 = g.tensor({v, o, v, o}, "pt2");
  for (int p = 0; p < np; ++p) m.pz.push_back(g.tensor({}, "pz"));
  for (int k = 0; k < ns; ++k) {
    m.pr.push_back(new_state(g, d, "pr"));
    m.pE.push_back(g.tensor({}, "pE"));
    m.lam.push_back(new_state(g, d, "lam"));
  }
  int lb = (int)g.ops.size();
  m.pres = build_residual(m, m.pt1, m.pt2, m.pz, m.pr);
  int le = (int)g.ops.size();
  std::vector<int> cons;
  for (int k = 0; k < ns; ++k) {
    SigmaOut s = build_sigma(m, lb, le, m.pres, m.pt1, m.pt2, m.pr[k]);
    int c0 = g.contract(",->", m.pE[k], m.pr[k].r0, -1.0, s.s0);
    int c1 = g.contract(",ai->ai", m.pE[k], m.pr[k].r1, -1.0, s.s1);
    int c2 = g.contract(",aibj->aibj", m.pE[k], m.pr[k].r2, -1.0, s.s2);
    m.pc.push_back({c0, c1, c2});
    int dt = full_dot(g, m.lam[k], m.pr[k]);
    m.pN.push_back(g.lincomb("", {{1.0, m.one, ""}, {-1.0, dt, ""}}));
  }
  for (int k = 0; k < ns; ++k)
    for (int l = k + 1; l < ns; ++l) m.pO.push_back(build_overlap(m, m.pt1, m.pt2, m.pr[k], m.pr[l]));
  m.fai = fock_vo(m, m.fock);
  int lag_end = (int)g.ops.size();
  // multipliers
  m.m1 = g.tensor({v, o}, "m1");
  m.m2 = g.tensor({v, o, v, o}, "m2");
  std::map<int, int> seeds = {{m.pres.O1, m.m1}, {m.pres.O2, m.m2}};
  for (int k = 0; k < ns; ++k) {
    StateT mm = new_state(g, d, "mk");
    m.mk.push_back({mm.r0, mm.r1, mm.r2});
    m.mN.push_back(g.tensor({}, "mN"));
    seeds[m.pc[k].s0] = mm.r0;
    seeds[m.pc[k].s1] = mm.r1;
    seeds[m.pc[k].s2] = mm.r2;
    seeds[m.pN[k]] = m.mN[k];
  }
  for (int p = 0; p < np; ++p) {
    m.mO.push_back(g.tensor({}, "mO"));
    seeds[m.pO[p]] = m.mO[p];
  }
  m.mF = g.tensor({v, o}, "mF");
  std::set<int> mult_in = {m.m1, m.m2, m.mF};
  for (auto& x : m.mk) {
    mult_in.insert(x.s0);
    mult_in.insert(x.s1);
    mult_in.insert(x.s2);
  }
  for (int x : m.mN) mult_in.insert(x);
  for (int x : m.mO) mult_in.insert(x);
  // J^T lambda-bar with respect to the CC parameters
  std::vector<int> params = {m.pt1, m.pt2};
  for (int z : m.pz) params.push_back(z);
  for (int k = 0; k < ns; ++k) {
    params.push_back(m.pr[k].r0);
    params.push_back(m.pr[k].r1);
    params.push_back(m.pr[k].r2);
    params.push_back(m.pE[k]);
  }
  {
    auto adj = g.vjp(0, lag_end, seeds, params);
    m.a_t1 = or_zeros(g, adj[m.pt1], {v, o});
    m.a_t2 = or_zeros(g, adj[m.pt2], {v, o, v, o});
    for (int z : m.pz) m.a_z.push_back(or_zeros(g, adj[z], {}));
    for (int k = 0; k < ns; ++k) {
      m.a_r.push_back({or_zeros(g, adj[m.pr[k].r0], {}), or_zeros(g, adj[m.pr[k].r1], {v, o}),
                       or_zeros(g, adj[m.pr[k].r2], {v, o, v, o})});
      m.a_E.push_back(or_zeros(g, adj[m.pE[k]], {}));
    }
    std::vector<int> outs = {m.a_t1, m.a_t2};
    for (int x : m.a_z) outs.push_back(x);
    for (auto& r : m.a_r) {
      outs.push_back(r.r0);
      outs.push_back(r.r1);
      outs.push_back(r.r2);
    }
    for (int x : m.a_E) outs.push_back(x);
    auto all = g.needed_ops(outs, have);
    m.p_lag = g.dependent_ops(all, mult_in);
    m.p_lag_pre = minus(all, m.p_lag);
    if (nbt > 1) {
      std::vector<int> ins;
      for (int x : mult_in)
        if (x != m.mF) ins.push_back(x);
      std::map<int, int> mp;
      m.p_lagB = g.batchify(m.p_lag, ins, nbt, mp);
      for (int x : ins) m.lagB[x] = mp.at(x);
      for (int x : outs)
        if (mp.count(x)) m.lagB[x] = mp.at(x);
    }
  }
  // orbital-rotation and integral adjoints (kappa-bar enters through F_ai)
  {
    std::map<int, int> s2 = seeds;
    s2[m.fai] = m.mF;
    auto adj = g.vjp(0, lag_end, s2, {m.kappa, m.h, m.L});
    m.a_kappa = or_zeros(g, adj[m.kappa], {v, o});
    m.a_h = or_zeros(g, adj[m.h], {n, n});
    m.a_L = or_zeros(g, adj[m.L], {J, n, n});
    auto allk = g.needed_ops({m.a_kappa}, have);
    m.p_kappa = g.dependent_ops(allk, mult_in);
    auto alli = g.needed_ops({m.a_h, m.a_L}, have);
    m.p_integral = g.dependent_ops(alli, mult_in);
    // A_HF^T kbar alone
    auto adjf = g.vjp(0, lag_end, {{m.fai, m.mF}}, {m.kappa});
    m.fk_adj = or_zeros(g, adjf[m.kappa], {v, o});
    auto allf = g.needed_ops({m.fk_adj}, have);
    m.p_fk = g.dependent_ops(allf, {m.mF});
    // primal values every adjoint program reads, computed once per solution
    std::set<int> pre(m.p_lag_pre.begin(), m.p_lag_pre.end());
    for (auto* pr : {&allk, &alli, &allf})
      for (int k : minus(*pr, g.dependent_ops(*pr, mult_in))) pre.insert(k);
    m.p_lag_pre.assign(pre.begin(), pre.end());
  }
  // fixed-basis Hamiltonian: Fock matrix of the closed-shell determinant
  // of orbitals Cmo, F = h + sum_J [2 L^J tr(L^J D) - L^J D L^J] with
  // D = C_occ C_occ^T; MO integrals C^T h C, C^T L^J C; densities back to
  // the fixed basis, C D1 C^T and C Z^J C^T
  {
    m.hao = g.tensor({n, n}, "h_fixed");
    m.Lao = g.tensor({J, n, n}, "L_fixed");
    m.Cmo = g.tensor({n, n}, "C");
    int b0 = (int)g.ops.size();
    int Cocc = g.slice(m.Cmo, {0, 0}, {n, o});
    int Dao = g.contract("pi,qi->pq", Cocc, Cocc);
    int dJ = g.contract("Jpq,pq->J", m.Lao, Dao);
    int X = g.contract("Jpr,rs->Jps", m.Lao, Dao);
    m.Fao = g.contract("Jps,Jsq->pq", X, m.Lao, -1.0, g.contract("Jpq,J->pq", m.Lao, dJ, 2.0, m.hao));
    int b1 = (int)g.ops.size();
    m.hmo = g.contract("pP,pQ->PQ", m.Cmo, g.contract("pq,qQ->pQ", m.hao, m.Cmo));
    m.Lmo = g.contract("pP,JpQ->JPQ", m.Cmo, g.contract("Jpq,qQ->JpQ", m.Lao, m.Cmo));
    int b2 = (int)g.ops.size();
    m.d1ao = g.contract("pP,Pq->pq", m.Cmo, g.contract("PQ,qQ->Pq", m.a_h, m.Cmo));
    m.zao = g.contract("pP,JPq->Jpq", m.Cmo, g.contract("JPQ,qQ->JPq", m.a_L, m.Cmo));
    int b3 = (int)g.ops.size();
    for (int k = b0; k < b1; ++k) m.p_aofock.push_back(k);
    for (int k = b1; k < b2; ++k) m.p_aotrans.push_back(k);
    for (int k = b2; k < b3; ++k) m.p_aodens.push_back(k);
  }
  // coupling targets O_mn for each ket state n
  m.nac_l = new_state(g, d, "nac_l");
  m.nac_t1c = g.tensor({v, o}, "nac_t1c");
  m.nac_t2c = g.tensor({v, o, v, o}, "nac_t2c");
  for (int k = 0; k < ns; ++k) {
    int begin = (int)g.ops.size();
    int d1 = g.lincomb("ai", {{1.0, m.pt1, "ai"}, {-1.0, m.nac_t1c, "ai"}});
    int d2 = g.lincomb("aibj", {{1.0, m.pt2, "aibj"}, {-1.0, m.nac_t2c, "aibj"}});
    StateT c = project_exp_t(m, d1, d2, m.pr[k]);
    int onac = full_dot(g, m.nac_l, c);
    int end = (int)g.ops.size();
    auto adj = g.vjp(begin, end, {{onac, m.one}}, {m.pt1, m.pt2, m.pr[k].r0, m.pr[k].r1, m.pr[k].r2});
    m.onac.push_back(onac);
    m.a_nac_t1.push_back(or_zeros(g, adj[m.pt1], {v, o}));
    m.a_nac_t2.push_back(or_zeros(g, adj[m.pt2], {v, o, v, o}));
    m.a_nac_r.push_back({or_zeros(g, adj[m.pr[k].r0], {}), or_zeros(g, adj[m.pr[k].r1], {v, o}),
                         or_zeros(g, adj[m.pr[k].r2], {v, o, v, o})});
    m.p_nac.push_back(g.needed_ops({m.onac[k], m.a_nac_t1[k], m.a_nac_t2[k], m.a_nac_r[k].r0,
                                    m.a_nac_r[k].r1, m.a_nac_r[k].r2},
                                   have));
  }
}

std::vector<int> host_tensors(const Model& m) {
  std::vector<int> r = {m.In,   m.Io,  m.one,     m.z2,      m.h,      m.L,      m.kappa,  m.hk,   m.Lk,
                        m.G,    m.fock, m.t1,     m.t2,      m.res.E,  m.res.O1, m.res.O2, m.sig.s0, m.sig.s1,
                        m.sig.s2, m.ovl, m.dens_hk, m.pt1, m.pt2,    m.fai,    m.m1,     m.m2,   m.mF,
                        m.a_t1, m.a_t2, m.a_kappa, m.a_h,     m.a_L,    m.fk_adj, m.nac_t1c, m.nac_t2c,
                        m.hao,  m.Lao,  m.Cmo,     m.Fao,     m.hmo,    m.Lmo,    m.d1ao,    m.zao};
  auto st = [&](const StateT& s) {
    r.push_back(s.r0);
    r.push_back(s.r1);
    r.push_back(s.r2);
  };
  auto sg = [&](const SigmaOut& s) {
    r.push_back(s.s0);
    r.push_back(s.s1);
    r.push_back(s.s2);
  };
  for (auto* v : {&m.zeta, &m.pz, &m.pE, &m.mN, &m.mO, &m.a_z, &m.a_E, &m.onac, &m.a_nac_t1, &m.a_nac_t2})
    r.insert(r.end(), v->begin(), v->end());
  for (auto* v : {&m.xs, &m.pr, &m.lam, &m.a_r, &m.a_nac_r})
    for (auto& s : *v) st(s);
  for (auto& s : m.mk) sg(s);
  for (const StateT* s : {&m.vin, &m.lin, &m.lout, &m.oa, &m.ob, &m.nac_l, &m.vinB, &m.sigB, &m.linB, &m.loutB})
    st(*s);
  for (auto& kv : m.lagB) r.push_back(kv.second);
  return r;
}

std::vector<const std::vector<int>*> programs(const Model& m) {
  std::vector<const std::vector<int>*> r = {&m.p_setup, &m.p_res,      &m.p_sig_pre, &m.p_sig,   &m.p_left,
                                            &m.p_ovl,   &m.p_dens,     &m.p_lag_pre, &m.p_lag,   &m.p_kappa,
                                            &m.p_fk,    &m.p_integral, &m.p_sigB,    &m.p_leftB,
                                            &m.p_aofock, &m.p_aotrans, &m.p_aodens, &m.p_lagB};
  for (auto& p : m.p_nac) r.push_back(&p);
  return r;
}

}  // namespace scc
