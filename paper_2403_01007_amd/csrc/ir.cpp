// Contraction-program graph, zero folding, and the JVP / VJP transforms.
#include "ir.hpp"

#include <algorithm>
#include <stdexcept>

namespace scc {

Spec parse_spec(const std::string& s) {
  Spec r;
  auto arrow = s.find("->");
  auto comma = s.find(',');
  if (arrow == std::string::npos || comma == std::string::npos || comma > arrow)
    throw std::runtime_error("bad contraction spec: " + s);
  r.la = s.substr(0, comma);
  r.lb = s.substr(comma + 1, arrow - comma - 1);
  r.lo = s.substr(arrow + 2);
  return r;
}

static void no_repeats(const std::string& l) {
  for (size_t i = 0; i < l.size(); ++i)
    for (size_t j = i + 1; j < l.size(); ++j)
      if (l[i] == l[j]) throw std::runtime_error("repeated index in " + l);
}

int Graph::tensor(const std::vector<int64_t>& dims, const std::string& name) {
  if (dims.size() > (size_t)MAXD) throw std::runtime_error("too many dims");
  TensorDesc d;
  d.nd = (int)dims.size();
  for (size_t i = 0; i < dims.size(); ++i) d.dim[i] = dims[i];
  d.name = name;
  t.push_back(d);
  return (int)t.size() - 1;
}

int Graph::zeros(const std::vector<int64_t>& dims) {
  int id = tensor(dims, "0");
  t[id].zero = true;
  return id;
}

std::vector<int64_t> Graph::dims(int id) const {
  return std::vector<int64_t>(t[id].dim.begin(), t[id].dim.begin() + t[id].nd);
}

void Graph::check_labels(const std::string& l, int id, const char* what) const {
  if ((int)l.size() != t[id].nd)
    throw std::runtime_error(std::string("label/rank mismatch in ") + what + " '" + l + "' for tensor " +
                             t[id].name);
  no_repeats(l);
}

int Graph::contract(const std::string& spec, int A, int B, double alpha, int c0, double beta) {
  Spec s = parse_spec(spec);
  check_labels(s.la, A, "contract A");
  check_labels(s.lb, B, "contract B");
  no_repeats(s.lo);
  std::map<char, int64_t> sz;
  auto reg = [&](const std::string& l, int id) {
    for (size_t i = 0; i < l.size(); ++i) {
      auto it = sz.find(l[i]);
      if (it != sz.end() && it->second != t[id].dim[i])
        throw std::runtime_error("dimension mismatch for index '" + std::string(1, l[i]) + "' in " + spec);
      sz[l[i]] = t[id].dim[i];
    }
  };
  reg(s.la, A);
  reg(s.lb, B);
  for (char c : s.la + s.lb + s.lo) {
    int n = (s.la.find(c) != std::string::npos) + (s.lb.find(c) != std::string::npos) +
            (s.lo.find(c) != std::string::npos);
    if (n < 2) throw std::runtime_error("index '" + std::string(1, c) + "' appears once in " + spec);
  }
  std::vector<int64_t> od;
  for (char c : s.lo) od.push_back(sz.at(c));
  if (c0 >= 0) {
    if (dims(c0) != od) throw std::runtime_error("addend shape mismatch in " + spec);
  }
  bool zero_prod = t[A].zero || t[B].zero || alpha == 0.0;
  if (zero_prod) {
    if (c0 >= 0 && !t[c0].zero && beta != 0.0) return beta == 1.0 ? c0 : scale(c0, beta);
    return zeros(od);
  }
  if (c0 >= 0 && (t[c0].zero || beta == 0.0)) c0 = -1;
  int out = tensor(od, "c");
  Op op;
  op.kind = OpKind::Contract;
  op.out = out;
  op.a = A;
  op.b = B;
  op.c0 = c0;
  op.alpha = alpha;
  op.beta = c0 >= 0 ? beta : 0.0;
  op.la = s.la;
  op.lb = s.lb;
  op.lo = s.lo;
  ops.push_back(op);
  return out;
}

int Graph::lincomb(const std::string& lo, const std::vector<Term>& terms) {
  no_repeats(lo);
  std::vector<int64_t> od(lo.size(), -1);
  std::vector<Term> keep;
  for (const auto& tm : terms) {
    check_labels(tm.labels, tm.id, "lincomb");
    for (size_t i = 0; i < tm.labels.size(); ++i) {
      auto p = lo.find(tm.labels[i]);
      if (p == std::string::npos) throw std::runtime_error("lincomb label not in output");
      if (od[p] >= 0 && od[p] != t[tm.id].dim[i]) throw std::runtime_error("lincomb dim mismatch");
      od[p] = t[tm.id].dim[i];
    }
    if (!t[tm.id].zero && tm.coef != 0.0) keep.push_back(tm);
  }
  for (auto d : od)
    if (d < 0) throw std::runtime_error("lincomb: undetermined output dim");
  if (keep.empty()) return zeros(od);
  if (keep.size() == 1 && keep[0].coef == 1.0 && keep[0].labels == lo) return keep[0].id;
  int out = tensor(od, "l");
  Op op;
  op.kind = OpKind::Lincomb;
  op.out = out;
  op.lo = lo;
  for (const auto& tm : keep) {
    op.ins.push_back(tm.id);
    op.coef.push_back(tm.coef);
    op.lin.push_back(tm.labels);
  }
  ops.push_back(op);
  return out;
}

static std::string default_labels(int nd) { return std::string("abcdef").substr(0, nd); }

int Graph::add(int A, int B, double ca, double cb) {
  std::string l = default_labels(t[A].nd);
  return lincomb(l, {{ca, A, l}, {cb, B, l}});
}

int Graph::scale(int A, double c) {
  std::string l = default_labels(t[A].nd);
  return lincomb(l, {{c, A, l}});
}

int Graph::slice(int in, const std::vector<int64_t>& off, const std::vector<int64_t>& sizes) {
  if ((int)off.size() != t[in].nd || sizes.size() != off.size()) throw std::runtime_error("slice rank");
  for (size_t i = 0; i < off.size(); ++i)
    if (off[i] < 0 || off[i] + sizes[i] > t[in].dim[i]) throw std::runtime_error("slice out of range");
  if (t[in].zero) return zeros(sizes);
  if (sizes == dims(in)) return in;
  int out = tensor(sizes, "s");
  Op op;
  op.kind = OpKind::Slice;
  op.out = out;
  op.a = in;
  for (size_t i = 0; i < off.size(); ++i) op.off[i] = off[i];
  ops.push_back(op);
  return out;
}

int Graph::embed(int in, const std::vector<int64_t>& off, const std::vector<int64_t>& outdims) {
  if ((int)off.size() != t[in].nd || outdims.size() != off.size()) throw std::runtime_error("embed rank");
  for (size_t i = 0; i < off.size(); ++i)
    if (off[i] < 0 || off[i] + t[in].dim[i] > outdims[i]) throw std::runtime_error("embed out of range");
  if (t[in].zero) return zeros(outdims);
  if (outdims == dims(in)) return in;
  int out = tensor(outdims, "e");
  Op op;
  op.kind = OpKind::Embed;
  op.out = out;
  op.a = in;
  for (size_t i = 0; i < off.size(); ++i) op.off[i] = off[i];
  ops.push_back(op);
  return out;
}

std::vector<int> Graph::jvp(int begin, int end, const std::map<int, int>& seeds) {
  std::vector<int> tan(t.size(), -1);
  for (auto& kv : seeds)
    if (!t[kv.second].zero) tan[kv.first] = kv.second;
  auto T = [&](int id) { return (id >= 0 && id < (int)tan.size()) ? tan[id] : -1; };
  for (int k = begin; k < end; ++k) {
    const Op op = ops[k];  // copy: ops may reallocate
    int res = -1;
    switch (op.kind) {
      case OpKind::Nop:
        break;
      case OpKind::Contract: {
        std::string spec = op.la + "," + op.lb + "->" + op.lo;
        int cur = -1;
        if (op.c0 >= 0 && T(op.c0) >= 0) cur = op.beta == 1.0 ? T(op.c0) : scale(T(op.c0), op.beta);
        if (T(op.a) >= 0) cur = contract(spec, T(op.a), op.b, op.alpha, cur, 1.0);
        if (T(op.b) >= 0) cur = contract(spec, op.a, T(op.b), op.alpha, cur, 1.0);
        res = cur;
        break;
      }
      case OpKind::Lincomb: {
        std::vector<Term> terms;
        for (size_t i = 0; i < op.ins.size(); ++i)
          if (T(op.ins[i]) >= 0) terms.push_back({op.coef[i], T(op.ins[i]), op.lin[i]});
        if (!terms.empty()) res = lincomb(op.lo, terms);
        break;
      }
      case OpKind::Slice:
        if (T(op.a) >= 0) {
          std::vector<int64_t> off(op.off.begin(), op.off.begin() + t[op.a].nd);
          res = slice(T(op.a), off, dims(op.out));
        }
        break;
      case OpKind::Embed:
        if (T(op.a) >= 0) {
          std::vector<int64_t> off(op.off.begin(), op.off.begin() + t[op.a].nd);
          res = embed(T(op.a), off, dims(op.out));
        }
        break;
    }
    if (res >= 0 && t[res].zero) res = -1;
    if (op.out < (int)tan.size()) tan[op.out] = res;
  }
  return tan;
}

std::map<int, int> Graph::vjp(int begin, int end, const std::map<int, int>& seeds,
                              const std::vector<int>& wanted) {
  const int nt = (int)t.size();
  std::vector<char> dep(nt, 0);
  for (int w : wanted) dep[w] = 1;
  for (int k = begin; k < end; ++k) {
    const Op& op = ops[k];
    bool d = false;
    if (op.kind == OpKind::Contract)
      d = dep[op.a] || dep[op.b] || (op.c0 >= 0 && dep[op.c0]);
    else if (op.kind == OpKind::Lincomb)
      for (int i : op.ins) d = d || dep[i];
    else
      d = dep[op.a];
    if (d) dep[op.out] = 1;
  }
  // Contributions to each tensor's adjoint are kept as terms (coefficient,
  // tensor, index map) and summed by one lincomb when the adjoint is needed
  // as a whole; a lone scaled or permuted term is passed on to the consuming
  // contraction or lincomb without being copied.
  std::map<int, std::vector<Term>> contrib;
  auto def = [&](int id) { return default_labels(t[id].nd); };
  for (auto& kv : seeds)
    if (!t[kv.second].zero) contrib[kv.first].push_back({1.0, kv.second, def(kv.second)});
  auto materialize = [&](int id) -> int {
    auto it = contrib.find(id);
    if (it == contrib.end() || it->second.empty()) return -1;
    const std::string l = def(id);
    if (it->second.size() == 1 && it->second[0].coef == 1.0 && it->second[0].labels == l) return it->second[0].id;
    int s = lincomb(l, it->second);
    it->second.assign(1, Term{1.0, s, l});
    return s;
  };
  auto term = [&](int id, Term& out) -> bool {
    auto it = contrib.find(id);
    if (it == contrib.end() || it->second.empty()) return false;
    if (it->second.size() > 1) materialize(id);
    out = it->second[0];
    return !t[out.id].zero;
  };
  for (int k = end - 1; k >= begin; --k) {
    const Op op = ops[k];
    if (!dep[op.out]) continue;
    switch (op.kind) {
      case OpKind::Nop:
        break;
      case OpKind::Contract: {
        Term g;
        if (!term(op.out, g)) break;
        // letters of the term's dimensions in the op's index names
        std::string lx;
        for (char c : g.labels) lx += op.lo[c - 'a'];
        if (dep[op.a]) {
          int r = contract(lx + "," + op.lb + "->" + op.la, g.id, op.b, op.alpha * g.coef);
          if (!t[r].zero) contrib[op.a].push_back({1.0, r, def(op.a)});
        }
        if (dep[op.b]) {
          int r = contract(op.la + "," + lx + "->" + op.lb, op.a, g.id, op.alpha * g.coef);
          if (!t[r].zero) contrib[op.b].push_back({1.0, r, def(op.b)});
        }
        if (op.c0 >= 0 && dep[op.c0]) contrib[op.c0].push_back({op.beta * g.coef, g.id, g.labels});
        break;
      }
      case OpKind::Lincomb: {
        Term g;
        if (!term(op.out, g)) break;
        for (size_t i = 0; i < op.ins.size(); ++i) {
          if (!dep[op.ins[i]]) continue;
          std::string l;
          for (char c : g.labels) l += (char)('a' + op.lin[i].find(op.lo[c - 'a']));
          contrib[op.ins[i]].push_back({op.coef[i] * g.coef, g.id, l});
        }
        break;
      }
      case OpKind::Slice:
        if (dep[op.a]) {
          int g = materialize(op.out);
          if (g < 0 || t[g].zero) break;
          std::vector<int64_t> off(op.off.begin(), op.off.begin() + t[op.a].nd);
          contrib[op.a].push_back({1.0, embed(g, off, dims(op.a)), def(op.a)});
        }
        break;
      case OpKind::Embed:
        if (dep[op.a]) {
          int g = materialize(op.out);
          if (g < 0 || t[g].zero) break;
          std::vector<int64_t> off(op.off.begin(), op.off.begin() + t[op.a].nd);
          contrib[op.a].push_back({1.0, slice(g, off, dims(op.a)), def(op.a)});
        }
        break;
    }
  }
  std::map<int, int> out;
  for (int w : wanted) out[w] = materialize(w);
  return out;
}

std::vector<int> Graph::batchify(const std::vector<int>& list, const std::vector<int>& inputs, int64_t nb,
                                 std::map<int, int>& map) {
  auto bdims = [&](int id) {
    std::vector<int64_t> d = {nb};
    for (auto x : dims(id)) d.push_back(x);
    return d;
  };
  for (int in : inputs) map[in] = tensor(bdims(in), t[in].name + "[Z]");
  auto B = [&](int id) -> int {
    auto it = map.find(id);
    return it == map.end() ? -1 : it->second;
  };
  size_t first = ops.size();
  for (int k : list) {
    const Op op = ops[k];  // copy: ops may reallocate
    int res = -1;
    switch (op.kind) {
      case OpKind::Nop:
        break;
      case OpKind::Contract: {
        int a = B(op.a), b = B(op.b), c0 = op.c0 >= 0 ? B(op.c0) : -1;
        if (a < 0 && b < 0) continue;
        if (a >= 0 && b >= 0) throw std::runtime_error("batchify: product of two batched tensors");
        if (op.c0 >= 0 && c0 < 0) throw std::runtime_error("batchify: unbatched addend of a batched product");
        std::string la = a >= 0 ? "Z" + op.la : op.la;
        std::string lb = b >= 0 ? "Z" + op.lb : op.lb;
        res = contract(la + "," + lb + "->Z" + op.lo, a >= 0 ? a : op.a, b >= 0 ? b : op.b, op.alpha,
                       op.c0 >= 0 ? c0 : -1, op.beta);
        break;
      }
      case OpKind::Lincomb: {
        std::vector<Term> terms;
        int nbat = 0;
        for (size_t i = 0; i < op.ins.size(); ++i) {
          int bi = B(op.ins[i]);
          if (bi >= 0) {
            ++nbat;
            terms.push_back({op.coef[i], bi, "Z" + op.lin[i]});
          }
        }
        if (nbat == 0) continue;
        if (nbat != (int)op.ins.size()) throw std::runtime_error("batchify: mixed linear combination");
        res = lincomb("Z" + op.lo, terms);
        break;
      }
      case OpKind::Slice:
      case OpKind::Embed: {
        int a = B(op.a);
        if (a < 0) continue;
        std::vector<int64_t> off = {0};
        for (int i = 0; i < t[op.a].nd; ++i) off.push_back(op.off[i]);
        res = op.kind == OpKind::Slice ? slice(a, off, bdims(op.out)) : embed(a, off, bdims(op.out));
        break;
      }
    }
    map[op.out] = res;
  }
  std::vector<int> out;
  for (size_t k = first; k < ops.size(); ++k) out.push_back((int)k);
  return out;
}

std::vector<int> Graph::needed_ops(const std::vector<int>& outputs, const std::set<int>& have) const {
  std::vector<char> need(t.size(), 0);
  for (int o : outputs)
    if (o >= 0 && !have.count(o)) need[o] = 1;
  std::vector<int> list;
  for (int k = (int)ops.size() - 1; k >= 0; --k) {
    const Op& op = ops[k];
    if (!need[op.out]) continue;
    list.push_back(k);
    auto mark = [&](int id) {
      if (id >= 0 && !have.count(id)) need[id] = 1;
    };
    if (op.kind == OpKind::Contract) {
      mark(op.a);
      mark(op.b);
      mark(op.c0);
    } else if (op.kind == OpKind::Lincomb) {
      for (int i : op.ins) mark(i);
    } else {
      mark(op.a);
    }
  }
  std::reverse(list.begin(), list.end());
  return list;
}

std::vector<int> Graph::dependent_ops(const std::vector<int>& list, const std::set<int>& vars) const {
  std::vector<char> dep(t.size(), 0);
  for (int v : vars) dep[v] = 1;
  std::vector<int> out;
  for (int k : list) {
    const Op& op = ops[k];
    bool d = false;
    if (op.kind == OpKind::Contract)
      d = dep[op.a] || dep[op.b] || (op.c0 >= 0 && dep[op.c0]);
    else if (op.kind == OpKind::Lincomb)
      for (int i : op.ins) d = d || dep[i];
    else
      d = dep[op.a];
    if (d) {
      dep[op.out] = 1;
      out.push_back(k);
    }
  }
  return out;
}

static std::vector<int> op_inputs(const Op& op) {
  std::vector<int> r;
  switch (op.kind) {
    case OpKind::Contract:
      r = {op.a, op.b};
      if (op.c0 >= 0) r.push_back(op.c0);
      for (const Seg& sg : op.segs) {
        r.push_back(sg.a);
        r.push_back(sg.b);
      }
      break;
    case OpKind::Nop:
      break;
    case OpKind::Lincomb:
      r = op.ins;
      break;
    case OpKind::Slice:
    case OpKind::Embed:
      r = {op.a};
      break;
  }
  return r;
}

int Graph::fuse_sums(const std::vector<const std::vector<int>*>& programs, const std::vector<int>& pinned) {
  constexpr size_t MAXSEG = 16;  // products per fused op (longer sums chain through the addend)
  const int64_t lim32 = (int64_t)1 << 31;
  const int nt = (int)t.size();
  std::vector<std::vector<int>> op_progs(ops.size());
  for (int p = 0; p < (int)programs.size(); ++p)
    for (int k : *programs[p])
      if (op_progs[k].empty() || op_progs[k].back() != p) op_progs[k].push_back(p);
  std::vector<int> nread(nt, 0), producer(nt, -1);
  std::vector<char> pin(nt, 0);
  for (int i : pinned)
    if (i >= 0 && i < nt) pin[i] = 1;
  for (size_t k = 0; k < ops.size(); ++k) {
    if (op_progs[k].empty()) continue;
    for (int in : op_inputs(ops[k])) ++nread[in];
    if (ops[k].out >= 0) producer[ops[k].out] = (int)k;
  }
  int absorbed = 0;
  for (size_t kl = 0; kl < ops.size(); ++kl) {
    if (ops[kl].kind != OpKind::Lincomb || op_progs[kl].empty()) continue;
    const Op L = ops[kl];
    // candidate terms grouped by how their output indices split between
    // batch, first-operand and second-operand indices (in L's names)
    std::map<std::string, std::vector<size_t>> groups;
    for (size_t i = 0; i < L.ins.size(); ++i) {
      const int ti = L.ins[i];
      const int kp = producer[ti];
      if (kp < 0 || kp >= (int)kl) continue;
      const Op& P = ops[kp];
      if (P.kind != OpKind::Contract || P.c0 >= 0 || !P.segs.empty()) continue;
      if (pin[ti] || nread[ti] != 1 || op_progs[kp] != op_progs[kl]) continue;
      if (t[P.a].size() >= lim32 || t[P.b].size() >= lim32 || t[ti].size() >= lim32) continue;
      std::string M, N, B;
      for (size_t q = 0; q < P.lo.size(); ++q) {
        const char c = P.lo[q], o = L.lin[i][q];
        const bool ia = P.la.find(c) != std::string::npos, ib = P.lb.find(c) != std::string::npos;
        (ia && ib ? B : ia ? M : N) += o;
      }
      // rows or columns fewer than a matrix-core tile: memory-bound shapes
      // that stay with their own kernels
      int64_t ms = 1, ns = 1;
      for (char c : M) ms *= t[L.out].dim[L.lo.find(c)];
      for (char c : N) ns *= t[L.out].dim[L.lo.find(c)];
      if (ms < 16 || ns < 16) continue;
      std::sort(M.begin(), M.end());
      std::sort(N.begin(), N.end());
      std::sort(B.begin(), B.end());
      groups[B + "|" + std::min(M, N) + "|" + std::max(M, N)].push_back(i);
    }
    std::vector<char> taken(L.ins.size(), 0);
    std::vector<Term> fused_terms;
    int nfused_groups = 0;
    for (auto& kv : groups) {
      std::vector<size_t> idx = kv.second;
      if (idx.size() < 2) continue;
      std::sort(idx.begin(), idx.end(), [&](size_t x, size_t y) { return producer[L.ins[x]] < producer[L.ins[y]]; });
      ++nfused_groups;
      // the first member's first-operand output indices set the orientation
      std::string mref;
      bool have_ref = false;
      int prev = -1;
      for (size_t c0 = 0; c0 < idx.size(); c0 += MAXSEG) {
        const size_t c1 = std::min(idx.size(), c0 + MAXSEG);
        std::vector<Seg> segs;
        for (size_t j = c0; j < c1; ++j) {
          const size_t i = idx[j];
          const Op& P = ops[producer[L.ins[i]]];
          // P's index names -> L's; summed indices get names unused by L
          std::map<char, char> ren;
          for (size_t q = 0; q < P.lo.size(); ++q) ren[P.lo[q]] = L.lin[i][q];
          std::string used = L.lo;
          char next = 'A';
          for (const std::string* l : {&P.la, &P.lb})
            for (char c : *l)
              if (!ren.count(c)) {
                while (used.find(next) != std::string::npos) ++next;
                ren[c] = next;
                used += next;
              }
          Seg sg{P.a, P.b, "", "", P.alpha * L.coef[i]};
          for (char c : P.la) sg.la += ren[c];
          for (char c : P.lb) sg.lb += ren[c];
          std::string am;
          for (char c : L.lo)
            if (sg.la.find(c) != std::string::npos && sg.lb.find(c) == std::string::npos) am += c;
          if (!have_ref) {
            mref = am;
            have_ref = true;
          }
          if (am != mref) {
            std::swap(sg.a, sg.b);
            std::swap(sg.la, sg.lb);
          }
          segs.push_back(sg);
        }
        const bool last = c1 == idx.size();
        const bool whole = last && idx.size() == L.ins.size();
        const int out = whole ? L.out : tensor(dims(L.out), "s");
        const int kf = producer[L.ins[idx[c1 - 1]]];
        for (size_t j = c0; j < c1; ++j) {
          const int kp = producer[L.ins[idx[j]]];
          t[L.ins[idx[j]]].unused = true;
          ops[kp] = Op{};
          ops[kp].kind = OpKind::Nop;
        }
        Op f;
        f.kind = OpKind::Contract;
        f.out = out;
        f.a = segs[0].a;
        f.b = segs[0].b;
        f.la = segs[0].la;
        f.lb = segs[0].lb;
        f.lo = L.lo;
        f.alpha = segs[0].alpha;
        f.c0 = prev;
        f.beta = 1.0;
        f.segs.assign(segs.begin() + 1, segs.end());
        ops[kf] = f;
        absorbed += (int)(c1 - c0);
        prev = out;
      }
      for (size_t i : idx) taken[i] = 1;
      fused_terms.push_back({1.0, prev, L.lo});
    }
    if (!nfused_groups) continue;
    if (nfused_groups == 1 && fused_terms[0].id == L.out) {
      ops[kl] = Op{};
      ops[kl].kind = OpKind::Nop;
      continue;
    }
    Op& Lm = ops[kl];
    Lm.ins.clear();
    Lm.coef.clear();
    Lm.lin.clear();
    for (size_t i = 0; i < L.ins.size(); ++i)
      if (!taken[i]) {
        Lm.ins.push_back(L.ins[i]);
        Lm.coef.push_back(L.coef[i]);
        Lm.lin.push_back(L.lin[i]);
      }
    for (const Term& tm : fused_terms) {
      Lm.ins.push_back(tm.id);
      Lm.coef.push_back(tm.coef);
      Lm.lin.push_back(tm.labels);
    }
  }
  return absorbed;
}

int64_t Graph::finalize(const std::vector<const std::vector<int>*>& programs, const std::vector<int>& pinned,
                        int64_t align, bool fuse) {
  if (fuse) fuse_sums(programs, pinned);
  auto rnd = [&](int64_t n) { return (n + align - 1) / align * align; };
  const int nt = (int)t.size();
  // owner program of each tensor's producer and of each consumer (-2: several)
  std::vector<int> prod_prog(nt, -1), use_prog(nt, -1), op_prog(ops.size(), -1);
  for (int p = 0; p < (int)programs.size(); ++p)
    for (int k : *programs[p]) op_prog[k] = op_prog[k] == -1 || op_prog[k] == p ? p : -2;
  for (size_t k = 0; k < ops.size(); ++k) {
    if (ops[k].kind == OpKind::Nop) continue;
    const int p = op_prog[k];
    int& pp = prod_prog[ops[k].out];
    pp = pp == -1 ? (p >= 0 ? p : -2) : -2;
    for (int in : op_inputs(ops[k])) {
      int& up = use_prog[in];
      if (p < 0)
        up = -2;
      else
        up = up == -1 || up == p ? p : -2;
    }
  }
  std::vector<char> temp(nt, 0), dead(nt, 0);
  for (size_t k = 0; k < ops.size(); ++k) {
    // produced by an op no program runs: never computed, needs no storage
    if (op_prog[k] == -1 && ops[k].out >= 0) dead[ops[k].out] = 1;
  }
  for (int i = 0; i < nt; ++i)
    if (t[i].unused) dead[i] = 1;
  for (size_t k = 0; k < ops.size(); ++k)
    if (op_prog[k] != -1)
      for (int in : op_inputs(ops[k]))
        if (dead[in]) throw std::runtime_error("a program reads a tensor no program computes");
  for (int i = 0; i < nt; ++i) temp[i] = !t[i].zero && prod_prog[i] >= 0 && use_prog[i] == prod_prog[i];
  for (int i : pinned)
    if (i >= 0 && i < nt) temp[i] = 0;
  // persistent storage
  int64_t pos = 0;
  for (int i = 0; i < nt; ++i) {
    t[i].offset = -1;
    if (t[i].zero || temp[i] || dead[i]) continue;
    t[i].offset = pos;
    pos += rnd(t[i].size());
  }
  // temporaries: liveness-based first fit within each program
  const int64_t base = pos;
  int64_t peak = 0;
  for (int p = 0; p < (int)programs.size(); ++p) {
    const auto& list = *programs[p];
    std::map<int, int> last;
    for (int j = 0; j < (int)list.size(); ++j)
      for (int in : op_inputs(ops[list[j]]))
        if (temp[in]) last[in] = j;
    std::map<int64_t, int64_t> used;  // offset -> size, live blocks
    std::vector<std::pair<int, int>> live;  // (last use, tensor)
    for (int j = 0; j < (int)list.size(); ++j) {
      // release temporaries whose last reader ran before op j
      for (size_t q = 0; q < live.size();) {
        if (live[q].first < j) {
          used.erase(t[live[q].second].offset - base);
          live[q] = live.back();
          live.pop_back();
        } else {
          ++q;
        }
      }
      const int out = ops[list[j]].out;
      if (out < 0 || !temp[out] || prod_prog[out] != p) continue;
      const int64_t need = rnd(t[out].size());
      int64_t at = 0;
      for (auto& b : used) {
        if (b.first - at >= need) break;
        at = std::max(at, b.first + b.second);
      }
      used[at] = need;
      t[out].offset = base + at;
      peak = std::max(peak, at + need);
      auto it = last.find(out);
      live.push_back({it == last.end() ? j : it->second, out});
    }
  }
  return base + peak;
}

}  // namespace scc
