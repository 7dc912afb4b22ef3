// Dump of the device programs of one problem size (test infrastructure):
// every tensor with its arena offset, every op (including the products of
// fused contractions), every program's op list and the tensors the host
// reads or writes.  The CPU interpreter in tests/test_graph_interp.py runs
// the programs from this dump in a flat arena laid out exactly as on the
// device, so that the storage plan (temporaries sharing memory by liveness)
// is exercised too.
//
// usage: graph_dump nocc nvirt nchol nstates fuse(0|1) out_file
#include <cstdio>
#include <cstdlib>

#include "../../paper_2403_01007_amd/csrc/model.hpp"

using namespace scc;

static const char* lab(const std::string& s) { return s.empty() ? "_" : s.c_str(); }

int main(int argc, char** argv) {
  if (argc != 7) {
    std::printf("usage: graph_dump nocc nvirt nchol nstates fuse out_file\n");
    return 2;
  }
  const int o = std::atoi(argv[1]), v = std::atoi(argv[2]);
  Dims d{o, v, o + v, std::atoi(argv[3]), std::atoi(argv[4])};
  Model m;
  build_model(m, d, d.ns + 2, d.ns + d.npairs());
  auto progs = programs(m);
  auto pinned = host_tensors(m);
  const long total = (long)m.g.finalize(progs, pinned, 32, std::atoi(argv[5]) != 0);
  FILE* f = std::fopen(argv[6], "w");
  if (!f) return 1;
  std::fprintf(f, "A %ld\n", total);
  for (size_t i = 0; i < m.g.t.size(); ++i) {
    const TensorDesc& t = m.g.t[i];
    std::fprintf(f, "T %zu %d %d %d", i, t.zero ? 1 : 0, t.unused ? 1 : 0, t.nd);
    for (int k = 0; k < t.nd; ++k) std::fprintf(f, " %ld", (long)t.dim[k]);
    std::fprintf(f, " %ld\n", (long)t.offset);
  }
  for (size_t k = 0; k < m.g.ops.size(); ++k) {
    const Op& op = m.g.ops[k];
    switch (op.kind) {
      case OpKind::Contract:
        std::fprintf(f, "C %d %d %d %d %.17g %.17g %s %s %s %zu", op.out, op.a, op.b, op.c0, op.alpha, op.beta,
                     lab(op.la), lab(op.lb), lab(op.lo), op.segs.size());
        for (const Seg& sg : op.segs)
          std::fprintf(f, " %d %d %s %s %.17g", sg.a, sg.b, lab(sg.la), lab(sg.lb), sg.alpha);
        std::fprintf(f, "\n");
        break;
      case OpKind::Lincomb:
        std::fprintf(f, "L %d %s %zu", op.out, lab(op.lo), op.ins.size());
        for (size_t i = 0; i < op.ins.size(); ++i)
          std::fprintf(f, " %d %.17g %s", op.ins[i], op.coef[i], lab(op.lin[i]));
        std::fprintf(f, "\n");
        break;
      case OpKind::Slice:
      case OpKind::Embed: {
        const int nd = m.g.t[op.a].nd;
        std::fprintf(f, "%s %d %d %d", op.kind == OpKind::Slice ? "SL" : "EM", op.out, op.a, nd);
        for (int i = 0; i < nd; ++i) std::fprintf(f, " %ld", (long)op.off[i]);
        std::fprintf(f, "\n");
        break;
      }
      case OpKind::Nop:
        std::fprintf(f, "N\n");
        break;
    }
  }
  for (size_t p = 0; p < progs.size(); ++p) {
    std::fprintf(f, "P %zu %zu", p, progs[p]->size());
    for (int k : *progs[p]) std::fprintf(f, " %d", k);
    std::fprintf(f, "\n");
  }
  // named tensors the host sets or reads around the residual program
  auto key = [&](const char* name, int id) { std::fprintf(f, "K %s %d\n", name, id); };
  key("In", m.In);
  key("Io", m.Io);
  key("one", m.one);
  key("z2", m.z2);
  key("h", m.h);
  key("L", m.L);
  key("kappa", m.kappa);
  key("t1", m.t1);
  key("t2", m.t2);
  key("E", m.res.E);
  key("O1", m.res.O1);
  key("O2", m.res.O2);
  auto state = [&](const char* name, int r0, int r1, int r2) { std::fprintf(f, "K %s %d %d %d\n", name, r0, r1, r2); };
  state("vin", m.vin.r0, m.vin.r1, m.vin.r2);
  state("sig", m.sig.s0, m.sig.s1, m.sig.s2);
  state("lin", m.lin.r0, m.lin.r1, m.lin.r2);
  state("lout", m.lout.r0, m.lout.r1, m.lout.r2);
  state("vinB", m.vinB.r0, m.vinB.r1, m.vinB.r2);
  state("sigB", m.sigB.r0, m.sigB.r1, m.sigB.r2);
  state("linB", m.linB.r0, m.linB.r1, m.linB.r2);
  state("loutB", m.loutB.r0, m.loutB.r1, m.loutB.r2);
  for (size_t p = 0; p < m.zeta.size(); ++p) std::fprintf(f, "K zeta%zu %d\n", p, m.zeta[p]);
  // multiplier inputs and adjoint outputs of the Lagrangian product and
  // their batched copies
  for (auto& kv : m.lagB) std::fprintf(f, "B %d %d\n", kv.first, kv.second);
  for (size_t k = 0; k < m.xs.size(); ++k)
    std::fprintf(f, "K xs%zu %d %d %d\n", k, m.xs[k].r0, m.xs[k].r1, m.xs[k].r2);
  std::fprintf(f, "H %zu", pinned.size());
  for (int i : pinned) std::fprintf(f, " %d", i);
  std::fprintf(f, "\n");
  std::fclose(f);
  return 0;
}
