// Host-side check of the contraction planner (test infrastructure).
//
// For every contraction of every device program of one problem size, the
// plan the executor would launch is rebuilt on the host (no device memory:
// the arena and scratch bases are null, so pointers are element offsets) and
// every operand and output address map of the matrix-core kernels is
// enumerated: each must visit every element of its tensor (or of its pack
// buffer in scratch) exactly once and stay in bounds.  Elementwise products
// must stay in bounds too.  Prints one summary line; exit status 1 on the
// first violation.
//
// usage: planner_check nocc nvirt nchol nstates
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../paper_2403_01007_amd/csrc/exec.hpp"
#include "../../paper_2403_01007_amd/csrc/model.hpp"

using namespace scc;

namespace {

// the device's index arithmetic, restated: quotient by magic multiply
int64_t group_offset(int64_t x, const IdxMap& m, int64_t si) {
  if (m.D == 0) return x * si;
  if (x >= ((int64_t)1 << 31)) {
    std::printf("index %lld beyond 32 bits\n", (long long)x);
    std::exit(1);
  }
  const uint32_t xx = (uint32_t)x;
  const int64_t q = (int64_t)((((uint64_t)xx * m.mag >> 32) + xx) >> m.sh);
  if (q != x / (int64_t)m.D) {
    std::printf("magic division %lld / %u wrong\n", (long long)x, m.D);
    std::exit(1);
  }
  return q * (int64_t)m.so + (x - q * (int64_t)m.D) * si;
}

int64_t elem(const void* p) { return (int64_t)((intptr_t)p / (intptr_t)sizeof(double)); }

// (batch, row, column) -> base + b sb + row map + column map is a bijection
// onto [base, base + size); returns false (and prints) otherwise
bool bijective(const char* what, int64_t base, int64_t size, int64_t B, int64_t sb, int64_t R, const IdxMap& mr,
               int64_t sr, int64_t C, const IdxMap& mc, int64_t sc) {
  if (B * R * C != size) {
    std::printf("%s: %lld elements visited, tensor holds %lld\n", what, (long long)(B * R * C), (long long)size);
    return false;
  }
  std::vector<uint8_t> hit(size, 0);
  for (int64_t b = 0; b < B; ++b)
    for (int64_t r = 0; r < R; ++r) {
      const int64_t o1 = b * sb + group_offset(r, mr, sr);
      for (int64_t c = 0; c < C; ++c) {
        const int64_t o = o1 + group_offset(c, mc, sc);
        if (o < 0 || o >= size || hit[o]++) {
          std::printf("%s: offset %lld out of range or visited twice (size %lld)\n", what, (long long)o,
                      (long long)size);
          return false;
        }
      }
    }
  (void)base;
  return true;
}

// an operand either lives at its tensor's arena offset or in a pack buffer
// inside the op's scratch
bool placed(const char* what, const void* p, const TensorDesc& d, int64_t scratch) {
  const int64_t e = elem(p);
  if (e == d.offset) return true;
  if (e >= 0 && e + d.size() <= scratch) return true;
  std::printf("%s: operand at %lld is neither the tensor (%lld) nor in scratch (%lld)\n", what, (long long)e,
              (long long)d.offset, (long long)scratch);
  return false;
}

}  // namespace

int main(int argc, char** argv) {
  if (argc != 5) {
    std::printf("usage: planner_check nocc nvirt nchol nstates\n");
    return 2;
  }
  const int o = std::atoi(argv[1]), v = std::atoi(argv[2]), nj = std::atoi(argv[3]), ns = std::atoi(argv[4]);
  Dims d{o, v, o + v, nj, ns};
  Model m;
  build_model(m, d, d.ns + 2, d.ns + d.npairs());
  m.g.finalize(programs(m), host_tensors(m));
  int gemm = 0, two = 0, outer = 0, multi = 0, products = 0;
  for (size_t k = 0; k < m.g.ops.size(); ++k) {
    const Op& op = m.g.ops[k];
    if (op.kind != OpKind::Contract) continue;
    const ContractPlan P = plan_contract(m.g, op, nullptr, nullptr);
    const TensorDesc& dO = m.g.t[op.out];
    if (P.kind == ContractKind::Outer) {
      const PermArgs& p = P.pc;
      int64_t ma = 0, mb = 0, mo = 0, tot = 1;
      for (int i = 0; i < p.nd; ++i) {
        ma += (p.dim[i] - 1) * p.istr[0][i];
        mb += (p.dim[i] - 1) * p.istr[1][i];
        mo += (p.dim[i] - 1) * p.ostr[i];
        tot *= p.dim[i];
      }
      if (!p.mul || ma >= m.g.t[op.a].size() || mb >= m.g.t[op.b].size() || mo != dO.size() - 1 || tot != p.total) {
        std::printf("op %zu: elementwise product out of bounds\n", k);
        return 1;
      }
      ++outer;
      continue;
    }
    if (P.kind == ContractKind::Multi) {
      const GemmArgs& G = P.g;
      int64_t ksum = 0;
      for (size_t q = 0; q < P.segs.size(); ++q) {
        const GemmSeg& S = P.segs[q];
        const Seg x = q == 0 ? Seg{op.a, op.b, op.la, op.lb, op.alpha} : op.segs[q - 1];
        const TensorDesc& dA = m.g.t[x.a];
        const TensorDesc& dB = m.g.t[x.b];
        if (S.k0 != ksum) {
          std::printf("op %zu: product %zu starts at %lld, expected %lld\n", k, q, (long long)S.k0, (long long)ksum);
          return 1;
        }
        ksum += S.K;
        if (!placed("A", S.A, dA, P.scratch) || !placed("B", S.B, dB, P.scratch) ||
            !bijective("A", elem(S.A), dA.size(), G.batch, S.sAb, G.M, S.mAm, S.sAm, S.K, S.mAk, S.sAk) ||
            !bijective("B", elem(S.B), dB.size(), G.batch, S.sBb, S.K, S.mBk, S.sBk, G.N, S.mBn, S.sBn)) {
          std::printf("op %zu (product %zu of %zu)\n", k, q, P.segs.size());
          return 1;
        }
      }
      if (ksum != G.K || !placed("C", G.C, dO, P.scratch) ||
          !bijective("C", elem(G.C), dO.size(), G.batch, G.sCb, G.M, G.mCm, G.sCm, G.N, G.mCn, G.sCn)) {
        std::printf("op %zu (multi-product output)\n", k);
        return 1;
      }
      ++multi;
      products += (int)P.segs.size();
      continue;
    }
    if (P.kind != ContractKind::Mfma || P.dot) continue;
    const GemmArgs& G = P.g;
    const TensorDesc& dA = m.g.t[op.a];
    const TensorDesc& dB = m.g.t[op.b];
    if (!placed("A", G.A, dA, P.scratch) || !placed("B", G.B, dB, P.scratch) || !placed("C", G.C, dO, P.scratch) ||
        !bijective("A", elem(G.A), dA.size(), G.batch, G.sAb, G.M, G.mAm, G.sAm, G.K, G.mAk, G.sAk) ||
        !bijective("B", elem(G.B), dB.size(), G.batch, G.sBb, G.K, G.mBk, G.sBk, G.N, G.mBn, G.sBn) ||
        !bijective("C", elem(G.C), dO.size(), G.batch, G.sCb, G.M, G.mCm, G.sCm, G.N, G.mCn, G.sCn)) {
      std::printf("op %zu: M %lld N %lld K %lld batch %lld\n", k, (long long)G.M, (long long)G.N, (long long)G.K,
                  (long long)G.batch);
      return 1;
    }
    if (G.splits > 1 && (elem(G.P) < 0 || elem(G.P) + G.splits * G.M * G.N > P.scratch)) {
      std::printf("op %zu: split-K partials outside scratch\n", k);
      return 1;
    }
    ++gemm;
    two += G.two ? 1 : 0;
  }
  std::printf("ok: %d GEMM plans (%d with two-run groups), %d multi-product plans (%d products), %d elementwise "
              "products\n",
              gemm, two, multi, products, outer);
  return 0;
}
