// Contraction programs over dense FP64 tensors, with forward-mode (JVP) and
// reverse-mode (VJP) program transforms.
//
// Every quantity of the SCCSD gradient / coupling path is a polynomial in the
// amplitudes and the integrals built from a handful of operations: binary
// tensor contractions, linear combinations of permuted tensors, and block
// slices/embeddings.  The coupled cluster residual is written once as such a
// program; the right and left excited-state transformations, the SCC triple
// excitation terms, the Lagrange-multiplier products and the effective
// densities are all derivatives of it, obtained by transforming the program.
// The programs run on the GPU through the executor in exec.hip.
#pragma once
#include <array>
#include <cstdint>
#include <map>
#include <set>
#include <string>
#include <vector>

namespace scc {

constexpr int MAXD = 6;

struct TensorDesc {
  int nd = 0;
  std::array<int64_t, MAXD> dim{};
  bool zero = false;        // identically zero: no storage, never read
  bool unused = false;      // no longer computed or read (fused away)
  int64_t offset = -1;      // arena offset in doubles (assigned by finalize)
  std::string name;
  int64_t size() const {
    int64_t s = 1;
    for (int i = 0; i < nd; ++i) s *= dim[i];
    return s;
  }
};

enum class OpKind { Contract, Lincomb, Slice, Embed, Nop };

// One more product summed into a contraction's output (same output indices)
struct Seg {
  int a, b;
  std::string la, lb;
  double alpha;
};

struct Op {
  OpKind kind;
  int out = -1;
  // Contract: out = alpha * sum A[la] B[lb] -> [lo]  (+ beta * c0)
  //               + sum over segs of s.alpha * sum A_s[s.la] B_s[s.lb]
  int a = -1, b = -1, c0 = -1;
  double alpha = 1.0, beta = 1.0;
  std::string la, lb, lo;
  std::vector<Seg> segs;
  // Lincomb: out[lo] = sum_i coef_i * ins_i[lin_i]
  std::vector<int> ins;
  std::vector<double> coef;
  std::vector<std::string> lin;
  // Slice: out = in[off : off + out.dim]; Embed: out = 0, out[off:] = in
  std::array<int64_t, MAXD> off{};
};

// A growing graph of tensors and ops.  Builder methods return tensor ids and
// fold identically-zero results (no op is emitted for them).
class Graph {
 public:
  std::vector<TensorDesc> t;
  std::vector<Op> ops;

  int tensor(const std::vector<int64_t>& dims, const std::string& name = "");
  int zeros(const std::vector<int64_t>& dims);
  bool is_zero(int id) const { return t[id].zero; }
  std::vector<int64_t> dims(int id) const;

  // einsum-style binary contraction, spec "ab,bc->ac" (single-letter
  // indices, none repeated within an operand, each index in exactly two of
  // the three operands or in all three = batch).  Optional addend c0.
  int contract(const std::string& spec, int A, int B, double alpha = 1.0,
               int c0 = -1, double beta = 1.0);
  struct Term {
    double coef;
    int id;
    std::string labels;
  };
  // out[lo] = sum coef * in[labels]; labels are permutations of lo.
  int lincomb(const std::string& lo, const std::vector<Term>& terms);
  int add(int A, int B, double ca = 1.0, double cb = 1.0);
  int scale(int A, double c);
  int slice(int in, const std::vector<int64_t>& off, const std::vector<int64_t>& sizes);
  int embed(int in, const std::vector<int64_t>& off, const std::vector<int64_t>& outdims);

  // Forward-mode transform of ops[begin, end): given tangents of some
  // tensors (seeds), emit tangent ops for every op in the range and return
  // tangent ids (-1 where the tangent is identically zero) indexed by tensor.
  std::vector<int> jvp(int begin, int end, const std::map<int, int>& seeds);

  // Reverse-mode transform of ops[begin, end): given cotangents of some
  // tensors, emit adjoint ops and return the adjoints of `wanted` (-1 where
  // identically zero).
  std::map<int, int> vjp(int begin, int end, const std::map<int, int>& seeds,
                         const std::vector<int>& wanted);

  // Batch transform: copy the ops of `list` that depend on `inputs`, giving
  // every tensor they produce a leading batch index of size nb (label 'Z').
  // The programs transformed are linear in those inputs, so no op ever
  // multiplies two batched tensors.  Returns the new op indices; `map` gets
  // tensor -> batched tensor for the inputs and every transformed output.
  std::vector<int> batchify(const std::vector<int>& list, const std::vector<int>& inputs, int64_t nb,
                            std::map<int, int>& map);

  // Ops needed (within [0, ops.size())) to compute `outputs`, excluding any
  // op whose output is in `have` (already computed by an earlier phase).
  std::vector<int> needed_ops(const std::vector<int>& outputs,
                              const std::set<int>& have = {}) const;
  // Ops in `list` that depend (transitively) on any tensor of `vars`.
  std::vector<int> dependent_ops(const std::vector<int>& list, const std::set<int>& vars) const;

  // Assign arena offsets to every non-zero tensor; returns doubles used.
  // Tensors produced and consumed within a single program of `programs`
  // (and read nowhere else) are temporaries: they share one region, reused
  // within each program by liveness (programs run one at a time).  All
  // other tensors get storage of their own.
  // Tensors in `pinned` (read or written by host code) always get storage of
  // their own.
  // First fuses sums of products (fuse_sums; skipped with fuse = false),
  // then assigns storage.
  int64_t finalize(const std::vector<const std::vector<int>*>& programs, const std::vector<int>& pinned,
                   int64_t align = 32, bool fuse = true);

  // Sums of products: where a lincomb adds the outputs of contractions that
  // nothing else reads and whose output indices split the same way between
  // their two operands, those contractions become the segments of one
  // contraction (the products accumulate in one pass over the output, no
  // intermediate tensors).  The absorbed ops become Nop, their outputs
  // unused.  Returns the number of contractions absorbed.
  int fuse_sums(const std::vector<const std::vector<int>*>& programs, const std::vector<int>& pinned);

 private:
  void check_labels(const std::string& l, int id, const char* what) const;
};

// Parsed einsum spec.
struct Spec {
  std::string la, lb, lo;
};
Spec parse_spec(const std::string& s);

}  // namespace scc
