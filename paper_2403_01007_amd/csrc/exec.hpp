// GPU executor for contraction programs (ir.hpp).
#pragma once
#include <hip/hip_runtime.h>

#include <array>
#include <cstdio>
#include <map>
#include <string>
#include <vector>

#include "ir.hpp"

namespace scc {

// Address of index x of a fused index group spanning two runs of a tensor's
// dimensions: (x / D) * so + (x % D) * s_inner (D = 0: one run, x * s_inner).
// mag, sh: 32-bit magic-number division by D.
struct IdxMap {
  uint32_t D = 0, so = 0, mag = 0, sh = 0;
};

// C[b][m][n] = alpha * sum_k A[b][m][k] B[b][k][n] + beta * Cin[b][m][n]
// with arbitrary element strides (one stride of each operand is normally 1);
// the m, n and k groups of each operand may span two runs (IdxMap, inner
// strides sAm, sAk, sBk, sBn, sCm, sCn).
struct GemmArgs {
  int64_t M, N, K, batch;
  double alpha, beta;
  const double* A;
  int64_t sAb, sAm, sAk;
  const double* B;
  int64_t sBb, sBk, sBn;
  const double* Cin;
  double* C;
  int64_t sCb, sCm, sCn;
  // split-K: `splits` > 1 writes alpha * partial sums over K chunks of
  // `kchunk` into P[split][m][n] (batch must be 1); a second pass adds them
  // in a fixed order into C (+ beta Cin).
  int64_t splits = 1, kchunk = 0;
  double* P = nullptr;
  IdxMap mAm, mAk, mBk, mBn, mCm, mCn;
  // some group spans two runs: the kernel takes 32-bit offsets (every
  // operand of fewer than 2^31 elements)
  bool two = false;
};

// out[idx] = sum_i coef_i * in_i[idx . istr_i] + beta * addend[idx . ostr]
// over the iteration shape `dim` (nd <= 6); out written at idx . ostr.
struct PermArgs {
  int nd;
  int64_t dim[MAXD];
  int nin;
  const double* in[4];
  int64_t istr[4][MAXD];
  double coef[4];
  double* out;
  int64_t ostr[MAXD];
  const double* addend;
  double beta;
  int64_t total;
  // mul: out = coef[0] * in[0] * in[1] (+ beta * addend), two inputs
  int mul;
};

void launch_gemm(const GemmArgs& a, hipStream_t s);
// the MFMA kernel alone, and the split-K reduction that follows it
void launch_gemm_main(const GemmArgs& a, hipStream_t s, bool f32 = false);
// One product of a multi-segment GEMM: C += alpha * A_s B_s over the
// segment's own summed extent K (positions k0 .. k0 + K - 1 of the
// concatenated summed index).  Every group may span two runs (IdxMap, single
// runs given as D = 2^31).
struct GemmSeg {
  const double* A;
  const double* B;
  int64_t K, k0;
  int64_t sAm, sAk, sBk, sBn, sAb, sBb;
  IdxMap mAm, mAk, mBk, mBn;
  double alpha;
};
constexpr int MAXSEG = 16;
// C = sum over segments (+ beta Cin): g holds the output, the total summed
// extent and the split-K plan (g.A, g.B unused, g.alpha = 1)
struct GemmMulti {
  GemmArgs g;
  int nseg;
  GemmSeg seg[MAXSEG];
};
void launch_gemm_multi(const GemmMulti& m, hipStream_t s, bool f32 = false);

// the GEMM kernels: FP64 or FP32 products, operand groups of one run each or
// of up to two runs, several products summed in one pass
enum GemmKernel { GEMM_F64 = 0, GEMM_F64_TWO = 1, GEMM_F32 = 2, GEMM_F32_TWO = 3, GEMM_F64_MULTI = 4,
                  GEMM_F32_MULTI = 5, NGEMMK = 6 };
inline int gemm_kernel_id(const GemmArgs& a, bool f32) { return (f32 ? 2 : 0) + (a.two ? 1 : 0); }
void launch_gemm_reduce(const GemmArgs& a, hipStream_t s);
// y[i] += sum_j coef[j] X[j][i] over X [k][n] (coef: host, k entries, read
// before the call returns)
void launch_combine(const double* X, int k, int64_t n, const double* coef, double* y, hipStream_t s);
void launch_perm(const PermArgs& a, hipStream_t s);
void launch_fill(double* p, int64_t n, double v, hipStream_t s);
// out[0] = alpha * sum x[i] y[i] + beta * addend[0]  (deterministic order);
// `partials` needs 1024 doubles.
void launch_dot(const double* x, const double* y, int64_t n, double alpha, const double* addend,
                double beta, double* out, double* partials, hipStream_t s);
// y = a x + b y (elementwise)
void launch_axpby(double a, const double* x, double b, double* y, int64_t n, hipStream_t s);
// y[i] = x[i] / max(|d[i] - shift|, floor) * sign(d[i] - shift)
void launch_precond(const double* x, const double* d, double shift, double floor_, double* y,
                    int64_t n, hipStream_t s);
// Symmetrise a doubles block in place: X[a,i,b,j] = (X[a,i,b,j] + X[b,j,a,i]) / 2
void launch_sym_pairs(double* x, int64_t nov, hipStream_t s);
// grad[k] = sum_p dh[k][p] D1[p] + sum_q dL[k][q] Z[q], k < ncoord
void launch_deriv_contract(const double* dh, int64_t nh, const double* D1, const double* dL, int64_t nl,
                           const double* Z, int ncoord, double* grad, double* partials, hipStream_t s);

// y[r] = alpha * sum_k Mt[r sr + k sk] x[k sx] + beta * yin[r sy]: a
// contraction with one free index (GEMV).  splits > 1 writes partial sums
// over K chunks into P[split][r]; a second pass adds them in a fixed order.
struct GemvArgs {
  int64_t R, K;
  const double* Mt;
  int64_t sr, sk;
  const double* x;
  int64_t sx;
  double alpha, beta;
  const double* yin;
  double* y;
  int64_t sy;
  int64_t splits = 1, kchunk = 0;
  double* P = nullptr;
  bool rows = false;  // k is the matrix's unit-stride index: one wave per row
};

void launch_gemv(const GemvArgs& g, hipStream_t s);
// K == 1: C[b][m][n] = alpha A[b][m] B[b][n] + beta Cin[b][m][n]

enum class ContractKind { Mfma, Dot, Gemv, Outer, Multi };

struct ContractPlan {
  // operand packs: -1 = use directly
  bool packA = false, packB = false, tmpC = false, dot = false;
  ContractKind kind = ContractKind::Mfma;
  GemvArgs gv{};
  GemmArgs g{};
  PermArgs pa{}, pb{}, pc{};
  int64_t scratch = 0;  // doubles of scratch needed
  // Multi: the products (g holds the output side) and their operand packs
  std::vector<GemmSeg> segs;
  std::vector<PermArgs> spacks;
};

class Executor {
 public:
  Executor(Graph& g, double* arena, double* scratch, int64_t scratch_doubles, double* partials)
      : g_(g), arena_(arena), scratch_(scratch), scratch_n_(scratch_doubles), partials_(partials) {}
  // plan every op (call after Graph::finalize); returns max scratch needed
  static int64_t plan_scratch(Graph& g);
  void plan_all();
  void run(const std::vector<int>& op_list, hipStream_t s);
  double* ptr(int id) const { return arena_ + g_.t[id].offset; }
  double flops(const std::vector<int>& op_list) const;
  // GEMM kernel timing with HIP events (off by default)
  void set_profile(bool on);
  bool profiling() const { return prof_; }
  // which GEMM kernels get events while profiling (bit k: GemmKernel k)
  void set_profile_mask(unsigned m) { prof_mask_ = m; }
  void flush_profile();
  // timed totals per GEMM kernel (GemmKernel): milliseconds, algorithmic
  // flops (2 M N K per launch), algorithmic bytes (operands read once, output
  // written once and read once if accumulated), launches
  double kernel_ms[NGEMMK] = {}, kernel_flops[NGEMMK] = {}, kernel_bytes[NGEMMK] = {};
  int64_t kernel_launches[NGEMMK] = {};
  // reduced precision: dense contractions (M, N, K >= 64) take FP32 products
  void set_lowp(bool on) { lowp_ = on; }
  bool lowp() const { return lowp_; }
  // Graph mode: each op list is captured once (per precision and profiling
  // setting) as a HIP graph and replayed; every tensor lives at a fixed
  // arena address, so the captured kernel arguments stay valid.
  void set_graphs(bool on) { graphs_ = on; }
  // per-shape totals of the timed launches, largest time first
  void shape_report(FILE* f, int top) const;
  ~Executor();

 private:
  Graph& g_;
  double* arena_;
  double* scratch_;
  int64_t scratch_n_;
  double* partials_;
  std::vector<ContractPlan> plans_;
  bool prof_ = false, lowp_ = false, graphs_ = false;
  unsigned prof_mask_ = ~0u;
  struct Captured {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // profiling variant: event pairs around the GEMM nodes
    std::vector<hipEvent_t> ev;
    std::vector<double> flops, bytes;
    std::vector<std::array<int64_t, 5>> shape;
    std::vector<char> kid;
  };
  std::map<std::array<int64_t, 3>, Captured> graphs_cache_;
  Captured* cap_ = nullptr;  // set while a graph is being captured
  void account(double ms, double flops, double bytes, const std::array<int64_t, 5>& shape, int kid);
  std::vector<char> ev_kid_;
  std::vector<hipEvent_t> ev_;
  std::vector<double> ev_flops_, ev_bytes_;
  std::vector<std::array<int64_t, 5>> ev_shape_;
  struct ShapeStat {
    int64_t n = 0;
    double ms = 0.0, flops = 0.0;
  };
  std::map<std::array<int64_t, 6>, ShapeStat> shapes_;
  size_t nev_ = 0;
  void run_op(int k, hipStream_t s);
  void timed_gemm(const GemmArgs& g, hipStream_t s, bool f32, const GemmMulti* multi = nullptr);
};

ContractPlan plan_contract(const Graph& g, const Op& op, double* arena, double* scratch);

}  // namespace scc
