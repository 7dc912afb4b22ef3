// libscc: context, solvers and the C ABI (include/scc.h).
//
// Iteration control runs on the host; every vector operation, every
// contraction and every reduction runs on the GPU.  Subspace problems (DIIS
// coefficients, Davidson subspace eigenproblem, GMRES least squares) are a
// few tens of numbers and are solved on the host in FP64.
#include "../../include/scc.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "exec.hpp"
#include "vec.hpp"
#include "model.hpp"
#include "singles.hpp"
#include "smalllinalg.hpp"

using namespace scc;

namespace {

struct SccError : std::runtime_error {
  int code;
  SccError(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

void hck(hipError_t e) {
  if (e != hipSuccess) throw SccError(SCC_EDEVICE, std::string("hip: ") + hipGetErrorString(e));
}

constexpr int NDIIS = 8;
constexpr int GMRES_M = 40;
constexpr int64_t PARTIALS = 1 << 18;

int64_t up(int64_t x, int64_t a = 32) { return (x + a - 1) / a * a; }

struct Sizes {
  int64_t nov, nvt, nst, nlag;
  int maxsub, nkeep, cap_lag, cap_k;
  int nbt, cap_b;        // targets per batched multiplier solve, Krylov capacity of each
  int64_t krylov;        // doubles of the Krylov region (single or batched solves)
  int64_t pool;
};

Sizes sizes_for(const Dims& d) {
  Sizes s;
  s.nov = d.nov();
  s.nvt = s.nov + s.nov * s.nov;
  s.nst = 1 + s.nvt;
  s.nlag = s.nvt + d.ns * (s.nst + 1) + d.npairs();
  // Davidson search space: 32 vectors per working root, at most 24 GB for
  // the vectors and their images; a thick restart keeps three Ritz vectors
  // per working root
  const int nwork = d.ns + 2;
  s.maxsub = std::max(40, std::min<int>(32 * nwork, (int)(24e9 / (16.0 * up(s.nvt)))));
  s.nkeep = std::min(s.maxsub / 2, 3 * nwork);
  int64_t p = 0;
  p += up(s.nvt) + up(s.nov);           // D, Dk
  p += 2 * d.ns * up(s.nst);            // R, L
  p += 2 * NDIIS * up(s.nvt) + 3 * up(s.nvt);
  p += 2 * (int64_t)s.maxsub * up(s.nvt) + (2 * (int64_t)s.nkeep + nwork + 3) * up(s.nvt);
  // recycled GCR spaces: Lagrangian (budget 32 GB) and orbital response
  // Krylov spaces of the multiplier solves share one region (96 GB budget):
  // one target with up to 400 directions, or nbt targets in lockstep
  const double budget = 96e9;
  s.cap_lag = (int)std::max<int64_t>(20, std::min<int64_t>(400, (int64_t)(budget / (16.0 * up(s.nlag)))));
  s.nbt = std::max(1, d.ns + d.npairs());
  s.cap_b = (int)std::max<int64_t>(20, std::min<int64_t>(400, (int64_t)(budget / (16.0 * up(s.nlag) * s.nbt))));
  s.krylov = std::max<int64_t>(2 * (int64_t)s.cap_lag * up(s.nlag), 2 * (int64_t)s.nbt * s.cap_b * up(s.nlag));
  // per-target vectors of the batched solve: b, x, r, z, w
  p += 5 * (int64_t)s.nbt * up(s.nlag) + (int64_t)s.nbt * up(s.cap_b);
  s.cap_k = 300;
  p += s.krylov + up(s.cap_lag) + 4 * up(s.nlag);
  // preconditioner of the multiplier equations: diag(D - omega_k)^-1 L_j for
  // every (k, j), the Schur vectors of the orthogonality multipliers and
  // three temporaries of its setup
  p += (int64_t)d.ns * d.ns * up(s.nst) + (2 * (int64_t)d.npairs() + 3) * up(s.nlag);
  // Anderson history of the SCC macro iteration (6 iterates: mixed states
  // and residuals) and the X3 input states
  p += (2 * 6 + 1) * (int64_t)d.ns * up(s.nst);
  // singles preconditioner: matrix, eigenvectors, eigenvalues, orbital
  // energies, eigensolver work space, temporaries of the shifted solves
  p += 2 * up(s.nov * s.nov) + up(s.nov) + up(d.n) + up(jacobi_work_doubles((int)s.nov)) + 2 * up(s.nov);
  p += 2 * (int64_t)s.cap_k * up(s.nov) + up(s.cap_k) + 4 * up(s.nov);
  p += 64;
  s.pool = p;
  return s;
}

// GCR recycling space (see gcr below)
struct Recycler {
  int64_t n = 0;
  int cap = 0, k = 0;
  double* U = nullptr;     // [cap][n] search directions
  double* C = nullptr;     // [cap][n] their images, orthonormal
  void reset() { k = 0; }
};

}  // namespace

struct scc_ctx {
  Model m;
  Sizes sz{};
  std::unique_ptr<Executor> ex;
  // all work runs on a stream of the context's own (graph capture needs a
  // stream other than the legacy default stream), ordered after the work
  // already enqueued on the caller's stream at the start of every call
  hipStream_t s = nullptr;
  hipStream_t user_s = nullptr;
  hipEvent_t entry_ev = nullptr;
  ~scc_ctx() {
    ex.reset();
    if (entry_ev) (void)hipEventDestroy(entry_ev);
    if (s) (void)hipStreamDestroy(s);
  }
  double* arena = nullptr;
  double* scratch = nullptr;
  int64_t scratch_n = 0;
  double* partials = nullptr;
  double* pool = nullptr;
  int64_t pool_used = 0;
  int64_t pool_base = 0;      // pool in use between calls (context-lifetime vectors)
  bool used_lowp = false;     // reduced-precision products ran during the current call
  void set_lowp(bool on) {
    ex->set_lowp(on);
    if (on) used_lowp = true;
  }
  scc_options opt{};
  std::string err;
  // persistent device vectors
  double* D = nullptr;        // diagonal preconditioner of the CC blocks [nov | nov^2]
  double* Dk = nullptr;       // diagonal of the orbital Hessian [nov]
  std::vector<double*> R, Lv; // states [r0 | r1 | r2]
  double* kbar = nullptr;
  double* dsc = nullptr;      // device scalars
  // singles preconditioner: eigenvectors U [nov][nov] and eigenvalues w
  // [nov] of the singlet singles matrix of the current geometry; once
  // diagonalised, the matrix's storage holds U^T; orbital energies on the
  // device
  double* cisA = nullptr;
  double* cisU = nullptr;
  double* cisW = nullptr;
  double* eps_d = nullptr;
  double* cis_work = nullptr;
  double* cis_tmp = nullptr;
  // y = U diag(1 / floor(w - shift)) U^T x on the singles block
  void singles_solve(const double* x, double shift, double fl, double* y) {
    launch_eig_shift_solve(cisU, cisA, cisW, (int)sz.nov, shift, fl, x, y, cis_tmp, s);
  }
  Recycler rec_lag, rec_k;    // recycled Krylov spaces of the multiplier solves
  std::vector<double> eps;
  bool have_h = false, have_ground = false, have_excited = false, have_mult = false;
  bool scc_on = false;        // the SCC constraint (zeta, O_kl) is part of the solution
  std::vector<double> Jz;     // zeta Jacobian dO/dzeta of the last SCC solve
  bool fixed_basis = false;   // Hamiltonian (and derivative integrals) in a fixed basis
  int last_ground_its = 0;    // iterations of the last ground-state solve
  double* krylov = nullptr;   // Krylov region of the multiplier solves
  double* batch_vec = nullptr;
  double E0 = 0.0, enuc = 0.0;
  std::vector<double> E, zeta;
  int mult_kind = -1, mult_m = -1, mult_n = -1;
  double flops = 0.0;

  double* alloc(int64_t n) {
    double* p = pool + pool_used;
    pool_used += up(n);
    if (pool_used > sz.pool) throw SccError(SCC_ENOMEM, "solver pool exhausted");
    return p;
  }
  double* tp(int id) { return ex->ptr(id); }
  bool zero(int id) const { return m.g.t[id].zero; }
  void run(const std::vector<int>& l) {
    ex->run(l, s);
    flops += ex->flops(l);
  }
  void sync() {
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) throw SccError(SCC_EDEVICE, std::string("hip: ") + hipGetErrorString(e));
  }
  void cp(double* dst, const double* src, int64_t n) {
    if (n <= 0) return;
    hipError_t e = hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) throw SccError(SCC_EDEVICE, "memcpy");
  }
  // copy tensor -> buffer (zeros for identically-zero tensors)
  void get(int id, double* dst) {
    int64_t n = m.g.t[id].size();
    if (zero(id))
      launch_fill(dst, n, 0.0, s);
    else
      cp(dst, tp(id), n);
  }
  void put(int id, const double* src) { cp(tp(id), src, m.g.t[id].size()); }
  // copy on the context's stream and wait for it (host buffers may be
  // pageable and short-lived)
  void xfer(void* dst, const void* src, size_t bytes, hipMemcpyKind kind) {
    hipError_t e = hipMemcpyAsync(dst, src, bytes, kind, s);
    if (e != hipSuccess) throw SccError(SCC_EDEVICE, std::string("hip: ") + hipGetErrorString(e));
    sync();
  }
  double host_scalar(const double* dp) {
    double v = 0;
    xfer(&v, dp, sizeof(double), hipMemcpyDeviceToHost);
    return v;
  }
  double tensor_scalar(int id) { return zero(id) ? 0.0 : host_scalar(tp(id)); }
  void set_scalar(int id, double v) { launch_fill(tp(id), 1, v, s); }
  void set_scalar_ptr(double* p, double v) { launch_fill(p, 1, v, s); }
  double dot(const double* x, const double* y, int64_t n) {
    launch_dot(x, y, n, 1.0, nullptr, 0.0, dsc, partials, s);
    return host_scalar(dsc);
  }
  void axpby(double a, const double* x, double b, double* y, int64_t n) { launch_axpby(a, x, b, y, n, s); }
  void fill(double* p, int64_t n, double v) { launch_fill(p, n, v, s); }
  // state <-> tensors
  void put_state(const StateT& st, const double* v) {
    put(st.r0, v);
    put(st.r1, v + 1);
    put(st.r2, v + 1 + sz.nov);
  }
  void get_state(const StateT& st, double* v) {
    get(st.r0, v);
    get(st.r1, v + 1);
    get(st.r2, v + 1 + sz.nov);
  }
  void sym_doubles(double* x) { launch_sym_pairs(x, sz.nov, s); }
  void log(const char* fmt, ...) __attribute__((format(printf, 2, 3)));
};

// Scoped use of the solver pool: everything allocated after construction is
// released when the scope ends, on every return and throw.
struct PoolMark {
  scc_ctx* c;
  int64_t mark;
  explicit PoolMark(scc_ctx* cc) : c(cc), mark(cc->pool_used) {}
  ~PoolMark() { c->pool_used = mark; }
  PoolMark(const PoolMark&) = delete;
  PoolMark& operator=(const PoolMark&) = delete;
};

void scc_ctx::log(const char* fmt, ...) {
  if (!opt.verbose) return;
  va_list ap;
  va_start(ap, fmt);
  vfprintf(stderr, fmt, ap);
  va_end(ap);
  fflush(stderr);
}

namespace {

// ---------------------------------------------------------------------------
// ground state: quasi-Newton steps (orbital-energy differences on the
// doubles, the inverse singles matrix on the singles) + DIIS
// ---------------------------------------------------------------------------
int ground_solve(scc_ctx* c, double tol, int maxit, double& rn) {
  Model& m = c->m;
  const int64_t nvt = c->sz.nvt, nov = c->sz.nov;
  PoolMark pm(c);
  double* x = c->alloc(nvt);
  double* r = c->alloc(nvt);
  double* e = c->alloc(nvt);
  std::vector<double*> X(NDIIS), Ev(NDIIS);
  for (int i = 0; i < NDIIS; ++i) {
    X[i] = c->alloc(nvt);
    Ev[i] = c->alloc(nvt);
  }
  c->get(m.t1, x);
  c->get(m.t2, x + nov);
  int nh = 0, head = 0, it = 0, since_best = 0;
  double best = 1e300;
  std::vector<double> B(NDIIS * NDIIS, 0.0);
  for (it = 0; it < maxit; ++it) {
    c->put(m.t1, x);
    c->put(m.t2, x + nov);
    c->run(m.p_res);
    c->get(m.res.O1, r);
    c->get(m.res.O2, r + nov);
    c->sym_doubles(r + nov);
    rn = std::sqrt(c->dot(r, r, nvt));
    c->log("  ground it %3d  |Omega| %.3e\n", it, rn);
    c->last_ground_its = it;
    if (rn < tol) break;
    // a residual that is not finite, or four orders of magnitude above the
    // best one reached, will not come back: stop at once
    if (!std::isfinite(rn) || (it > 0 && rn > 1e4 * best)) {
      c->last_ground_its = it;
      c->err = "ground-state iterations diverged";
      return SCC_ENOCONV;
    }
    // restart the extrapolation when it stagnates
    if (rn < best) {
      best = rn;
      since_best = 0;
    } else if (++since_best >= 8) {
      nh = 0;
      head = 0;
      since_best = 0;
      best = rn;
    }
    launch_precond(r, c->D, 0.0, 1e-8, e, nvt, c->s);
    c->singles_solve(r, 0.0, 1e-8, e);
    int slot = head;
    head = (head + 1) % NDIIS;
    nh = std::min(nh + 1, NDIIS);
    c->cp(X[slot], x, nvt);
    c->axpby(-1.0, e, 1.0, X[slot], nvt);
    c->cp(Ev[slot], e, nvt);
    for (int i = 0; i < nh; ++i) {
      double v = c->dot(Ev[slot], Ev[i], nvt);
      B[slot * NDIIS + i] = B[i * NDIIS + slot] = v;
    }
    int n1 = nh + 1;
    std::vector<double> A(n1 * n1, 0.0), b(n1, 0.0);
    double scale = 0;
    for (int i = 0; i < nh; ++i) scale = std::max(scale, B[i * NDIIS + i]);
    if (scale <= 0) scale = 1;
    for (int i = 0; i < nh; ++i) {
      for (int j = 0; j < nh; ++j) A[i * n1 + j] = B[i * NDIIS + j] / scale;
      A[i * n1 + nh] = A[nh * n1 + i] = -1.0;
    }
    b[nh] = -1.0;
    if (!solve_linear(n1, A, b)) {
      c->cp(x, X[slot], nvt);
      continue;
    }
    c->fill(x, nvt, 0.0);
    for (int i = 0; i < nh; ++i) c->axpby(b[i], X[i], 1.0, x, nvt);
    c->sym_doubles(x + nov);
  }
  c->put(m.t1, x);
  c->put(m.t2, x + nov);
  c->run(m.p_res);
  if (it >= maxit) {
    c->err = "ground-state iterations did not converge";
    return SCC_ENOCONV;
  }
  return SCC_OK;
}

// out[i] = C[i] . r for i < k (host copy returned)
std::vector<double> multi_dot(scc_ctx* c, const double* Cb, int k, int64_t n, const double* r) {
  std::vector<double> h(k);
  if (k == 0) return h;
  PoolMark pm(c);
  double* tmp = c->alloc(k);
  launch_deriv_contract(Cb, n, r, Cb, 0, r, k, tmp, c->partials, c->s);
  c->xfer(h.data(), tmp, k * sizeof(double), hipMemcpyDeviceToHost);
  return h;
}

// Dot products (x . y) and multi-dots (C[i] . r, i < k) queued on the stream
// and read back with one wait; each result comes from the same kernels as
// dot() and multi_dot(), so the values are the same.
struct DotBatch {
  struct Req {
    const double* a;
    int k;  // -1: dot(a, r); -2: the device value a[0]
    const double* r;
  };
  std::vector<Req> reqs;
  int dot(const double* x, const double* y) {
    reqs.push_back({x, -1, y});
    return (int)reqs.size() - 1;
  }
  int multi(const double* Cb, int k, const double* r) {
    reqs.push_back({Cb, k, r});
    return (int)reqs.size() - 1;
  }
  int value(const double* p) {
    reqs.push_back({p, -2, nullptr});
    return (int)reqs.size() - 1;
  }
  // results in request order (a dot gives one value)
  std::vector<std::vector<double>> run(scc_ctx* c, int64_t n) {
    std::vector<std::vector<double>> out(reqs.size());
    int total = 0;
    for (const Req& q : reqs) total += q.k < 0 ? 1 : q.k;
    if (total == 0) {
      reqs.clear();
      return out;
    }
    PoolMark pm(c);
    double* tmp = c->alloc(total);
    int off = 0;
    for (const Req& q : reqs) {
      if (q.k == -2) {
        c->cp(tmp + off, q.a, 1);
        off += 1;
      } else if (q.k < 0) {
        launch_dot(q.a, q.r, n, 1.0, nullptr, 0.0, tmp + off, c->partials, c->s);
        off += 1;
      } else if (q.k > 0) {
        launch_deriv_contract(q.a, n, q.r, q.a, 0, q.r, q.k, tmp + off, c->partials, c->s);
        off += q.k;
      }
    }
    std::vector<double> h(total);
    c->xfer(h.data(), tmp, total * sizeof(double), hipMemcpyDeviceToHost);
    off = 0;
    for (size_t i = 0; i < reqs.size(); ++i) {
      const int k = reqs[i].k < 0 ? 1 : reqs[i].k;
      out[i].assign(h.begin() + off, h.begin() + off + k);
      off += k;
    }
    reqs.clear();
    return out;
  }
};

// y += sum_i coef_i X_i for vectors at arbitrary addresses (a few terms)
void multi_axpy_list(scc_ctx* c, const std::vector<const double*>& X, int64_t n, const std::vector<double>& coef,
                     double* y) {
  for (size_t i = 0; i < X.size(); ++i)
    if (coef[i] != 0.0) launch_axpby(coef[i], X[i], 1.0, y, n, c->s);
}

// y += sum_i coef_i X[i] (X [k][n]) in one streaming pass
void multi_axpy(scc_ctx* c, const double* Xb, int k, int64_t n, const std::vector<double>& coef, double* y) {
  if (k == 0) return;
  launch_combine(Xb, k, n, coef.data(), y, c->s);
}

// ---------------------------------------------------------------------------
// nonsymmetric Davidson on the excited-excited block (r0 = 0): right
// eigenvectors of Hbar (left = false) or of Hbar^T (left = true)
// ---------------------------------------------------------------------------
void apply_block(scc_ctx* c, bool left, const double* v, double* w) {
  Model& m = c->m;
  const int64_t nov = c->sz.nov;
  if (!left) {
    c->set_scalar(m.vin.r0, 0.0);
    c->put(m.vin.r1, v);
    c->put(m.vin.r2, v + nov);
    c->run(m.p_sig);
    c->get(m.sig.s1, w);
    c->get(m.sig.s2, w + nov);
  } else {
    c->set_scalar(m.lin.r0, 0.0);
    c->put(m.lin.r1, v);
    c->put(m.lin.r2, v + nov);
    c->run(m.p_left);
    c->get(m.lout.r1, w);
    c->get(m.lout.r2, w + nov);
  }
  c->sym_doubles(w + nov);
}

// w_i = A v_i for i < cnt through the batched programs (nb vectors a pass)
void apply_many(scc_ctx* c, bool left, double* const* v, double* const* w, int cnt) {
  Model& m = c->m;
  const int64_t nov = c->sz.nov, n2 = nov * nov;
  const int nb = m.nb;
  if (nb <= 1) {
    for (int i = 0; i < cnt; ++i) apply_block(c, left, v[i], w[i]);
    return;
  }
  const StateT& in = left ? m.linB : m.vinB;
  const StateT& out = left ? m.loutB : m.sigB;
  for (int b0 = 0; b0 < cnt; b0 += nb) {
    const int nc = std::min(nb, cnt - b0);
    std::vector<CopyItem> ci = {{c->tp(in.r0), nullptr, nb}};
    for (int j = 0; j < nb; ++j) {
      double* r1 = c->tp(in.r1) + j * nov;
      double* r2 = c->tp(in.r2) + j * n2;
      ci.push_back({r1, j < nc ? v[b0 + j] : nullptr, nov});
      ci.push_back({r2, j < nc ? v[b0 + j] + nov : nullptr, n2});
    }
    launch_copy_list(ci, c->s);
    c->run(left ? m.p_leftB : m.p_sigB);
    std::vector<CopyItem> co;
    for (int j = 0; j < nc; ++j) {
      co.push_back({w[b0 + j], c->tp(out.r1) + j * nov, nov});
      co.push_back({w[b0 + j] + nov, c->tp(out.r2) + j * n2, n2});
    }
    launch_copy_list(co, c->s);
    for (int j = 0; j < nc; ++j) c->sym_doubles(w[b0 + j] + nov);
  }
}

int davidson(scc_ctx* c, bool left, int nroots, const std::vector<const double*>& guess, double tol, int maxit,
             std::vector<double>& evals, std::vector<double*>& out, int& iters) {
  const int64_t nvt = c->sz.nvt, nov = c->sz.nov;
  const int maxsub = c->sz.maxsub;
  // nwork Ritz pairs are refined; the nbuf above the requested ones only
  // keep a nearby root from slowing the convergence of the last requested one
  const int nbuf = 2;
  const int nwork = nroots + nbuf;
  const int nkeep = std::min(c->sz.nkeep, maxsub / 2);
  const double pfloor = 0.05;
  PoolMark pm(c);
  std::vector<double*> V(maxsub), W(maxsub);
  double* Vb = c->alloc((int64_t)maxsub * nvt);
  double* Wb = c->alloc((int64_t)maxsub * nvt);
  for (int i = 0; i < maxsub; ++i) {
    V[i] = Vb + (int64_t)i * nvt;
    W[i] = Wb + (int64_t)i * nvt;
  }
  std::vector<double*> Xr(nkeep), Xw(nkeep), Rs(nwork);
  for (int i = 0; i < nkeep; ++i) {
    Xr[i] = c->alloc(nvt);
    Xw[i] = c->alloc(nvt);
  }
  for (int i = 0; i < nwork; ++i) Rs[i] = c->alloc(nvt);
  double* q = c->alloc(nvt);
  int nv = 0;
  auto add_vector = [&](double* src) -> bool {
    double n0 = std::sqrt(c->dot(src, src, nvt));
    if (!(n0 > 0)) return false;
    c->axpby(0.0, src, 1.0 / n0, src, nvt);
    for (int pass = 0; pass < 2; ++pass) {
      auto h = multi_dot(c, Vb, nv, nvt, src);
      for (auto& x : h) x = -x;
      multi_axpy(c, Vb, nv, nvt, h, src);
    }
    double nr = std::sqrt(c->dot(src, src, nvt));
    if (nr < 1e-8) return false;
    c->cp(V[nv], src, nvt);
    c->axpby(0.0, src, 1.0 / nr, V[nv], nvt);
    ++nv;
    return true;
  };
  for (auto* gv : guess) {
    c->cp(q, gv + 1, nvt);
    add_vector(q);
  }
  if (nv < nwork) {
    // the lowest eigenvectors of the singlet singles matrix
    std::vector<double> wh(nov);
    c->xfer(wh.data(), c->cisW, nov * sizeof(double), hipMemcpyDeviceToHost);
    std::vector<int> idx(nov);
    for (int64_t i = 0; i < nov; ++i) idx[i] = (int)i;
    std::sort(idx.begin(), idx.end(), [&](int a, int b) { return wh[a] < wh[b]; });
    for (int64_t k = 0; k < nov && nv < std::max(nwork, nroots + 2); ++k) {
      c->fill(q, nvt, 0.0);
      launch_eig_column(c->cisU, (int)nov, idx[k], q, c->s);
      add_vector(q);
    }
  }
  const int nw_ = std::min<int>(nwork, nv);
  std::vector<double> G(maxsub * maxsub, 0.0);
  int nw = 0, ng = 0;
  iters = 0;
  double stag_ref = 1e300;
  int stag_it = 0;
  for (int it = 0; it < maxit; ++it) {
    iters = it + 1;
    if (nw < nv) {
      apply_many(c, left, &V[nw], &W[nw], nv - nw);
      nw = nv;
    }
    // new rows and columns of the subspace matrix G_ij = V_i . W_j
    {
      DotBatch db;
      for (int j = ng; j < nv; ++j) db.multi(Vb, nv, W[j]);
      for (int i = ng; i < nv; ++i) db.multi(Wb, ng, V[i]);
      auto res = db.run(c, nvt);
      int q = 0;
      for (int j = ng; j < nv; ++j, ++q)
        for (int i = 0; i < nv; ++i) G[i * maxsub + j] = res[q][i];
      for (int i = ng; i < nv; ++i, ++q)
        for (int j = 0; j < ng; ++j) G[i * maxsub + j] = res[q][j];
    }
    ng = nv;
    std::vector<double> Gs(nv * nv);
    for (int i = 0; i < nv; ++i)
      for (int j = 0; j < nv; ++j) Gs[i * nv + j] = G[i * maxsub + j];
    std::vector<cplx> w, Y;
    if (!eig_nonsym_real(nv, Gs, w) && !eig_nonsym(nv, Gs, w, Y, false))
      throw SccError(SCC_ENOCONV, "subspace eigensolver failed");
    std::vector<int> ord(nv);
    for (int i = 0; i < nv; ++i) ord[i] = i;
    std::sort(ord.begin(), ord.end(), [&](int a, int b) { return w[a].real() < w[b].real(); });
    const int nr_now = std::min(nw_, nv);
    const int nx = std::max(nr_now, std::min(nkeep, nv));
    // Ritz vectors Xr[k] = V y_k and images Xw[k] = W y_k of the k-th lowest
    // Ritz value: the working roots every iteration, the rest of the kept
    // ones only for a thick restart
    Y.assign(nv * nv, 0.0);
    std::vector<double> th(nx);
    std::vector<char> conv(nx, 0), cplx_k(nx, 0);
    auto ritz = [&](int k) {
      std::vector<cplx> yc;
      const int col = ord[k];
      eig_nonsym_vector(nv, Gs, w[col], yc);
      for (int j = 0; j < nv; ++j) Y[j * nv + col] = yc[j];
      th[k] = w[col].real();
      // a complex-conjugate Ritz pair contributes Re(y) and Im(y)
      const bool cplx_pair = std::fabs(w[col].imag()) > 1e-10 * std::max(1.0, std::fabs(w[col].real()));
      const bool use_imag = cplx_pair && w[col].imag() < 0;
      std::vector<double> y(nv);
      double yn = 0;
      for (int j = 0; j < nv; ++j) {
        y[j] = use_imag ? yc[j].imag() : yc[j].real();
        yn += y[j] * y[j];
      }
      yn = std::sqrt(yn);
      c->fill(Xr[k], nvt, 0.0);
      c->fill(Xw[k], nvt, 0.0);
      for (auto& yy : y) yy /= yn;
      multi_axpy(c, Vb, nv, nvt, y, Xr[k]);
      multi_axpy(c, Wb, nv, nvt, y, Xw[k]);
      if (k < nr_now) {
        c->cp(Rs[k], Xw[k], nvt);
        c->axpby(-th[k], Xr[k], 1.0, Rs[k], nvt);
        cplx_k[k] = cplx_pair;
      }
    };
    for (int k = 0; k < nr_now; ++k) ritz(k);
    double maxres = 0;
    // residual norms of the working roots, read back together
    {
      DotBatch db;
      for (int k = 0; k < std::min(nr_now, nx); ++k) db.dot(Rs[k], Rs[k]);
      auto res = db.run(c, nvt);
      for (int k = 0; k < std::min(nr_now, nx); ++k) {
        const double rn = std::sqrt(res[k][0]);
        if (k < nroots) maxres = std::max(maxres, rn);
        conv[k] = rn < tol && !cplx_k[k];
      }
    }
    // A wanted root that is one of a complex-conjugate Ritz pair: its
    // residual is that of the complex vector x = V(yr + i yi) with
    // theta = a + ib, i.e. W yr - a V yr + b V yi and W yi - b V yr - a V yi.
    // Converged, the excited-state energy is complex: an error, not a root.
    for (int k = 0; k < std::min(nroots, std::min(nr_now, nx)); ++k) {
      if (!cplx_k[k]) continue;
      const int col = ord[k];
      PoolMark pk(c);
      double* rr = c->alloc(nvt);
      double* ri = c->alloc(nvt);
      std::vector<double> yr(nv), yi(nv);
      double yn = 0;
      for (int j = 0; j < nv; ++j) {
        yr[j] = Y[j * nv + col].real();
        yi[j] = Y[j * nv + col].imag();
        yn += yr[j] * yr[j] + yi[j] * yi[j];
      }
      yn = std::sqrt(yn);
      for (int j = 0; j < nv; ++j) {
        yr[j] /= yn;
        yi[j] /= yn;
      }
      const double a = w[col].real(), b = w[col].imag();
      std::vector<double> cr(nv), ci(nv);
      for (int j = 0; j < nv; ++j) {
        cr[j] = -a * yr[j] + b * yi[j];  // V part of the real residual
        ci[j] = -b * yr[j] - a * yi[j];  // V part of the imaginary residual
      }
      c->fill(rr, nvt, 0.0);
      c->fill(ri, nvt, 0.0);
      multi_axpy(c, Wb, nv, nvt, yr, rr);
      multi_axpy(c, Vb, nv, nvt, cr, rr);
      multi_axpy(c, Wb, nv, nvt, yi, ri);
      multi_axpy(c, Vb, nv, nvt, ci, ri);
      DotBatch dbc;
      const int i1 = dbc.dot(rr, rr), i2 = dbc.dot(ri, ri);
      const auto res = dbc.run(c, nvt);
      const double rn = std::sqrt(res[i1][0] + res[i2][0]);
      if (rn < tol) {
        char msg[160];
        std::snprintf(msg, sizeof msg, "excited state %d converged to a complex energy %.10f %+.3ei", k, a, b);
        throw SccError(SCC_ECOMPLEX, msg);
      }
    }
    // stagnation (e.g. a complex pair that neither converges nor separates):
    // no halving of the largest wanted residual in 60 steps ends the solve
    if (maxres < 0.5 * stag_ref) {
      stag_ref = maxres;
      stag_it = it;
    } else if (it - stag_it >= 60) {
      throw SccError(SCC_ENOCONV, "Davidson iterations stagnated");
    }
    if (c->opt.verbose) {
      c->log("  %s davidson it %3d  nv %2d  max|r| %.3e", left ? "left " : "right", it, nv, maxres);
      for (int k = 0; k < nroots; ++k) c->log("  w%d %.8f%s", k, th[k] - c->E0, conv[k] ? "*" : "");
      c->log("\n");
    }
    bool done = true;
    for (int k = 0; k < nroots; ++k) done = done && conv[k];
    if (done) {
      evals.assign(th.begin(), th.begin() + nroots);
      for (int k = 0; k < nroots; ++k) c->cp(out[k], Xr[k], nvt);
      return SCC_OK;
    }
    int nnew = 0;
    for (int k = 0; k < nr_now; ++k)
      if (!conv[k]) ++nnew;
    if (nv + nnew > maxsub) {
      // thick restart on the lowest nkeep Ritz vectors (orthonormalised)
      for (int k = nr_now; k < nx; ++k) ritz(k);
      nv = 0;
      for (int k = 0; k < nx; ++k) {
        for (int pass = 0; pass < 2; ++pass) {
          auto h = multi_dot(c, Vb, nv, nvt, Xr[k]);
          for (auto& x : h) x = -x;
          multi_axpy(c, Vb, nv, nvt, h, Xr[k]);
          multi_axpy(c, Wb, nv, nvt, h, Xw[k]);
        }
        double nr = std::sqrt(c->dot(Xr[k], Xr[k], nvt));
        if (nr < 1e-8) continue;
        c->cp(V[nv], Xr[k], nvt);
        c->axpby(0.0, Xr[k], 1.0 / nr, V[nv], nvt);
        c->cp(W[nv], Xw[k], nvt);
        c->axpby(0.0, Xw[k], 1.0 / nr, W[nv], nvt);
        ++nv;
      }
      nw = nv;
      ng = 0;
    }
    for (int k = 0; k < nr_now; ++k) {
      if (conv[k]) continue;
      // (D - omega)^-1 with omega = theta - E0 (Hbar carries E0 on its
      // diagonal); on the singles, the shifted inverse of the singles matrix
      launch_precond(Rs[k], c->D, th[k] - c->E0, pfloor, q, nvt, c->s);
      c->singles_solve(Rs[k], th[k] - c->E0, pfloor, q);
      c->sym_doubles(q + nov);
      if (nv < maxsub) add_vector(q);
    }
  }
  c->err = "Davidson iterations did not converge";
  return SCC_ENOCONV;
}

// ---------------------------------------------------------------------------
// excited states with normalisation O_kk = 1, L.R = 1 and phase convention
// ---------------------------------------------------------------------------
double state_overlap(scc_ctx* c, const double* a, const double* b) {
  Model& m = c->m;
  c->put_state(m.oa, a);
  c->put_state(m.ob, b);
  c->run(m.p_ovl);
  return c->tensor_scalar(m.ovl);
}

int excited_at_fixed_zeta(scc_ctx* c, double tol, int maxit, bool warm, int& iters, bool need_left = true) {
  Model& m = c->m;
  const int ns = c->m.d.ns;
  const int64_t nvt = c->sz.nvt, nov = c->sz.nov, nst = c->sz.nst;
  double rn = 0;
  int rc = ground_solve(c, tol, maxit, rn);
  if (rc) return rc;
  iters += c->last_ground_its;
  c->E0 = c->tensor_scalar(m.res.E);
  c->run(m.p_sig_pre);
  std::vector<const double*> gr, gl;
  if (warm)
    for (int k = 0; k < ns; ++k) {
      gr.push_back(c->R[k]);
      gl.push_back(c->Lv[k]);
    }
  PoolMark pm(c);
  std::vector<double*> outR(ns), outL(ns);
  for (int k = 0; k < ns; ++k) {
    outR[k] = c->alloc(nst);
    outL[k] = c->alloc(nst);
  }
  std::vector<double*> oR(ns), oL(ns);
  for (int k = 0; k < ns; ++k) {
    oR[k] = outR[k] + 1;
    oL[k] = outL[k] + 1;
  }
  std::vector<double> ER, EL;
  int itR = 0, itL = 0;
  rc = davidson(c, false, ns, gr, tol, maxit, ER, oR, itR);
  if (rc) return rc;
  if (need_left) {
    rc = davidson(c, true, ns, gl, tol, maxit, EL, oL, itL);
    if (rc) return rc;
  }
  iters += itR + itL;
  c->E.assign(ns, 0.0);
  for (int k = 0; k < ns; ++k) {
    if (need_left && std::fabs(ER[k] - EL[k]) > 1e-6 * std::max(1.0, std::fabs(ER[k])))
      throw SccError(SCC_ENOCONV, "left and right excitation energies differ");
    c->E[k] = ER[k];
    double om = ER[k] - c->E0;
    if (std::fabs(om) < 1e-10) throw SccError(SCC_ESINGULAR, "excitation energy ~ 0");
    // R0 = eta.R / omega from the reference row of calHbar
    c->fill(outR[k], 1, 0.0);
    c->put_state(m.vin, outR[k]);
    c->run(m.p_sig);
    double etaR = c->tensor_scalar(m.sig.s0);
    launch_fill(outR[k], 1, etaR / om, c->s);
    // O_kk = 1
    double okk = state_overlap(c, outR[k], outR[k]);
    c->axpby(0.0, outR[k], 1.0 / std::sqrt(okk), outR[k], nst);
    // phase
    if (warm) {
      double ov = c->dot(c->R[k], outR[k], nst);
      if (ov < 0) c->axpby(0.0, outR[k], -1.0, outR[k], nst);
    } else {
      std::vector<double> r1(nov);
      c->sync();
      c->xfer(r1.data(), outR[k] + 1, nov * sizeof(double), hipMemcpyDeviceToHost);
      int64_t im = 0;
      for (int64_t i = 1; i < nov; ++i)
        if (std::fabs(r1[i]) > std::fabs(r1[im])) im = i;
      if (r1[im] < 0) c->axpby(0.0, outR[k], -1.0, outR[k], nst);
    }
    if (need_left) {
      // L0 = 0, L.R = 1
      c->fill(outL[k], 1, 0.0);
      double lr = c->dot(outL[k], outR[k], nst);
      c->axpby(0.0, outL[k], 1.0 / lr, outL[k], nst);
    }
  }
  for (int k = 0; k < ns; ++k) {
    c->cp(c->R[k], outR[k], nst);
    if (need_left) c->cp(c->Lv[k], outL[k], nst);
  }
  (void)nvt;
  return SCC_OK;
}

void set_scc_inputs(scc_ctx* c, const std::vector<double>& zeta, bool states) {
  Model& m = c->m;
  for (size_t p = 0; p < m.zeta.size(); ++p) c->set_scalar(m.zeta[p], p < zeta.size() ? zeta[p] : 0.0);
  if (states)
    for (int k = 0; k < m.d.ns; ++k) c->put_state(m.xs[k], c->R[k]);
}

std::vector<double> pair_overlaps(scc_ctx* c) {
  std::vector<double> O;
  const int ns = c->m.d.ns;
  for (int k = 0; k < ns; ++k)
    for (int l = k + 1; l < ns; ++l) O.push_back(state_overlap(c, c->R[k], c->R[l]));
  return O;
}

// Canonical phase of converged states: the largest-magnitude R1 element of
// every right vector is positive, whatever the start (plain or a guess) and
// the path of the iteration.  Flipping R_k flips L_k, the overlaps O_kl and
// X3^{kl} of every pair with k; zeta_kl changes sign with them (zeta_kl X3^{kl}
// and so the amplitudes stay as they are), as do the matching rows and
// columns of the zeta Jacobian.
void canonical_phase(scc_ctx* c) {
  const int ns = c->m.d.ns, np = c->m.d.npairs();
  const int64_t nov = c->sz.nov, nst = c->sz.nst;
  std::vector<int> sg(ns, 1);
  std::vector<double> r1(nov);
  bool any = false;
  c->sync();
  for (int k = 0; k < ns; ++k) {
    c->xfer(r1.data(), c->R[k] + 1, nov * sizeof(double), hipMemcpyDeviceToHost);
    int64_t im = 0;
    for (int64_t i = 1; i < nov; ++i)
      if (std::fabs(r1[i]) > std::fabs(r1[im])) im = i;
    if (r1[im] < 0) {
      sg[k] = -1;
      any = true;
      c->axpby(0.0, c->R[k], -1.0, c->R[k], nst);
      c->axpby(0.0, c->Lv[k], -1.0, c->Lv[k], nst);
    }
  }
  if (!any || np == 0) return;
  std::vector<int> sp;
  for (int k = 0; k < ns; ++k)
    for (int l = k + 1; l < ns; ++l) sp.push_back(sg[k] * sg[l]);
  if ((int)c->zeta.size() == np)
    for (int p = 0; p < np; ++p) c->zeta[p] *= sp[p];
  if ((int)c->Jz.size() == np * np)
    for (int p = 0; p < np; ++p)
      for (int q = 0; q < np; ++q) c->Jz[p * np + q] *= sp[p] * sp[q];
  if (c->scc_on) set_scc_inputs(c, c->zeta, true);
}

int excited_pass_run(scc_ctx* c, double tol, double tol_overlap, bool warm, int& iters);

// One solve of the excited states, returned in the canonical phase.  warm:
// continue from the zeta, amplitudes, vectors and zeta Jacobian of a previous
// pass (the FP64 refinement of a reduced-precision solve, or a guess);
// otherwise start from CCSD at zeta = 0.
int excited_pass(scc_ctx* c, double tol, double tol_overlap, bool warm, int& iters) {
  const int rc = excited_pass_run(c, tol, tol_overlap, warm, iters);
  if (rc == SCC_OK) canonical_phase(c);
  return rc;
}

// residual tolerance of the solves behind the finite-difference zeta
// Jacobian (step 1e-4: O to about 1e-8 gives the Jacobian to about 1e-4)
constexpr double FD_TOL = 1e-8;

int excited_pass_run(scc_ctx* c, double tol, double tol_overlap, bool warm, int& iters) {
  const int ns = c->m.d.ns, np = c->m.d.npairs();
  const int maxit = c->opt.max_iter;
  const bool use_scc = c->opt.scc && c->m.d.o >= 2 && np > 0;
  c->scc_on = use_scc;
  int rc = SCC_OK;
  if (!warm) {
    c->zeta.assign(np, 0.0);
    c->Jz.clear();
    set_scc_inputs(c, c->zeta, false);
    // with the constraint active, the CCSD states are only the starting
    // point (solved to 1e-8, the accuracy of the finite-difference Jacobian
    // that follows): left vectors are solved once, at the converged SCC point
    rc = excited_at_fixed_zeta(c, use_scc ? std::max(tol, FD_TOL) : tol, maxit, false, iters, !use_scc);
    if (rc) return rc;
  } else if (!use_scc) {
    for (int k = 0; k < ns; ++k) c->cp(c->Lv[k], c->R[k], c->sz.nst);
    return excited_at_fixed_zeta(c, tol, maxit, true, iters, true);
  }
  if (use_scc) {
    // The SCC macro iteration is a fixed-point map x -> G(x) on x = (zeta,
    // X3 states): the ground and excited states are solved at (zeta, X3),
    // giving right vectors R' and overlaps O; G(x) = (zeta - J^-1 O, R') with
    // J = dO/dzeta at fixed X3 (finite differences once, or the previous
    // solve's).  Its fixed point is the SCC solution.  Anderson mixing of the
    // last NAND iterates (the combination of the G(x_i) whose residuals
    // G(x_i) - x_i have the least norm, weights summing to one) replaces the
    // plain step x <- G(x): the X3 states lag one iteration behind the
    // states they are built from, and the plain iteration converges only
    // linearly.
    constexpr int NAND = 6;
    const int64_t nst = c->sz.nst;
    PoolMark pm(c);
    std::vector<double*> Rx(ns);                                 // X3 input states of this iteration
    for (int k = 0; k < ns; ++k) {
      Rx[k] = c->alloc(nst);
      c->cp(Rx[k], c->R[k], nst);
    }
    std::vector<std::vector<double*>> Rg(NAND, std::vector<double*>(ns)), Rf = Rg;
    for (int i = 0; i < NAND; ++i)
      for (int k = 0; k < ns; ++k) {
        Rg[i][k] = c->alloc(nst);
        Rf[i][k] = c->alloc(nst);
      }
    std::vector<std::vector<double>> zg(NAND), zf(NAND);
    std::vector<double> Bm(NAND * NAND, 0.0);
    int nh = 0, head = 0;
    std::vector<double>& Jz = c->Jz;
    std::vector<double> z = c->zeta;
    bool conv = false;
    double omax_prev = 1.0, best = 1e300;
    for (int it = 0; it < c->opt.max_iter && !conv; ++it) {
      // inexact inner solves while the constraint is far from satisfied;
      // the pass that is the base point of a finite-difference Jacobian is
      // as tight as its displaced solves (a Jacobian carried over from a
      // previous solve needs none)
      const bool fd_base = it == 0 && Jz.empty();
      const double tol_it = fd_base ? std::max(tol, FD_TOL) : std::max(tol, std::min(1e-5, 1e-3 * omax_prev));
      for (size_t p = 0; p < c->m.zeta.size(); ++p) c->set_scalar(c->m.zeta[p], z[p]);
      for (int k = 0; k < ns; ++k) c->put_state(c->m.xs[k], Rx[k]);
      rc = excited_at_fixed_zeta(c, tol_it, maxit, true, iters, false);
      if (rc) return rc;
      std::vector<double> O = pair_overlaps(c);
      // residual of the X3 states: R' - Rx (new slot of the history)
      const int slot = head;
      head = (head + 1) % NAND;
      nh = std::min(nh + 1, NAND);
      double dR = 0, omax = 0;
      {
        DotBatch db;
        std::vector<int> id(ns);
        for (int k = 0; k < ns; ++k) {
          c->cp(Rg[slot][k], c->R[k], nst);
          c->cp(Rf[slot][k], c->R[k], nst);
          c->axpby(-1.0, Rx[k], 1.0, Rf[slot][k], nst);
          id[k] = db.dot(Rf[slot][k], Rf[slot][k]);
        }
        const auto r = db.run(c, nst);
        for (int k = 0; k < ns; ++k) dR = std::max(dR, std::sqrt(r[id[k]][0]));
      }
      for (double x : O) omax = std::max(omax, std::fabs(x));
      c->log(" scc it %2d  max|O| %.3e  |dR| %.3e  zeta0 %.8f  (inner tol %.1e, history %d)\n", it, omax, dR, z[0],
             tol_it, nh);
      omax_prev = omax;
      if (omax < tol_overlap && dR < 10 * tol && tol_it <= tol) {
        conv = true;
        break;
      }
      if (Jz.empty()) {
        // finite-difference Jacobian dO/dzeta with the X3 states held fixed
        Jz.assign(np * np, 0.0);
        const double h = 1e-4;
        PoolMark pk(c);
        std::vector<double*> keepR(ns), keepL(ns);
        for (int k = 0; k < ns; ++k) {
          keepR[k] = c->alloc(nst);
          keepL[k] = c->alloc(nst);
          c->cp(keepR[k], c->R[k], nst);
          c->cp(keepL[k], c->Lv[k], nst);
        }
        // the displaced solves need O to ~1e-8 only (h = 1e-4)
        const double tol_fd = std::max(tol_it, FD_TOL);
        for (int p = 0; p < np; ++p) {
          std::vector<double> zp = z;
          zp[p] += h;
          for (size_t q = 0; q < c->m.zeta.size(); ++q) c->set_scalar(c->m.zeta[q], zp[q]);
          rc = excited_at_fixed_zeta(c, tol_fd, maxit, true, iters, false);
          if (rc) return rc;
          std::vector<double> Op = pair_overlaps(c);
          for (int q = 0; q < np; ++q) Jz[q * np + p] = (Op[q] - O[q]) / h;
          for (int k = 0; k < ns; ++k) {
            c->cp(c->R[k], keepR[k], nst);
            c->cp(c->Lv[k], keepL[k], nst);
          }
        }
      }
      std::vector<double> step = O;
      if (!solve_linear(np, Jz, step)) throw SccError(SCC_ESINGULAR, "zeta Jacobian singular");
      zg[slot].resize(np);
      zf[slot].resize(np);
      for (int p = 0; p < np; ++p) {
        zg[slot][p] = z[p] - step[p];
        zf[slot][p] = -step[p];
      }
      // a clear setback restarts the history from this iterate
      if (omax < best) {
        best = omax;
      } else if (omax > 10 * best) {
        nh = 1;
        best = omax;
        for (int i = 0; i < NAND; ++i)
          if (i != slot) zg[i].clear();
      }
      // Gram matrix of the residuals (R parts on the device, zeta parts here)
      {
        DotBatch db;
        std::vector<std::vector<int>> id(NAND, std::vector<int>(ns, -1));
        for (int i = 0; i < NAND; ++i) {
          if (zg[i].empty() || (nh < NAND && ((slot - i + NAND) % NAND) >= nh)) continue;
          for (int k = 0; k < ns; ++k) id[i][k] = db.dot(Rf[slot][k], Rf[i][k]);
        }
        const auto r = db.run(c, nst);
        for (int i = 0; i < NAND; ++i) {
          if (id[i][0] < 0) continue;
          double v = 0;
          for (int k = 0; k < ns; ++k) v += r[id[i][k]][0];
          for (int p = 0; p < np; ++p) v += zf[slot][p] * zf[i][p];
          Bm[slot * NAND + i] = Bm[i * NAND + slot] = v;
        }
      }
      std::vector<int> use;
      for (int d = 0; d < nh; ++d) use.push_back((slot - d + NAND) % NAND);
      const int nu = (int)use.size(), n1 = nu + 1;
      std::vector<double> A(n1 * n1, 0.0), w(n1, 0.0);
      double sc = 0;
      for (int i = 0; i < nu; ++i) sc = std::max(sc, Bm[use[i] * NAND + use[i]]);
      if (!(sc > 0)) sc = 1;
      for (int i = 0; i < nu; ++i) {
        for (int j = 0; j < nu; ++j) A[i * n1 + j] = Bm[use[i] * NAND + use[j]] / sc;
        A[i * n1 + nu] = A[nu * n1 + i] = -1.0;
      }
      w[nu] = -1.0;
      if (nu == 1 || !solve_linear(n1, A, w)) {
        std::fill(w.begin(), w.end(), 0.0);
        w[0] = 1.0;  // plain step from the newest iterate
      }
      // next iterate: sum_i w_i G(x_i)
      for (int p = 0; p < np; ++p) {
        double v = 0;
        for (int i = 0; i < nu; ++i) v += w[i] * zg[use[i]][p];
        z[p] = v;
      }
      for (int k = 0; k < ns; ++k) {
        std::vector<const double*> src(nu);
        std::vector<double> cf(nu);
        for (int i = 0; i < nu; ++i) {
          src[i] = Rg[use[i]][k];
          cf[i] = w[i];
        }
        c->fill(Rx[k], nst, 0.0);
        multi_axpy_list(c, src, nst, cf, Rx[k]);
      }
    }
    c->zeta = z;
    if (!conv) {
      c->err = "SCC iterations did not converge";
      return SCC_ENOCONV;
    }
    // left eigenvectors once, at the converged (zeta, X3) point, started
    // from the right vectors
    set_scc_inputs(c, z, false);
    for (int k = 0; k < ns; ++k) c->cp(c->Lv[k], c->R[k], nst);
    rc = excited_at_fixed_zeta(c, tol, maxit, true, iters, true);
    if (rc) return rc;
  }
  return SCC_OK;
}

// reduced-precision mode: FP32-product pass to this tolerance, then FP64
constexpr double LOWP_TOL = 1e-6;

int excited_solve(scc_ctx* c, scc_info* info) {
  const double tol = c->opt.tol_residual, tov = c->opt.tol_overlap;
  int iters = 0, rc;
  if (c->opt.precision == 1) {
    c->set_lowp(true);
    try {
      rc = excited_pass(c, std::max(tol, LOWP_TOL), std::max(tov, LOWP_TOL), false, iters);
    } catch (const SccError& e) {
      rc = e.code;
    }
    c->ex->set_lowp(false);
    // a reduced-precision pass that stalls at its own rounding level still
    // leaves a good starting point for the FP64 refinement
    if (rc && rc != SCC_ENOCONV) return rc;
    rc = excited_pass(c, tol, tov, true, iters);
  } else {
    rc = excited_pass(c, tol, tov, false, iters);
  }
  if (rc) return rc;
  if (info) {
    info->iterations = iters;
    info->converged = 1;
  }
  return SCC_OK;
}

using LinOp = std::function<void(const double*, double*)>;

// ---------------------------------------------------------------------------
// GCR with recycling: pairs (u_i, c_i = A u_i), c_i orthonormal, kept across
// right-hand sides of the same operator (all gradient / coupling targets share
// the Lagrangian Jacobian).  Equivalent to unrestarted GMRES for one RHS.
// ---------------------------------------------------------------------------
int gcr(scc_ctx* c, Recycler& rc, const LinOp& A, const LinOp& Minv, const double* b, double* x, double tol,
        int maxit, int& iters, double& relres, bool warm = false) {
  const int64_t n = rc.n;
  PoolMark pm(c);
  double* r = c->alloc(n);
  double* z = c->alloc(n);
  double* w = c->alloc(n);
  double bn = std::sqrt(c->dot(b, b, n));
  if (warm) {
    // continue from the given x: r = b - A x
    A(x, w);
    c->cp(r, b, n);
    c->axpby(-1.0, w, 1.0, r, n);
  } else {
    c->fill(x, n, 0.0);
    c->cp(r, b, n);
  }
  iters = 0;
  relres = 1.0;
  if (bn == 0) {
    relres = 0;
    return SCC_OK;
  }
  rc.reset();
  if (rc.k > 0) {
    auto al = multi_dot(c, rc.C, rc.k, n, r);
    multi_axpy(c, rc.U, rc.k, n, al, x);
    for (auto& v : al) v = -v;
    multi_axpy(c, rc.C, rc.k, n, al, r);
  }
  int checks = 0;
  for (int it = 0; it < maxit; ++it) {
    relres = std::sqrt(c->dot(r, r, n)) / bn;
    if (it % 10 == 0) c->log("  gcr it %3d (stored %d)  rel. residual %.3e\n", it, rc.k, relres);
    if (relres < tol) {
      // confirm with the true residual b - A x before accepting
      A(x, w);
      c->cp(r, b, n);
      c->axpby(-1.0, w, 1.0, r, n);
      double tr = std::sqrt(c->dot(r, r, n)) / bn;
      c->log("  gcr it %3d  true rel. residual %.3e\n", it, tr);
      if (tr < 10 * tol || ++checks > 3) {
        relres = tr;
        if (tr < 10 * tol) return SCC_OK;
        c->err = "Krylov solve: true residual stays above the tolerance";
        return SCC_ENOCONV;
      }
      // continue from the true residual (its direction re-seeds the space)
      Minv(r, z);
      A(z, w);
      for (int pass = 0; pass < 2; ++pass) {
        auto be = multi_dot(c, rc.C, rc.k, n, w);
        for (auto& v : be) v = -v;
        multi_axpy(c, rc.C, rc.k, n, be, w);
        multi_axpy(c, rc.U, rc.k, n, be, z);
      }
      double wn = std::sqrt(c->dot(w, w, n));
      if (!(wn > 0) || rc.k >= rc.cap) break;
      double* un = rc.U + (int64_t)rc.k * n;
      double* cn = rc.C + (int64_t)rc.k * n;
      c->cp(un, z, n);
      c->axpby(0.0, z, 1.0 / wn, un, n);
      c->cp(cn, w, n);
      c->axpby(0.0, w, 1.0 / wn, cn, n);
      ++rc.k;
      // project the true residual on the whole stored space
      auto al = multi_dot(c, rc.C, rc.k, n, r);
      multi_axpy(c, rc.U, rc.k, n, al, x);
      for (auto& v : al) v = -v;
      multi_axpy(c, rc.C, rc.k, n, al, r);
      continue;
    }
    if (rc.k >= rc.cap) break;
    // next direction from the last orthonormal image (the Krylov space of
    // GMRES); starting from the residual alone stalls when A M^-1 r is
    // orthogonal to r, which happens for the bordered multiplier system
    ++iters;
    if (it == 0 || rc.k == 0)
      Minv(r, z);
    else
      Minv(rc.C + (int64_t)(rc.k - 1) * n, z);
    A(z, w);
    const double w0 = std::sqrt(c->dot(w, w, n));
    // orthogonalise w against the stored c_i, mirror on z; a second pass
    // only when the first removed most of w ("twice is enough")
    double wn = w0;
    for (int pass = 0; pass < 2; ++pass) {
      const double before = wn;
      auto be = multi_dot(c, rc.C, rc.k, n, w);
      std::vector<double> nb(be.size());
      for (size_t i = 0; i < be.size(); ++i) nb[i] = -be[i];
      multi_axpy(c, rc.C, rc.k, n, nb, w);
      multi_axpy(c, rc.U, rc.k, n, nb, z);
      wn = std::sqrt(c->dot(w, w, n));
      if (wn > 0.5 * before) break;
    }
    if (!(wn > 1e-12 * w0)) {
      // the Krylov space is (numerically) invariant: confirm with the true residual
      relres = 0.0;
      continue;
    }
    double* un = rc.U + (int64_t)rc.k * n;
    double* cn = rc.C + (int64_t)rc.k * n;
    c->cp(un, z, n);
    c->axpby(0.0, z, 1.0 / wn, un, n);
    c->cp(cn, w, n);
    c->axpby(0.0, w, 1.0 / wn, cn, n);
    ++rc.k;
    double al = c->dot(cn, r, n);
    c->axpby(al, un, 1.0, x, n);
    c->axpby(-al, cn, 1.0, r, n);
  }
  if (relres < tol) return SCC_OK;
  c->err = "Krylov solve: iteration limit or space capacity reached";
  return SCC_ENOCONV;
}

// ---------------------------------------------------------------------------
// Lagrangian: parameters, multipliers, targets
// ---------------------------------------------------------------------------
struct Seg {
  int mult;   // multiplier tensor (cotangent input)
  int adj;    // adjoint output tensor (parameter row)
  int64_t n;
  int kind;   // 0: t block, 1+k: state k block, -1: E / zeta
  int comp;   // 0 scalar, 1 singles, 2 doubles
  bool active = true;  // false: zeta / O_kl of a solution without the SCC constraint
};

std::vector<Seg> lag_segments(scc_ctx* c) {
  Model& m = c->m;
  const int64_t nov = c->sz.nov;
  std::vector<Seg> s;
  s.push_back({m.m1, m.a_t1, nov, 0, 1});
  s.push_back({m.m2, m.a_t2, nov * nov, 0, 2});
  for (int k = 0; k < m.d.ns; ++k) {
    s.push_back({m.mk[k].s0, m.a_r[k].r0, 1, 1 + k, 0});
    s.push_back({m.mk[k].s1, m.a_r[k].r1, nov, 1 + k, 1});
    s.push_back({m.mk[k].s2, m.a_r[k].r2, nov * nov, 1 + k, 2});
    s.push_back({m.mN[k], m.a_E[k], 1, -1, 0});
  }
  for (int p = 0; p < m.d.npairs(); ++p) s.push_back({m.mO[p], m.a_z[p], 1, -1, 0, c->scc_on});
  return s;
}

void set_lagrangian_point(scc_ctx* c) {
  Model& m = c->m;
  const int64_t nov = c->sz.nov;
  const int ns = m.d.ns;
  {
    PoolMark pm(c);
    double* tmp = c->alloc(c->sz.nvt);
    c->get(m.t1, tmp);
    c->get(m.t2, tmp + nov);
    c->put(m.pt1, tmp);
    c->put(m.pt2, tmp + nov);
    c->put(m.nac_t1c, tmp);
    c->put(m.nac_t2c, tmp + nov);
  }
  for (int p = 0; p < m.d.npairs(); ++p) c->set_scalar(m.pz[p], c->zeta[p]);
  for (int k = 0; k < ns; ++k) {
    c->put_state(m.pr[k], c->R[k]);
    c->set_scalar(m.pE[k], c->E[k]);
    c->put_state(m.lam[k], c->Lv[k]);
  }
  c->fill(c->tp(m.mF), nov, 0.0);
  c->run(m.p_lag_pre);
}

// right-hand side b = -dTarget/dlambda (parameter layout) of the gradient of
// E_n (kind 0) or the coupling target O_mn (kind 1)
void lag_rhs(scc_ctx* c, const std::vector<int64_t>& offs, int kind, int mm, int nn, double* b) {
  Model& m = c->m;
  const int64_t n = c->sz.nlag;
  c->fill(b, n, 0.0);
  if (kind == 0) {
    // gradient of E_n: unit vector on the E_n parameter
    int idx = 2 + 4 * nn + 3;
    launch_fill(b + offs[idx], 1, -1.0, c->s);
  } else {
    c->put_state(m.nac_l, c->Lv[mm]);
    c->run(m.p_nac[nn]);
    c->get(m.a_nac_t1[nn], b + offs[0]);
    c->get(m.a_nac_t2[nn], b + offs[1]);
    int base = 2 + 4 * nn;
    c->get(m.a_nac_r[nn].r0, b + offs[base]);
    c->get(m.a_nac_r[nn].r1, b + offs[base + 1]);
    c->get(m.a_nac_r[nn].r2, b + offs[base + 2]);
    c->axpby(0.0, b, -1.0, b, n);
  }
}

// out = J^T in: one Lagrangian product (single-target program)
void lag_apply_single(scc_ctx* c, const std::vector<Seg>& segs, const std::vector<int64_t>& offs, const double* in,
                      double* out) {
  Model& m = c->m;
  for (size_t i = 0; i < segs.size(); ++i) {
    if (segs[i].active)
      c->put(segs[i].mult, in + offs[i]);
    else
      c->fill(c->tp(segs[i].mult), segs[i].n, 0.0);
  }
  c->run(m.p_lag);
  for (size_t i = 0; i < segs.size(); ++i) {
    if (!segs[i].active) {
      c->fill(out + offs[i], segs[i].n, 0.0);
      continue;
    }
    c->get(segs[i].adj, out + offs[i]);
    if (segs[i].comp == 2) c->sym_doubles(out + offs[i]);
  }
}

// Preconditioner of the multiplier equations J^T lambda = b (parameter-space
// residual in, multiplier space out), a block elimination with three parts.
//  * Amplitude rows (t) <-> Omega multipliers: orbital-energy differences D.
//  * Each excited state k: the bordered block
//        [ (Hbar - E_k)^T   -Lam_k ] [lambda_k]   [f]   (rows of calR_k)
//        [ -R_k^T             0    ] [  mu_k  ] = [g]   (row of E_k)
//    solved exactly on the span of the known states and approximately on
//    the rest: with c_j = R_j . f and the biorthonormal pairs (R_j, L_j),
//    (Hbar - E_k)^T L_j = (E_j - E_k) L_j, so
//        mu = -c_k,   lambda = -g L_k + sum_{j != k} c_j / (E_j - E_k) L_j
//                              + Q diag(D - omega_k)^-1 Q f,
//    Q removing the components along every L_j (Q f = f - sum_j c_j L_j).
//  * Orthogonality multipliers gamma_p: they do not enter the zeta rows
//    directly, only through the blocks above, so they come from the Schur
//    complement of the zeta rows, S = C^T M^-1 G with G_p = J^T e_gamma_p (the
//    gradient of O_p over the parameters) and C_p = J e_zeta_p (the zeta
//    derivative of every constraint): with y = M^-1 v,
//        gamma = S^-1 (C^T y - v_zeta),   lambda = y - sum_p gamma_p M^-1 G_p.
// The blocks' couplings (F-bar terms, zeta-scaled X3 derivatives) are left to
// the Krylov iteration.
struct LagPrec {
  std::vector<double*> DL;       // diag(D - omega_k)^-1 L_j, [k * ns + j], each [nst]
  int np = 0;                    // orthogonality multipliers in the Schur step (0: none)
  std::vector<double*> MG;       // M^-1 G_p, multiplier layout [nlag]
  std::vector<double*> C;        // C_p, multiplier layout [nlag]
  std::vector<double> S;         // np x np, row q = C_q
  int seg_zeta0 = 0;             // first zeta / O segment
};

void lag_state_dinv(scc_ctx* c, int k, const double* in, double* out) {
  const int64_t nov = c->sz.nov;
  double* dzero = c->dsc + 8;
  const double shift = c->E[k] - c->E0;
  launch_precond(in, dzero, shift, 0.05, out, 1, c->s);
  c->singles_solve(in + 1, shift, 0.05, out + 1);
  launch_precond(in + 1 + nov, c->D + nov, shift, 0.05, out + 1 + nov, nov * nov, c->s);
}

// M^-1 of the block-diagonal part (gamma rows left at zero)
void lag_prec_blocks(scc_ctx* c, const LagPrec& P, const std::vector<Seg>& segs, const std::vector<int64_t>& offs,
                     const double* in, double* out) {
  const int64_t nov = c->sz.nov, nst = c->sz.nst;
  const int ns = c->m.d.ns;
  c->fill(c->dsc + 8, 1, 0.0);
  for (size_t i = 0; i < segs.size(); ++i) {
    const Seg& sg = segs[i];
    if (sg.kind != 0) continue;
    if (sg.comp == 1)
      c->singles_solve(in + offs[i], 0.0, 0.05, out + offs[i]);
    else
      launch_precond(in + offs[i], c->D + nov, 0.0, 0.05, out + offs[i], sg.n, c->s);
  }
  for (size_t i = 2 + 4 * (size_t)ns; i < segs.size(); ++i) c->fill(out + offs[i], segs[i].n, 0.0);
  // c_j = R_j . f for every state block, and g, read back together
  DotBatch d1;
  std::vector<std::vector<int>> ic(ns, std::vector<int>(ns));
  std::vector<int> ig(ns);
  for (int k = 0; k < ns; ++k) {
    const int64_t sb = offs[2 + 4 * k], eb = offs[2 + 4 * k + 3];
    for (int j = 0; j < ns; ++j) ic[k][j] = d1.dot(c->R[j], in + sb);
    ig[k] = d1.value(in + eb);
  }
  const auto r1 = d1.run(c, nst);
  // z = diag(D - omega_k)^-1 (f - sum_j c_j L_j), then R_j . z
  DotBatch d2;
  std::vector<std::vector<int>> iz(ns, std::vector<int>(ns));
  for (int k = 0; k < ns; ++k) {
    double* z = out + offs[2 + 4 * k];
    lag_state_dinv(c, k, in + offs[2 + 4 * k], z);
    std::vector<double> cf(ns);
    for (int j = 0; j < ns; ++j) cf[j] = -r1[ic[k][j]][0];
    multi_axpy_list(c, std::vector<const double*>(P.DL.begin() + k * ns, P.DL.begin() + (k + 1) * ns), nst, cf, z);
    for (int j = 0; j < ns; ++j) iz[k][j] = d2.dot(c->R[j], z);
  }
  const auto r2 = d2.run(c, nst);
  // lambda = Q z - g L_k + sum_{j != k} c_j / (E_j - E_k) L_j,  mu = -c_k
  for (int k = 0; k < ns; ++k) {
    double* z = out + offs[2 + 4 * k];
    const double g = r1[ig[k]][0];
    std::vector<double> cf(ns);
    for (int j = 0; j < ns; ++j) {
      cf[j] = -r2[iz[k][j]][0];
      if (j == k)
        cf[j] -= g;
      else
        cf[j] += r1[ic[k][j]][0] / (c->E[j] - c->E[k]);
    }
    multi_axpy_list(c, std::vector<const double*>(c->Lv.begin(), c->Lv.end()), nst, cf, z);
    c->set_scalar_ptr(out + offs[2 + 4 * k + 3], -r1[ic[k][k]][0]);
  }
}

// Setup at the current solution.  DL by diagonal scaling of the left
// vectors.  With the SCC constraint active, the Schur step of the
// orthogonality multipliers: G_p = J^T e_gamma_p by Lagrangian products with
// unit gamma_p, and C_p (the zeta_p derivative of every constraint) from the
// residual and right-transformation programs at zeta = e_p and zeta = 0,
// both affine in zeta, with the X3 states at calR.  The vectors stay in the
// solver pool of the caller's scope.
LagPrec lag_prec_setup(scc_ctx* c, const std::vector<Seg>& segs, const std::vector<int64_t>& offs) {
  LagPrec P;
  Model& m = c->m;
  const int ns = m.d.ns, np = m.d.npairs();
  const int64_t n = c->sz.nlag, nov = c->sz.nov, nst = c->sz.nst, nvt = c->sz.nvt;
  P.seg_zeta0 = 2 + 4 * ns;
  c->fill(c->dsc + 8, 1, 0.0);
  for (int k = 0; k < ns; ++k)
    for (int j = 0; j < ns; ++j) {
      double* q = c->alloc(nst);
      lag_state_dinv(c, k, c->Lv[j], q);
      P.DL.push_back(q);
    }
  if (!c->scc_on || np == 0) return P;
  P.np = np;
  for (int p = 0; p < np; ++p) {
    P.MG.push_back(c->alloc(n));
    P.C.push_back(c->alloc(n));
  }
  {
    PoolMark tmp_mark(c);
    double* e = c->alloc(n);
    double* G = c->alloc(n);
    for (int p = 0; p < np; ++p) {
      c->fill(e, n, 0.0);
      launch_fill(e + offs[P.seg_zeta0 + p], 1, 1.0, c->s);
      lag_apply_single(c, segs, offs, e, G);
      lag_prec_blocks(c, P, segs, offs, G, P.MG[p]);
    }
    // constraint values at zeta = 0 and at zeta = e_p
    auto eval = [&](const std::vector<double>& z, double* dst) {
      c->fill(dst, n, 0.0);
      set_scc_inputs(c, z, true);
      c->run(m.p_res);
      c->get(m.res.O1, dst + offs[0]);
      c->get(m.res.O2, dst + offs[1]);
      c->sym_doubles(dst + offs[1]);
      c->run(m.p_sig_pre);
      for (int k = 0; k < ns; ++k) {
        c->put_state(m.vin, c->R[k]);
        c->run(m.p_sig);
        c->get(m.sig.s0, dst + offs[2 + 4 * k]);
        c->get(m.sig.s1, dst + offs[3 + 4 * k]);
        c->get(m.sig.s2, dst + offs[4 + 4 * k]);
        c->sym_doubles(dst + offs[4 + 4 * k]);
      }
    };
    double* base = c->alloc(n);
    eval(std::vector<double>(np, 0.0), base);
    for (int p = 0; p < np; ++p) {
      std::vector<double> z(np, 0.0);
      z[p] = 1.0;
      eval(z, P.C[p]);
      c->axpby(-1.0, base, 1.0, P.C[p], n);
    }
    // back to the solution's zeta (and its residual / transformation state)
    set_scc_inputs(c, c->zeta, true);
    c->run(m.p_res);
    c->run(m.p_sig_pre);
  }
  DotBatch db;
  std::vector<std::vector<int>> id(np, std::vector<int>(np));
  for (int q = 0; q < np; ++q)
    for (int p = 0; p < np; ++p) id[q][p] = db.dot(P.C[q], P.MG[p]);
  const auto r = db.run(c, n);
  P.S.assign((size_t)np * np, 0.0);
  for (int q = 0; q < np; ++q)
    for (int p = 0; p < np; ++p) P.S[(size_t)q * np + p] = r[id[q][p]][0];
  (void)nov;
  (void)nvt;
  return P;
}

void lag_prec(scc_ctx* c, const LagPrec& P, const std::vector<Seg>& segs, const std::vector<int64_t>& offs,
              const double* in, double* out) {
  lag_prec_blocks(c, P, segs, offs, in, out);
  if (!P.np) return;
  const int np = P.np;
  const int64_t n = c->sz.nlag;
  DotBatch db;
  std::vector<int> ic(np), iv(np);
  for (int q = 0; q < np; ++q) {
    ic[q] = db.dot(P.C[q], out);
    iv[q] = db.value(in + offs[P.seg_zeta0 + q]);
  }
  const auto r = db.run(c, n);
  std::vector<double> gam(np);
  for (int q = 0; q < np; ++q) gam[q] = r[ic[q]][0] - r[iv[q]][0];
  if (!solve_linear(np, P.S, gam)) return;  // singular Schur complement: block part alone
  std::vector<double> cf(np);
  for (int p = 0; p < np; ++p) cf[p] = -gam[p];
  multi_axpy_list(c, std::vector<const double*>(P.MG.begin(), P.MG.end()), n, cf, out);
  for (int p = 0; p < np; ++p) c->set_scalar_ptr(out + offs[P.seg_zeta0 + p], gam[p]);
}

// with the multipliers x of one target: orbital multipliers
// A_HF^T kbar = -(eta_kappa + dTarget/dkappa); leaves the multipliers in
// their tensors and kbar in c->kbar
int orbital_response(scc_ctx* c, const std::vector<Seg>& segs, const std::vector<int64_t>& offs, const double* x,
                     int kind, int mm, int nn, int& itk, double& relk) {
  Model& m = c->m;
  const int64_t nov = c->sz.nov;
  for (size_t i = 0; i < segs.size(); ++i) {
    if (segs[i].active)
      c->put(segs[i].mult, x + offs[i]);
    else
      c->fill(c->tp(segs[i].mult), segs[i].n, 0.0);
  }
  PoolMark pm(c);
  c->fill(c->tp(m.mF), nov, 0.0);
  c->run(m.p_kappa);
  double* rhs = c->alloc(nov);
  c->get(m.a_kappa, rhs);
  if (kind == 1) {
    // coupling: dO_mn/dkappa_ai = -(d_ai - d_ia) with d = d(calL_m, calR_n)
    c->run(m.p_sig_pre);
    c->put_state(m.vin, c->R[nn]);
    c->put_state(m.lin, c->Lv[mm]);
    c->run(m.p_dens);
    std::vector<double> dh((size_t)m.d.n * m.d.n, 0.0);
    if (!c->zero(m.dens_hk)) c->xfer(dh.data(), c->tp(m.dens_hk), dh.size() * sizeof(double), hipMemcpyDeviceToHost);
    std::vector<double> ck(nov);
    const int o = m.d.o, v = m.d.v, N = m.d.n;
    for (int a = 0; a < v; ++a)
      for (int i = 0; i < o; ++i) ck[a * o + i] = -(dh[(o + a) * N + i] - dh[i * N + o + a]);
    double* dck = c->alloc(nov);
    c->xfer(dck, ck.data(), nov * sizeof(double), hipMemcpyHostToDevice);
    c->axpby(1.0, dck, 1.0, rhs, nov);
  }
  c->axpby(0.0, rhs, -1.0, rhs, nov);
  auto applyF = [&](const double* in, double* out) {
    c->put(m.mF, in);
    c->run(m.p_fk);
    c->get(m.fk_adj, out);
  };
  auto precF = [&](const double* in, double* out) { launch_precond(in, c->Dk, 0.0, 1e-3, out, nov, c->s); };
  c->fill(c->kbar, nov, 0.0);
  int rc = gcr(c, c->rec_k, applyF, precF, rhs, c->kbar, c->opt.tol_residual, std::max(c->opt.max_iter, c->rec_k.cap),
               itk, relk);
  c->put(m.mF, c->kbar);
  if (rc) return rc;
  c->have_mult = true;
  c->mult_kind = kind;
  c->mult_m = mm;
  c->mult_n = nn;
  return SCC_OK;
}

// One target's multipliers.  guess (device, [nlag], may be NULL) is used as
// the starting point if its residual is below that of the zero start (else
// *rejected = true); xout (device, may be NULL) receives the multipliers.
int multipliers_solve(scc_ctx* c, int kind, int mm, int nn, scc_info* info, const double* guess = nullptr,
                      double* xout = nullptr, bool* rejected = nullptr) {
  Model& m = c->m;
  const int64_t n = c->sz.nlag;
  set_lagrangian_point(c);
  auto segs = lag_segments(c);
  PoolMark pm(c);
  double* b = c->alloc(n);
  double* x = c->alloc(n);
  c->fill(x, n, 0.0);
  int64_t off = 0;
  std::vector<int64_t> offs;
  for (auto& sg : segs) {
    offs.push_back(off);
    off += sg.n;
  }
  lag_rhs(c, offs, kind, mm, nn, b);
  LagPrec lp = lag_prec_setup(c, segs, offs);
  auto prec = [&](const double* in, double* out) { lag_prec(c, lp, segs, offs, in, out); };
  auto apply = [&](const double* in, double* out) { lag_apply_single(c, segs, offs, in, out); };
  int iters = 0;
  double rel = 0;
  const int maxg = std::max(c->opt.max_iter, c->rec_lag.cap);
  int rc;
  // The multiplier equations are solved in FP64 in every precision mode:
  // with FP32 products the Krylov recurrence of this bordered system drifts
  // away from its true residual (directions of large norm amplify the
  // product rounding), so a reduced-precision pass is no usable start.
  bool warm = false;
  if (guess) {
    PoolMark pg(c);
    double* r = c->alloc(n);
    c->cp(x, guess, n);
    apply(x, r);
    c->axpby(1.0, b, -1.0, r, n);
    DotBatch db;
    const int ir = db.dot(r, r), ib = db.dot(b, b);
    const auto res = db.run(c, n);
    warm = std::isfinite(res[ir][0]) && res[ir][0] < res[ib][0];
    if (!warm) {
      c->fill(x, n, 0.0);
      if (rejected) *rejected = true;
    }
  }
  rc = gcr(c, c->rec_lag, apply, prec, b, x, c->opt.tol_residual, maxg, iters, rel, warm);
  if (rc) return rc;
  if (xout) c->cp(xout, x, n);
  int itk = 0;
  double relk = 0;
  rc = orbital_response(c, segs, offs, x, kind, mm, nn, itk, relk);
  if (rc) return rc;
  if (info) {
    info->iterations = iters + itk;
    info->residual = std::max(rel, relk);
    info->converged = 1;
  }
  return SCC_OK;
}


int integral_adjoints(scc_ctx* c) {
  Model& m = c->m;
  c->put(m.mF, c->kbar);
  c->run(m.p_integral);
  return SCC_OK;
}

// Effective densities of the current multipliers contracted with the
// derivative integrals: out[k] = <dh_k, D1> + <dL_k, Z>
void contract_derivatives(scc_ctx* c, int ncoord, const double* dh, const double* dchol, double* out) {
  integral_adjoints(c);
  const int64_t N = c->m.d.n, J = c->m.d.nj;
  int d1id = c->m.a_h, zid = c->m.a_L;
  if (c->fixed_basis) {
    // derivative integrals in the fixed basis: densities C D1 C^T, C Z C^T
    c->run(c->m.p_aodens);
    d1id = c->m.d1ao;
    zid = c->m.zao;
  }
  double* D1 = c->zero(d1id) ? nullptr : c->tp(d1id);
  double* Z = c->zero(zid) ? nullptr : c->tp(zid);
  if (!D1 || !Z) throw SccError(SCC_EDEVICE, "empty density");
  launch_deriv_contract(dh, N * N, D1, dchol, J * N * N, Z, ncoord, out, c->partials, c->s);
}

struct Target {
  int kind, m, n;
  double* out;
};

// Multiplier equations of several targets solved in lockstep: one pass of
// the batched Lagrangian products (p_lagB) serves up to nbt targets per
// Krylov step; each target keeps its own GCR/ORTHODIR recurrence (the same
// steps as gcr() above).  Then orbital response and derivative contraction
// per target.  Targets that do not converge within the batched capacity are
// solved alone.
int targets_solve(scc_ctx* c, const std::vector<Target>& tg, int ncoord, const double* dh, const double* dchol,
                  int& iters_total, const double* guess, double* mult, bool& rejected) {
  Model& m = c->m;
  const int64_t n = c->sz.nlag, un = up(c->sz.nlag);
  const int nbt = c->sz.nbt, cap = c->sz.cap_b;
  const double tol = c->opt.tol_residual;
  set_lagrangian_point(c);
  auto segs = lag_segments(c);
  std::vector<int64_t> offs;
  {
    int64_t off = 0;
    for (auto& sg : segs) {
      offs.push_back(off);
      off += sg.n;
    }
  }
  PoolMark pm(c);
  LagPrec lp = lag_prec_setup(c, segs, offs);
  auto prec = [&](const double* in, double* out) { lag_prec(c, lp, segs, offs, in, out); };
  // out_j = J^T in_j for the listed slots (at most nbt), other slots zero
  auto applyB = [&](const std::vector<const double*>& in, const std::vector<double*>& out) {
    std::vector<CopyItem> ci;
    for (size_t i = 0; i < segs.size(); ++i) {
      const Seg& sg = segs[i];
      double* base = c->tp(m.lagB.at(sg.mult));
      for (int j = 0; j < nbt; ++j) {
        const bool use = j < (int)in.size() && in[j] && sg.active;
        ci.push_back({base + (int64_t)j * sg.n, use ? in[j] + offs[i] : nullptr, sg.n});
      }
    }
    launch_copy_list(ci, c->s);
    c->run(m.p_lagB);
    std::vector<CopyItem> co;
    std::vector<double*> sym;
    for (size_t i = 0; i < segs.size(); ++i) {
      const Seg& sg = segs[i];
      auto it = m.lagB.find(sg.adj);
      for (int j = 0; j < (int)out.size(); ++j) {
        if (!out[j]) continue;
        if (!sg.active || it == m.lagB.end()) {
          co.push_back({out[j] + offs[i], nullptr, sg.n});
          continue;
        }
        co.push_back({out[j] + offs[i], c->tp(it->second) + (int64_t)j * sg.n, sg.n});
        if (sg.comp == 2) sym.push_back(out[j] + offs[i]);
      }
    }
    launch_copy_list(co, c->s);
    for (double* p : sym) c->sym_doubles(p);
  };
  const int maxg = std::max(c->opt.max_iter, cap);
  std::vector<int> failed;
  for (size_t b0 = 0; b0 < tg.size(); b0 += nbt) {
    const int nb = (int)std::min<size_t>(nbt, tg.size() - b0);
    std::vector<double*> B(nb), X(nb), R(nb), Z(nb), W(nb), U(nb), C(nb);
    std::vector<int> k(nb, 0), done(nb, 0), checks(nb, 0);
    std::vector<char> first(nb, 1), reseed(nb, 0), force(nb, 0);
    std::vector<double> bn(nb);
    for (int j = 0; j < nb; ++j) {
      B[j] = c->batch_vec + (0 * (int64_t)nbt + j) * un;
      X[j] = c->batch_vec + (1 * (int64_t)nbt + j) * un;
      R[j] = c->batch_vec + (2 * (int64_t)nbt + j) * un;
      Z[j] = c->batch_vec + (3 * (int64_t)nbt + j) * un;
      W[j] = c->batch_vec + (4 * (int64_t)nbt + j) * un;
      U[j] = c->krylov + (2 * (int64_t)j) * cap * un;
      C[j] = c->krylov + (2 * (int64_t)j + 1) * cap * un;
      const Target& t = tg[b0 + j];
      lag_rhs(c, offs, t.kind, t.m, t.n, B[j]);
      c->fill(X[j], n, 0.0);
      c->cp(R[j], B[j], n);
      bn[j] = std::sqrt(c->dot(B[j], B[j], n));
      if (bn[j] == 0) done[j] = 1;
    }
    if (guess) {
      // starting points judged by their residuals: b - J^T x0 for all targets
      // with one batched product; a guess no better than zero is dropped
      std::vector<const double*> gin(nb);
      std::vector<double*> gout(nb);
      for (int j = 0; j < nb; ++j) {
        c->cp(X[j], guess + (int64_t)(b0 + j) * n, n);
        gin[j] = X[j];
        gout[j] = W[j];
      }
      applyB(gin, gout);
      DotBatch db;
      std::vector<int> ir(nb);
      for (int j = 0; j < nb; ++j) {
        c->cp(Z[j], B[j], n);
        c->axpby(-1.0, W[j], 1.0, Z[j], n);
        ir[j] = db.dot(Z[j], Z[j]);
      }
      const auto res = db.run(c, n);
      for (int j = 0; j < nb; ++j) {
        const double rn = std::sqrt(res[ir[j]][0]);
        if (std::isfinite(rn) && rn < bn[j]) {
          c->cp(R[j], Z[j], n);
          if (bn[j] > 0 && rn < tol * bn[j]) force[j] = 1;  // confirm on the true residual at once
        } else {
          c->fill(X[j], n, 0.0);
          rejected = true;
        }
      }
    }
    int it = 0;
    for (; it < maxg; ++it) {
      // convergence, confirmed on the true residual b - A x
      std::vector<const double*> cin(nb, nullptr);
      std::vector<double*> cout(nb, nullptr);
      bool any = false;
      DotBatch drr;
      std::vector<int> irr(nb, -1);
      for (int j = 0; j < nb; ++j)
        if (!done[j] && !force[j]) irr[j] = drr.dot(R[j], R[j]);
      const auto rr = drr.run(c, n);
      for (int j = 0; j < nb; ++j) {
        if (done[j]) continue;
        const double rel = force[j] ? 0.0 : std::sqrt(rr[irr[j]][0]) / bn[j];
        if (it % 10 == 0) c->log("  batched gcr it %3d target %d (stored %d)  rel. residual %.3e\n", it, j, k[j], rel);
        if (rel < tol) {
          cin[j] = X[j];
          cout[j] = W[j];
          any = true;
        }
        force[j] = 0;
      }
      if (any) {
        applyB(cin, cout);
        for (int j = 0; j < nb; ++j) {
          if (!cin[j]) continue;
          c->cp(R[j], B[j], n);
          c->axpby(-1.0, W[j], 1.0, R[j], n);
          const double tr = std::sqrt(c->dot(R[j], R[j], n)) / bn[j];
          c->log("  batched gcr it %3d target %d  true rel. residual %.3e\n", it, j, tr);
          if (tr < 10 * tol)
            done[j] = 1;
          else if (++checks[j] > 3)
            done[j] = -1;
          else
            reseed[j] = 1;
        }
      }
      std::vector<const double*> zin(nb, nullptr);
      std::vector<double*> wout(nb, nullptr);
      bool running = false;
      for (int j = 0; j < nb; ++j) {
        if (done[j]) continue;
        if (k[j] >= cap) {
          done[j] = -1;
          continue;
        }
        running = true;
        const double* dir = (first[j] || reseed[j] || k[j] == 0) ? R[j] : C[j] + (int64_t)(k[j] - 1) * n;
        prec(dir, Z[j]);
        zin[j] = Z[j];
        wout[j] = W[j];
      }
      if (!running) break;
      applyB(zin, wout);
      // Orthogonalisation of the new images, all targets at a time: the dot
      // products of every target are read back with one wait per phase.
      std::vector<double> w0(nb, 0.0), wn(nb, 0.0);
      {
        DotBatch db;
        std::vector<int> iw(nb, -1), ib(nb, -1);
        for (int j = 0; j < nb; ++j) {
          if (!zin[j]) continue;
          first[j] = 0;
          iw[j] = db.dot(W[j], W[j]);
          ib[j] = db.multi(C[j], k[j], W[j]);
        }
        auto res = db.run(c, n);
        for (int j = 0; j < nb; ++j) {
          if (!zin[j]) continue;
          w0[j] = std::sqrt(res[iw[j]][0]);
          auto be = res[ib[j]];
          for (auto& v : be) v = -v;
          multi_axpy(c, C[j], k[j], n, be, W[j]);
          multi_axpy(c, U[j], k[j], n, be, Z[j]);
          iw[j] = db.dot(W[j], W[j]);
        }
        res = db.run(c, n);
        for (int j = 0; j < nb; ++j) {
          if (!zin[j]) continue;
          wn[j] = std::sqrt(res[iw[j]][0]);
          // second pass only where the first one cancelled
          if (!(wn[j] > 0.5 * w0[j])) {
            auto be2 = multi_dot(c, C[j], k[j], n, W[j]);
            for (auto& v : be2) v = -v;
            multi_axpy(c, C[j], k[j], n, be2, W[j]);
            multi_axpy(c, U[j], k[j], n, be2, Z[j]);
            wn[j] = std::sqrt(c->dot(W[j], W[j], n));
          }
        }
      }
      DotBatch dal;
      std::vector<int> ial(nb, -1);
      for (int j = 0; j < nb; ++j) {
        if (!zin[j]) continue;
        if (!(wn[j] > 1e-12 * w0[j])) {
          force[j] = 1;  // invariant space: confirm on the true residual
          continue;
        }
        double* un_ = U[j] + (int64_t)k[j] * n;
        double* cn_ = C[j] + (int64_t)k[j] * n;
        c->cp(un_, Z[j], n);
        c->axpby(0.0, Z[j], 1.0 / wn[j], un_, n);
        c->cp(cn_, W[j], n);
        c->axpby(0.0, W[j], 1.0 / wn[j], cn_, n);
        ++k[j];
        if (reseed[j]) {
          // project the true residual on the whole stored space
          auto al = multi_dot(c, C[j], k[j], n, R[j]);
          multi_axpy(c, U[j], k[j], n, al, X[j]);
          for (auto& v : al) v = -v;
          multi_axpy(c, C[j], k[j], n, al, R[j]);
          reseed[j] = 0;
        } else {
          ial[j] = dal.dot(cn_, R[j]);
        }
      }
      {
        auto res = dal.run(c, n);
        for (int j = 0; j < nb; ++j) {
          if (ial[j] < 0) continue;
          const double al = res[ial[j]][0];
          double* un_ = U[j] + (int64_t)(k[j] - 1) * n;
          double* cn_ = C[j] + (int64_t)(k[j] - 1) * n;
          c->axpby(al, un_, 1.0, X[j], n);
          c->axpby(-al, cn_, 1.0, R[j], n);
        }
      }
    }
    iters_total += it;
    // orbital response and contraction, target by target
    for (int j = 0; j < nb; ++j) {
      const Target& t = tg[b0 + j];
      if (done[j] != 1) {
        failed.push_back((int)(b0 + j));
        continue;
      }
      if (mult) c->cp(mult + (int64_t)(b0 + j) * n, X[j], n);
      int itk = 0;
      double relk = 0;
      int rc = orbital_response(c, segs, offs, X[j], t.kind, t.m, t.n, itk, relk);
      if (rc) return rc;
      iters_total += itk;
      contract_derivatives(c, ncoord, dh, dchol, t.out);
    }
  }
  // targets beyond the batched capacity: alone, with the full Krylov region
  for (int f : failed) {
    const Target& t = tg[f];
    c->log("  target %d solved alone\n", f);
    scc_info inf{};
    int rc = multipliers_solve(c, t.kind, t.m, t.n, &inf, guess ? guess + (int64_t)f * n : nullptr,
                               mult ? mult + (int64_t)f * n : nullptr, &rejected);
    if (rc) return rc;
    iters_total += inf.iterations;
    contract_derivatives(c, ncoord, dh, dchol, t.out);
  }
  return SCC_OK;
}

template <class F>
int guarded(scc_ctx* c, scc_info* info, F&& f) {
  auto t0 = std::chrono::steady_clock::now();
  double f0 = c ? c->flops : 0;
  int rc;
  if (c) c->used_lowp = false;
  try {
    if (c) {
      // order after the caller's stream
      hck(hipEventRecord(c->entry_ev, c->user_s));
      hck(hipStreamWaitEvent(c->s, c->entry_ev, 0));
    }
    rc = f();
    if (c) {
      c->ex->flush_profile();
      c->sync();
    }
  } catch (const SccError& e) {
    if (c) c->err = e.what();
    rc = e.code;
  } catch (const std::exception& e) {
    if (c) c->err = e.what();
    rc = SCC_EDEVICE;
  }
  // every call leaves the executor in FP64 mode and the solver pool as it
  // found it; a call that did not release its pool use is an internal error
  if (c) {
    c->ex->set_lowp(false);
    if (c->pool_used != c->pool_base) {
      if (rc == SCC_OK) {
        c->err = "internal error: solver pool not released (" + std::to_string(c->pool_used - c->pool_base) +
                 " doubles)";
        rc = SCC_EDEVICE;
      }
      c->pool_used = c->pool_base;
    }
  }
  if (info) {
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    info->flops_mfma = c ? c->flops - f0 : 0;
    info->precision = c && c->used_lowp ? 1 : 0;
    if (rc) info->converged = 0;
  }
  return rc;
}

bool valid_dims(const scc_dims* d) {
  return d && d->nocc >= 1 && d->nvirt >= 1 && d->nchol >= 1 && d->nstates >= 1 && d->nstates <= 16;
}

void default_opts(const scc_options* o, scc_options& out) {
  out.tol_residual = 1e-10;
  out.tol_overlap = 1e-11;
  out.max_iter = 200;
  out.scc = 1;
  out.verbose = 0;
  out.precision = 0;
  out.eager = 0;
  if (o) out = *o;
  if (out.tol_residual <= 0) out.tol_residual = 1e-10;
  if (out.tol_overlap <= 0) out.tol_overlap = 1e-11;
  if (out.max_iter <= 0) out.max_iter = 200;
}

struct Plan {
  std::unique_ptr<Model> m;
  int64_t arena, scratch, pool;
  size_t bytes;
};

Plan make_plan(const scc_dims* d) {
  Plan p;
  p.m = std::make_unique<Model>();
  Dims dd{d->nocc, d->nvirt, d->nocc + d->nvirt, d->nchol, d->nstates};
  build_model(*p.m, dd, dd.ns + 2, dd.ns + dd.npairs());
  p.arena = up(p.m->g.finalize(programs(*p.m), host_tensors(*p.m)), 32);
  p.scratch = up(std::max<int64_t>(Executor::plan_scratch(p.m->g), 32));
  p.pool = up(sizes_for(dd).pool);
  p.bytes = (size_t)(p.arena + p.scratch + PARTIALS + p.pool) * sizeof(double) + 256;
  return p;
}

}  // namespace

namespace {
int install_mo_hamiltonian_impl(scc_ctx* c, double e_nuc);
// MO-basis integrals are in m.h / m.L: derived quantities, checks, reset
int install_mo_hamiltonian(scc_ctx* c, double e_nuc) { return install_mo_hamiltonian_impl(c, e_nuc); }
}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

int scc_multiplier_length(const scc_dims* dims, long long* n) {
  if (!valid_dims(dims) || !n) return SCC_EINVAL;
  const long long nov = (long long)dims->nocc * dims->nvirt, ns = dims->nstates;
  *n = nov + nov * nov + ns * (2 + nov + nov * nov) + ns * (ns - 1) / 2;
  return SCC_OK;
}

int scc_workspace_bytes(const scc_dims* dims, const scc_options* opts, size_t* bytes) {
  (void)opts;
  if (!valid_dims(dims) || !bytes) return SCC_EINVAL;
  try {
    Plan p = make_plan(dims);
    *bytes = p.bytes;
  } catch (...) {
    return SCC_EINVAL;
  }
  return SCC_OK;
}

int scc_create(const scc_dims* dims, const scc_options* opts, void* workspace, size_t bytes, void* hip_stream,
               scc_ctx** ctx) {
  if (!valid_dims(dims) || !workspace || !ctx) return SCC_EINVAL;
  *ctx = nullptr;
  try {
    Plan p = make_plan(dims);
    if (bytes < p.bytes) return SCC_ENOMEM;
    auto c = std::make_unique<scc_ctx>();
    c->m = std::move(*p.m);
    Dims dd = c->m.d;
    c->sz = sizes_for(dd);
    default_opts(opts, c->opt);
    c->user_s = (hipStream_t)hip_stream;
    hck(hipStreamCreateWithFlags(&c->s, hipStreamNonBlocking));
    hck(hipEventCreateWithFlags(&c->entry_ev, hipEventDisableTiming));
    uintptr_t base = ((uintptr_t)workspace + 255) & ~(uintptr_t)255;
    c->arena = (double*)base;
    c->scratch = c->arena + p.arena;
    c->scratch_n = p.scratch;
    c->partials = c->scratch + p.scratch;
    c->pool = c->partials + PARTIALS;
    c->sz.pool = p.pool;
    c->ex = std::make_unique<Executor>(c->m.g, c->arena, c->scratch, c->scratch_n, c->partials);
    c->ex->plan_all();
    c->ex->set_graphs(c->opt.eager == 0);
    c->D = c->alloc(c->sz.nvt);
    c->Dk = c->alloc(c->sz.nov);
    for (int k = 0; k < dd.ns; ++k) {
      c->R.push_back(c->alloc(c->sz.nst));
      c->Lv.push_back(c->alloc(c->sz.nst));
    }
    c->kbar = c->alloc(c->sz.nov);
    c->dsc = c->alloc(32);
    c->rec_lag.n = c->sz.nlag;
    c->rec_lag.cap = c->sz.cap_lag;
    c->krylov = c->alloc(c->sz.krylov);
    c->rec_lag.U = c->krylov;
    c->rec_lag.C = c->krylov + (int64_t)c->sz.cap_lag * up(c->sz.nlag);
    c->batch_vec = c->alloc(5 * (int64_t)c->sz.nbt * up(c->sz.nlag));
    c->rec_k.n = c->sz.nov;
    c->rec_k.cap = c->sz.cap_k;
    c->rec_k.U = c->alloc((int64_t)c->sz.cap_k * up(c->sz.nov));
    c->rec_k.C = c->alloc((int64_t)c->sz.cap_k * up(c->sz.nov));
    c->cisA = c->alloc(c->sz.nov * c->sz.nov);
    c->cisU = c->alloc(c->sz.nov * c->sz.nov);
    c->cisW = c->alloc(c->sz.nov);
    c->eps_d = c->alloc(dd.n);
    c->cis_work = c->alloc(jacobi_work_doubles((int)c->sz.nov));
    c->cis_tmp = c->alloc(c->sz.nov);
    c->pool_base = c->pool_used;
    // constants
    Model& m = c->m;
    std::vector<double> In((size_t)dd.n * dd.n, 0.0), Io((size_t)dd.o * dd.o, 0.0);
    for (int i = 0; i < dd.n; ++i) In[(size_t)i * dd.n + i] = 1.0;
    for (int i = 0; i < dd.o; ++i) Io[(size_t)i * dd.o + i] = 1.0;
    c->xfer(c->tp(m.In), In.data(), In.size() * sizeof(double), hipMemcpyHostToDevice);
    c->xfer(c->tp(m.Io), Io.data(), Io.size() * sizeof(double), hipMemcpyHostToDevice);
    c->set_scalar(m.one, 1.0);
    c->fill(c->tp(m.z2), m.g.t[m.z2].size(), 0.0);
    c->fill(c->tp(m.kappa), c->sz.nov, 0.0);
    c->fill(c->tp(m.t1), c->sz.nov, 0.0);
    c->fill(c->tp(m.t2), c->sz.nov * c->sz.nov, 0.0);
    for (int z : m.zeta) c->set_scalar(z, 0.0);
    for (auto& xs : m.xs) {
      c->fill(c->tp(xs.r0), 1, 0.0);
      c->fill(c->tp(xs.r1), c->sz.nov, 0.0);
      c->fill(c->tp(xs.r2), c->sz.nov * c->sz.nov, 0.0);
    }
    c->sync();
    *ctx = c.release();
  } catch (const SccError& e) {
    return e.code;
  } catch (const std::exception& e) {
    fprintf(stderr, "scc_create: %s\n", e.what());
    return SCC_EDEVICE;
  }
  return SCC_OK;
}

void scc_destroy(scc_ctx* ctx) { delete ctx; }

const char* scc_last_error(const scc_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int scc_set_hamiltonian(scc_ctx* c, const double* h, const double* chol, double e_nuc) {
  if (!c || !h || !chol) return SCC_EINVAL;
  // a failed call leaves the context without a Hamiltonian
  c->have_h = c->have_ground = c->have_excited = c->have_mult = false;
  return guarded(c, nullptr, [&]() -> int {
    Model& m = c->m;
    c->cp(c->tp(m.h), h, m.g.t[m.h].size());
    c->cp(c->tp(m.L), chol, m.g.t[m.L].size());
    c->fixed_basis = false;
    return install_mo_hamiltonian(c, e_nuc);
  });
}

int scc_set_hamiltonian_fixed_basis(scc_ctx* c, const double* h, const double* chol, double e_nuc,
                                    const double* orbitals_guess, double* orbitals, scc_info* info) {
  if (!c || !h || !chol) return SCC_EINVAL;
  c->have_h = c->have_ground = c->have_excited = c->have_mult = false;
  return guarded(c, info, [&]() -> int {
    Model& m = c->m;
    const int N = m.d.n, o = m.d.o;
    c->cp(c->tp(m.hao), h, m.g.t[m.hao].size());
    c->cp(c->tp(m.Lao), chol, m.g.t[m.Lao].size());
    // reference orbitals: the guess (phase reference too) or the basis itself
    std::vector<double> ref((size_t)N * N, 0.0), C, F((size_t)N * N), w, V;
    if (orbitals_guess) {
      c->sync();
      c->xfer(ref.data(), orbitals_guess, ref.size() * sizeof(double), hipMemcpyDeviceToHost);
    } else {
      for (int p = 0; p < N; ++p) ref[(size_t)p * N + p] = 1.0;
    }
    C = ref;
    // Roothaan iterations: F(C) diagonalised, occupied = lowest o orbitals,
    // until the Fock matrix commutes with the density, max |F D - D F| < tol.
    // The matrix diagonalised is Pulay's DIIS extrapolation of the last
    // eight Fock matrices (error vectors F D - D F): plain Roothaan steps
    // oscillate with growing amplitude for some systems.
    const double tol = std::min(1e-12, 1e-2 * c->opt.tol_residual);
    int it = 0;
    double comm = 1.0;
    const int ndiis = 8;
    std::vector<std::vector<double>> Fh, Eh;
    for (; it < 500; ++it) {
      c->xfer(c->tp(m.Cmo), C.data(), C.size() * sizeof(double), hipMemcpyHostToDevice);
      c->run(m.p_aofock);
      c->sync();
      c->xfer(F.data(), c->tp(m.Fao), F.size() * sizeof(double), hipMemcpyDeviceToHost);
      std::vector<double> D((size_t)N * N, 0.0);
      for (int p = 0; p < N; ++p)
        for (int q = 0; q < N; ++q) {
          double x = 0;
          for (int i = 0; i < o; ++i) x += C[(size_t)p * N + i] * C[(size_t)q * N + i];
          D[(size_t)p * N + q] = x;
        }
      comm = 0;
      std::vector<double> err((size_t)N * N);
      for (int p = 0; p < N; ++p)
        for (int q = 0; q < N; ++q) {
          double x = 0;
          for (int r = 0; r < N; ++r) x += F[(size_t)p * N + r] * D[(size_t)r * N + q] - D[(size_t)p * N + r] * F[(size_t)r * N + q];
          err[(size_t)p * N + q] = x;
          comm = std::max(comm, std::fabs(x));
        }
      const bool done = comm < tol;
      if (done) {
        // canonical orbitals of the converged Fock matrix (a rotation within
        // the occupied and within the virtual blocks; D is unchanged)
        eig_sym(N, F, w, V);
        for (int k = 0; k < N; ++k) {
          double sgn = 0;
          for (int p = 0; p < N; ++p) sgn += ref[(size_t)p * N + k] * V[(size_t)p * N + k];
          if (sgn < 0)
            for (int p = 0; p < N; ++p) V[(size_t)p * N + k] = -V[(size_t)p * N + k];
        }
        C = V;
        break;
      }
      Fh.push_back(F);
      Eh.push_back(err);
      if ((int)Fh.size() > ndiis) {
        Fh.erase(Fh.begin());
        Eh.erase(Eh.begin());
      }
      const int nh = (int)Fh.size(), n1 = nh + 1;
      std::vector<double> B((size_t)n1 * n1, -1.0), cf(n1, 0.0);
      B[(size_t)nh * n1 + nh] = 0.0;
      double bscale = 0;
      for (int i = 0; i < nh; ++i)
        for (int j = 0; j <= i; ++j) {
          double x = 0;
          for (size_t e = 0; e < err.size(); ++e) x += Eh[i][e] * Eh[j][e];
          B[(size_t)i * n1 + j] = B[(size_t)j * n1 + i] = x;
          if (i == j) bscale = std::max(bscale, x);
        }
      if (bscale > 0)
        for (int i = 0; i < nh; ++i)
          for (int j = 0; j < nh; ++j) B[(size_t)i * n1 + j] /= bscale;
      cf[nh] = -1.0;
      std::vector<double> Fx = F;
      if (solve_linear(n1, B, cf)) {
        std::fill(Fx.begin(), Fx.end(), 0.0);
        for (int i = 0; i < nh; ++i)
          for (size_t e = 0; e < Fx.size(); ++e) Fx[e] += cf[i] * Fh[i][e];
      }
      eig_sym(N, Fx, w, V);
      // phase: each orbital overlaps its reference orbital positively
      for (int k = 0; k < N; ++k) {
        double sgn = 0;
        for (int p = 0; p < N; ++p) sgn += ref[(size_t)p * N + k] * V[(size_t)p * N + k];
        if (sgn < 0)
          for (int p = 0; p < N; ++p) V[(size_t)p * N + k] = -V[(size_t)p * N + k];
      }
      C = V;
    }
    if (comm >= tol) throw SccError(SCC_ENOCONV, "RHF iterations did not converge");
    c->log(" RHF converged in %d iterations (max |FD - DF| %.2e)\n", it, comm);
    c->xfer(c->tp(m.Cmo), C.data(), C.size() * sizeof(double), hipMemcpyHostToDevice);
    if (orbitals) c->xfer(orbitals, C.data(), C.size() * sizeof(double), hipMemcpyHostToDevice);
    c->run(m.p_aotrans);
    c->cp(c->tp(m.h), c->tp(m.hmo), m.g.t[m.h].size());
    c->cp(c->tp(m.L), c->tp(m.Lmo), m.g.t[m.L].size());
    c->fixed_basis = true;
    if (info) {
      info->iterations = it;
      info->residual = comm;
      info->converged = 1;
    }
    return install_mo_hamiltonian(c, e_nuc);
  });
}

namespace {
int install_mo_hamiltonian_impl(scc_ctx* c, double e_nuc) {
    Model& m = c->m;
    c->fill(c->tp(m.kappa), c->sz.nov, 0.0);
    c->run(m.p_setup);
    // orbital energies from the Fock diagonal
    const int N = m.d.n, o = m.d.o, v = m.d.v;
    std::vector<double> F((size_t)N * N);
    c->sync();
    c->xfer(F.data(), c->tp(m.fock), F.size() * sizeof(double), hipMemcpyDeviceToHost);
    c->eps.resize(N);
    for (int p = 0; p < N; ++p) c->eps[p] = F[(size_t)p * N + p];
    double fai = 0;
    for (int a = 0; a < v; ++a)
      for (int i = 0; i < o; ++i) fai = std::max(fai, std::fabs(F[(size_t)(o + a) * N + i]));
    if (fai > 1e-6) throw SccError(SCC_EINVAL, "integrals are not in a Hartree-Fock basis (max|F_ai| > 1e-6)");
    // Diagonal preconditioners.  Doubles: orbital-energy differences.
    // Singles: the diagonal of the singlet singles-singles block at t = 0,
    //   eps_a - eps_i + 2 (ai|ai) - (aa|ii),
    // which differs from eps_a - eps_i by terms of the size of the low
    // excitation energies themselves.  Orbital response: the diagonal of
    // the closed-shell RHF Hessian, eps_a - eps_i + 3 (ai|ai) - (aa|ii).
    const int J = m.d.nj;
    std::vector<double> Lh((size_t)J * N * N);
    c->xfer(Lh.data(), c->tp(m.L), Lh.size() * sizeof(double), hipMemcpyDeviceToHost);
    std::vector<double> D(c->sz.nvt), Dk(c->sz.nov);
    const int64_t nov = c->sz.nov;
    for (int a = 0; a < v; ++a)
      for (int i = 0; i < o; ++i) {
        double coul = 0, exch = 0;
        for (int j = 0; j < J; ++j) {
          const double* Lj = Lh.data() + (size_t)j * N * N;
          double lai = Lj[(size_t)(o + a) * N + i];
          coul += lai * lai;
          exch += Lj[(size_t)(o + a) * N + o + a] * Lj[(size_t)i * N + i];
        }
        const double de = c->eps[o + a] - c->eps[i];
        D[a * o + i] = de + 2.0 * coul - exch;
        Dk[a * o + i] = de + 3.0 * coul - exch;
      }
    for (int64_t p = 0; p < nov; ++p) {
      const int64_t ap = p / o, ip = p % o;
      for (int64_t q = 0; q < nov; ++q) {
        const int64_t aq = q / o, iq = q % o;
        D[nov + p * nov + q] = c->eps[o + ap] - c->eps[ip] + c->eps[o + aq] - c->eps[iq];
      }
    }
    c->xfer(c->D, D.data(), D.size() * sizeof(double), hipMemcpyHostToDevice);
    c->xfer(c->Dk, Dk.data(), Dk.size() * sizeof(double), hipMemcpyHostToDevice);
    // singles preconditioner of this geometry
    c->xfer(c->eps_d, c->eps.data(), N * sizeof(double), hipMemcpyHostToDevice);
    launch_cis_matrix(c->tp(m.L), J, o, v, c->eps_d, c->cisA, c->s);
    const int sweeps = sym_eig_jacobi(c->cisA, c->cisU, c->cisW, (int)nov, c->cis_work, c->s);
    launch_transpose(c->cisU, (int)nov, c->cisA, c->s);
    c->log(" singles matrix diagonalised in %d Jacobi sweeps\n", sweeps);
    // every geometry starts cold: t = 0 (the first Jacobi step is MP2), zeta = 0
    c->fill(c->tp(m.t1), nov, 0.0);
    c->fill(c->tp(m.t2), nov * nov, 0.0);
    c->enuc = e_nuc;
    c->have_h = true;
    c->have_ground = c->have_excited = c->have_mult = false;
    c->rec_lag.reset();
    c->rec_k.reset();
    return SCC_OK;
}
}  // namespace

int scc_ground(scc_ctx* c, const double* guess_t, double* e0, scc_info* info) {
  if (!c) return SCC_EINVAL;
  if (!c->have_h) {
    c->err = "scc_ground before scc_set_hamiltonian";
    return SCC_ESTATE;
  }
  return guarded(c, info, [&]() -> int {
    Model& m = c->m;
    const int64_t nov = c->sz.nov, nvt = c->sz.nvt;
    for (int z : m.zeta) c->set_scalar(z, 0.0);
    if (guess_t) {
      // the residual judges the guess: it is used only if its residual is
      // below that of the plain start (the MP2 amplitudes, the first step
      // from t = 0)
      PoolMark pm(c);
      double* r = c->alloc(nvt);
      double* tm = c->alloc(nvt);
      auto resnorm = [&](const double* t) {
        c->put(m.t1, t);
        c->put(m.t2, t + nov);
        c->run(m.p_res);
        c->get(m.res.O1, r);
        c->get(m.res.O2, r + nov);
        c->sym_doubles(r + nov);
        return std::sqrt(c->dot(r, r, nvt));
      };
      c->fill(tm, nvt, 0.0);
      resnorm(tm);
      launch_precond(r, c->D, 0.0, 1e-8, tm, nvt, c->s);
      c->axpby(0.0, tm, -1.0, tm, nvt);
      const double r_plain = resnorm(tm);
      const double r_guess = resnorm(guess_t);
      const bool use = std::isfinite(r_guess) && r_guess < r_plain;
      c->log(" ground guess: residual %.3e (plain start %.3e) -> %s\n", r_guess, r_plain, use ? "used" : "rejected");
      if (!use) {
        c->put(m.t1, tm);
        c->put(m.t2, tm + nov);
        if (info) info->fallback_used = 1;
      }
    }
    double rn = 0;
    int rc = ground_solve(c, c->opt.tol_residual, c->opt.max_iter, rn);
    c->E0 = c->tensor_scalar(m.res.E) + c->enuc;
    if (e0) launch_fill(e0, 1, c->E0, c->s);
    if (info) {
      info->iterations = c->last_ground_its;
      info->residual = rn;
      info->converged = rc == SCC_OK;
    }
    c->E0 -= c->enuc;
    if (rc == SCC_OK) c->have_ground = true;
    return rc;
  });
}

int scc_excited(scc_ctx* c, int nstates, const double* guess, double* energies, double* zeta, scc_info* info) {
  if (!c) return SCC_EINVAL;
  if (nstates != c->m.d.ns) {
    c->err = "nstates must equal the context's nstates";
    return SCC_EINVAL;
  }
  if (!c->have_h) {
    c->err = "scc_excited before scc_set_hamiltonian";
    return SCC_ESTATE;
  }
  return guarded(c, info, [&]() -> int {
    int rc = SCC_ENOCONV;
    if (guess) {
      // start from the given states and zeta; fall back to the plain start
      // (CCSD states at zeta = 0) if that solve fails
      const int ns = c->m.d.ns, np = c->m.d.npairs();
      const int64_t nst = c->sz.nst;
      for (int k = 0; k < ns; ++k) c->cp(c->R[k], guess + k * nst, nst);
      std::vector<double> z(np, 0.0);
      if (np) c->xfer(z.data(), guess + (int64_t)ns * nst, np * sizeof(double), hipMemcpyDeviceToHost);
      bool finite = true;
      for (double x : z) finite = finite && std::isfinite(x);
      if (finite) {
        c->zeta = z;
        // the zeta Jacobian of the previous solve (a nearby geometry along a
        // trajectory) seeds the Newton/Broyden iteration
        if (c->Jz.size() != (size_t)np * np) c->Jz.clear();
        try {
          int iters = 0;
          rc = excited_pass(c, c->opt.tol_residual, c->opt.tol_overlap, true, iters);
          if (info) info->iterations = iters;
        } catch (const SccError& e) {
          rc = e.code;
        }
      }
      c->log(" excited-state guess %s\n", rc == SCC_OK ? "used" : "rejected");
      if (rc != SCC_OK && info) info->fallback_used = 1;
    }
    if (rc != SCC_OK) {
      int fb = info ? info->fallback_used : 0;
      rc = excited_solve(c, info);
      if (info) info->fallback_used = fb;
    }
    if (rc) return rc;
    c->have_ground = c->have_excited = true;
    c->have_mult = false;
    c->rec_lag.reset();
    c->rec_k.reset();
    if (energies) {
      std::vector<double> e(c->E);
      for (auto& x : e) x += c->enuc;
      c->xfer(energies, e.data(), e.size() * sizeof(double), hipMemcpyHostToDevice);
    }
    if (zeta && !c->zeta.empty()) c->xfer(zeta, c->zeta.data(), c->zeta.size() * sizeof(double), hipMemcpyHostToDevice);
    return SCC_OK;
  });
}

int scc_multipliers(scc_ctx* c, int kind, int m, int n, const double* guess, double* multipliers, scc_info* info) {
  if (!c) return SCC_EINVAL;
  const int ns = c->m.d.ns;
  if (kind < 0 || kind > 1 || n < 0 || n >= ns || (kind == 1 && (m < 0 || m >= ns || m == n))) {
    c->err = "bad target";
    return SCC_EINVAL;
  }
  if (!c->have_excited) {
    c->err = "scc_multipliers before scc_excited";
    return SCC_ESTATE;
  }
  return guarded(c, info, [&]() -> int {
    bool rejected = false;
    const int rc = multipliers_solve(c, kind, m, n, info, guess, multipliers, &rejected);
    if (info && rejected) info->fallback_used = 1;
    return rc;
  });
}

int scc_densities(scc_ctx* c, int kind, int mm, int nn, double* d1, double* z3, double* kappa_bar) {
  if (!c) return SCC_EINVAL;
  const int ns = c->m.d.ns;
  if (kind < 0 || kind > 1 || nn < 0 || nn >= ns || (kind == 1 && (mm < 0 || mm >= ns || mm == nn))) {
    c->err = "bad target";
    return SCC_EINVAL;
  }
  if (!c->have_excited) {
    c->err = "scc_densities before scc_excited";
    return SCC_ESTATE;
  }
  return guarded(c, nullptr, [&]() -> int {
    if (!(c->have_mult && c->mult_kind == kind && c->mult_n == nn && (kind == 0 || c->mult_m == mm))) {
      int rc = multipliers_solve(c, kind, mm, nn, nullptr);
      if (rc) return rc;
    }
    integral_adjoints(c);
    if (c->fixed_basis) {
      c->run(c->m.p_aodens);
      if (d1) c->get(c->m.d1ao, d1);
      if (z3) c->get(c->m.zao, z3);
    } else {
      if (d1) c->get(c->m.a_h, d1);
      if (z3) c->get(c->m.a_L, z3);
    }
    if (kappa_bar) c->cp(kappa_bar, c->kbar, c->sz.nov);
    return SCC_OK;
  });
}

static int derivative(scc_ctx* c, int kind, int mm, int nn, int ncoord, const double* dh, const double* dchol,
                      double* out, scc_info* info) {
  if (!c) return SCC_EINVAL;
  const int ns = c->m.d.ns;
  if (!dh || !dchol || !out || ncoord < 0 || (int64_t)ncoord * 256 > PARTIALS) {
    c->err = "bad derivative-integral arguments";
    return SCC_EINVAL;
  }
  if (nn < 0 || nn >= ns || (kind == 1 && (mm < 0 || mm >= ns || mm == nn))) {
    c->err = "bad target state";
    return SCC_EINVAL;
  }
  if (!c->have_excited) {
    c->err = "gradient or coupling before scc_excited";
    return SCC_ESTATE;
  }
  return guarded(c, info, [&]() -> int {
    if (!(c->have_mult && c->mult_kind == kind && c->mult_n == nn && (kind == 0 || c->mult_m == mm))) {
      int rc = multipliers_solve(c, kind, mm, nn, info);
      if (rc) return rc;
    }
    contract_derivatives(c, ncoord, dh, dchol, out);
    return SCC_OK;
  });
}

int scc_gradient(scc_ctx* c, int n, int ncoord, const double* dh, const double* dchol, double* grad, scc_info* info) {
  if (c && (n < 0 || n >= c->m.d.ns)) return SCC_EINVAL;
  return derivative(c, 0, -1, n, ncoord, dh, dchol, grad, info);
}

int scc_nac(scc_ctx* c, int m, int n, int ncoord, const double* dh, const double* dchol, double* nac, scc_info* info) {
  if (c && (n < 0 || n >= c->m.d.ns || m < 0 || m >= c->m.d.ns || m == n)) return SCC_EINVAL;
  return derivative(c, 1, m, n, ncoord, dh, dchol, nac, info);
}

int scc_gradients_and_couplings(scc_ctx* c, int ngrad, const int* states, int npair, const int* pairs, int ncoord,
                                const double* dh, const double* dchol, const double* guess, double* multipliers,
                                double* grads, double* nacs, scc_info* info) {
  if (!c) return SCC_EINVAL;
  const int ns = c->m.d.ns;
  if (ngrad < 0 || npair < 0 || (ngrad > 0 && (!states || !grads)) || (npair > 0 && (!pairs || !nacs)) || !dh ||
      !dchol || ncoord < 0 || (int64_t)ncoord * 256 > PARTIALS) {
    c->err = "bad arguments";
    return SCC_EINVAL;
  }
  std::vector<Target> tg;
  for (int i = 0; i < ngrad; ++i) {
    if (states[i] < 0 || states[i] >= ns) {
      c->err = "bad state index";
      return SCC_EINVAL;
    }
    tg.push_back({0, -1, states[i], grads + (int64_t)i * ncoord});
  }
  for (int i = 0; i < npair; ++i) {
    const int mm = pairs[2 * i], nn = pairs[2 * i + 1];
    if (mm < 0 || mm >= ns || nn < 0 || nn >= ns || mm == nn) {
      c->err = "bad state pair";
      return SCC_EINVAL;
    }
    tg.push_back({1, mm, nn, nacs + (int64_t)i * ncoord});
  }
  if (!c->have_excited) {
    c->err = "gradients or couplings before scc_excited";
    return SCC_ESTATE;
  }
  return guarded(c, info, [&]() -> int {
    int iters = 0;
    bool rejected = false;
    int rc = SCC_OK;
    if (c->m.nbt > 1) {
      rc = targets_solve(c, tg, ncoord, dh, dchol, iters, guess, multipliers, rejected);
    } else {
      const int64_t n = c->sz.nlag;
      for (size_t i = 0; i < tg.size(); ++i) {
        const Target& t = tg[i];
        scc_info inf{};
        rc = multipliers_solve(c, t.kind, t.m, t.n, &inf, guess ? guess + (int64_t)i * n : nullptr,
                               multipliers ? multipliers + (int64_t)i * n : nullptr, &rejected);
        if (rc) break;
        iters += inf.iterations;
        contract_derivatives(c, ncoord, dh, dchol, t.out);
      }
    }
    if (info) {
      info->iterations = iters;
      info->converged = rc == SCC_OK;
      info->fallback_used = rejected ? 1 : 0;
    }
    return rc;
  });
}

int scc_get(scc_ctx* c, int field, int k, double* out) {
  if (!c || !out) return SCC_EINVAL;
  return guarded(c, nullptr, [&]() -> int {
    Model& m = c->m;
    const int64_t nov = c->sz.nov;
    switch (field) {
      case SCC_FIELD_T:
        c->get(m.t1, out);
        c->get(m.t2, out + nov);
        return SCC_OK;
      case SCC_FIELD_R:
      case SCC_FIELD_L:
        if (!c->have_excited || k < 0 || k >= m.d.ns) return SCC_ESTATE;
        c->cp(out, field == SCC_FIELD_R ? c->R[k] : c->Lv[k], c->sz.nst);
        return SCC_OK;
      case SCC_FIELD_E0:
        launch_fill(out, 1, c->E0 + c->enuc, c->s);
        return SCC_OK;
      case SCC_FIELD_OMEGA:
        c->run(m.p_res);
        c->get(m.res.O1, out);
        c->get(m.res.O2, out + nov);
        return SCC_OK;
    }
    return SCC_EINVAL;
  });
}

int scc_profile(scc_ctx* c, int enable, int kernel, double* gemm_ms, double* gemm_flops, long long* gemm_launches,
                double* gemm_bytes) {
  if (!c || kernel < 0 || kernel >= NGEMMK) return SCC_EINVAL;
  return guarded(c, nullptr, [&]() -> int {
    const bool was_on = c->ex->profiling();
    c->ex->flush_profile();
    c->ex->set_profile(enable != 0);
    if (!enable && was_on && c->opt.verbose) c->ex->shape_report(stderr, 25);
    if (gemm_ms) *gemm_ms = c->ex->kernel_ms[kernel];
    if (gemm_flops) *gemm_flops = c->ex->kernel_flops[kernel];
    if (gemm_launches) *gemm_launches = (long long)c->ex->kernel_launches[kernel];
    if (gemm_bytes) *gemm_bytes = c->ex->kernel_bytes[kernel];
    return SCC_OK;
  });
}

int scc_profile_kernels(scc_ctx* c, unsigned mask) {
  if (!c) return SCC_EINVAL;
  return guarded(c, nullptr, [&]() -> int {
    c->ex->flush_profile();
    c->ex->set_profile_mask(mask);
    return SCC_OK;
  });
}

int scc_eval_residual(scc_ctx* c, const double* t, const double* zeta, const double* xs, double* out) {
  if (!c || !t || !out) return SCC_EINVAL;
  if (!c->have_h) return SCC_ESTATE;
  return guarded(c, nullptr, [&]() -> int {
    Model& m = c->m;
    const int64_t nov = c->sz.nov;
    c->put(m.t1, t);
    c->put(m.t2, t + nov);
    for (size_t p = 0; p < m.zeta.size(); ++p) {
      if (zeta)
        c->cp(c->tp(m.zeta[p]), zeta + p, 1);
      else
        c->set_scalar(m.zeta[p], 0.0);
    }
    for (int k = 0; k < m.d.ns; ++k) {
      if (xs)
        c->put_state(m.xs[k], xs + k * c->sz.nst);
      else {
        c->fill(c->tp(m.xs[k].r0), 1, 0.0);
        c->fill(c->tp(m.xs[k].r1), nov, 0.0);
        c->fill(c->tp(m.xs[k].r2), nov * nov, 0.0);
      }
    }
    c->set_lowp(c->opt.precision == 1);
    c->run(m.p_res);
    c->ex->set_lowp(false);
    c->get(m.res.E, out);
    c->get(m.res.O1, out + 1);
    c->get(m.res.O2, out + 1 + nov);
    return SCC_OK;
  });
}

int scc_eval_sigma(scc_ctx* c, const double* vec, double* out) {
  if (!c || !vec || !out) return SCC_EINVAL;
  if (!c->have_h) return SCC_ESTATE;
  return guarded(c, nullptr, [&]() -> int {
    Model& m = c->m;
    c->run(m.p_sig_pre);
    c->put_state(m.vin, vec);
    c->run(m.p_sig);
    c->get(m.sig.s0, out);
    c->get(m.sig.s1, out + 1);
    c->get(m.sig.s2, out + 1 + c->sz.nov);
    return SCC_OK;
  });
}

int scc_eval_left(scc_ctx* c, const double* vec, double* out) {
  if (!c || !vec || !out) return SCC_EINVAL;
  if (!c->have_h) return SCC_ESTATE;
  return guarded(c, nullptr, [&]() -> int {
    Model& m = c->m;
    c->run(m.p_sig_pre);
    c->put_state(m.lin, vec);
    c->run(m.p_left);
    c->get(m.lout.r0, out);
    c->get(m.lout.r1, out + 1);
    c->get(m.lout.r2, out + 1 + c->sz.nov);
    c->sym_doubles(out + 1 + c->sz.nov);
    return SCC_OK;
  });
}

}  // extern "C"
