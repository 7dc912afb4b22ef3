// Singles-space preconditioner of the solvers: the closed-shell singlet
// singles matrix of the Hamiltonian (the singles-singles block of the
// coupled cluster Jacobian at T = 0),
//     A_ai,bj = (eps_a - eps_i) d_ab d_ij + 2 (ai|jb) - (ab|ij),
// built from the MO Cholesky vectors, diagonalised once per geometry in FP64
// on the device by a parallel two-sided Jacobi iteration, and applied for any
// shift theta as U diag(1 / (w - theta)) U^T (floored denominators).  The
// synthetic Hamiltonians couple all singles strongly, so the low excited
// states spread over many (ai) and a diagonal preconditioner alone resolves
// them slowly.
#include <hip/hip_runtime.h>

#include <cmath>
#include <stdexcept>
#include <string>
#include <vector>

#include "exec.hpp"
#include "singles.hpp"

namespace scc {
namespace {

void hck(hipError_t e, const char* what) {
  if (e != hipSuccess) throw std::runtime_error(std::string(what) + ": " + hipGetErrorString(e));
}

// A[(a o + i)][(b o + j)], one thread per element, the Cholesky index summed
// in order
__global__ __launch_bounds__(256) void cis_matrix_kernel(const double* __restrict__ L, int nj, int o, int v,
                                                         const double* __restrict__ eps, double* __restrict__ A) {
  const int N = o + v;
  const int64_t nov = (int64_t)o * v;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nov * nov) return;
  const int64_t row = idx / nov, col = idx - row * nov;
  const int a = (int)(row / o), i = (int)(row - (int64_t)a * o);
  const int b = (int)(col / o), j = (int)(col - (int64_t)b * o);
  const int64_t NN = (int64_t)N * N;
  const int64_t o_ai = (int64_t)(o + a) * N + i, o_jb = (int64_t)j * N + o + b;
  const int64_t o_ab = (int64_t)(o + a) * N + o + b, o_ij = (int64_t)i * N + j;
  double coul = 0.0, exch = 0.0;
  for (int J = 0; J < nj; ++J) {
    const double* LJ = L + J * NN;
    coul += LJ[o_ai] * LJ[o_jb];
    exch += LJ[o_ab] * LJ[o_ij];
  }
  double val = 2.0 * coul - exch;
  if (row == col) val += eps[o + a] - eps[i];
  A[idx] = val;
}

// round-robin pairing of m (even) indices, round r in [0, m - 1): every
// index meets every other once per sweep; index m - 1 stays fixed
__device__ __forceinline__ void rr_pair(int r, int k, int m, int& p, int& q) {
  if (k == 0) {
    p = m - 1;
    q = r;
  } else {
    p = (r + k) % (m - 1);
    q = (r - k + (m - 1)) % (m - 1);
  }
  if (p > q) {
    const int t = p;
    p = q;
    q = t;
  }
}

// Jacobi rotations of one round: J = [[c, s], [-s, c]] on (p, q) zeroes
// A_pq in J^T A J (symmetric 2 x 2 Schur decomposition); pairs that involve
// the padding index n (odd n) or whose A_pq is already negligible do nothing
__global__ void jacobi_angles_kernel(const double* __restrict__ A, int n, int m, int r, double* cs, double* sn,
                                     int* pp, int* qq) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m / 2) return;
  int p, q;
  rr_pair(r, k, m, p, q);
  double c = 1.0, s = 0.0;
  if (q < n) {
    const double apq = A[(int64_t)p * n + q];
    const double app = A[(int64_t)p * n + p], aqq = A[(int64_t)q * n + q];
    if (fabs(apq) > 1e-300 && fabs(apq) > 1e-18 * sqrt(fabs(app * aqq))) {
      const double tau = (aqq - app) / (2.0 * apq);
      const double t = tau >= 0.0 ? 1.0 / (tau + sqrt(1.0 + tau * tau)) : -1.0 / (-tau + sqrt(1.0 + tau * tau));
      c = 1.0 / sqrt(1.0 + t * t);
      s = t * c;
    }
  } else {
    q = -1;
  }
  cs[k] = c;
  sn[k] = s;
  pp[k] = p;
  qq[k] = q;
}

// rows p, q of A <- J^T A (one thread per (pair, column))
__global__ void jacobi_rows_kernel(double* __restrict__ A, int n, int npair, const double* cs, const double* sn,
                                   const int* pp, const int* qq) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)npair * n) return;
  const int k = (int)(idx / n), jcol = (int)(idx - (int64_t)k * n);
  const int q = qq[k];
  const double s = sn[k];
  if (q < 0 || s == 0.0) return;
  const int p = pp[k];
  const double c = cs[k];
  double* ap = A + (int64_t)p * n + jcol;
  double* aq = A + (int64_t)q * n + jcol;
  const double x = *ap, y = *aq;
  *ap = c * x - s * y;
  *aq = s * x + c * y;
}

// columns p, q of A <- A J and of V <- V J (one thread per (row, pair))
__global__ void jacobi_cols_kernel(double* __restrict__ A, double* __restrict__ V, int n, int npair,
                                   const double* cs, const double* sn, const int* pp, const int* qq) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)npair * n) return;
  const int i = (int)(idx / npair), k = (int)(idx - (int64_t)i * npair);
  const int q = qq[k];
  const double s = sn[k];
  if (q < 0 || s == 0.0) return;
  const int p = pp[k];
  const double c = cs[k];
  double* a = A + (int64_t)i * n;
  const double x = a[p], y = a[q];
  a[p] = c * x - s * y;
  a[q] = s * x + c * y;
  double* vv = V + (int64_t)i * n;
  const double vx = vv[p], vy = vv[q];
  vv[p] = c * vx - s * vy;
  vv[q] = s * vx + c * vy;
}

constexpr int NORM_BLOCKS = 256;

// partial sums of squares: off-diagonal and all elements, per block
__global__ __launch_bounds__(256) void offdiag_kernel(const double* __restrict__ A, int n, double* part) {
  __shared__ double so[256], sa[256];
  double off = 0.0, all = 0.0;
  const int64_t total = (int64_t)n * n;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const double x = A[idx];
    const int64_t r = idx / n;
    all += x * x;
    if (idx - r * n != r) off += x * x;
  }
  so[threadIdx.x] = off;
  sa[threadIdx.x] = all;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      so[threadIdx.x] += so[threadIdx.x + w];
      sa[threadIdx.x] += sa[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = so[0];
    part[2 * blockIdx.x + 1] = sa[0];
  }
}

__global__ void diag_kernel(const double* __restrict__ A, int n, double* w) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) w[i] = A[(int64_t)i * n + i];
}

// u_k = (sum_i UT[k][i] x_i) / floor(w_k - shift) with UT = U^T, one wave
// per k (rows of UT are contiguous)
__global__ __launch_bounds__(256) void eig_proj_kernel(const double* __restrict__ UT, const double* __restrict__ w,
                                                       int n, double shift, double fl, const double* __restrict__ x,
                                                       double* __restrict__ u) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int k = blockIdx.x * 4 + wave;
  if (k >= n) return;  // the whole wave leaves together (no barriers below)
  const double* row = UT + (int64_t)k * n;
  double acc = 0.0;
  for (int i = lane; i < n; i += 64) acc += row[i] * x[i];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if (lane == 0) {
    double d = w[k] - shift;
    if (fabs(d) < fl) d = d < 0.0 ? -fl : fl;
    u[k] = acc / d;
  }
}

// UT = U^T (32 x 32 tiles through LDS)
__global__ void transpose_kernel(const double* __restrict__ U, int n, double* __restrict__ UT) {
  __shared__ double tile[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 256 threads: 32 x 8
  for (int r = ty; r < 32; r += 8) {
    const int i = by + r, j = bx + tx;
    if (i < n && j < n) tile[r][tx] = U[(int64_t)i * n + j];
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int i = bx + r, j = by + tx;
    if (i < n && j < n) UT[(int64_t)i * n + j] = tile[tx][r];
  }
}

// y_i = sum_k U[i][k] u_k, one wave per row
__global__ __launch_bounds__(256) void eig_back_kernel(const double* __restrict__ U, int n,
                                                       const double* __restrict__ u, double* __restrict__ y) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + wave;
  if (i >= n) return;
  const double* row = U + (int64_t)i * n;
  double acc = 0.0;
  for (int k = lane; k < n; k += 64) acc += row[k] * u[k];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if (lane == 0) y[i] = acc;
}

__global__ void column_kernel(const double* __restrict__ U, int n, int k, double* y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = U[(int64_t)i * n + k];
}

__global__ void identity_kernel(double* V, int n) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < (int64_t)n * n) V[idx] = (idx / n == idx % n) ? 1.0 : 0.0;
}

unsigned blocks(int64_t work) { return (unsigned)((work + 255) / 256); }

}  // namespace

void launch_cis_matrix(const double* L, int nj, int o, int v, const double* eps, double* A, hipStream_t s) {
  const int64_t nov = (int64_t)o * v;
  hipLaunchKernelGGL(cis_matrix_kernel, dim3(blocks(nov * nov)), dim3(256), 0, s, L, nj, o, v, eps, A);
  hck(hipGetLastError(), "cis matrix launch");
}

int64_t jacobi_work_doubles(int n) {
  const int m = n + (n & 1);
  return 2 * (int64_t)m + 2 * NORM_BLOCKS + (int64_t)m;  // cs, sn, partial sums, pp / qq (as doubles)
}

int sym_eig_jacobi(double* A, double* V, double* w, int n, double* work, hipStream_t s, double tol, int max_sweeps) {
  if (n <= 0) return 0;
  const int m = n + (n & 1), npair = m / 2;
  double* cs = work;
  double* sn = cs + m / 2 + 1;
  double* part = work + 2 * (int64_t)m;
  int* pp = (int*)(part + 2 * NORM_BLOCKS);
  int* qq = pp + npair;
  hipLaunchKernelGGL(identity_kernel, dim3(blocks((int64_t)n * n)), dim3(256), 0, s, V, n);
  hck(hipGetLastError(), "jacobi identity");
  std::vector<double> h(2 * NORM_BLOCKS);
  auto norms = [&](double& off, double& all) {
    hipLaunchKernelGGL(offdiag_kernel, dim3(NORM_BLOCKS), dim3(256), 0, s, A, n, part);
    hck(hipGetLastError(), "jacobi norm");
    hck(hipMemcpyAsync(h.data(), part, h.size() * sizeof(double), hipMemcpyDeviceToHost, s), "jacobi norm copy");
    hck(hipStreamSynchronize(s), "jacobi norm sync");
    off = all = 0.0;
    for (int b = 0; b < NORM_BLOCKS; ++b) {
      off += h[2 * b];
      all += h[2 * b + 1];
    }
  };
  double off = 0, all = 0;
  norms(off, all);
  int sweep = 0;
  for (; sweep < max_sweeps && off > tol * tol * all && n > 1; ++sweep) {
    for (int r = 0; r < m - 1; ++r) {
      hipLaunchKernelGGL(jacobi_angles_kernel, dim3(blocks(npair)), dim3(256), 0, s, A, n, m, r, cs, sn, pp, qq);
      hipLaunchKernelGGL(jacobi_rows_kernel, dim3(blocks((int64_t)npair * n)), dim3(256), 0, s, A, n, npair, cs, sn,
                         pp, qq);
      hipLaunchKernelGGL(jacobi_cols_kernel, dim3(blocks((int64_t)npair * n)), dim3(256), 0, s, A, V, n, npair, cs,
                         sn, pp, qq);
    }
    hck(hipGetLastError(), "jacobi sweep");
    norms(off, all);
  }
  if (off > tol * tol * all && n > 1) throw std::runtime_error("Jacobi eigensolver did not converge");
  hipLaunchKernelGGL(diag_kernel, dim3(blocks(n)), dim3(256), 0, s, A, n, w);
  hck(hipGetLastError(), "jacobi diag");
  return sweep;
}

void launch_eig_column(const double* U, int n, int k, double* y, hipStream_t s) {
  hipLaunchKernelGGL(column_kernel, dim3(blocks(n)), dim3(256), 0, s, U, n, k, y);
  hck(hipGetLastError(), "eigenvector column");
}

void launch_transpose(const double* U, int n, double* UT, hipStream_t s) {
  dim3 grid((unsigned)((n + 31) / 32), (unsigned)((n + 31) / 32));
  hipLaunchKernelGGL(transpose_kernel, grid, dim3(256), 0, s, U, n, UT);
  hck(hipGetLastError(), "transpose");
}

void launch_eig_shift_solve(const double* U, const double* UT, const double* w, int n, double shift, double fl,
                            const double* x, double* y, double* tmp, hipStream_t s) {
  hipLaunchKernelGGL(eig_proj_kernel, dim3((n + 3) / 4), dim3(256), 0, s, UT, w, n, shift, fl, x, tmp);
  hipLaunchKernelGGL(eig_back_kernel, dim3((n + 3) / 4), dim3(256), 0, s, U, n, tmp, y);
  hck(hipGetLastError(), "eig shift solve");
}

}  // namespace scc
