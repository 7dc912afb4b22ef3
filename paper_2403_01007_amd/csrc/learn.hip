// Learned initial-guess model on the device: PCA of solution vectors (FP64,
// through the Gram matrix on the FP64 matrix-core GEMM) and a tanh
// perceptron in FP32 with its backward pass and Adam updates.  Every
// reduction runs in a fixed order, so results are deterministic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "scc_learn.h"
#include "exec.hpp"
#include "smalllinalg.hpp"

namespace scc {
namespace {

constexpr int OK = 0, EINVAL_ = -1, EDEVICE_ = -6, ENOMEM_ = -7;

struct HipError : std::runtime_error {
  using std::runtime_error::runtime_error;
};

void hk(hipError_t e, const char* what) {
  if (e != hipSuccess) throw HipError(std::string(what) + ": " + hipGetErrorString(e));
}

unsigned blocks_for(int64_t n) { return (unsigned)std::min<int64_t>((n + 255) / 256, 16384); }

// ---------------------------------------------------------------------------
// FP32 kernels of the perceptron
// ---------------------------------------------------------------------------
// C[M][N] = alpha * op(A) op(B) + beta * C, op(A)[m][k] = tA ? A[k][m] : A[m][k]
// (leading dimensions = row lengths of the stored matrices); 16 x 16 tiles
// staged through LDS, one output element per thread, k in fixed order.
__global__ __launch_bounds__(256) void sgemm_kernel(int M, int N, int K, float alpha, const float* A, int lda, int tA,
                                                   const float* B, int ldb, int tB, float beta, float* C, int ldc) {
  __shared__ float As[16][17];
  __shared__ float Bs[16][17];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int m = blockIdx.y * 16 + ty, n = blockIdx.x * 16 + tx;
  float acc = 0.0f;
  for (int k0 = 0; k0 < K; k0 += 16) {
    {
      const int mm = blockIdx.y * 16 + ty, kk = k0 + tx;
      float a = 0.0f;
      if (mm < M && kk < K) a = tA ? A[(int64_t)kk * lda + mm] : A[(int64_t)mm * lda + kk];
      As[ty][tx] = a;
      const int kb = k0 + ty, nb = blockIdx.x * 16 + tx;
      float b = 0.0f;
      if (kb < K && nb < N) b = tB ? B[(int64_t)nb * ldb + kb] : B[(int64_t)kb * ldb + nb];
      Bs[ty][tx] = b;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) acc += As[ty][kk] * Bs[kk][tx];
    __syncthreads();
  }
  if (m < M && n < N) {
    float v = alpha * acc;
    if (beta != 0.0f) v += beta * C[(int64_t)m * ldc + n];
    C[(int64_t)m * ldc + n] = v;
  }
}

void sgemm(int M, int N, int K, float alpha, const float* A, int lda, bool tA, const float* B, int ldb, bool tB,
           float beta, float* C, int ldc, hipStream_t s) {
  if (M <= 0 || N <= 0) return;
  dim3 grid((N + 15) / 16, (M + 15) / 16);
  hipLaunchKernelGGL(sgemm_kernel, grid, dim3(256), 0, s, M, N, K, alpha, A, lda, tA ? 1 : 0, B, ldb, tB ? 1 : 0,
                     beta, C, ldc);
  hk(hipGetLastError(), "sgemm launch");
}

// Z[b][j] = tanh(Z[b][j] + bias[j]) (act = 1) or Z + bias (act = 0)
__global__ void bias_act_kernel(float* Z, const float* bias, int B, int n, int act) {
  const int64_t total = (int64_t)B * n;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    float z = Z[i] + bias[i % n];
    Z[i] = act ? tanhf(z) : z;
  }
}

// D = D * (1 - H^2)
__global__ void tanh_back_kernel(float* D, const float* H, int64_t total) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x)
    D[i] *= 1.0f - H[i] * H[i];
}

// g[j] = sum_b D[b][j] (b ascending)
__global__ void colsum_kernel(const float* D, int B, int n, float* g) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  float acc = 0.0f;
  for (int b = 0; b < B; ++b) acc += D[(int64_t)b * n + j];
  g[j] = acc;
}

// E = (Y - T) / B in place of Y; loss = sum (Y - T)^2 / (2 B) (one block)
__global__ __launch_bounds__(256) void mse_kernel(float* Y, const float* T, int B, int n, float* loss) {
  __shared__ float sh[256];
  const int64_t total = (int64_t)B * n;
  float acc = 0.0f;
  for (int64_t i = threadIdx.x; i < total; i += 256) {
    const float e = Y[i] - T[i];
    acc += e * e;
    Y[i] = e / (float)B;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0 && loss) *loss = 0.5f * sh[0] / (float)B;
}

__global__ void adam_kernel(float* p, const float* g, float* m, float* v, int64_t n, float lr, float c1, float c2) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float mi = 0.9f * m[i] + 0.1f * g[i];
    const float vi = 0.999f * v[i] + 0.001f * g[i] * g[i];
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
  }
}

// rows of X, T picked by idx into Xb, Tb
__global__ void gather_kernel(const float* X, const float* T, const int* idx, int B, int nin, int nout, int n,
                              float* Xb, float* Tb) {
  const int b = blockIdx.x;
  if (b >= B) return;
  const int r = idx[b];
  if (r < 0 || r >= n) return;  // rejected on the host before launch
  for (int j = threadIdx.x; j < nin; j += blockDim.x) Xb[(int64_t)b * nin + j] = X[(int64_t)r * nin + j];
  for (int j = threadIdx.x; j < nout; j += blockDim.x) Tb[(int64_t)b * nout + j] = T[(int64_t)r * nout + j];
}

struct Mlp {
  int nin, nh, nout;
  int64_t oW1, ob1, oW2, ob2, oW3, ob3, count;
  explicit Mlp(const scc_mlp_dims& d) : nin(d.nin), nh(d.nhidden), nout(d.nout) {
    oW1 = 0;
    ob1 = oW1 + (int64_t)nh * nin;
    oW2 = ob1 + nh;
    ob2 = oW2 + (int64_t)nh * nh;
    oW3 = ob2 + nh;
    ob3 = oW3 + (int64_t)nout * nh;
    count = ob3 + nout;
  }
  // activations h1, h2 [B][nh], output y [B][nout], deltas d1, d2 [B][nh],
  // batch copies xb [B][nin], tb [B][nout]
  int64_t ws_floats(int B) const {
    return 4 * (int64_t)B * nh + 2 * (int64_t)B * nout + (int64_t)B * nin + 64;
  }
};

bool valid(const scc_mlp_dims* d) { return d && d->nin > 0 && d->nhidden > 0 && d->nout > 0; }

// forward of B samples; h1, h2, y in the workspace
void mlp_forward(const Mlp& M, const float* p, int B, const float* X, float* h1, float* h2, float* y, hipStream_t s) {
  sgemm(B, M.nh, M.nin, 1.0f, X, M.nin, false, p + M.oW1, M.nin, true, 0.0f, h1, M.nh, s);
  hipLaunchKernelGGL(bias_act_kernel, dim3(blocks_for((int64_t)B * M.nh)), dim3(256), 0, s, h1, p + M.ob1, B, M.nh, 1);
  sgemm(B, M.nh, M.nh, 1.0f, h1, M.nh, false, p + M.oW2, M.nh, true, 0.0f, h2, M.nh, s);
  hipLaunchKernelGGL(bias_act_kernel, dim3(blocks_for((int64_t)B * M.nh)), dim3(256), 0, s, h2, p + M.ob2, B, M.nh, 1);
  sgemm(B, M.nout, M.nh, 1.0f, h2, M.nh, false, p + M.oW3, M.nh, true, 0.0f, y, M.nout, s);
  hipLaunchKernelGGL(bias_act_kernel, dim3(blocks_for((int64_t)B * M.nout)), dim3(256), 0, s, y, p + M.ob3, B, M.nout,
                     0);
  hk(hipGetLastError(), "mlp forward");
}

// loss and gradient of one batch
void mlp_loss_grad(const Mlp& M, const float* p, int B, const float* X, const float* T, float* loss, float* g,
                   float* ws, hipStream_t s) {
  float* h1 = ws;
  float* h2 = h1 + (int64_t)B * M.nh;
  float* d1 = h2 + (int64_t)B * M.nh;
  float* d2 = d1 + (int64_t)B * M.nh;
  float* y = d2 + (int64_t)B * M.nh;
  mlp_forward(M, p, B, X, h1, h2, y, s);
  hipLaunchKernelGGL(mse_kernel, dim3(1), dim3(256), 0, s, y, T, B, M.nout, loss);  // y <- dY
  // layer 3: gW3 = dY^T h2, gb3 = colsum dY, d2 = (dY W3) * (1 - h2^2)
  sgemm(M.nout, M.nh, B, 1.0f, y, M.nout, true, h2, M.nh, false, 0.0f, g + M.oW3, M.nh, s);
  hipLaunchKernelGGL(colsum_kernel, dim3((M.nout + 255) / 256), dim3(256), 0, s, y, B, M.nout, g + M.ob3);
  sgemm(B, M.nh, M.nout, 1.0f, y, M.nout, false, p + M.oW3, M.nh, false, 0.0f, d2, M.nh, s);
  hipLaunchKernelGGL(tanh_back_kernel, dim3(blocks_for((int64_t)B * M.nh)), dim3(256), 0, s, d2, h2, (int64_t)B * M.nh);
  // layer 2
  sgemm(M.nh, M.nh, B, 1.0f, d2, M.nh, true, h1, M.nh, false, 0.0f, g + M.oW2, M.nh, s);
  hipLaunchKernelGGL(colsum_kernel, dim3((M.nh + 255) / 256), dim3(256), 0, s, d2, B, M.nh, g + M.ob2);
  sgemm(B, M.nh, M.nh, 1.0f, d2, M.nh, false, p + M.oW2, M.nh, false, 0.0f, d1, M.nh, s);
  hipLaunchKernelGGL(tanh_back_kernel, dim3(blocks_for((int64_t)B * M.nh)), dim3(256), 0, s, d1, h1, (int64_t)B * M.nh);
  // layer 1
  sgemm(M.nh, M.nin, B, 1.0f, d1, M.nh, true, X, M.nin, false, 0.0f, g + M.oW1, M.nin, s);
  hipLaunchKernelGGL(colsum_kernel, dim3((M.nh + 255) / 256), dim3(256), 0, s, d1, B, M.nh, g + M.ob1);
  hk(hipGetLastError(), "mlp backward");
}

template <class F>
int guard(F&& f) {
  try {
    return f();
  } catch (const HipError&) {
    return EDEVICE_;
  } catch (const std::invalid_argument&) {
    return EINVAL_;
  } catch (const std::exception&) {
    return EDEVICE_;
  }
}

// ---------------------------------------------------------------------------
// Forward pass without a caller workspace: the two hidden-layer activation
// buffers live in one file-scope device array (4 MiB on every device the
// library runs on, held until the process ends).  Host code never passes the
// array's name to a kernel: its device address is looked up once per device.
// ---------------------------------------------------------------------------
constexpr int64_t NOALLOC_FLOATS = (int64_t)1 << 20;
constexpr int MAX_DEVICES = 64;
std::mutex noalloc_mu;
float* noalloc_ptr[MAX_DEVICES] = {};

// ---------------------------------------------------------------------------
// PCA kernels
// ---------------------------------------------------------------------------
// mean[j] = (1/n) sum_i X[i][j]; Xc = X - mean
__global__ void center_kernel(const double* X, int n, int64_t d, double* mean, double* Xc) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < d; j += (int64_t)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int i = 0; i < n; ++i) acc += X[(int64_t)i * d + j];
    const double m = acc / n;
    mean[j] = m;
    for (int i = 0; i < n; ++i) Xc[(int64_t)i * d + j] = X[(int64_t)i * d + j] - m;
  }
}

// row r of U: index of the largest |U[r][j]| (smallest j on ties), then the
// row is negated if that element is negative
__global__ __launch_bounds__(256) void sign_fix_kernel(double* U, int64_t d) {
  __shared__ double sv[256];
  __shared__ int64_t si[256];
  double* row = U + (int64_t)blockIdx.x * d;
  double best = -1.0;
  int64_t bi = 0;
  for (int64_t j = threadIdx.x; j < d; j += 256) {
    const double a = fabs(row[j]);
    if (a > best) {
      best = a;
      bi = j;
    }
  }
  sv[threadIdx.x] = best;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      const double a = sv[threadIdx.x + w];
      const int64_t ai = si[threadIdx.x + w];
      if (a > sv[threadIdx.x] || (a == sv[threadIdx.x] && ai < si[threadIdx.x])) {
        sv[threadIdx.x] = a;
        si[threadIdx.x] = ai;
      }
    }
    __syncthreads();
  }
  const bool flip = row[si[0]] < 0.0;
  __syncthreads();
  if (flip)
    for (int64_t j = threadIdx.x; j < d; j += 256) row[j] = -row[j];
}

// out[r][j] = mean[j] + sum_i coef[r][i] basis[i][j]
__global__ void expand_kernel(int m, int64_t d, int k, const double* mean, const double* basis, const double* coef,
                              double* out) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < d; j += (int64_t)gridDim.x * blockDim.x)
    for (int r = 0; r < m; ++r) {
      double acc = mean[j];
      for (int i = 0; i < k; ++i) acc += coef[(int64_t)r * k + i] * basis[(int64_t)i * d + j];
      out[(int64_t)r * d + j] = acc;
    }
}

// FP64 GEMM on the matrix cores (the contraction kernel of the executor),
// with split-K partial sums when the output is small and K long
void dgemm(int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t sAm, int64_t sAk, const double* B,
           int64_t sBk, int64_t sBn, double* C, int64_t ldc, double* partials, int64_t partial_cap, hipStream_t s) {
  GemmArgs g{};
  g.M = M;
  g.N = N;
  g.K = K;
  g.batch = 1;
  g.alpha = alpha;
  g.beta = 0.0;
  g.A = A;
  g.sAm = sAm;
  g.sAk = sAk;
  g.B = B;
  g.sBk = sBk;
  g.sBn = sBn;
  g.C = C;
  g.sCm = ldc;
  g.sCn = 1;
  const int64_t tiles = ((M + 63) / 64) * ((N + 63) / 64);
  int64_t sp = std::min<int64_t>(std::max<int64_t>(1, 1024 / std::max<int64_t>(tiles, 1)), K / 256);
  sp = std::min<int64_t>(sp, partial_cap / std::max<int64_t>(M * N, 1));
  if (sp > 1) {
    int64_t kc = (K + sp - 1) / sp;
    kc = (kc + 15) / 16 * 16;
    sp = (K + kc - 1) / kc;
    if (sp > 1) {
      g.splits = sp;
      g.kchunk = kc;
      g.P = partials;
    }
  }
  launch_gemm(g, s);
}

int64_t pca_partial_cap(int n, int k) { return std::max<int64_t>((int64_t)n * n, (int64_t)n * k) * 64; }

}  // namespace
}  // namespace scc

__device__ __align__(256) float scratch[scc::NOALLOC_FLOATS];

namespace scc {
namespace {
// device address of `scratch` on device dev (current), looked up once
float* noalloc_scratch(int dev) {
  std::lock_guard<std::mutex> lk(noalloc_mu);
  if (!noalloc_ptr[dev]) {
    void* p = nullptr;
    hk(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (!p) throw HipError("hipGetSymbolAddress(scratch) returned null");
    noalloc_ptr[dev] = (float*)p;
  }
  return noalloc_ptr[dev];
}
}  // namespace
}  // namespace scc

using namespace scc;

extern "C" {

int scc_mlp_param_count(const scc_mlp_dims* d, long long* count) {
  if (!valid(d) || !count) return EINVAL_;
  *count = (long long)Mlp(*d).count;
  return OK;
}

int scc_mlp_workspace_bytes(const scc_mlp_dims* d, int max_batch, size_t* bytes) {
  if (!valid(d) || max_batch <= 0 || !bytes) return EINVAL_;
  *bytes = (size_t)Mlp(*d).ws_floats(max_batch) * sizeof(float) + 256;
  return OK;
}

int scc_mlp_forward(const scc_mlp_dims* d, const float* params, int n, const float* X, float* Y, void* workspace,
                    size_t bytes, void* hip_stream) {
  if (!valid(d) || !params || n <= 0 || !X || !Y || !workspace) return EINVAL_;
  Mlp M(*d);
  if (bytes < (size_t)M.ws_floats(n) * sizeof(float)) return ENOMEM_;
  return guard([&]() -> int {
    hipStream_t s = (hipStream_t)hip_stream;
    float* h1 = (float*)workspace;
    float* h2 = h1 + (int64_t)n * M.nh;
    mlp_forward(M, params, n, X, h1, h2, Y, s);
    hk(hipStreamSynchronize(s), "sync");
    return OK;
  });
}

int scc_mlp_forward_noalloc(const scc_mlp_dims* d, const float* params, int n, const float* X, float* Y,
                            void* hip_stream) {
  if (!valid(d) || !params || n <= 0 || !X || !Y) return EINVAL_;
  Mlp M(*d);
  if (2 * (int64_t)n * M.nh > NOALLOC_FLOATS) return ENOMEM_;
  return guard([&]() -> int {
    hipStream_t s = (hipStream_t)hip_stream;
    int dev = 0;
    hk(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= MAX_DEVICES) throw std::invalid_argument("device index");
    float* h1 = noalloc_scratch(dev);
    float* h2 = h1 + (int64_t)n * M.nh;
    mlp_forward(M, params, n, X, h1, h2, Y, s);
    hk(hipStreamSynchronize(s), "sync");
    return OK;
  });
}

int scc_mlp_loss_grad(const scc_mlp_dims* d, const float* params, int n, const float* X, const float* T, float* loss,
                      float* grad, void* workspace, size_t bytes, void* hip_stream) {
  if (!valid(d) || !params || n <= 0 || !X || !T || !loss || !grad || !workspace) return EINVAL_;
  Mlp M(*d);
  if (bytes < (size_t)M.ws_floats(n) * sizeof(float)) return ENOMEM_;
  return guard([&]() -> int {
    hipStream_t s = (hipStream_t)hip_stream;
    mlp_loss_grad(M, params, n, X, T, loss, grad, (float*)workspace, s);
    hk(hipStreamSynchronize(s), "sync");
    return OK;
  });
}

int scc_mlp_train(const scc_mlp_dims* d, float* params, float* adam_m, float* adam_v, int n, const float* X,
                  const float* T, int nsteps, int batch, const int* order, float lr, int step0, float* losses,
                  void* workspace, size_t bytes, void* hip_stream) {
  if (!valid(d) || !params || !adam_m || !adam_v || n <= 0 || !X || !T || nsteps < 0 || batch <= 0 || !order ||
      !workspace || step0 < 0 || !(lr > 0))
    return EINVAL_;
  Mlp M(*d);
  // workspace: loss/grad scratch for a batch, then the batch copies and the gradient
  const int64_t need = M.ws_floats(batch) + (int64_t)batch * (M.nin + M.nout) + M.count + 64;
  if (bytes < (size_t)need * sizeof(float)) return ENOMEM_;
  return guard([&]() -> int {
    hipStream_t s = (hipStream_t)hip_stream;
    // indices are checked on the host: every one must address a sample
    std::vector<int> ho((size_t)nsteps * batch);
    if (!ho.empty()) {
      hk(hipMemcpyAsync(ho.data(), order, ho.size() * sizeof(int), hipMemcpyDeviceToHost, s), "order d2h");
      hk(hipStreamSynchronize(s), "sync");
    }
    for (int i : ho)
      if (i < 0 || i >= n) throw std::invalid_argument("sample index out of range");
    float* ws = (float*)workspace;
    float* xb = ws + M.ws_floats(batch);
    float* tb = xb + (int64_t)batch * M.nin;
    float* g = tb + (int64_t)batch * M.nout;
    for (int st = 0; st < nsteps; ++st) {
      hipLaunchKernelGGL(gather_kernel, dim3(batch), dim3(64), 0, s, X, T, order + (int64_t)st * batch, batch, M.nin,
                         M.nout, n, xb, tb);
      mlp_loss_grad(M, params, batch, xb, tb, losses ? losses + st : nullptr, g, ws, s);
      const int step = step0 + st + 1;
      const float c1 = 1.0f - powf(0.9f, (float)step), c2 = 1.0f - powf(0.999f, (float)step);
      hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(M.count)), dim3(256), 0, s, params, g, adam_m, adam_v, M.count,
                         lr, c1, c2);
      hk(hipGetLastError(), "adam");
    }
    hk(hipStreamSynchronize(s), "sync");
    return OK;
  });
}

int scc_pca_workspace_bytes(int n, long long d, int k, size_t* bytes) {
  if (n <= 0 || d <= 0 || k <= 0 || k > n || !bytes) return EINVAL_;
  // centred data, Gram matrix, eigenvectors, split-K partial sums
  *bytes = (size_t)((int64_t)n * d + (int64_t)n * n + (int64_t)n * k + pca_partial_cap(n, k) + 64) * sizeof(double) + 256;
  return OK;
}

int scc_pca_fit(int n, long long d, int k, const double* X, double* mean, double* basis, double* coef,
                double* eigenvalues, void* workspace, size_t bytes, void* hip_stream) {
  size_t need = 0;
  if (scc_pca_workspace_bytes(n, d, k, &need) != OK || !X || !mean || !basis || !coef || !workspace) return EINVAL_;
  if (bytes < need) return ENOMEM_;
  return guard([&]() -> int {
    hipStream_t s = (hipStream_t)hip_stream;
    uintptr_t base = ((uintptr_t)workspace + 255) & ~(uintptr_t)255;
    double* Xc = (double*)base;
    double* G = Xc + (int64_t)n * d;
    double* Vk = G + (int64_t)n * n;
    double* P = Vk + (int64_t)n * k;
    const int64_t pcap = pca_partial_cap(n, k);
    hipLaunchKernelGGL(center_kernel, dim3(blocks_for(d)), dim3(256), 0, s, X, n, (int64_t)d, mean, Xc);
    hk(hipGetLastError(), "center");
    // Gram matrix G = Xc Xc^T
    dgemm(n, n, d, 1.0, Xc, d, 1, Xc, 1, d, G, n, P, pcap, s);
    std::vector<double> Gh((size_t)n * n), w, V;
    hk(hipMemcpyAsync(Gh.data(), G, Gh.size() * sizeof(double), hipMemcpyDeviceToHost, s), "gram d2h");
    hk(hipStreamSynchronize(s), "sync");
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < i; ++j) Gh[(size_t)i * n + j] = Gh[(size_t)j * n + i] = 0.5 * (Gh[(size_t)i * n + j] + Gh[(size_t)j * n + i]);
    eig_sym(n, Gh, w, V);
    // leading k (descending): Vk[i][c] = V[i][n-1-c] / sqrt(w), so that
    // U = Vk^T Xc has orthonormal rows
    std::vector<double> vk((size_t)n * k);
    for (int c = 0; c < k; ++c) {
      const double lam = w[n - 1 - c];
      if (!(lam > 0)) throw std::invalid_argument("PCA rank below k");
      if (eigenvalues) eigenvalues[c] = lam;
      for (int i = 0; i < n; ++i) vk[(size_t)i * k + c] = V[(size_t)i * n + (n - 1 - c)] / std::sqrt(lam);
    }
    hk(hipMemcpyAsync(Vk, vk.data(), vk.size() * sizeof(double), hipMemcpyHostToDevice, s), "vk h2d");
    // U [k][d] = Vk^T Xc
    dgemm(k, d, n, 1.0, Vk, 1, k, Xc, d, 1, basis, d, P, pcap, s);
    hipLaunchKernelGGL(sign_fix_kernel, dim3(k), dim3(256), 0, s, basis, (int64_t)d);
    hk(hipGetLastError(), "sign fix");
    // C [n][k] = Xc U^T
    dgemm(n, k, d, 1.0, Xc, d, 1, basis, 1, d, coef, k, P, pcap, s);
    hk(hipStreamSynchronize(s), "sync");
    return OK;
  });
}

int scc_pca_expand(int m, long long d, int k, const double* mean, const double* basis, const double* coef, double* out,
                   void* hip_stream) {
  if (m <= 0 || d <= 0 || k <= 0 || !mean || !basis || !coef || !out) return EINVAL_;
  return guard([&]() -> int {
    hipStream_t s = (hipStream_t)hip_stream;
    hipLaunchKernelGGL(expand_kernel, dim3(blocks_for(d)), dim3(256), 0, s, m, (int64_t)d, k, mean, basis, coef, out);
    hk(hipGetLastError(), "expand");
    hk(hipStreamSynchronize(s), "sync");
    return OK;
  });
}

}  // extern "C"
