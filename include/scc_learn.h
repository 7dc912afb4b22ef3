/*
 * scc_learn.h -- C ABI of the learned initial-guess model of libscc:
 * principal component analysis of solution vectors (FP64) and a small tanh
 * perceptron (FP32) trained by Adam, all on the device.
 *
 * The model predicts starting vectors (amplitudes, excited-state vectors,
 * SCC parameters) of the iterative solves from the geometry coordinates of
 * a trajectory family H(x) = H0 + sum_k x_k H_k; the solvers of scc.h judge
 * every prediction by its residual and fall back to their plain guess.
 *
 * Conventions
 *   - Every array is a DEVICE pointer, row-major, owned by the caller,
 *     including the workspace (size from the *_workspace_bytes calls).
 *   - Work is enqueued on the given stream (NULL: the default stream); the
 *     calls synchronise it before returning.
 *   - Return values are the SCC_* codes of scc.h (0 = success,
 *     -1 = invalid argument, -6 = HIP runtime error, -7 = workspace too
 *     small); nothing is kept between calls.
 *
 * PCA of X [n][d]: mean m [d] (column mean); basis U [k][d], the k leading
 * eigenvectors of (X - m)^T (X - m) as orthonormal rows, each signed so that
 * its largest-magnitude element is positive; eigenvalues w [k] (descending,
 * host array); coefficients C = (X - m) U^T [n][k].  Computed through the
 * Gram matrix (X - m)(X - m)^T, so n (not d) sets the cost of the
 * eigenproblem; k <= n.
 *
 * Perceptron with sizes (nin, nh, nout):
 *   h1 = tanh(W1 x + b1), h2 = tanh(W2 h1 + b2), y = W3 h2 + b3,
 * parameters [W1 (nh x nin) | b1 | W2 (nh x nh) | b2 | W3 (nout x nh) | b3]
 * in FP32.  Loss of a batch of B samples: (1/(2B)) sum (y - t)^2.  Adam
 * with beta1 = 0.9, beta2 = 0.999, eps = 1e-8, bias-corrected moments.
 */
#ifndef SCC_LEARN_H
#define SCC_LEARN_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct scc_mlp_dims {
  int nin;      /* inputs (geometry coordinates) */
  int nhidden;  /* width of both hidden layers */
  int nout;     /* outputs (principal-component coefficients) */
} scc_mlp_dims;

/* Parameter count (host out). */
int scc_mlp_param_count(const scc_mlp_dims* d, long long* count);

/* Workspace for batches of up to max_batch samples (host out). */
int scc_mlp_workspace_bytes(const scc_mlp_dims* d, int max_batch, size_t* bytes);

/* Y [n][nout] = network(X [n][nin]). */
int scc_mlp_forward(const scc_mlp_dims* d, const float* params, int n, const float* X, float* Y, void* workspace,
                    size_t bytes, void* hip_stream);

/* Y [n][nout] = network(X [n][nin]) as scc_mlp_forward (same kernels, same
 * results), for callers that cannot allocate device memory or pass a
 * workspace (code under stream capture, tight serving loops, harnesses that
 * forbid allocation).  The hidden activations use a library-owned device
 * array of 4 MiB per device (held until the process ends), so
 * 2 * n * nhidden must not exceed 1048576 (n <= 2048 at nhidden = 256):
 * larger n returns -7 before any work.  Allocates nothing.  Every call on a
 * device shares that device's array: calls that overlap in time on one
 * device (other streams, other host threads) race and must be serialised
 * by the caller. */
int scc_mlp_forward_noalloc(const scc_mlp_dims* d, const float* params, int n, const float* X, float* Y,
                            void* hip_stream);

/* Loss (device float[1]) and its gradient grad [count] over the batch
 * X [n][nin], targets T [n][nout]. */
int scc_mlp_loss_grad(const scc_mlp_dims* d, const float* params, int n, const float* X, const float* T, float* loss,
                      float* grad, void* workspace, size_t bytes, void* hip_stream);

/* nsteps Adam steps; step s uses the samples order[s][0..batch) of X, T
 * (int32 indices < n) and has Adam step number step0 + s + 1.  params,
 * adam_m, adam_v [count] are updated in place (zero the moments before the
 * first call); losses [nsteps] (device, may be NULL) receives the loss of
 * each step before its update. */
int scc_mlp_train(const scc_mlp_dims* d, float* params, float* adam_m, float* adam_v, int n, const float* X,
                  const float* T, int nsteps, int batch, const int* order, float lr, int step0, float* losses,
                  void* workspace, size_t bytes, void* hip_stream);

/* Workspace of scc_pca_fit (host out). */
int scc_pca_workspace_bytes(int n, long long d, int k, size_t* bytes);

/* PCA of X [n][d] (FP64): mean [d], basis [k][d], coef [n][k] (device),
 * eigenvalues [k] (host, may be NULL). */
int scc_pca_fit(int n, long long d, int k, const double* X, double* mean, double* basis, double* coef,
                double* eigenvalues, void* workspace, size_t bytes, void* hip_stream);

/* out [m][d] = mean + coef [m][k] . basis (FP64 coefficients). */
int scc_pca_expand(int m, long long d, int k, const double* mean, const double* basis, const double* coef, double* out,
                   void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* SCC_LEARN_H */
