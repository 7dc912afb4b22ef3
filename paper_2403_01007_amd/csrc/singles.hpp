// Singles-space preconditioner: the closed-shell singlet singles matrix of
// the Hamiltonian, its eigendecomposition on the device and shifted solves
// (singles.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace scc {

// A [nov][nov], A_ai,bj = (eps_a - eps_i) d_ab d_ij + 2 (ai|jb) - (ab|ij)
// with (pq|rs) = sum_J L[J][p][q] L[J][r][s]; L [nj][N][N] MO Cholesky
// vectors and eps [N] on the device; (ai) = a * o + i.
void launch_cis_matrix(const double* L, int nj, int o, int v, const double* eps, double* A, hipStream_t s);

// Device work space (doubles) of sym_eig_jacobi for order n.
int64_t jacobi_work_doubles(int n);

// Symmetric A [n][n] (overwritten: converges to diag(w)) = V diag(w) V^T by
// parallel two-sided Jacobi sweeps (round-robin pair ordering), until the
// off-diagonal Frobenius norm is below tol times the whole norm.  V [n][n]
// (eigenvectors in its columns) and w [n] on the device.  Returns the number
// of sweeps; throws std::runtime_error after max_sweeps.
int sym_eig_jacobi(double* A, double* V, double* w, int n, double* work, hipStream_t s, double tol = 1e-12,
                   int max_sweeps = 40);

// y [n] = column k of U [n][n].
void launch_eig_column(const double* U, int n, int k, double* y, hipStream_t s);

// UT [n][n] = U^T (device).
void launch_transpose(const double* U, int n, double* UT, hipStream_t s);

// y = U diag(1 / d_k) U^T x, d_k = w_k - shift floored to |d_k| >= fl (sign
// kept), with UT = U^T stored; tmp [n] device scratch; y may alias x only
// if tmp does not.
void launch_eig_shift_solve(const double* U, const double* UT, const double* w, int n, double shift, double fl,
                            const double* x, double* y, double* tmp, hipStream_t s);

}  // namespace scc
