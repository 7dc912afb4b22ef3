/*
 * scc.h -- C ABI of libscc: SCCSD(E) energies, nuclear gradients and
 * nonadiabatic derivative couplings on one AMD Instinct MI355X (gfx950).
 *
 * Method: similarity constrained coupled cluster singles and doubles with the
 * natural projection, gradients and couplings from the Lagrangian (Z-vector)
 * method of Kjonstad, Angelico and Koch, "Coupled cluster theory for
 * nonadiabatic dynamics: nuclear gradients and nonadiabatic couplings in
 * similarity constrained coupled cluster theory" (arXiv:2403.01007).
 *
 * Conventions shared by every call
 *   - Closed-shell restricted reference, o occupied and v virtual spatial
 *     orbitals, N = o + v; occupied orbitals first.
 *   - H = sum h_pq E_pq + 1/2 sum g_pqrs (E_pq E_rs - d_qr E_ps),
 *     g_pqrs = sum_J L^J_pq L^J_rs (Cholesky-factored two-electron integrals).
 *   - Amplitude layouts (row-major FP64): t1[a][i] (v x o) and
 *     t2[a][i][b][j] (v x o x v x o), symmetric under (ai) <-> (bj), with
 *     T2 = 1/2 sum_aibj t_aibj E_ai E_bj.  An excited-state vector is
 *     [R0 | R1 (v*o) | R2 (v*o*v*o)].  Left vectors pair with right vectors
 *     through the plain dot product over this full layout.
 *   - Units: Hartree; coordinates are dimensionless.
 *
 * Memory and streams
 *   - Every array argument is a DEVICE pointer (HIP global memory) unless a
 *     comment says "host".  The caller owns all buffers, including the
 *     workspace; the library never allocates device memory and never keeps a
 *     caller pointer after a call returns (the Hamiltonian is copied into the
 *     workspace).
 *   - Every call orders its work after the work already enqueued on the
 *     stream given to scc_create, runs it on a stream of the context's own
 *     (created with default priority) and is blocking: it synchronises that
 *     stream before returning, because the solvers read residual norms back
 *     to the host.  Outputs are complete when a call returns.
 *
 * Errors: every int-returning call returns one of the SCC_* codes below and
 * never throws.  On error, outputs other than scc_info are unspecified and
 * scc_last_error() describes the failure.
 */
#ifndef SCC_H
#define SCC_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  SCC_OK = 0,
  SCC_EINVAL = -1,     /* bad dimensions, NULL pointer or option */
  SCC_ESTATE = -2,     /* call made out of order */
  SCC_ENOCONV = -3,    /* iteration limit reached */
  SCC_ECOMPLEX = -4,   /* a converged excited-state energy is complex */
  SCC_ESINGULAR = -5,  /* singular linear system (e.g. omega_m ~ 0) */
  SCC_EDEVICE = -6,    /* HIP runtime error */
  SCC_ENOMEM = -7      /* workspace smaller than scc_workspace_bytes */
};

typedef struct scc_dims {
  int nocc;     /* o */
  int nvirt;    /* v */
  int nchol;    /* Cholesky rank N_J */
  int nstates;  /* excited states in the constrained set K (>= 1) */
} scc_dims;

typedef struct scc_options {
  double tol_residual;   /* max-norm of CC / EOM / multiplier residuals (e.g. 1e-10) */
  double tol_overlap;    /* |O_kl| threshold of the SCC constraint (e.g. 1e-11) */
  int max_iter;          /* iteration limit of each solver */
  int scc;               /* 1: SCCSD(E); 0: plain CCSD / EOM-CCSD */
  int verbose;           /* 1: per-iteration log on stderr */
  int precision;         /* 0: FP64 throughout.  1: in the ground and
                            excited-state solves the dense contractions
                            (every GEMM with M, N, K >= 64: ladder, ring,
                            hole-hole, Fock-dressed) take FP32 products with
                            FP32 accumulation on the matrix cores until the
                            solve reaches max(tol_residual, 1e-6); it is then
                            refined in FP64 from that point.  Residual norms,
                            DIIS, subspace eigenproblems, orthogonalisation
                            and the multiplier equations stay in FP64. */
  int eager;             /* 0: every device program (the residual, the
                            transformations, the Lagrangian products...) is
                            captured once as a HIP graph and replayed.
                            1: kernels are launched one by one.  Results are
                            identical. */
} scc_options;

typedef struct scc_info {
  int iterations;        /* solver iterations of the call (ground-state steps plus
                            Davidson steps, or Krylov steps) */
  int converged;         /* 1 on success */
  int fallback_used;     /* 1 if a supplied guess was rejected */
  double residual;       /* final residual norm */
  double seconds;        /* wall time of the call */
  double flops_mfma;     /* contraction flops executed by the call */
  int precision;         /* 0: every contraction of the call took FP64
                            products; 1: part of the call ran with
                            reduced-precision products (options.precision =
                            1) before its FP64 refinement */
} scc_info;

typedef struct scc_ctx scc_ctx;

/* Workspace size (bytes) for the given dimensions.  Host pointers; pure
 * host computation.  Returns SCC_EINVAL for bad dimensions. */
int scc_workspace_bytes(const scc_dims* dims, const scc_options* opts, size_t* bytes);

/* Create a context.  workspace: device buffer of >= scc_workspace_bytes
 * bytes (256-byte aligned); hip_stream: hipStream_t (NULL = default stream).
 * Returns SCC_ENOMEM if the workspace is too small. */
int scc_create(const scc_dims* dims, const scc_options* opts, void* workspace, size_t bytes,
               void* hip_stream, scc_ctx** ctx);
void scc_destroy(scc_ctx* ctx);
/* Message of the last failure of this context (host string, owned by ctx). */
const char* scc_last_error(const scc_ctx* ctx);

/* Hamiltonian of the current geometry (Theory, coupled cluster section: the
 * electronic Hamiltonian in second quantization, one-electron integrals h_pq
 * with the singlet excitation operators E_pq and two-electron integrals
 * g_pqrs with e_pqrs, plus the nuclear repulsion e_nuc; the same H enters the
 * transition-density form of <L|Hbar^(1)|R> in the gradient section) in its
 * canonical restricted Hartree-Fock molecular-orbital basis (orbital
 * energies ascending within the occupied and the virtual blocks):
 *   h    [N][N]         one-electron integrals,
 *   chol [N_J][N][N]    Cholesky vectors, symmetric in the last two indices.
 * Copies into the workspace; invalidates every cached solution and resets
 * the amplitudes (t = 0, so the first ground-state step is MP2). Returns
 * SCC_EINVAL if max |F_ai| > 1e-6 (not a Hartree-Fock basis). */
int scc_set_hamiltonian(scc_ctx* ctx, const double* h, const double* chol, double e_nuc);

/* Hamiltonian of the current geometry in a fixed orthonormal basis (for
 * example the orbitals of a reference geometry): h [N][N], chol [N_J][N][N]
 * as in scc_set_hamiltonian but in that basis.  Solves the closed-shell RHF
 * equations on the device (Fock builds from the Cholesky vectors, Roothaan
 * iterations until max |F D - D F| < min(1e-12, 1e-2 tol_residual)),
 * transforms the integrals to the canonical MO basis (Theory, orbitals of
 * the current geometry; eq. H-bar-with-kappa at kappa = 0) and then acts as
 * scc_set_hamiltonian.  orbitals_guess: NULL (start from the basis itself)
 * or [N][N] starting orbitals (columns), e.g. those of the previous
 * geometry; each converged orbital is signed to overlap its starting
 * orbital positively.  orbitals: NULL or [N][N] converged orbitals out.
 * After this call, scc_gradient / scc_nac take their derivative integrals
 * in the same fixed basis and scc_densities returns densities in it.
 * info (host, may be NULL): RHF iterations and final commutator norm.
 * Returns SCC_ENOCONV if the RHF iterations do not converge in 500 steps. */
int scc_set_hamiltonian_fixed_basis(scc_ctx* ctx, const double* h, const double* chol, double e_nuc,
                                    const double* orbitals_guess, double* orbitals, scc_info* info);

/* Ground state Omega(t) = 0 of CCSD (zeta = 0) (coupled cluster section,
 * eq. for Omega_mu).  guess_t: NULL or [t1 | t2]; a guess is used only if
 * its residual norm is below that of the plain start (the MP2 amplitudes),
 * else info->fallback_used = 1.  e0: device double[1].  The converged
 * amplitudes are the starting point of a following scc_excited.
 * SCC_ENOCONV at the iteration limit, or at once when the residual norm is
 * not finite or has grown 10^4 times above the best one reached. */
int scc_ground(scc_ctx* ctx, const double* guess_t, double* e0, scc_info* info);

/* Excited states of the constrained set: EOM right/left eigenvectors with the
 * SCC orthogonality conditions O_kl = <psi_k|P|psi_l> = 0 imposed through
 * zeta_kl X3^kl, ground and excited states solved simultaneously (SCC
 * section; natural projection).  Normalisation: O_kk = 1 and calL_k.calR_k =
 * 1; phase: the largest-magnitude R1 element of each converged right vector
 * is positive, whatever the start (zeta_kl changes sign with a flipped state,
 * so zeta_kl X3^kl does not); order: ascending energy.
 * energies: device double[nstates] (total energies);
 * zeta: device double[nstates*(nstates-1)/2] (pairs k<l, row-major).
 * guess: NULL (plain start: CCSD states at zeta = 0, Davidson started from
 * the lowest eigenvectors of the singles block of calHbar at t = 0) or
 * [nstates][1 + nov + nov^2] right vectors followed
 * by [npairs] zeta values; the solve then starts there (amplitudes from the
 * preceding scc_ground or scc_excited; the SCC Jacobian dO/dzeta of the
 * context's previous solve, if any, seeds the zeta updates) and falls back
 * to the plain start, with info->fallback_used = 1, if it does not
 * converge. */
int scc_excited(scc_ctx* ctx, int nstates, const double* guess, double* energies, double* zeta, scc_info* info);

/* Lagrange multipliers of the gradient of state n (kind = 0, m ignored) or
 * of the coupling d_mn (kind = 1): the stationarity conditions of the
 * gradient / coupling Lagrangians (eqs. Lagrangian_gradient,
 * Lagrangian_coupling) solved for the amplitude, excited-state and
 * orthogonality multipliers first, then the orbital multipliers.
 * guess: NULL or device double[scc_multiplier_length] starting multipliers,
 * used only if the residual b - J^T x0 is below that of the zero start (else
 * info->fallback_used = 1).  multipliers: NULL or device
 * double[scc_multiplier_length], receives the converged multipliers (layout
 * at scc_multiplier_length). */
int scc_multipliers(scc_ctx* ctx, int kind, int m, int n, const double* guess, double* multipliers,
                    scc_info* info);

/* Effective densities of one target: the gradient of state n (kind = 0, m
 * ignored) or the coupling d_mn (kind = 1).  They are the one- and
 * two-electron densities that the gradient and coupling expressions
 * (eqs. gradient_expression, coupling_expression) contract with the
 * derivative Hamiltonian: the transition densities d_pq, d_pqrs of the
 * effective bras K_k (eqs. K-gradients, K-couplings) with the right states,
 * plus those of L0-bar^k with calR_k and of zeta-bar with HF, plus the orbital
 * multipliers kappa-bar, which contract with F_ai^(1).  With Cholesky
 * integrals the two-electron part is returned factorised:
 *   d1 [N][N]          = dL/dh_pq,
 *   z3 [N_J][N][N]     = dL/dL^J_pq  (= 2 sum_rs d_pqrs L^J_rs, symmetrised),
 *   kappa_bar [v][o]   orbital multipliers,
 * in the MO basis, or the fixed basis after scc_set_hamiltonian_fixed_basis.
 * Any output may be NULL.  Solves the target's multipliers first unless they
 * are those of the last scc_multipliers / scc_gradient / scc_nac call.
 * SCC_EINVAL for a bad target; SCC_ESTATE before scc_excited. */
int scc_densities(scc_ctx* ctx, int kind, int m, int n, double* d1, double* z3, double* kappa_bar);

/* Gradient g_n (eq. gradient_expression) along ncoord coordinates whose
 * derivative integrals, in the same MO basis, are dh [ncoord][N][N] and
 * dchol [ncoord][N_J][N][N]: g[k] = <dh_k, d1> + <dchol_k, z3>.
 * grad: device double[ncoord]. */
int scc_gradient(scc_ctx* ctx, int n, int ncoord, const double* dh, const double* dchol, double* grad,
                 scc_info* info);

/* Derivative coupling d_mn = <psi_m| d psi_n / dx> (derivative on the ket;
 * eq. coupling_expression with a fixed orthonormal basis, so O^(1)_mn = 0). */
int scc_nac(scc_ctx* ctx, int m, int n, int ncoord, const double* dh, const double* dchol, double* nac,
            scc_info* info);

/* Gradients of several states and couplings of several pairs in one call
 * (same quantities as scc_gradient / scc_nac): the multiplier equations of
 * up to nstates + npairs targets are solved in lockstep, so that one pass of
 * the Lagrangian products (the transposed Jacobian of the constraints)
 * serves all of them; each target keeps its own Krylov recurrence.
 * states: host int[ngrad]; pairs: host int[2 * npair] as (m, n);
 * grads: device double[ngrad][ncoord]; nacs: device double[npair][ncoord].
 * Targets are ordered gradients first, then couplings.
 * guess: NULL or device double[ngrad + npair][scc_multiplier_length]
 * starting multipliers (e.g. predicted by the learned model); each is used
 * only if its residual is below that of the zero start, else it is dropped
 * and info->fallback_used = 1.  multipliers: NULL or device
 * double[ngrad + npair][scc_multiplier_length], receives the converged
 * multipliers.  The multiplier equations are solved in FP64 in every
 * precision mode. */
int scc_gradients_and_couplings(scc_ctx* ctx, int ngrad, const int* states, int npair, const int* pairs, int ncoord,
                                const double* dh, const double* dchol, const double* guess, double* multipliers,
                                double* grads, double* nacs, scc_info* info);

/* Length of one target's multiplier vector (host out).  Layout, row-major
 * FP64, doubles blocks in the full symmetric [a][i][b][j] layout:
 *   [ zeta-bar: singles (v*o) | doubles (v*o*v*o)       multipliers of Omega
 *   | for each state k: L0-bar^k (1) | L-bar^k singles | L-bar^k doubles
 *   |                   E-bar_k (1)                     multipliers of the
 *                                                        eigenvalue equations
 *                                                        and normalisation
 *   | gamma-bar_kl for pairs k < l (row-major) ]        orthogonality
 * (eqs. Lagrangian_gradient, Lagrangian_coupling); zero in the gamma-bar
 * slots when the SCC constraint is inactive. */
int scc_multiplier_length(const scc_dims* dims, long long* n);

/* Export solution fields to device buffers:
 *   SCC_FIELD_T      [t1 | t2]
 *   SCC_FIELD_R      right vector k  [R0 | R1 | R2]
 *   SCC_FIELD_L      left vector k   [L0 | L1 | L2]
 *   SCC_FIELD_E0     ground-state energy (1)
 *   SCC_FIELD_OMEGA  residual [Omega1 | Omega2] at the current amplitudes */
enum { SCC_FIELD_T = 0, SCC_FIELD_R = 1, SCC_FIELD_L = 2, SCC_FIELD_E0 = 3, SCC_FIELD_OMEGA = 4 };
int scc_get(scc_ctx* ctx, int field, int k, double* out);

/* Profiling of the MFMA contraction kernels: enable = 1 starts timing every
 * GEMM launch with HIP events on the context's stream (0 stops and clears
 * nothing).  kernel selects the totals returned:
 *   SCC_GEMM_F64      gemm_f64_kernel (FP64; each operand index group one
 *                     run of dimensions)
 *   SCC_GEMM_F64_TWO  gemm_f64_two_kernel (FP64; some group spans two runs)
 *   SCC_GEMM_F64_MULTI  gemm_f64_multi_kernel (FP64; several products
 *                     summed into one output in one pass)
 *   SCC_GEMM_F32, SCC_GEMM_F32_TWO, SCC_GEMM_F32_MULTI  the FP32-product
 *                     variants (precision 1)
 * On return (host pointers, any may be NULL): accumulated kernel
 * milliseconds, algorithmic flops (2 M N K per launch), launches, and
 * algorithmic bytes (operands read once, the output written once and read
 * once when accumulated) since the context was created.  SCC_EINVAL for another kernel value.  With the
 * verbose option, enable = 0 on a profiling context also prints the time per
 * GEMM shape on stderr. */
enum { SCC_GEMM_F64 = 0, SCC_GEMM_F64_TWO = 1, SCC_GEMM_F32 = 2, SCC_GEMM_F32_TWO = 3, SCC_GEMM_F64_MULTI = 4,
       SCC_GEMM_F32_MULTI = 5 };
int scc_profile(scc_ctx* ctx, int enable, int kernel, double* gemm_ms, double* gemm_flops, long long* gemm_launches,
                double* gemm_bytes);

/* Which GEMM kernels scc_profile times: bit k of mask selects kernel k of
 * the enumeration above (default: all).  Launches of the other kernels run
 * without events (and add nothing to their totals), which keeps the event
 * overhead off the timed work when one kernel is of interest. */
int scc_profile_kernels(scc_ctx* ctx, unsigned mask);

/* Test hooks on the device programs (inputs/outputs device pointers):
 *   residual at given amplitudes (and zeta / X3 states when nstates > 1):
 *     t [t1|t2], zeta [npairs], xs [nstates][1+nov+nov^2] (may be NULL);
 *     out [E0 | Omega1 | Omega2]
 *   right transformation of vec [R0|R1|R2] at the current amplitudes
 *     -> out [sigma0 | sigma1 | sigma2]
 *   left transformation of vec -> out (same layout; doubles part symmetrised,
 *   i.e. the transformation restricted to (ai)<->(bj) symmetric vectors).
 * With precision = 1 the residual hook evaluates with FP32 products in the
 * dense contractions (the reduced-precision pass of the solvers). */
int scc_eval_residual(scc_ctx* ctx, const double* t, const double* zeta, const double* xs, double* out);
int scc_eval_sigma(scc_ctx* ctx, const double* vec, double* out);
int scc_eval_left(scc_ctx* ctx, const double* vec, double* out);

#ifdef __cplusplus
}
#endif
#endif /* SCC_H */
