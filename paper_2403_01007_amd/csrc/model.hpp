// Construction of the SCCSD(E) programs on a contraction graph.
#pragma once
#include <map>
#include <vector>

#include "ir.hpp"

namespace scc {

struct Dims {
  int o, v, n, nj, ns;  // occupied, virtual, orbitals, Cholesky rank, states
  int npairs() const { return ns * (ns - 1) / 2; }
  int64_t nov() const { return (int64_t)o * v; }
};

struct StateT {
  int r0, r1, r2;  // 0-d, [v,o], [v,o,v,o]
};

struct CCOut {
  int E, O1, O2;
};

struct SigmaOut {
  int s0, s1, s2;
};

// All tensors and op lists of one context.
struct Model {
  Dims d{};
  Graph g;
  // constants
  int In = -1, Io = -1, one = -1, z2 = -1;
  // integrals (MO basis at the current geometry) and orbital rotation
  int h = -1, L = -1, kappa = -1;
  int hk = -1, Lk = -1;                 // rotated integrals
  int G = -1, Govvv = -1, Govov = -1;   // bare blocks of the rotated integrals
  int fock = -1;                        // Fock matrix of the rotated integrals
  // --- ground state / residual program
  int t1 = -1, t2 = -1;
  std::vector<int> zeta;                // 0-d per pair
  std::vector<StateT> xs;               // states entering X3
  CCOut res{};
  int res_begin = 0, res_end = 0;
  // --- right transformation of one vector
  StateT vin{};
  SigmaOut sig{};
  int sig_end = 0;
  // --- left transformation: cotangents in, adjoints out
  StateT lin{};
  StateT lout{};
  // --- overlap O(a, b) of two states at the current t
  StateT oa{}, ob{};
  int ovl = -1;
  // --- one-electron density of <calL| Hbar |calR> (for the coupling's
  //     orbital term): cotangents lin on sig outputs, adjoint w.r.t. hk
  int dens_hk = -1;
  // --- Lagrangian (parameters, constraints, multipliers, adjoints)
  int pt1 = -1, pt2 = -1;
  std::vector<int> pz;
  std::vector<StateT> pr;
  std::vector<int> pE;
  std::vector<StateT> lam;              // normalisation vectors (constants)
  CCOut pres{};
  std::vector<SigmaOut> pc;             // (calHbar - E_k) calR_k
  std::vector<int> pN;                  // 1 - Lam_k . calR_k
  std::vector<int> pO;                  // O_kl, k < l
  int fai = -1;                         // F_ai(kappa), [v,o]
  // multiplier (cotangent) inputs
  int m1 = -1, m2 = -1;
  std::vector<SigmaOut> mk;
  std::vector<int> mN, mO;
  int mF = -1;
  // adjoints of the Lagrangian w.r.t. the parameters (J^T lambda-bar)
  int a_t1 = -1, a_t2 = -1;
  std::vector<int> a_z;
  std::vector<StateT> a_r;
  std::vector<int> a_E;
  int a_kappa = -1;                     // from the constraints (eta-kappa)
  int a_h = -1, a_L = -1;               // effective densities
  int fk_adj = -1;                      // A_HF^T kbar (kappa adjoint of F_ai)
  // coupling target O_mn = calL_m . P exp(T - T0) calR_n, one program per n
  StateT nac_l{};                       // calL_m (constant input)
  int nac_t1c = -1, nac_t2c = -1;       // reference amplitudes (constants)
  std::vector<int> onac;                // per n
  std::vector<int> a_nac_t1, a_nac_t2;  // per n
  std::vector<StateT> a_nac_r;          // per n
  std::vector<std::vector<int>> p_nac;  // per n

  // --- Hamiltonian given in a fixed orthonormal basis: RHF Fock matrix for
  //     orbitals Cmo (columns), the MO transformation, and the effective
  //     densities transformed back to the fixed basis
  int hao = -1, Lao = -1, Cmo = -1;
  int Fao = -1, hmo = -1, Lmo = -1, d1ao = -1, zao = -1;
  std::vector<int> p_aofock, p_aotrans, p_aodens;

  // --- right / left transformations of a block of nb vectors at once
  //     (leading batch index on every input, output and intermediate)
  int nb = 1;
  StateT vinB{}, sigB{}, linB{}, loutB{};
  std::vector<int> p_sigB, p_leftB;
  // --- Lagrangian products J^T lambda-bar for nbt targets at once: batched
  //     copy of p_lag; lagB maps each multiplier input and adjoint output to
  //     its batched tensor [nbt, ...]
  int nbt = 1;
  std::map<int, int> lagB;
  std::vector<int> p_lagB;

  // op lists
  std::vector<int> p_setup, p_res, p_sig_pre, p_sig, p_left, p_ovl, p_dens, p_lag_pre, p_lag, p_kappa, p_fk,
      p_integral;
};

void build_model(Model& m, const Dims& d, int nb = 1, int nbt = 1);

// Every op list the context runs (the storage plan relies on this list).
std::vector<const std::vector<int>*> programs(const Model& m);
// Every tensor the host reads or writes between programs (never reused as a
// program temporary).
std::vector<int> host_tensors(const Model& m);

}  // namespace scc
