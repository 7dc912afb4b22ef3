// Host check of the subspace eigensolvers (test infrastructure): the real
// double-shift QR eigenvalues equal those of the complex single-shift QR for
// random nonsymmetric matrices with real and complex eigenvalues (as
// multisets, to 1e-10 relative), and every eigenvalue makes A - lambda
// singular to working precision (the inverse-iteration vector has a small
// residual).  Prints one summary line; exit status 1 on the first failure.
#include <algorithm>
#include <cstdio>
#include <random>
#include <vector>

#include "../../paper_2403_01007_amd/csrc/smalllinalg.hpp"

using namespace scc;

int main() {
  std::mt19937 gen(12345);
  std::normal_distribution<double> nd;
  int cases = 0;
  for (int n : {1, 2, 3, 5, 8, 17, 40, 61, 80, 120}) {
    for (int rep = 0; rep < 4; ++rep) {
      std::vector<double> A((size_t)n * n);
      for (auto& x : A) x = nd(gen);
      if (rep % 2 == 1)  // a spread, mostly real spectrum (as in the Davidson subspaces)
        for (int i = 0; i < n; ++i) A[(size_t)i * n + i] += 0.5 * i;
      std::vector<cplx> wr, wc, V;
      if (!eig_nonsym_real(n, A, wr) || !eig_nonsym(n, A, wc, V, false)) {
        std::printf("n %d rep %d: no convergence\n", n, rep);
        return 1;
      }
      double scale = 1.0;
      for (auto& z : wc) scale = std::max(scale, std::abs(z));
      std::vector<char> used(n, 0);
      for (int i = 0; i < n; ++i) {
        int best = -1;
        double bd = 1e300;
        for (int j = 0; j < n; ++j)
          if (!used[j] && std::abs(wr[i] - wc[j]) < bd) {
            bd = std::abs(wr[i] - wc[j]);
            best = j;
          }
        used[best] = 1;
        if (bd > 1e-10 * scale) {
          std::printf("n %d rep %d: eigenvalue %.15g%+.15gi unmatched (%.2e)\n", n, rep, wr[i].real(), wr[i].imag(), bd);
          return 1;
        }
        std::vector<cplx> x;
        eig_nonsym_vector(n, A, wr[i], x);
        double res = 0, nx = 0;
        for (int r = 0; r < n; ++r) {
          cplx acc = -wr[i] * x[r];
          for (int c = 0; c < n; ++c) acc += A[(size_t)r * n + c] * x[c];
          res = std::max(res, std::abs(acc));
          nx = std::max(nx, std::abs(x[r]));
        }
        if (res > 1e-8 * scale * nx) {
          std::printf("n %d rep %d: eigenvector residual %.2e\n", n, rep, res);
          return 1;
        }
      }
      ++cases;
    }
  }
  std::printf("ok: %d matrices\n", cases);
  return 0;
}
