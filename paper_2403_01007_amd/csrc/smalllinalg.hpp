// Small dense linear algebra for the solvers' subspace problems (dimensions
// of a few tens): pivoted Gaussian elimination, nonsymmetric eigensolvers
// (Householder reduction to Hessenberg form, then real double-shift QR, or
// complex single-shift QR with Wilkinson shifts; eigenvectors by inverse
// iteration) and a cyclic Jacobi symmetric eigensolver.
#pragma once
#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

namespace scc {

using cplx = std::complex<double>;

// Solve A x = b in place (A row-major n x n, overwritten). Returns false if
// a pivot vanishes.
inline bool solve_linear(int n, std::vector<double> A, std::vector<double>& b) {
  for (int k = 0; k < n; ++k) {
    int p = k;
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(A[i * n + k]) > std::fabs(A[p * n + k])) p = i;
    if (A[p * n + k] == 0.0) return false;
    if (p != k) {
      for (int j = 0; j < n; ++j) std::swap(A[k * n + j], A[p * n + j]);
      std::swap(b[k], b[p]);
    }
    for (int i = k + 1; i < n; ++i) {
      double f = A[i * n + k] / A[k * n + k];
      for (int j = k; j < n; ++j) A[i * n + j] -= f * A[k * n + j];
      b[i] -= f * b[k];
    }
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = b[i];
    for (int j = i + 1; j < n; ++j) s -= A[i * n + j] * b[j];
    b[i] = s / A[i * n + i];
  }
  return true;
}

inline bool solve_complex(int n, std::vector<cplx> A, std::vector<cplx>& b) {
  for (int k = 0; k < n; ++k) {
    int p = k;
    for (int i = k + 1; i < n; ++i)
      if (std::abs(A[i * n + k]) > std::abs(A[p * n + k])) p = i;
    if (std::abs(A[p * n + k]) == 0.0) return false;
    if (p != k) {
      for (int j = 0; j < n; ++j) std::swap(A[k * n + j], A[p * n + j]);
      std::swap(b[k], b[p]);
    }
    for (int i = k + 1; i < n; ++i) {
      cplx f = A[i * n + k] / A[k * n + k];
      for (int j = k; j < n; ++j) A[i * n + j] -= f * A[k * n + j];
      b[i] -= f * b[k];
    }
  }
  for (int i = n - 1; i >= 0; --i) {
    cplx s = b[i];
    for (int j = i + 1; j < n; ++j) s -= A[i * n + j] * b[j];
    b[i] = s / A[i * n + i];
  }
  return true;
}

// Eigenvalues w[n] and right eigenvectors V (column k = V[i*n+k]) of a real
// nonsymmetric matrix A (row-major).  Returns false if QR fails to converge.
// One eigenvector of A (n x n, row-major) for the eigenvalue lam, by inverse
// iteration: one LU factorisation of A - lam' (lam nudged off the exact
// eigenvalue), three solves; normalised, largest component real positive.
inline void eig_nonsym_vector_real(int n, const std::vector<double>& A, double lam, std::vector<cplx>& x);

inline void eig_nonsym_vector(int n, const std::vector<double>& A, cplx lam, std::vector<cplx>& x) {
  if (lam.imag() == 0.0) {
    eig_nonsym_vector_real(n, A, lam.real(), x);
    return;
  }
  double anorm = 0;
  for (int i = 0; i < n * n; ++i) anorm = std::max(anorm, std::fabs(A[i]));
  lam += cplx(1e-13 * (anorm + 1.0), 0.0);
  std::vector<cplx> M(n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) M[i * n + j] = A[i * n + j] - (i == j ? lam : cplx(0.0));
  std::vector<int> piv(n);
  bool ok = true;
  for (int k = 0; k < n && ok; ++k) {
    int p = k;
    for (int i = k + 1; i < n; ++i)
      if (std::abs(M[i * n + k]) > std::abs(M[p * n + k])) p = i;
    piv[k] = p;
    if (std::abs(M[p * n + k]) == 0.0) {
      ok = false;
      break;
    }
    if (p != k)
      for (int j = 0; j < n; ++j) std::swap(M[k * n + j], M[p * n + j]);
    for (int i = k + 1; i < n; ++i) {
      const cplx f = M[i * n + k] / M[k * n + k];
      M[i * n + k] = f;
      for (int j = k + 1; j < n; ++j) M[i * n + j] -= f * M[k * n + j];
    }
  }
  x.assign(n, 0.0);
  for (int i = 0; i < n; ++i) x[i] = cplx(1.0 + 0.1 * i, 0.0);
  for (int it = 0; it < 3 && ok; ++it) {
    for (int k = 0; k < n; ++k) {
      if (piv[k] != k) std::swap(x[k], x[piv[k]]);
      for (int i = k + 1; i < n; ++i) x[i] -= M[i * n + k] * x[k];
    }
    for (int i = n - 1; i >= 0; --i) {
      cplx sum = x[i];
      for (int j = i + 1; j < n; ++j) sum -= M[i * n + j] * x[j];
      x[i] = sum / M[i * n + i];
    }
    double nr = 0;
    for (auto& z : x) nr += std::norm(z);
    nr = std::sqrt(nr);
    for (auto& z : x) z /= nr;
  }
  int im = 0;
  for (int i = 1; i < n; ++i)
    if (std::abs(x[i]) > std::abs(x[im])) im = i;
  const cplx ph = std::abs(x[im]) > 0 ? std::conj(x[im]) / std::abs(x[im]) : cplx(1.0);
  for (int i = 0; i < n; ++i) x[i] *= ph;
}

// The same for a real eigenvalue, in real arithmetic (a quarter of the work).
inline void eig_nonsym_vector_real(int n, const std::vector<double>& A, double lam, std::vector<cplx>& xc) {
  double anorm = 0;
  for (int i = 0; i < n * n; ++i) anorm = std::max(anorm, std::fabs(A[i]));
  lam += 1e-13 * (anorm + 1.0);
  std::vector<double> M(A);
  for (int i = 0; i < n; ++i) M[(size_t)i * n + i] -= lam;
  std::vector<int> piv(n);
  bool ok = true;
  for (int k = 0; k < n && ok; ++k) {
    int p = k;
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(M[(size_t)i * n + k]) > std::fabs(M[(size_t)p * n + k])) p = i;
    piv[k] = p;
    if (M[(size_t)p * n + k] == 0.0) {
      ok = false;
      break;
    }
    if (p != k)
      for (int j = 0; j < n; ++j) std::swap(M[(size_t)k * n + j], M[(size_t)p * n + j]);
    for (int i = k + 1; i < n; ++i) {
      const double f = M[(size_t)i * n + k] / M[(size_t)k * n + k];
      M[(size_t)i * n + k] = f;
      for (int j = k + 1; j < n; ++j) M[(size_t)i * n + j] -= f * M[(size_t)k * n + j];
    }
  }
  std::vector<double> x(n);
  for (int i = 0; i < n; ++i) x[i] = 1.0 + 0.1 * i;
  for (int it = 0; it < 3 && ok; ++it) {
    for (int k = 0; k < n; ++k) {
      if (piv[k] != k) std::swap(x[k], x[piv[k]]);
      for (int i = k + 1; i < n; ++i) x[i] -= M[(size_t)i * n + k] * x[k];
    }
    for (int i = n - 1; i >= 0; --i) {
      double sum = x[i];
      for (int j = i + 1; j < n; ++j) sum -= M[(size_t)i * n + j] * x[j];
      x[i] = sum / M[(size_t)i * n + i];
    }
    double nr = 0;
    for (double z : x) nr += z * z;
    nr = std::sqrt(nr);
    for (double& z : x) z /= nr;
  }
  int im = 0;
  for (int i = 1; i < n; ++i)
    if (std::fabs(x[i]) > std::fabs(x[im])) im = i;
  const double sg = x[im] < 0 ? -1.0 : 1.0;
  xc.assign(n, 0.0);
  for (int i = 0; i < n; ++i) xc[i] = sg * x[i];
}

// Eigenvalues of a real non-symmetric matrix (Hessenberg reduction, shifted
// complex QR); with vectors, also every eigenvector (columns of V).
inline bool eig_nonsym(int n, const std::vector<double>& A, std::vector<cplx>& w, std::vector<cplx>& V,
                       bool vectors = true) {
  std::vector<cplx> H(n * n);
  for (int i = 0; i < n * n; ++i) H[i] = A[i];
  // Householder reduction to upper Hessenberg form
  for (int k = 0; k + 2 < n; ++k) {
    double alpha = 0;
    for (int i = k + 1; i < n; ++i) alpha += std::norm(H[i * n + k]);
    alpha = std::sqrt(alpha);
    if (alpha == 0.0) continue;
    std::vector<cplx> u(n, 0.0);
    cplx x0 = H[(k + 1) * n + k];
    cplx ph = std::abs(x0) > 0 ? x0 / std::abs(x0) : cplx(1.0);
    for (int i = k + 1; i < n; ++i) u[i] = H[i * n + k];
    u[k + 1] += ph * alpha;
    double un = 0;
    for (int i = k + 1; i < n; ++i) un += std::norm(u[i]);
    if (un == 0.0) continue;
    // H = (I - 2uu*/un) H (I - 2uu*/un)
    for (int j = 0; j < n; ++j) {
      cplx s = 0;
      for (int i = k + 1; i < n; ++i) s += std::conj(u[i]) * H[i * n + j];
      s *= 2.0 / un;
      for (int i = k + 1; i < n; ++i) H[i * n + j] -= u[i] * s;
    }
    for (int i = 0; i < n; ++i) {
      cplx s = 0;
      for (int j = k + 1; j < n; ++j) s += H[i * n + j] * u[j];
      s *= 2.0 / un;
      for (int j = k + 1; j < n; ++j) H[i * n + j] -= s * std::conj(u[j]);
    }
  }
  // complex shifted QR on the Hessenberg matrix
  w.assign(n, 0.0);
  int hi = n - 1, iter = 0;
  while (hi >= 0) {
    if (hi == 0) {
      w[0] = H[0];
      break;
    }
    int lo = hi;
    while (lo > 0) {
      double s = std::abs(H[(lo - 1) * n + lo - 1]) + std::abs(H[lo * n + lo]);
      if (s == 0.0) s = 1.0;
      if (std::abs(H[lo * n + lo - 1]) < 1e-15 * s) {
        H[lo * n + lo - 1] = 0.0;
        break;
      }
      --lo;
    }
    if (lo == hi) {
      w[hi] = H[hi * n + hi];
      --hi;
      iter = 0;
      continue;
    }
    if (++iter > 300 * n) return false;
    // Wilkinson shift from the trailing 2x2 block
    cplx a = H[(hi - 1) * n + hi - 1], b = H[(hi - 1) * n + hi], c = H[hi * n + hi - 1], d = H[hi * n + hi];
    cplx tr = a + d, det = a * d - b * c;
    cplx disc = std::sqrt(tr * tr - 4.0 * det);
    cplx l1 = 0.5 * (tr + disc), l2 = 0.5 * (tr - disc);
    cplx mu = std::abs(l1 - d) < std::abs(l2 - d) ? l1 : l2;
    if (iter % 11 == 10) mu += cplx(0.7 * std::abs(c), 0.0);  // exceptional shift
    for (int i = lo; i <= hi; ++i) H[i * n + i] -= mu;
    std::vector<cplx> cs(n), sn(n);
    for (int k = lo; k < hi; ++k) {
      cplx x = H[k * n + k], y = H[(k + 1) * n + k];
      double r = std::sqrt(std::norm(x) + std::norm(y));
      cplx cc = r == 0 ? cplx(1.0) : x / r, ss = r == 0 ? cplx(0.0) : y / r;
      cs[k] = cc;
      sn[k] = ss;
      for (int j = k; j < n; ++j) {
        cplx h1 = H[k * n + j], h2 = H[(k + 1) * n + j];
        H[k * n + j] = std::conj(cc) * h1 + std::conj(ss) * h2;
        H[(k + 1) * n + j] = -ss * h1 + cc * h2;
      }
    }
    for (int k = lo; k < hi; ++k) {
      cplx cc = cs[k], ss = sn[k];
      for (int i = 0; i <= std::min(k + 2, hi); ++i) {
        cplx h1 = H[i * n + k], h2 = H[i * n + k + 1];
        H[i * n + k] = h1 * cc + h2 * ss;
        H[i * n + k + 1] = -h1 * std::conj(ss) + h2 * std::conj(cc);
      }
    }
    for (int i = lo; i <= hi; ++i) H[i * n + i] += mu;
  }
  if (!vectors) return true;
  V.assign(n * n, 0.0);
  std::vector<cplx> x;
  for (int k = 0; k < n; ++k) {
    eig_nonsym_vector(n, A, w[k], x);
    for (int i = 0; i < n; ++i) V[i * n + k] = x[i];
  }
  return true;
}

// Eigenvalues of a real nonsymmetric matrix in real arithmetic: Householder
// reduction to upper Hessenberg form, then implicitly shifted QR steps with
// the two eigenvalues of the trailing 2 x 2 block as a double shift (a 3 x 3
// Householder reflector introduces the bulge, further reflectors chase it down
// the subdiagonal), with deflation at negligible subdiagonal elements; a
// trailing 2 x 2 block gives a real pair or a complex-conjugate pair.  About
// a quarter of the work of the complex single-shift iteration.  Returns false
// if some eigenvalue needs more than 60 steps.
inline bool eig_nonsym_real(int n, const std::vector<double>& A, std::vector<cplx>& w) {
  std::vector<double> H(A);
  auto h = [&](int i, int j) -> double& { return H[(size_t)i * n + j]; };
  for (int k = 0; k + 2 < n; ++k) {
    double alpha = 0;
    for (int i = k + 1; i < n; ++i) alpha += h(i, k) * h(i, k);
    alpha = std::sqrt(alpha);
    if (alpha == 0.0) continue;
    std::vector<double> u(n, 0.0);
    for (int i = k + 1; i < n; ++i) u[i] = h(i, k);
    u[k + 1] += h(k + 1, k) >= 0 ? alpha : -alpha;
    double un = 0;
    for (int i = k + 1; i < n; ++i) un += u[i] * u[i];
    if (un == 0.0) continue;
    for (int j = 0; j < n; ++j) {  // H = (I - 2 u u^T / un) H
      double sdot = 0;
      for (int i = k + 1; i < n; ++i) sdot += u[i] * h(i, j);
      sdot *= 2.0 / un;
      for (int i = k + 1; i < n; ++i) h(i, j) -= u[i] * sdot;
    }
    for (int i = 0; i < n; ++i) {  // H = H (I - 2 u u^T / un)
      double sdot = 0;
      for (int j = k + 1; j < n; ++j) sdot += h(i, j) * u[j];
      sdot *= 2.0 / un;
      for (int j = k + 1; j < n; ++j) h(i, j) -= sdot * u[j];
    }
    for (int i = k + 2; i < n; ++i) h(i, k) = 0.0;
  }
  w.assign(n, 0.0);
  // P = I - 2 v v^T / (v.v) applied to rows r0..r0+m-1 (columns c0..c1) and
  // to the same columns (rows q0..q1); v of length m (2 or 3)
  auto reflect = [&](const double* v, int m, int r0, int c0, int c1, int q0, int q1) {
    double vv = 0;
    for (int i = 0; i < m; ++i) vv += v[i] * v[i];
    if (vv == 0.0) return;
    const double f = 2.0 / vv;
    for (int j = c0; j <= c1; ++j) {
      double sdot = 0;
      for (int i = 0; i < m; ++i) sdot += v[i] * h(r0 + i, j);
      sdot *= f;
      for (int i = 0; i < m; ++i) h(r0 + i, j) -= v[i] * sdot;
    }
    for (int i = q0; i <= q1; ++i) {
      double sdot = 0;
      for (int j = 0; j < m; ++j) sdot += h(i, r0 + j) * v[j];
      sdot *= f;
      for (int j = 0; j < m; ++j) h(i, r0 + j) -= sdot * v[j];
    }
  };
  // Householder vector v with (I - 2 v v^T / v.v) x = -+|x| e1
  auto house = [](const double* x, int m, double* v) {
    double nx = 0;
    for (int i = 0; i < m; ++i) nx += x[i] * x[i];
    nx = std::sqrt(nx);
    for (int i = 0; i < m; ++i) v[i] = x[i];
    v[0] += x[0] >= 0 ? nx : -nx;
  };
  int hi = n - 1, its = 0;
  while (hi >= 0) {
    int l = hi;
    for (; l > 0; --l) {
      const double sc = std::fabs(h(l - 1, l - 1)) + std::fabs(h(l, l));
      if (std::fabs(h(l, l - 1)) <= 1e-15 * (sc > 0 ? sc : 1.0)) {
        h(l, l - 1) = 0.0;
        break;
      }
    }
    if (l == hi) {  // one real eigenvalue
      w[hi] = h(hi, hi);
      --hi;
      its = 0;
      continue;
    }
    if (l == hi - 1) {  // a 2 x 2 block
      const double a = h(hi - 1, hi - 1), b = h(hi - 1, hi), c = h(hi, hi - 1), d = h(hi, hi);
      const double tr = 0.5 * (a + d), det = a * d - b * c, disc = tr * tr - det;
      if (disc >= 0) {
        const double r = std::sqrt(disc), e1 = tr + (tr >= 0 ? r : -r);
        w[hi - 1] = e1;
        w[hi] = e1 != 0.0 ? det / e1 : tr - (tr >= 0 ? r : -r);
      } else {
        const double r = std::sqrt(-disc);
        w[hi - 1] = cplx(tr, r);
        w[hi] = cplx(tr, -r);
      }
      hi -= 2;
      its = 0;
      continue;
    }
    if (++its > 60) return false;
    // double shift from the trailing 2 x 2 block (exceptional shifts after
    // 10 and 20 steps without deflation)
    double s = h(hi - 1, hi - 1) + h(hi, hi);
    double t = h(hi - 1, hi - 1) * h(hi, hi) - h(hi - 1, hi) * h(hi, hi - 1);
    if (its == 10 || its == 20) {
      const double e = std::fabs(h(hi, hi - 1)) + std::fabs(h(hi - 1, hi - 2));
      s = 1.5 * e;
      t = e * e;
    }
    double x[3] = {h(l, l) * h(l, l) + h(l, l + 1) * h(l + 1, l) - s * h(l, l) + t,
                   h(l + 1, l) * (h(l, l) + h(l + 1, l + 1) - s), h(l + 1, l) * h(l + 2, l + 1)};
    for (int k = l; k <= hi - 2; ++k) {
      double v[3];
      house(x, 3, v);
      const int c0 = k > l ? k - 1 : l;
      reflect(v, 3, k, c0, hi, l, std::min(k + 3, hi));
      x[0] = h(k + 1, k);
      x[1] = h(k + 2, k);
      if (k < hi - 2) x[2] = h(k + 3, k);
    }
    double v[3];
    house(x, 2, v);
    reflect(v, 2, hi - 1, hi - 2, hi, l, hi);
  }
  return true;
}

// Symmetric eigenproblem A = V diag(w) V^T (row-major n x n) by cyclic
// Jacobi rotations; eigenvalues ascending, eigenvectors in the columns of V.
inline void eig_sym(int n, std::vector<double> A, std::vector<double>& w, std::vector<double>& V) {
  V.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
  auto a = [&](int i, int j) -> double& { return A[(size_t)i * n + j]; };
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        tot += a(i, j) * a(i, j);
        if (i != j) off += a(i, j) * a(i, j);
      }
    if (off <= 1e-30 * tot || off == 0.0) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = a(p, q);
        if (std::fabs(apq) < 1e-300) continue;
        // rotation angle that zeroes a(p,q): tan(2 phi) = 2 a_pq / (a_qq - a_pp)
        const double theta = (a(q, q) - a(p, p)) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
        for (int k = 0; k < n; ++k) {  // columns p, q
          const double akp = a(k, p), akq = a(k, q);
          a(k, p) = cs * akp - sn * akq;
          a(k, q) = sn * akp + cs * akq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          const double apk = a(p, k), aqk = a(q, k);
          a(p, k) = cs * apk - sn * aqk;
          a(q, k) = sn * apk + cs * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
          V[(size_t)k * n + p] = cs * vkp - sn * vkq;
          V[(size_t)k * n + q] = sn * vkp + cs * vkq;
        }
      }
  }
  std::vector<int> ord(n);
  for (int i = 0; i < n; ++i) ord[i] = i;
  std::sort(ord.begin(), ord.end(), [&](int x, int y) { return a(x, x) < a(y, y); });
  std::vector<double> W((size_t)n * n);
  w.resize(n);
  for (int j = 0; j < n; ++j) {
    w[j] = a(ord[j], ord[j]);
    for (int i = 0; i < n; ++i) W[(size_t)i * n + j] = V[(size_t)i * n + ord[j]];
  }
  V.swap(W);
}

}  // namespace scc
