// Exercises the library's host-side setup code (fd_host.cpp, fd_geometry.cpp)
// under AddressSanitizer and UndefinedBehaviorSanitizer: univariate assembly
// over degrees, regularities, boundary treatments and weights; the
// generalized eigensolve up to order 256; the coefficient matrices, their
// separable fit and the operator diagonals in 2D and 3D; and the argument
// checks of each routine. Prints "ok" and exits 0 when every property checked
// here holds; the sanitizers abort on the first memory or UB error.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../paper_1712_00403_amd/csrc/fd_host.h"

static int failures = 0;
#define CHECK(c)                                                        \
  do {                                                                  \
    if (!(c)) {                                                         \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
      ++failures;                                                       \
    }                                                                   \
  } while (0)

static double sym_err(int m, const std::vector<double>& A) {
  double e = 0.0, s = 0.0;
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      e = std::fmax(e, std::fabs(A[i + m * j] - A[j + m * i]));
      s = std::fmax(s, std::fabs(A[i + m * j]));
    }
  return e / s;
}

int main() {
  // ---- assembly: every degree 1..8, every regularity, both boundary treatments
  for (int deg = 1; deg <= 8; ++deg)
    for (int reg = -1; reg < deg; ++reg)
      for (int dir = 0; dir < 2; ++dir)
        for (int n_el : {1, 2, 5, 17}) {
          int m = 0;
          if (fdh::assemble_1d(n_el, deg, reg, dir, 0, nullptr, nullptr, &m, nullptr, nullptr) != 0) {
            CHECK(dir == 1);  // only a space emptied by the boundary condition is refused
            continue;
          }
          std::vector<double> K(size_t(m) * m), M(size_t(m) * m);
          const int npts = deg + 1 + (n_el % 3);
          std::vector<double> tau(size_t(n_el) * npts), mu(size_t(n_el) * npts);
          for (size_t q = 0; q < tau.size(); ++q) {
            tau[q] = 1.0 + 0.3 * std::sin(0.7 * double(q));
            mu[q] = 2.0 + std::cos(0.3 * double(q));
          }
          CHECK(fdh::assemble_1d(n_el, deg, reg, dir, npts, tau.data(), mu.data(), &m, K.data(), M.data()) == 0);
          CHECK(sym_err(m, K) < 1e-13 && sym_err(m, M) < 1e-13);
          for (int i = 0; i < m; ++i) CHECK(M[i + size_t(m) * i] > 0.0);
        }
  // argument checks
  int m = 0;
  CHECK(fdh::assemble_1d(0, 2, 1, 0, 0, nullptr, nullptr, &m, nullptr, nullptr) == 1);
  CHECK(fdh::assemble_1d(4, 0, 0, 0, 0, nullptr, nullptr, &m, nullptr, nullptr) == 1);
  CHECK(fdh::assemble_1d(4, 3, 3, 0, 0, nullptr, nullptr, &m, nullptr, nullptr) == 1);
  CHECK(fdh::assemble_1d(4, 3, 1, 0, 17, nullptr, nullptr, &m, nullptr, nullptr) == 1);

  // ---- Nitsche-modified stiffness: symmetric, argument checks
  for (int deg = 1; deg <= 6; ++deg)
    for (int n_el : {1, 2, 9}) {
      CHECK(fdh::nitsche_stiffness_1d(n_el, deg, deg - 1, 5.0 * deg, &m, nullptr) == 0);
      std::vector<double> K(size_t(m) * m);
      CHECK(fdh::nitsche_stiffness_1d(n_el, deg, deg - 1, 5.0 * deg, &m, K.data()) == 0);
      CHECK(sym_err(m, K) < 1e-13);
    }
  CHECK(fdh::nitsche_stiffness_1d(3, 2, 1, -1.0, &m, nullptr) == 1);

  // ---- banded Cholesky of mass matrices: L L^T = M on the band
  for (int deg = 1; deg <= 6; ++deg)
    for (int n_el : {1, 4, 11}) {
      CHECK(fdh::assemble_1d(n_el, deg, deg - 1, 0, 0, nullptr, nullptr, &m, nullptr, nullptr) == 0);
      std::vector<double> M(size_t(m) * m);
      CHECK(fdh::assemble_1d(n_el, deg, deg - 1, 0, 0, nullptr, nullptr, &m, nullptr, M.data()) == 0);
      int bw = -1;
      CHECK(fdh::band_cholesky(m, M.data(), 16, &bw, nullptr, nullptr) == 0 && bw == std::min(deg, m - 1));
      std::vector<double> fac(size_t(bw + 1) * m);
      CHECK(fdh::band_cholesky(m, M.data(), 16, &bw, fac.data(), fac.data()) == 0);
      auto L = [&](int i, int j) { return i == j ? 1.0 / fac[i] : (i - j >= 1 && i - j <= bw ? fac[size_t(i - j) * m + i] : 0.0); };
      double err = 0.0;
      for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) {
          double s = 0.0;
          for (int c = 0; c < m; ++c) s += L(i, c) * L(j, c);
          err = std::fmax(err, std::fabs(s - M[i + size_t(m) * j]));
        }
      CHECK(err < 1e-14);
    }
  {
    std::vector<double> B = {1.0, 2.0, 2.0, 1.0}, f(4);
    int bw = 0;
    CHECK(fdh::band_cholesky(2, B.data(), 16, &bw, f.data(), f.data()) == 2);
    CHECK(fdh::band_cholesky(2, B.data(), 0, &bw, nullptr, nullptr) == 1);
  }

  // ---- eigensolve: U^T M U = I, K U = M U diag(d) for orders up to 256
  for (int n_el : {1, 3, 16, 64, 127}) {
    std::vector<double> K, M;
    CHECK(fdh::assemble_1d(n_el, 3, 1, 1, 0, nullptr, nullptr, &m, nullptr, nullptr) == 0);
    K.assign(size_t(m) * m, 0.0);
    M.assign(size_t(m) * m, 0.0);
    CHECK(fdh::assemble_1d(n_el, 3, 1, 1, 0, nullptr, nullptr, &m, K.data(), M.data()) == 0);
    std::vector<double> U(size_t(m) * m), d(m);
    const char* why = nullptr;
    CHECK(fdh::factor_1d(m, K.data(), M.data(), U.data(), d.data(), &why) == 0);
    double orth = 0.0;
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) {
        double s = 0.0;
        for (int a = 0; a < m; ++a)
          for (int b = 0; b < m; ++b) s += U[a + size_t(m) * i] * M[a + size_t(m) * b] * U[b + size_t(m) * j];
        orth = std::fmax(orth, std::fabs(s - (i == j ? 1.0 : 0.0)));
      }
    CHECK(orth < 1e-10);
    for (int i = 1; i < m; ++i) CHECK(d[i] >= d[i - 1]);
    std::vector<double> U0(size_t(m) * m), d0(m);
    CHECK(fdh::factor_1d(m, nullptr, M.data(), U0.data(), d0.data(), &why) == 0);
    for (int i = 0; i < m; ++i) CHECK(d0[i] == 0.0);
  }
  {
    // not positive definite, asymmetric, bad order
    std::vector<double> M = {1.0, 2.0, 2.0, 1.0}, K = {1.0, 0.0, 0.0, 1.0}, U(4), d(2);
    const char* why = nullptr;
    CHECK(fdh::factor_1d(2, K.data(), M.data(), U.data(), d.data(), &why) == 2 && why);
    std::vector<double> A = {2.0, 1.0, 0.0, 2.0};
    CHECK(fdh::factor_1d(2, K.data(), A.data(), U.data(), d.data(), &why) == 1);
    CHECK(fdh::factor_1d(0, K.data(), K.data(), U.data(), d.data(), &why) == 1);
  }

  // ---- coefficient-aware setup on small 2D and 3D grids
  for (int dim = 2; dim <= 3; ++dim) {
    const int n_el[3] = {3, 4, 2}, deg = 3, reg = 1, npts = deg + 1;
    int nq[3] = {1, 1, 1};
    int64_t P = 1;
    for (int j = 0; j < dim; ++j) {
      nq[j] = n_el[j] * npts;
      P *= nq[j];
    }
    std::vector<double> xq[3];
    for (int j = 0; j < dim; ++j) {
      xq[j].resize(nq[j]);
      std::vector<double> w(nq[j]);
      fdh::element_quadrature(n_el[j], npts, xq[j].data(), w.data());
    }
    // a curved map with a full Jacobian, a positive non-separable viscosity
    std::vector<double> jac(size_t(P) * dim * dim, 0.0), nu(P);
    for (int64_t p = 0; p < P; ++p) {
      int64_t r = p;
      double e[3] = {0, 0, 0};
      for (int j = 0; j < dim; ++j) {
        e[j] = xq[j][r % nq[j]];
        r /= nq[j];
      }
      double* J = &jac[size_t(p) * dim * dim];
      for (int a = 0; a < dim; ++a) J[a * dim + a] = 1.0 + 0.1 * e[(a + 1) % dim];
      J[0 * dim + 1] = 0.2 * e[1];
      nu[p] = 1.0 + 0.5 * std::sin(6.28 * e[0]) * std::cos(6.28 * e[1]);
    }
    std::vector<double> C(size_t(dim) * dim * dim * P), qw(P);
    CHECK(fdh::geometry_coefficients(dim, P, jac.data(), nu.data(), -1, C.data(), qw.data()) == 0);
    for (int64_t p = 0; p < P; ++p) CHECK(qw[p] > 0.0);
    for (int k = 0; k < dim; ++k) {
      std::vector<double> Ck(size_t(dim) * dim * P);
      CHECK(fdh::geometry_coefficients(dim, P, jac.data(), nu.data(), k, Ck.data(), qw.data()) == 0);
      std::vector<double> tau(nq[0] + nq[1] + (dim == 3 ? nq[2] : 0)), mu(tau.size());
      CHECK(fdh::separable_factors(dim, nq, Ck.data(), int64_t(dim + 1) * P, 20, 1e-12, tau.data(), mu.data()) == 0);
      for (size_t i = 0; i < tau.size(); ++i)
        CHECK(tau[i] > 0.0 && std::isfinite(tau[i]) && mu[i] > 0.0 && std::isfinite(mu[i]));
      int64_t N = 1;
      for (int j = 0; j < dim; ++j) {
        CHECK(fdh::assemble_1d(n_el[j], deg + 1, reg, 1, npts, nullptr, nullptr, &m, nullptr, nullptr) == 0);
        N *= m;
      }
      std::vector<double> diag(N);
      CHECK(fdh::operator_diagonal(dim, n_el, deg + 1, reg, 1, npts, 1, Ck.data(), diag.data()) == 0);
      for (double v : diag) CHECK(v > 0.0 && std::isfinite(v));
    }
    // a singular Jacobian is refused
    std::vector<double> bad(jac);
    for (int a = 0; a < dim * dim; ++a) bad[a] = 0.0;
    CHECK(fdh::geometry_coefficients(dim, P, bad.data(), nu.data(), -1, C.data(), qw.data()) == 2);
  }
  if (failures) {
    std::fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  std::printf("ok\n");
  return 0;
}
