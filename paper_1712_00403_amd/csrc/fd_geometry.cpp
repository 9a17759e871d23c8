// Host FP64 setup of the coefficient-aware blocks (Sec. 6 and Appendix):
// pointwise coefficient matrices, the separable approximation of their
// diagonal entries, and the diagonals of the Galerkin operators that the
// diagonal scalings D_V and D_Q restore.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <limits>
#include <thread>
#include <vector>

#include "fd_host.h"

namespace fdh {

namespace {

int host_threads() {
  static const int n = [] {
    int t = int(std::thread::hardware_concurrency());
    if (const char* e = std::getenv("FD_HOST_THREADS")) t = std::atoi(e);
    return std::max(1, std::min(t, 64));
  }();
  return n;
}

// Run body(lo, hi) over [0, count) split into contiguous chunks, one per thread.
template <class F>
void parallel_for(int64_t count, F body) {
  const int nt = int(std::min<int64_t>(host_threads(), count));
  if (nt <= 1) {
    if (count > 0) body(int64_t(0), count);
    return;
  }
  std::vector<std::thread> pool;
  for (int i = 0; i < nt; ++i) {
    const int64_t lo = count * i / nt, hi = count * (i + 1) / nt;
    pool.emplace_back([=, &body] { body(lo, hi); });
  }
  for (auto& th : pool) th.join();
}

}  // namespace

// C_k = nu (J^{-1} J^{-T} + D_k D_k^T) |det J| with D_k = J^{-1} e_k
// (Sec. 3, eq. Q_TH) and the pressure-mass weight nu^{-1} |det J|
// (eq. weighted-pressure-mass), point by point.
int geometry_coefficients(int d, int64_t P, const double* jac, const double* nu, int component, double* C,
                          double* qw) {
  if ((d != 2 && d != 3) || P < 1 || !jac || !nu || (!C && !qw) || component < -1 || component >= d) return 1;
  const int k0 = component < 0 ? 0 : component, k1 = component < 0 ? d : component + 1;
  std::atomic<int> bad{0};
  parallel_for(P, [&](int64_t lo, int64_t hi) {
    int local_bad = 0;
    for (int64_t p = lo; p < hi; ++p) {
      const double* J = jac + p * d * d;
      double inv[9], det;
      if (d == 2) {
        det = J[0] * J[3] - J[1] * J[2];
        inv[0] = J[3] / det;
        inv[1] = -J[1] / det;
        inv[2] = -J[2] / det;
        inv[3] = J[0] / det;
      } else {
        // adjugate (cofactor transpose) over the determinant
        const double c00 = J[4] * J[8] - J[5] * J[7];
        const double c01 = J[5] * J[6] - J[3] * J[8];
        const double c02 = J[3] * J[7] - J[4] * J[6];
        det = J[0] * c00 + J[1] * c01 + J[2] * c02;
        inv[0] = c00 / det;
        inv[3] = c01 / det;
        inv[6] = c02 / det;
        inv[1] = (J[2] * J[7] - J[1] * J[8]) / det;
        inv[4] = (J[0] * J[8] - J[2] * J[6]) / det;
        inv[7] = (J[1] * J[6] - J[0] * J[7]) / det;
        inv[2] = (J[1] * J[5] - J[2] * J[4]) / det;
        inv[5] = (J[2] * J[3] - J[0] * J[5]) / det;
        inv[8] = (J[0] * J[4] - J[1] * J[3]) / det;
      }
      const double v = nu[p];
      if (!(det != 0.0) || !std::isfinite(det) || !(v > 0.0)) {
        local_bad = 1;
        continue;
      }
      const double adet = std::fabs(det);
      if (qw) qw[p] = adet / v;
      if (!C) continue;
      for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) {
          double g = 0.0;  // (J^{-1} J^{-T})_{ab}
          for (int c = 0; c < d; ++c) g += inv[a * d + c] * inv[b * d + c];
          for (int k = k0; k < k1; ++k) {
            const double dk = inv[a * d + k] * inv[b * d + k];  // (D_k D_k^T)_{ab}
            C[((int64_t(k - k0) * d + a) * d + b) * P + p] = v * (g + dk) * adet;
          }
        }
    }
    if (local_bad) bad.store(1);
  });
  return bad.load() ? 2 : 0;
}

// Diliberto-Straus alternating midrange fit of one field (log values) on a
// tensor grid: f_i(eta_i) <- midrange over the other axes of
// (L - sum_{l != i} f_l), axis by axis, until no factor moves by more than
// tol or after `sweeps` sweeps.
static void midrange_fit(int d, const int* nq, const std::vector<double>& L, int sweeps, double tol,
                         std::vector<std::vector<double>>& f) {
  const int n0 = nq[0], n1 = nq[1], n2 = d == 3 ? nq[2] : 1;
  f.assign(d, {});
  for (int i = 0; i < d; ++i) f[i].assign(nq[i], 0.0);
  const double inf = std::numeric_limits<double>::infinity();
  const int nt = std::max(1, std::min(host_threads(), n2 * n1));
  for (int s = 0; s < sweeps; ++s) {
    double moved = 0.0;
    for (int i = 0; i < d; ++i) {
      // per-thread partial max/min over slabs of the outer index
      std::vector<std::vector<double>> mx(nt, std::vector<double>(nq[i], -inf)),
          mn(nt, std::vector<double>(nq[i], inf));
      const int64_t outer = int64_t(n2) * n1;
      std::vector<std::thread> pool;
      for (int t = 0; t < nt; ++t) {
        const int64_t lo = outer * t / nt, hi = outer * (t + 1) / nt;
        pool.emplace_back([&, t, lo, hi] {
          double* MX = mx[t].data();
          double* MN = mn[t].data();
          for (int64_t o = lo; o < hi; ++o) {
            const int i2 = int(o / n1), i1 = int(o % n1);
            double base = 0.0;
            if (i != 1) base += f[1][i1];
            if (d == 3 && i != 2) base += f[2][i2];
            const double* row = L.data() + o * n0;
            if (i == 0) {
              for (int i0 = 0; i0 < n0; ++i0) {
                const double v = row[i0] - base;
                MX[i0] = std::max(MX[i0], v);
                MN[i0] = std::min(MN[i0], v);
              }
            } else {
              const int ix = i == 1 ? i1 : i2;
              double lmx = -inf, lmn = inf;
              for (int i0 = 0; i0 < n0; ++i0) {
                const double v = row[i0] - base - f[0][i0];
                lmx = std::max(lmx, v);
                lmn = std::min(lmn, v);
              }
              MX[ix] = std::max(MX[ix], lmx);
              MN[ix] = std::min(MN[ix], lmn);
            }
          }
        });
      }
      for (auto& th : pool) th.join();
      for (int x = 0; x < nq[i]; ++x) {
        double a = -inf, b = inf;
        for (int t = 0; t < nt; ++t) {
          a = std::max(a, mx[t][x]);
          b = std::min(b, mn[t][x]);
        }
        const double nv = 0.5 * (a + b);
        moved = std::max(moved, std::fabs(nv - f[i][x]));
        f[i][x] = nv;
      }
    }
    if (moved < tol) break;
  }
}

// tau^k_j and mu^k_j of one coefficient matrix C_k (Appendix): every diagonal
// entry c_jj is fitted as tau_j(eta_j) prod_{i != j} mu_i(eta_i); the
// non-tau factors are normalised to geometric mean 1 (constant moved into
// tau_j) and mu_i is the geometric mean of its estimates from the entries
// j != i.
int separable_factors(int d, const int* nq, const double* c, int64_t stride, int sweeps, double tol,
                      double* tau, double* mu) {
  if ((d != 2 && d != 3) || !nq || !c || !tau || !mu || sweeps < 1) return 1;
  int64_t P = 1;
  for (int i = 0; i < d; ++i) {
    if (nq[i] < 1) return 1;
    P *= nq[i];
  }
  if (stride < P) return 1;
  std::vector<std::vector<std::vector<double>>> est(d);  // est[j][i]
  std::vector<double> L(P);
  for (int j = 0; j < d; ++j) {
    const double* cj = c + j * stride;
    for (int64_t p = 0; p < P; ++p) {
      if (!(cj[p] > 0.0) || !std::isfinite(cj[p])) return 2;
      L[p] = std::log(cj[p]);
    }
    std::vector<std::vector<double>> f;
    midrange_fit(d, nq, L, sweeps, tol, f);
    double shift = 0.0;
    for (int i = 0; i < d; ++i) {
      if (i == j) continue;
      double m = 0.0;
      for (double v : f[i]) m += v;
      m /= nq[i];
      for (double& v : f[i]) v -= m;
      shift += m;
    }
    for (double& v : f[j]) v += shift;
    est[j] = std::move(f);
  }
  int64_t off = 0;
  for (int i = 0; i < d; ++i) {
    for (int x = 0; x < nq[i]; ++x) {
      tau[off + x] = std::exp(est[i][i][x]);
      double s = 0.0;
      for (int j = 0; j < d; ++j)
        if (j != i) s += est[j][i][x];
      mu[off + x] = std::exp(s / (d - 1));
    }
    off += nq[i];
  }
  return 0;
}

// Diagonal of sum_{a,b} int c_ab d_a B_i d_b B_i (order 1) or of
// int c B_i^2 (order 0) over a tensor-product spline space, by sum
// factorisation over the quadrature grid: one contraction per direction,
// each restricted to the support of the univariate function.
int operator_diagonal(int d, const int* n_el, int degree, int regularity, int dirichlet, int npts,
                      int order, const double* coef, double* diag) {
  if ((d != 2 && d != 3) || !n_el || !coef || !diag || (order != 0 && order != 1)) return 1;
  if (npts <= 0) npts = degree + 1;
  std::vector<int> m(d), nq(d);
  std::vector<std::vector<double>> B(d), dB(d), W(d);
  std::vector<std::vector<int>> qlo(d), qhi(d);
  for (int t = 0; t < d; ++t) {
    if (basis_tables(n_el[t], degree, regularity, dirichlet, npts, &m[t], B[t], dB[t], qlo[t], qhi[t]))
      return 1;
    nq[t] = n_el[t] * npts;
    std::vector<double> xq(nq[t]);
    W[t].resize(nq[t]);
    element_quadrature(n_el[t], npts, xq.data(), W[t].data());
  }
  int64_t P = 1, N = 1;
  for (int t = 0; t < d; ++t) {
    P *= nq[t];
    N *= m[t];
  }
  std::fill(diag, diag + N, 0.0);
  // X_t[i][q] = w_q (B or B')_i(q) (B or B')_i(q), by how many of a, b are t
  auto table = [&](int t, int nder) {
    std::vector<double> X(size_t(m[t]) * nq[t]);
    for (int i = 0; i < m[t]; ++i)
      for (int q = 0; q < nq[t]; ++q) {
        const size_t k = size_t(i) * nq[t] + q;
        const double u = nder >= 1 ? dB[t][k] : B[t][k];
        const double v = nder >= 2 ? dB[t][k] : B[t][k];
        X[k] = W[t][q] * u * v;
      }
    return X;
  };
  const int npairs = order == 0 ? 1 : d * d;
  const int n0 = m[0], q0 = nq[0], n1 = m[1], q1 = nq[1];
  const int n2 = d == 3 ? m[2] : 1, q2 = d == 3 ? nq[2] : 1;
  std::vector<double> T1(size_t(q2) * q1 * n0), T2(size_t(q2) * n1 * n0);
  for (int pr = 0; pr < npairs; ++pr) {
    const int a = order == 0 ? -1 : pr / d, b = order == 0 ? -1 : pr % d;
    const double* C = coef + int64_t(pr) * P;
    bool zero = true;
    for (int64_t p = 0; p < P && zero; ++p) zero = C[p] == 0.0;
    if (zero) continue;
    std::vector<double> X[3];
    for (int t = 0; t < d; ++t) X[t] = table(t, (t == a) + (t == b));
    // T1[q3][q2][i1] = sum_{q1 in supp i1} X1[i1][q1] C[q1 + nq1 (q2 + nq2 q3)]
    parallel_for(int64_t(q2) * q1, [&](int64_t lo, int64_t hi) {
      for (int64_t o = lo; o < hi; ++o) {
        const double* row = C + o * q0;
        double* out = T1.data() + o * n0;
        for (int i = 0; i < n0; ++i) {
          const double* x = X[0].data() + size_t(i) * q0;
          double s = 0.0;
          for (int q = qlo[0][i]; q < qhi[0][i]; ++q) s += x[q] * row[q];
          out[i] = s;
        }
      }
    });
    // T2[q3][i2][i1] = sum_{q2 in supp i2} X2[i2][q2] T1[q3][q2][i1]
    parallel_for(q2, [&](int64_t lo, int64_t hi) {
      for (int64_t s3 = lo; s3 < hi; ++s3)
        for (int j = 0; j < n1; ++j) {
          double* out = T2.data() + (s3 * n1 + j) * n0;
          std::fill(out, out + n0, 0.0);
          const double* x = X[1].data() + size_t(j) * q1;
          for (int q = qlo[1][j]; q < qhi[1][j]; ++q) {
            const double xv = x[q];
            const double* in = T1.data() + (s3 * q1 + q) * n0;
            for (int i = 0; i < n0; ++i) out[i] += xv * in[i];
          }
        }
    });
    if (d == 2) {
      for (int64_t k = 0; k < int64_t(n1) * n0; ++k) diag[k] += T2[k];
      continue;
    }
    // diag[i3][i2][i1] += sum_{q3 in supp i3} X3[i3][q3] T2[q3][i2][i1]
    parallel_for(n2, [&](int64_t lo, int64_t hi) {
      for (int64_t k = lo; k < hi; ++k) {
        double* out = diag + k * n1 * n0;
        const double* x = X[2].data() + size_t(k) * q2;
        for (int q = qlo[2][k]; q < qhi[2][k]; ++q) {
          const double xv = x[q];
          const double* in = T2.data() + int64_t(q) * n1 * n0;
          for (int64_t i = 0; i < int64_t(n1) * n0; ++i) out[i] += xv * in[i];
        }
      }
    });
  }
  return 0;
}

}  // namespace fdh
