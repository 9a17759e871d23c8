// Host-side FP64 setup of the FD library: univariate B-spline factors, the
// generalized eigendecomposition of each pencil (Algorithm 1, step 1) and the
// packing of the factors into MFMA fragment order. Pure C++ (no HIP), so it
// can be built and checked on a machine without a GPU.
#include "fd_host.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

namespace fdh {

// ------------------------------------------------------------------ quadrature

// Gauss-Legendre rule on [-1, 1]: Newton iteration on the Legendre polynomial
// P_n from the three-term recurrence, weights 2 / ((1 - x^2) P_n'(x)^2).
void gauss_legendre(int n, double* x, double* w) {
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double z = std::cos(pi * (i + 0.75) / (n + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = z; p0 = 1.0; }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-17) break;
    }
    // recompute the derivative at the converged node
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
      double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    if (n == 1) { p1 = z; p0 = 1.0; }
    dp = n * (z * p1 - p0) / (z * z - 1.0);
    double wi = 2.0 / ((1.0 - z * z) * dp * dp);
    x[i] = -z;
    x[n - 1 - i] = z;
    w[i] = wi;
    w[n - 1 - i] = wi;
  }
  if (n % 2 == 1) x[n / 2] = 0.0;
}

void element_quadrature(int n_el, int npts, double* xq, double* wq) {
  double g[32], gw[32];
  gauss_legendre(npts, g, gw);
  const double h = 1.0 / n_el;
  for (int e = 0; e < n_el; ++e)
    for (int q = 0; q < npts; ++q) {
      xq[e * npts + q] = (e + 0.5 * (g[q] + 1.0)) * h;
      wq[e * npts + q] = 0.5 * h * gw[q];
    }
}

// ------------------------------------------------------------------ B-splines

// Open knot vector: degree+1 end knots, interior breakpoints e/n_el repeated
// degree - regularity times (continuity + multiplicity = degree).
static std::vector<double> knots_open_uniform(int n_el, int degree, int regularity) {
  const int mult = degree - regularity;
  std::vector<double> t;
  for (int i = 0; i <= degree; ++i) t.push_back(0.0);
  for (int e = 1; e < n_el; ++e)
    for (int r = 0; r < mult; ++r) t.push_back(double(e) / n_el);
  for (int i = 0; i <= degree; ++i) t.push_back(1.0);
  return t;
}

// The degree+1 B-splines that do not vanish on knot span `span`
// (t[span] <= x < t[span+1]), by the triangular form of the Cox-de Boor
// recursion; N[j] is the value of function span - degree + j.
static void nonzero_basis(const std::vector<double>& t, int span, int degree, double x, double* N) {
  double left[32], right[32];
  N[0] = 1.0;
  for (int j = 1; j <= degree; ++j) {
    left[j] = x - t[span + 1 - j];
    right[j] = t[span + j] - x;
    double saved = 0.0;
    for (int r = 0; r < j; ++r) {
      const double den = right[r + 1] + left[j - r];
      const double tmp = den != 0.0 ? N[r] / den : 0.0;
      N[r] = saved + right[r + 1] * tmp;
      saved = left[j - r] * tmp;
    }
    N[j] = saved;
  }
}

// Values N and first derivatives dN of the degree+1 functions that do not
// vanish on knot span `span`; derivative by differentiating the recursion:
// b'_{k,p} = p/(t_{k+p}-t_k) b_{k,p-1} - p/(t_{k+p+1}-t_{k+1}) b_{k+1,p-1}.
static void nonzero_basis_ders(const std::vector<double>& t, int span, int degree, double x, double* N,
                               double* dN) {
  double Nl[32];
  nonzero_basis(t, span, degree, x, N);
  nonzero_basis(t, span, degree - 1, x, Nl);  // functions span-degree+1 .. span
  for (int j = 0; j <= degree; ++j) {
    const int k = span - degree + j;
    const double lo = (j >= 1) ? Nl[j - 1] : 0.0;        // b_{k,p-1}
    const double hi = (j <= degree - 1) ? Nl[j] : 0.0;   // b_{k+1,p-1}
    const double d1 = t[k + degree] - t[k];
    const double d2 = t[k + degree + 1] - t[k + 1];
    dN[j] = (d1 != 0.0 ? degree / d1 * lo : 0.0) - (d2 != 0.0 ? degree / d2 * hi : 0.0);
  }
}

int basis_tables(int n_el, int degree, int regularity, int dirichlet, int npts, int* m_out,
                 std::vector<double>& B, std::vector<double>& dB, std::vector<int>& qlo,
                 std::vector<int>& qhi) {
  if (n_el < 1 || degree < 1 || degree > 12 || regularity < -1 || regularity >= degree) return 1;
  if (npts <= 0 || npts > 16) return 1;
  const std::vector<double> t = knots_open_uniform(n_el, degree, regularity);
  const int m_full = int(t.size()) - degree - 1;
  const int off = dirichlet ? 1 : 0;
  const int m = m_full - 2 * off;
  if (m < 1) return 1;
  *m_out = m;
  const int nq = n_el * npts;
  B.assign(size_t(m) * nq, 0.0);
  dB.assign(size_t(m) * nq, 0.0);
  qlo.assign(m, nq);
  qhi.assign(m, 0);
  std::vector<double> xq(nq), wq(nq);
  element_quadrature(n_el, npts, xq.data(), wq.data());
  const int mult = degree - regularity;
  double N[32], dN[32];
  for (int e = 0; e < n_el; ++e) {
    const int span = degree + mult * e;
    for (int q = 0; q < npts; ++q) {
      const int iq = e * npts + q;
      nonzero_basis_ders(t, span, degree, xq[iq], N, dN);
      for (int j = 0; j <= degree; ++j) {
        const int r = span - degree + j - off;
        if (r < 0 || r >= m) continue;
        B[size_t(r) * nq + iq] = N[j];
        dB[size_t(r) * nq + iq] = dN[j];
      }
    }
    for (int j = 0; j <= degree; ++j) {
      const int r = span - degree + j - off;
      if (r < 0 || r >= m) continue;
      qlo[r] = std::min(qlo[r], e * npts);
      qhi[r] = std::max(qhi[r], (e + 1) * npts);
    }
  }
  return 0;
}

int assemble_1d(int n_el, int degree, int regularity, int dirichlet, int npts, const double* tau_q,
                const double* mu_q, int* m_out, double* K, double* M) {
  if (n_el < 1 || degree < 1 || degree > 12 || regularity < -1 || regularity >= degree) return 1;
  if (npts <= 0) npts = degree + 1;
  if (npts > 16) return 1;
  const std::vector<double> t = knots_open_uniform(n_el, degree, regularity);
  const int m_full = int(t.size()) - degree - 1;
  const int off = dirichlet ? 1 : 0;
  const int m = m_full - 2 * off;
  if (m < 1) return 1;
  *m_out = m;
  if (!K && !M) return 0;
  std::vector<double> Kf(size_t(m_full) * m_full, 0.0), Mf(size_t(m_full) * m_full, 0.0);
  std::vector<double> xq(size_t(n_el) * npts), wq(size_t(n_el) * npts);
  element_quadrature(n_el, npts, xq.data(), wq.data());
  const int mult = degree - regularity;
  double N[32], dN[32];
  for (int e = 0; e < n_el; ++e) {
    const int span = degree + mult * e;  // last knot index equal to e / n_el
    for (int q = 0; q < npts; ++q) {
      const size_t iq = size_t(e) * npts + q;
      const double x = xq[iq];
      nonzero_basis_ders(t, span, degree, x, N, dN);
      const double wk = wq[iq] * (tau_q ? tau_q[iq] : 1.0);
      const double wm = wq[iq] * (mu_q ? mu_q[iq] : 1.0);
      for (int a = 0; a <= degree; ++a)
        for (int b = 0; b <= degree; ++b) {
          const size_t idx = size_t(span - degree + a) + size_t(m_full) * (span - degree + b);
          Kf[idx] += wk * dN[a] * dN[b];
          Mf[idx] += wm * N[a] * N[b];
        }
    }
  }
  for (int c = 0; c < m; ++c)
    for (int r = 0; r < m; ++r) {
      const size_t src = size_t(r + off) + size_t(m_full) * (c + off);
      if (K) K[r + size_t(m) * c] = Kf[src];
      if (M) M[r + size_t(m) * c] = Mf[src];
    }
  return 0;
}

// Nitsche-modified stiffness of the RT velocity blocks (Sec. 5, the factor
// K~ below eq. prec3D_RT): the full-space stiffness plus the one-direction
// face terms of the parametric Nitsche form,
//   K~_ls = K_ls - [b'_l b_s + b'_s b_l]_0^1 + 2 (c_pen / h) (b_l b_s (1) + b_l b_s (0)),
// h = 1 / n_el. End values come from the first and the last knot span (the
// last one closed at x = 1).
int nitsche_stiffness_1d(int n_el, int degree, int regularity, double c_pen, int* m_out, double* K) {
  if (!(c_pen >= 0.0)) return 1;
  int m = 0;
  if (assemble_1d(n_el, degree, regularity, 0, 0, nullptr, nullptr, &m, nullptr, nullptr) != 0) return 1;
  *m_out = m;
  if (!K) return 0;
  if (assemble_1d(n_el, degree, regularity, 0, 0, nullptr, nullptr, &m, K, nullptr) != 0) return 1;
  const std::vector<double> t = knots_open_uniform(n_el, degree, regularity);
  const double h = 1.0 / n_el;
  double N[32], dN[32];
  // (span, point, sign of the outer normal's contribution)
  const int spans[2] = {degree, m - 1};
  const double xs[2] = {0.0, 1.0}, sg[2] = {-1.0, 1.0};
  for (int e = 0; e < 2; ++e) {
    nonzero_basis_ders(t, spans[e], degree, xs[e], N, dN);
    const int f0 = spans[e] - degree;
    for (int a = 0; a <= degree; ++a)
      for (int b = 0; b <= degree; ++b) {
        const int l = f0 + a, s = f0 + b;
        K[l + size_t(m) * s] += -sg[e] * (dN[a] * N[b] + dN[b] * N[a]) + 2.0 * c_pen / h * N[a] * N[b];
      }
  }
  return 0;
}

// Banded Cholesky factor of a symmetric positive definite matrix (the
// route of Sec. 5.2 for P_Q: each M_i has bandwidth degree, so its solve is
// O(degree n)). M: n x n column-major; the bandwidth b is the largest |i - j|
// with M_ij != 0. L (lower, M = L L^T) is returned as band[j * n + i] =
// L(i, i - j) for j = 1..b and rdiag[i] = 1 / L(i, i). 0, 1 (arguments,
// asymmetry or b > max_band) or 2 (not positive definite).
int band_cholesky(int n, const double* M, int max_band, int* b_out, double* band, double* rdiag) {
  if (n < 1 || !M || max_band < 0) return 1;
  int b = 0;
  double amax = 0.0;
  for (int c = 0; c < n; ++c)
    for (int r = 0; r < n; ++r) amax = std::max(amax, std::fabs(M[r + size_t(n) * c]));
  for (int c = 0; c < n; ++c)
    for (int r = 0; r < n; ++r) {
      const double v = M[r + size_t(n) * c];
      if (std::fabs(v - M[c + size_t(n) * r]) > 1e-12 * amax) return 1;
      if (v != 0.0) b = std::max(b, std::abs(r - c));
    }
  if (b > max_band) return 1;
  *b_out = b;
  if (!band || !rdiag) return 0;
  // dense lower factor restricted to the band, row by row
  std::vector<double> L(size_t(n) * (b + 1), 0.0);  // L[i * (b+1) + j] = L(i, i - j)
  for (int i = 0; i < n; ++i) {
    for (int j = std::min(b, i); j >= 0; --j) {
      const int k = i - j;  // column
      double s = M[i + size_t(n) * k];
      for (int t = 1; t <= b; ++t) {
        // sum over columns c < k inside both bands: L(i, c) L(k, c), c = k - t
        const int c = k - t;
        if (c < 0 || i - c > b) continue;
        s -= L[size_t(i) * (b + 1) + (i - c)] * L[size_t(k) * (b + 1) + (k - c)];
      }
      if (j == 0) {
        if (!(s > 0.0)) return 2;
        L[size_t(i) * (b + 1)] = std::sqrt(s);
      } else {
        L[size_t(i) * (b + 1) + j] = s / L[size_t(k) * (b + 1)];
      }
    }
  }
  for (int i = 0; i < n; ++i) {
    rdiag[i] = 1.0 / L[size_t(i) * (b + 1)];
    for (int j = 1; j <= b; ++j) band[size_t(j) * n + i] = L[size_t(i) * (b + 1) + j];
  }
  return 0;
}

// Mixed univariate integrals X[l][m] = int b_{a,l}^(da) b_{b,m}^(db) over all
// functions of two spline spaces on the same uniform mesh (da, db in {0, 1}:
// value or first derivative), by Gauss quadrature with npts points per
// element; X is ma x mb column-major. The blocks of the Stokes system that
// couple different spaces or a derivative with a value (Sec. 3) are Kronecker
// products of these. 0, or 1 on bad arguments.
int mixed_1d(int n_el, int deg_a, int reg_a, int da, int deg_b, int reg_b, int db, int npts, int* ma, int* mb,
             double* X) {
  if ((da != 0 && da != 1) || (db != 0 && db != 1)) return 1;
  std::vector<double> Ba, dBa, Bb, dBb;
  std::vector<int> la, ha, lb, hb;
  if (basis_tables(n_el, deg_a, reg_a, 0, npts, ma, Ba, dBa, la, ha) != 0) return 1;
  if (basis_tables(n_el, deg_b, reg_b, 0, npts, mb, Bb, dBb, lb, hb) != 0) return 1;
  if (!X) return 0;
  const int nq = n_el * npts;
  std::vector<double> xq(nq), wq(nq);
  element_quadrature(n_el, npts, xq.data(), wq.data());
  const std::vector<double>& Ta = da ? dBa : Ba;
  const std::vector<double>& Tb = db ? dBb : Bb;
  for (int m = 0; m < *mb; ++m)
    for (int l = 0; l < *ma; ++l) {
      double s = 0.0;
      const int q0 = std::max(la[l], lb[m]), q1 = std::min(ha[l], hb[m]);
      for (int q = q0; q < q1; ++q) s += wq[q] * Ta[size_t(l) * nq + q] * Tb[size_t(m) * nq + q];
      X[l + size_t(*ma) * m] = s;
    }
  return 0;
}

// ------------------------------------------------------------------ eigensolve

// Symmetric eigenproblem by cyclic Jacobi (row-cyclic ordering), with the
// relative off-diagonal threshold |a_pq| <= eps sqrt(|a_pp a_qq|), which keeps
// the small eigenvalues to high relative accuracy. A is n*n column-major and
// overwritten; V receives the orthonormal eigenvectors.
static void jacobi_sym(int n, double* A, double* V) {
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) V[i + size_t(n) * j] = (i == j) ? 1.0 : 0.0;
  auto a = [&](int i, int j) -> double& { return A[i + size_t(n) * j]; };
  for (int sweep = 0; sweep < 100; ++sweep) {
    bool rotated = false;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = a(p, q);
        if (std::fabs(apq) <= 1e-16 * std::sqrt(std::fabs(a(p, p) * a(q, q))) || apq == 0.0) continue;
        rotated = true;
        const double theta = (a(q, q) - a(p, p)) / (2.0 * apq);
        double tt;
        if (std::isinf(theta)) tt = 0.0;
        else tt = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::hypot(theta, 1.0));
        const double c = 1.0 / std::sqrt(tt * tt + 1.0), s = tt * c;
        for (int k = 0; k < n; ++k) {  // columns p, q
          const double akp = a(k, p), akq = a(k, q);
          a(k, p) = c * akp - s * akq;
          a(k, q) = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          const double apk = a(p, k), aqk = a(q, k);
          a(p, k) = c * apk - s * aqk;
          a(q, k) = s * apk + c * aqk;
        }
        a(p, q) = 0.0;
        a(q, p) = 0.0;
        for (int k = 0; k < n; ++k) {
          const double vkp = V[k + size_t(n) * p], vkq = V[k + size_t(n) * q];
          V[k + size_t(n) * p] = c * vkp - s * vkq;
          V[k + size_t(n) * q] = s * vkp + c * vkq;
        }
      }
    if (!rotated) break;
  }
}

int factor_1d(int n, const double* K, const double* M, double* U, double* d, const char** why) {
  *why = "";
  if (n < 1 || !M || !U || !d) { *why = "fd_factor_1d: bad arguments"; return 1; }
  auto idx = [n](int i, int j) { return size_t(i) + size_t(n) * j; };
  double scaleM = 0.0, scaleK = 0.0;
  for (size_t i = 0; i < size_t(n) * n; ++i) {
    scaleM = std::max(scaleM, std::fabs(M[i]));
    if (K) scaleK = std::max(scaleK, std::fabs(K[i]));
  }
  for (int j = 0; j < n; ++j)
    for (int i = j + 1; i < n; ++i) {
      if (std::fabs(M[idx(i, j)] - M[idx(j, i)]) > 1e-12 * scaleM) { *why = "M is not symmetric"; return 1; }
      if (K && std::fabs(K[idx(i, j)] - K[idx(j, i)]) > 1e-12 * scaleK) { *why = "K is not symmetric"; return 1; }
    }
  // Cholesky M = L L^T (lower, column-major), symmetric part of M.
  std::vector<double> L(size_t(n) * n, 0.0);
  for (int j = 0; j < n; ++j) {
    double s = 0.5 * (M[idx(j, j)] + M[idx(j, j)]);
    for (int k = 0; k < j; ++k) s -= L[idx(j, k)] * L[idx(j, k)];
    if (!(s > 0.0)) { *why = "M is not positive definite"; return 2; }
    const double ljj = std::sqrt(s);
    L[idx(j, j)] = ljj;
    for (int i = j + 1; i < n; ++i) {
      double v = 0.5 * (M[idx(i, j)] + M[idx(j, i)]);
      for (int k = 0; k < j; ++k) v -= L[idx(i, k)] * L[idx(j, k)];
      L[idx(i, j)] = v / ljj;
    }
  }
  // C = L^{-1} Ks L^{-T}: first X = L^{-1} Ks (forward substitution on columns),
  // then C = L^{-1} X^T (X^T = Ks L^{-T} since Ks is symmetric).
  std::vector<double> X(size_t(n) * n, 0.0), C(size_t(n) * n, 0.0), V(size_t(n) * n);
  for (int c = 0; c < n; ++c)
    for (int i = 0; i < n; ++i) {
      double v = K ? 0.5 * (K[idx(i, c)] + K[idx(c, i)]) : 0.0;
      for (int k = 0; k < i; ++k) v -= L[idx(i, k)] * X[idx(k, c)];
      X[idx(i, c)] = v / L[idx(i, i)];
    }
  for (int c = 0; c < n; ++c)
    for (int i = 0; i < n; ++i) {
      double v = X[idx(c, i)];
      for (int k = 0; k < i; ++k) v -= L[idx(i, k)] * C[idx(k, c)];
      C[idx(i, c)] = v / L[idx(i, i)];
    }
  for (int j = 0; j < n; ++j)
    for (int i = j + 1; i < n; ++i) {
      const double s = 0.5 * (C[idx(i, j)] + C[idx(j, i)]);
      C[idx(i, j)] = s;
      C[idx(j, i)] = s;
    }
  jacobi_sym(n, C.data(), V.data());
  // sort ascending
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return C[idx(a, a)] < C[idx(b, b)]; });
  // U = L^{-T} V (back substitution with L^T)
  for (int jj = 0; jj < n; ++jj) {
    const int j = order[jj];
    d[jj] = C[idx(j, j)];
    for (int i = n - 1; i >= 0; --i) {
      double v = V[idx(i, j)];
      for (int k = i + 1; k < n; ++k) v -= L[idx(k, i)] * U[idx(k, jj)];
      U[idx(i, jj)] = v / L[idx(i, i)];
    }
  }
  if (!K)
    for (int i = 0; i < n; ++i) d[i] = 0.0;
  return 0;
}

}  // namespace fdh
