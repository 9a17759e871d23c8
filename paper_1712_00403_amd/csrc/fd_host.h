// Host-side FP64 setup routines of the FD library (no HIP dependency).
#pragma once
#include <cstddef>
#include <cstdint>
#include <vector>

namespace fdh {

// Gauss-Legendre rule with n points on [-1, 1], ascending nodes.
void gauss_legendre(int n, double* x, double* w);

// Per-element Gauss points/weights on the uniform mesh of [0, 1] with n_el
// elements (element-major arrays of n_el * npts).
void element_quadrature(int n_el, int npts, double* xq, double* wq);

// Univariate stiffness/mass factors (weighted by tau/mu at the quadrature
// points when given). Returns 0 on success, 1 on bad arguments. K/M may be
// null to query the order m only.
int assemble_1d(int n_el, int degree, int regularity, int dirichlet, int npts, const double* tau_q,
                const double* mu_q, int* m_out, double* K, double* M);

// Nitsche-modified stiffness K~ of the RT velocity blocks over all m functions
// of the space (column-major m x m). 0 on success, 1 on bad arguments; K may
// be null to query m.
int nitsche_stiffness_1d(int n_el, int degree, int regularity, double c_pen, int* m_out, double* K);

// Mixed univariate integrals int b_a^(da) b_b^(db) over all functions of two
// spaces (X: ma x mb column-major; null to query the sizes). 0, or 1.
int mixed_1d(int n_el, int deg_a, int reg_a, int da, int deg_b, int reg_b, int db, int npts, int* ma, int* mb,
             double* X);

// Banded Cholesky M = L L^T of an SPD matrix of bandwidth b <= max_band:
// band[j*n + i] = L(i, i-j) (j = 1..b; row j = 0 unused), rdiag[i] = 1/L(i,i).
// band/rdiag may be null to query b. 0, 1 (arguments, asymmetry, b too
// large) or 2 (not positive definite).
int band_cholesky(int n, const double* M, int max_band, int* b_out, double* band, double* rdiag);

// Generalized eigendecomposition K U = M U diag(d), U^T M U = I, d ascending.
// K may be null (d = 0). Returns 0, 1 (bad argument / asymmetric) or
// 2 (M not positive definite); *why names the failure.
int factor_1d(int n, const double* K, const double* M, double* U, double* d, const char** why);

// Dense tables of the kept univariate functions at the quadrature points:
// B, dB are m x (n_el*npts) row-major (row = function after dropping the end
// functions when `dirichlet`), [qlo[i], qhi[i]) the quadrature points of the
// elements in the support of function i. Returns 0, or 1 on bad arguments.
int basis_tables(int n_el, int degree, int regularity, int dirichlet, int npts, int* m_out,
                 std::vector<double>& B, std::vector<double>& dB, std::vector<int>& qlo,
                 std::vector<int>& qhi);

// Coefficient matrices C_k of the velocity blocks and the pressure-mass
// weight at P points (fd_geometry_coefficients). 0, 1 (arguments) or
// 2 (singular Jacobian or nu <= 0 at some point).
int geometry_coefficients(int d, int64_t P, const double* jac, const double* nu, int component, double* C,
                          double* qw);

// Separable factors of the d diagonal entries of one C_k (fd_separable_factors).
// 0, 1 (arguments) or 2 (an entry <= 0).
int separable_factors(int d, const int* nq, const double* c, int64_t stride, int sweeps, double tol,
                      double* tau, double* mu);

// Diagonal of a tensor-product Galerkin operator (fd_operator_diagonal). 0 or 1.
int operator_diagonal(int d, const int* n_el, int degree, int regularity, int dirichlet, int npts,
                      int order, const double* coef, double* diag);

}  // namespace fdh
