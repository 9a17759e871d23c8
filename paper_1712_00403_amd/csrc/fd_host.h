// Host-side FP64 setup routines of the FD library (no HIP dependency).
#pragma once
#include <cstddef>
#include <cstdint>

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

// Generalized eigendecomposition K U = M U diag(d), U^T M U = I, d ascending.
// K may be null (d = 0). Returns 0, 1 (bad argument / asymmetric) or
// 2 (M not positive definite); *why names the failure.
int factor_1d(int n, const double* K, const double* M, double* U, double* d, const char** why);

}  // namespace fdh
