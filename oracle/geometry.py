"""Coefficient-aware blocks: geometry and viscosity in P_V and P_Q (Sec. 6, Appendix).

Test infrastructure only (see ``oracle/__init__``).

Velocity block k (TH): the stiffness A_kk has the coefficient matrix
C_k = nu (J^{-1} J^{-T} + D_k D_k^T) |det J| with D_k = J^{-1} e_k
(Sec. 3, eq. Q_TH). The Appendix drops the off-diagonal entries of C_k and
replaces each diagonal entry c^k_jj by a product tau^k_j(eta_j) prod_{i!=j}
mu^k_i(eta_i), computed at the quadrature points. The resulting block is the
unit-weight Kronecker sum of the weighted pairs (K^k_j[tau^k_j], M^k_j[mu^k_j]),
so Algorithm 1 applies to it, and the diagonal scaling
D_V = diag(A_kk) / diag(P_breve) (Sec. 6) restores the diagonal of A_kk.
Pressure: Q = int nu^{-1} B_i B_j |det J| (eq. weighted-pressure-mass), P_Q is
the plain mass Kronecker product and D_Q = diag(Q) / diag(P_Q) (Sec. 6).

Readings (the paper names the approximation's references but states no
algorithm, norm, stopping rule or reconciliation of the mu factors shared by
two diagonal entries):

* the separable fit of each c^k_jj is the Diliberto-Straus alternating
  midrange iteration on log c^k_jj over the quadrature grid: for every axis
  in turn, the factor of that axis becomes the midrange (half of max plus
  min) over all other axes of log c minus the other factors; at most
  ``sweeps`` sweeps, or until no factor moves by more than ``tol``;
* each non-tau factor is normalised to geometric mean 1 over its quadrature
  points and the constant is moved into tau^k_j;
* mu^k_i is the geometric mean of the estimates of axis i obtained from the
  entries j != i (one estimate in 2D, two in 3D);
* quadrature: degree + 1 Gauss points per element for both the velocity
  (degree p + 1) and the pressure (degree p) spaces.

The approximation quality for non-separable coefficients has no pin in the
paper (parity unpinned for that part); it is exact when every c^k_jj is a
product of one-variable functions, and the tests pin it there.
"""
import numpy as np

from .assemble import assemble_1d
from .bspline import (basis_derivatives, basis_values, element_quadrature,
                      open_uniform_knots)


def coefficient_matrices(J, nu):
    """C_k = nu (J^{-1} J^{-T} + D_k D_k^T) |det J|, D_k = J^{-1} e_k (eq. Q_TH).

    J: (P, d, d) with J[p, a, b] = dG_a/deta_b; nu: (P,). Returns (d, P, d, d),
    entry [k, p] the matrix C_k at point p.
    """
    J = np.asarray(J, dtype=np.float64)
    P, d, _ = J.shape
    Ji = np.linalg.inv(J)                          # per point (library routine on a stack)
    det = np.abs(np.linalg.det(J))
    base = Ji @ np.swapaxes(Ji, 1, 2)              # J^{-1} J^{-T}
    w = (np.asarray(nu, dtype=np.float64) * det)[:, None, None]
    out = np.zeros((d, P, d, d))
    for k in range(d):
        Dk = Ji[:, :, k]                           # J^{-1} e_k
        out[k] = w * (base + Dk[:, :, None] * Dk[:, None, :])
    return out


def pressure_weight(J, nu):
    """nu^{-1} |det J| at each point: the weight of the TH pressure mass Q (eq. weighted-pressure-mass)."""
    J = np.asarray(J, dtype=np.float64)
    return np.abs(np.linalg.det(J)) / np.asarray(nu, dtype=np.float64)


def separable_fit(logc, sweeps=20, tol=1e-12):
    """Diliberto-Straus midrange iteration: log c ~ f_1(eta_1) + ... + f_d(eta_d).

    ``logc`` has one axis per direction (axis j indexes the quadrature points
    of direction j). Returns the list of 1D arrays f_j.
    """
    logc = np.asarray(logc, dtype=np.float64)
    d = logc.ndim
    f = [np.zeros(logc.shape[j]) for j in range(d)]
    for _ in range(sweeps):
        moved = 0.0
        for i in range(d):
            rest = logc.copy()
            for l in range(d):
                if l != i:
                    shape = [1] * d
                    shape[l] = -1
                    rest = rest - f[l].reshape(shape)
            other = tuple(a for a in range(d) if a != i)
            new = 0.5 * (rest.max(axis=other) + rest.min(axis=other))
            moved = max(moved, float(np.max(np.abs(new - f[i]))))
            f[i] = new
        if moved < tol:
            break
    return f


def separable_factors(cdiag, sweeps=20, tol=1e-12):
    """tau^k_j and mu^k_j from the diagonal entries c^k_jj of one C_k (Appendix).

    ``cdiag[j]`` is c^k_jj on the quadrature grid (one axis per direction).
    Returns (tau, mu): lists of 1D arrays over the quadrature points of each
    direction, with c^k_jj ~ tau_j(eta_j) prod_{i!=j} mu_i(eta_i).
    """
    d = len(cdiag)
    est = [[None] * d for _ in range(d)]  # est[j][i]: log factor of axis i from entry j
    for j in range(d):
        f = separable_fit(np.log(cdiag[j]), sweeps, tol)
        shift = 0.0
        for i in range(d):
            if i != j:
                m = float(np.mean(f[i]))
                est[j][i] = f[i] - m
                shift += m
        est[j][j] = f[j] + shift
    tau = [np.exp(est[j][j]) for j in range(d)]
    mu = [np.exp(np.mean([est[j][i] for j in range(d) if j != i], axis=0)) for i in range(d)]
    return tau, mu


def grid_axes(n_el, npts):
    """Quadrature points and weights of each direction (element-major, as assemble_1d uses them)."""
    out = []
    for ne in n_el:
        x, w = element_quadrature(ne, npts)
        out.append((x.ravel(), w.ravel()))
    return out


def _space_tables(n_el, degree, regularity, dirichlet, npts):
    """Per direction: basis values and derivatives at the quadrature points, kept functions only."""
    tabs = []
    for ne in n_el:
        knots = open_uniform_knots(ne, degree, regularity)
        x, _ = element_quadrature(ne, npts)
        B = basis_values(knots, degree, x.ravel())
        dB = basis_derivatives(knots, degree, x.ravel())
        if dirichlet:
            B, dB = B[1:-1], dB[1:-1]
        tabs.append((B, dB))
    return tabs


def operator_diagonal(n_el, degree, regularity, dirichlet, npts, coef, order):
    """Diagonal of a tensor-product Galerkin operator with pointwise coefficients.

    order 1: [A]_ii = sum_q w_q sum_{a,b} c_ab(q) d_a B_i(q) d_b B_i(q) with
    ``coef`` of shape (d, d, nq_1, .., nq_d) (the full coefficient matrix,
    off-diagonal entries included); order 0: [Q]_ii = sum_q w_q c(q) B_i(q)^2
    with ``coef`` of shape (nq_1, .., nq_d). B_i is the tensor product of the
    univariate functions, d_a B_i differentiates the factor of direction a.
    The sum over the grid is one numpy einsum per (a, b) (the library picks
    the order of the contraction). Returns the diagonal as a vector with i_1
    fastest.
    """
    d = len(n_el)
    tabs = _space_tables(n_el, degree, regularity, dirichlet, npts)
    wts = [w for _, w in grid_axes(n_el, npts)]
    letters_q = "abc"[:d]
    letters_i = "ijk"[:d]
    spec = letters_q + "," + ",".join(f"{letters_i[t]}{letters_q[t]}" for t in range(d)) + "->" + letters_i

    def table(t, da, db):
        B, dB = tabs[t]
        return (dB if da else B) * (dB if db else B) * wts[t][None, :]

    if order == 0:
        D = np.einsum(spec, coef, *[table(t, False, False) for t in range(d)], optimize=True)
    else:
        D = 0.0
        for a in range(d):
            for b in range(d):
                D = D + np.einsum(spec, coef[a, b], *[table(t, t == a, t == b) for t in range(d)], optimize=True)
    return np.reshape(D, -1, order="F")


def kron_diag(diags):
    """Diagonal of A_d (x) .. (x) A_1 from the diagonals of the factors (i_1 fastest)."""
    out = np.ones(1)
    for v in diags:  # direction 1 first, so it ends in the rightmost slot
        out = np.kron(v, out)
    return out


def tensor_grid(axes):
    """Every point of the tensor grid of the 1D point arrays ``axes`` as rows (P, d), axis 1 fastest."""
    d = len(axes)
    sizes = [len(a) for a in axes]
    P = int(np.prod(sizes))
    pts = np.empty((P, d))
    for j, a in enumerate(axes):
        inner = int(np.prod(sizes[:j]))          # points of the faster axes
        outer = P // (inner * sizes[j])
        pts[:, j] = np.tile(np.repeat(np.asarray(a, dtype=np.float64), inner), outer)
    return pts


def _grid_fields(geometry, n_el, npts):
    """J and nu on the tensor quadrature grid (axis 1 fastest)."""
    axes = [x for x, _ in grid_axes(n_el, npts)]
    eta = tensor_grid(axes)
    J = geometry.jacobian(eta)
    nu = geometry.nu(geometry.map(eta))
    shape = tuple(len(a) for a in axes)
    return J, nu, shape


class GeometryBlocks:
    """Everything the coefficient-aware P_D needs for one TH patch (Sec. 6, Appendix).

    For velocity block k: the weighted univariate pairs (K^k_j, M^k_j), the
    diagonal of A_kk, of the Kronecker sum P_breve_k, and the scale
    D_V^{-1/2}. For the pressure: the plain mass factors and D_Q^{-1/2}.
    """

    def __init__(self, n_el, p, geometry, sweeps=20, tol=1e-12):
        d = len(n_el)
        self.ndim, self.n_el, self.p = d, tuple(n_el), p
        vdeg, vreg, vpts = p + 1, p - 1, p + 2
        J, nu, shape = _grid_fields(geometry, n_el, vpts)
        C = coefficient_matrices(J, nu)  # (d, P, d, d)
        self.vel_K, self.vel_M, self.diagA, self.diagP, self.vel_scales = [], [], [], [], []
        self.tau, self.mu = [], []
        for k in range(d):
            cdiag = [np.reshape(C[k, :, j, j], shape, order="F") for j in range(d)]
            tau, mu = separable_factors(cdiag, sweeps, tol)
            Ks, Ms = [], []
            for j in range(d):
                K, _ = assemble_1d(n_el[j], vdeg, vreg, True, tau=tau[j].reshape(n_el[j], vpts),
                                   npts=vpts)
                _, M = assemble_1d(n_el[j], vdeg, vreg, True, mu=mu[j].reshape(n_el[j], vpts),
                                   npts=vpts)
                Ks.append(K)
                Ms.append(M)
            coef = np.stack([np.stack([np.reshape(C[k, :, a, b], shape, order="F") for b in range(d)])
                             for a in range(d)])
            dA = operator_diagonal(n_el, vdeg, vreg, True, vpts, coef, 1)
            dP = 0.0
            for j in range(d):
                dP = dP + kron_diag([np.diag(Ks[i]) if i == j else np.diag(Ms[i]) for i in range(d)])
            self.tau.append(tau)
            self.mu.append(mu)
            self.vel_K.append(Ks)
            self.vel_M.append(Ms)
            self.diagA.append(dA)
            self.diagP.append(dP)
            self.vel_scales.append(1.0 / np.sqrt(dA / dP))
        qdeg, qreg, qpts = p, p - 1, p + 1
        Jq, nuq, qshape = _grid_fields(geometry, n_el, qpts)
        wq = np.reshape(pressure_weight(Jq, nuq), qshape, order="F")
        self.pres_M = [assemble_1d(n_el[j], qdeg, qreg, False, npts=qpts)[1] for j in range(d)]
        self.diagQ = operator_diagonal(n_el, qdeg, qreg, False, qpts, wq, 0)
        self.diagPQ = kron_diag([np.diag(M) for M in self.pres_M])
        self.pres_scale = 1.0 / np.sqrt(self.diagQ / self.diagPQ)
