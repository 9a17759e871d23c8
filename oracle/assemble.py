"""Univariate stiffness and mass factors (Sec. 5 and Appendix).

Test infrastructure only (see ``oracle/__init__``).
"""
import numpy as np

from .bspline import (basis_derivatives, basis_values, element_quadrature,
                      open_uniform_knots, space_dim)


def assemble_1d(n_el, degree, regularity, dirichlet, tau=None, mu=None, npts=None):
    """Univariate factors K and M on a uniform mesh of [0, 1].

    [K]_{ls} = int tau b'_l b'_s and [M]_{ls} = int mu b_l b_s (Sec. 5, the
    factors K_k^TH, M_k^TH below eq. prec3D_TH and M_k below eq. precQ; the
    weights tau, mu are the Appendix's weighted pairs K^d_k[tau], M^d_k[mu]).
    With ``dirichlet`` the first and last B-spline are dropped (indices
    l, s = 2..m-1 in the paper), as for the TH velocity; the pressure keeps
    all m functions.

    ``tau``/``mu`` are None (weight 1) or arrays of shape (n_el, npts) holding
    the weight at the quadrature points returned by ``element_quadrature``
    (the Appendix computes the separable factors directly at those points).
    ``npts`` defaults to degree + 1 Gauss points per element (reading of a
    point the paper leaves open).

    Returns dense FP64 (K, M).
    """
    if npts is None:
        npts = degree + 1
    knots = open_uniform_knots(n_el, degree, regularity)
    m = space_dim(knots, degree)
    xq, wq = element_quadrature(n_el, npts)
    x = xq.ravel()
    w = wq.ravel()
    B = basis_values(knots, degree, x)          # (m, nq)
    dB = basis_derivatives(knots, degree, x)    # (m, nq)
    wk = w * (np.ones_like(x) if tau is None else np.asarray(tau, dtype=np.float64).ravel())
    wm = w * (np.ones_like(x) if mu is None else np.asarray(mu, dtype=np.float64).ravel())
    K = np.zeros((m, m))
    M = np.zeros((m, m))
    for q in range(x.size):
        K += wk[q] * np.outer(dB[:, q], dB[:, q])
        M += wm[q] * np.outer(B[:, q], B[:, q])
    if dirichlet:
        K = K[1:-1, 1:-1]
        M = M[1:-1, 1:-1]
    return K, M


def taylor_hood_velocity_1d(n_el, p, tau=None, mu=None):
    """TH velocity factors: degree p+1, regularity p-1, Dirichlet (Sec. 2.2.1, Sec. 5).

    p is the pressure degree (Sec. 7: p always refers to the pressure space)
    and the regularity is alpha = p - 1, so interior knots of the degree p+1
    velocity space are doubled.
    """
    return assemble_1d(n_el, p + 1, p - 1, True, tau=tau, mu=mu)


def pressure_1d(n_el, p, mu=None):
    """TH pressure mass factor: degree p, regularity p-1, no boundary condition (eq. precQ)."""
    return assemble_1d(n_el, p, p - 1, False, mu=mu)[1]


def nitsche_stiffness_1d(n_el, degree, regularity, c_pen):
    """The Nitsche-modified stiffness factor K~ of the RT velocity blocks (Sec. 5, factors below eq. prec3D_RT).

    Over all m B-splines of the degree/regularity space (no function dropped):
    [K~]_ls = int b'_l b'_s
              - ( b'_l(1) b_s(1) - b'_l(0) b_s(0) + b'_s(1) b_l(1) - b'_s(0) b_l(0) )
              + 2 (c_pen / h) ( b_l(1) b_s(1) + b_l(0) b_s(0) ),
    h = 1 / n_el. These are the symmetric-gradient face terms of the
    parametric Nitsche form sigma-hat (Sec. 5, the definition above eq.
    precVth) restricted to one direction. End-point values use the closed last
    span (reading of the half-open spans, see ``basis_values``).
    """
    K, _ = assemble_1d(n_el, degree, regularity, False)
    knots = open_uniform_knots(n_el, degree, regularity)
    ends = np.array([0.0, 1.0])
    B = basis_values(knots, degree, ends)
    dB = basis_derivatives(knots, degree, ends)
    b0, b1 = B[:, 0], B[:, 1]
    d0, d1 = dB[:, 0], dB[:, 1]
    h = 1.0 / n_el
    consistency = np.outer(d1, b1) - np.outer(d0, b0) + np.outer(b1, d1) - np.outer(b0, d0)
    penalty = 2.0 * c_pen / h * (np.outer(b1, b1) + np.outer(b0, b0))
    return K - consistency + penalty


def rt_penalty(p):
    """C_pen = 5 (alpha + 1) with alpha = p - 1, the value of the experiments (Sec. 7)."""
    return 5.0 * p


def raviart_thomas_velocity_1d(n_el, p, k, c_pen=None):
    """Per-direction (K, M) of the RT velocity block P_V,k^RT (eq. prec3D_RT) and its weights.

    Direction k: degree p+1, regularity alpha+1 = p, first and last function
    dropped (the normal component vanishes on the faces normal to e_k):
    K_k^RT, M_k^RT. Every other direction j: degree p, regularity
    alpha = p-1, all functions: the Nitsche factor K~_j and the mass M~_j.
    Weights 2 on direction k and 1 elsewhere (T_k = I + e_k e_k^T).
    ``n_el`` lists the elements per direction; h of direction j is 1/n_el[j].
    Returns (Ks, Ms, weights).
    """
    c_pen = rt_penalty(p) if c_pen is None else c_pen
    d = len(n_el)
    Ks, Ms = [], []
    for j in range(d):
        if j == k:
            K, M = assemble_1d(n_el[j], p + 1, p, True)
        else:
            K = nitsche_stiffness_1d(n_el[j], p, p - 1, c_pen)
            M = assemble_1d(n_el[j], p, p - 1, False)[1]
        Ks.append(K)
        Ms.append(M)
    w = np.ones(d)
    w[k] = 2.0
    return Ks, Ms, w
