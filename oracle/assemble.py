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
