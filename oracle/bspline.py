"""Univariate B-splines on open uniform knot vectors (Sec. 2.1).

Test infrastructure only (see ``oracle/__init__``).
"""
import numpy as np


def open_uniform_knots(n_el, degree, regularity):
    """Open knot vector on [0, 1] with ``n_el`` uniform elements (Sec. 2.1).

    The end knots are repeated degree+1 times (open knot vector). Each interior
    breakpoint j/n_el is repeated degree - regularity times, since continuity
    plus multiplicity equals the degree at every breakpoint (Sec. 2.1).
    Returns the knot vector; its length is m + degree + 1 with m the dimension
    of the spline space.
    """
    if n_el < 1 or degree < 0 or regularity < -1 or regularity >= degree:
        raise ValueError("need n_el>=1, degree>=0, -1<=regularity<degree")
    mult = degree - regularity
    knots = [0.0] * (degree + 1)
    for j in range(1, n_el):
        knots += [j / n_el] * mult
    knots += [1.0] * (degree + 1)
    return np.array(knots, dtype=np.float64)


def space_dim(knots, degree):
    """m = number of B-splines on the knot vector (length is m + degree + 1)."""
    return len(knots) - degree - 1


def _ratio(num, den):
    """num/den with the Cox-de Boor convention 0/0 = 0 (Sec. 2.1).

    A zero denominator only occurs for repeated knots, where the B-spline it
    multiplies is identically zero, so returning 0 is the convention.
    """
    return np.where(den == 0.0, 0.0, num / np.where(den == 0.0, 1.0, den))


def basis_values(knots, degree, x):
    """Values of all m B-splines of the given degree at the points ``x``.

    Cox-de Boor recursion exactly as defined in Sec. 2.1: degree 0 is the
    indicator of the half-open knot span [xi_i, xi_{i+1}); degree q combines
    two degree q-1 functions with the knot-ratio weights and 0/0 = 0.
    Reading of the paper (half-open spans make every function vanish at
    x = 1): the last non-empty span is closed, so evaluation at the right end
    point is the limit from the left.  Returns an array of shape (m, len(x)).
    """
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    t = knots
    nspan = len(t) - 1
    B = np.zeros((nspan, x.size))
    last = max(i for i in range(nspan) if t[i] < t[i + 1])
    for i in range(nspan):
        if t[i] < t[i + 1]:
            inside = (t[i] <= x) & (x < t[i + 1])
            if i == last:
                inside |= x == t[i + 1]
            B[i] = inside.astype(np.float64)
    for q in range(1, degree + 1):
        Bn = np.zeros((nspan - q, x.size))
        for i in range(nspan - q):
            left = _ratio(x - t[i], np.full_like(x, t[i + q] - t[i]))
            right = _ratio(t[i + q + 1] - x, np.full_like(x, t[i + q + 1] - t[i + 1]))
            Bn[i] = left * B[i] + right * B[i + 1]
        B = Bn
    return B


def basis_derivatives(knots, degree, x):
    """First derivatives of all m B-splines at ``x`` (shape (m, len(x))).

    The paper does not state the derivative formula; this is the textbook one
    obtained by differentiating the recursion:
    b'_{i,q} = q/(xi_{i+q}-xi_i) b_{i,q-1} - q/(xi_{i+q+1}-xi_{i+1}) b_{i+1,q-1},
    with 0/0 = 0.
    """
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    if degree == 0:
        return np.zeros((space_dim(knots, 0), x.size))
    t = knots
    Bl = basis_values(knots, degree - 1, x)  # m + 1 functions of degree q-1
    m = space_dim(knots, degree)
    dB = np.zeros((m, x.size))
    q = degree
    for i in range(m):
        a = _ratio(np.float64(q), np.float64(t[i + q] - t[i]))
        b = _ratio(np.float64(q), np.float64(t[i + q + 1] - t[i + 1]))
        dB[i] = a * Bl[i] - b * Bl[i + 1]
    return dB


def gauss_legendre(npts):
    """Gauss-Legendre nodes and weights on [-1, 1] (library routine)."""
    return np.polynomial.legendre.leggauss(npts)


def element_quadrature(n_el, npts):
    """Per-element Gauss points and weights on the uniform mesh of [0, 1].

    Returns (x, w) of shape (n_el, npts). The paper does not state the rule;
    the reading used throughout is npts = degree + 1 points per element, which
    integrates products of two degree-q splines (or their derivatives) exactly.
    """
    g, gw = gauss_legendre(npts)
    h = 1.0 / n_el
    left = np.arange(n_el, dtype=np.float64) * h
    x = left[:, None] + 0.5 * h * (g[None, :] + 1.0)
    w = np.broadcast_to(0.5 * h * gw[None, :], x.shape).copy()
    return x, w
