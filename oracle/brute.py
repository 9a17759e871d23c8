"""Explicit Kronecker-sum assembly and direct solve (tiny grids only).

Test infrastructure only (see ``oracle/__init__``). This is the plain
definition the FD method reaches exactly: P = sum_i w_i (M_d (x) .. K_i .. (x)
M_1) (eq. sylv_eq, eq. prec3D_TH) or P = M_d (x) .. (x) M_1 (eq. precQ),
formed as a matrix with the Kronecker product of Sec. 2.3 and solved.
"""
import numpy as np
import scipy.sparse


def kron_list(mats):
    """A_1 (x) A_2 (x) ... (Sec. 2.3 definition), as a sparse matrix."""
    out = scipy.sparse.csr_matrix(mats[0])
    for A in mats[1:]:
        out = scipy.sparse.kron(out, scipy.sparse.csr_matrix(A), format="csr")
    return out


def assemble_operator(Ks, Ms, weights=None):
    """P with direction 1 in the rightmost slot (i_1 fastest).

    For d = 3: P = w_1 M_3(x)M_2(x)K_1 + w_2 M_3(x)K_2(x)M_1 + w_3 K_3(x)M_2(x)M_1.
    ``Ks=None`` gives M_d (x) .. (x) M_1.
    """
    d = len(Ms)
    if Ks is None:
        return kron_list([Ms[j] for j in reversed(range(d))])
    w = np.ones(d) if weights is None else weights
    P = None
    for i in range(d):
        term = kron_list([(Ks[j] if j == i else Ms[j]) for j in reversed(range(d))]) * w[i]
        P = term if P is None else P + term
    return P


def solve(Ks, Ms, r, weights=None, scale=None):
    """z = P^{-1} r by a dense Cholesky solve of the assembled P.

    ``scale`` (optional) holds D^{-1/2} of the scaled form
    P^G = D^{1/2} P D^{1/2} (Sec. 6): z = D^{-1/2} P^{-1} D^{-1/2} r.
    """
    P = assemble_operator(Ks, Ms, weights).toarray()
    rhs = np.asarray(r, dtype=np.float64)
    if scale is not None:
        rhs = scale * rhs
    L = np.linalg.cholesky(P)
    z = np.linalg.solve(L.T, np.linalg.solve(L, rhs))
    if scale is not None:
        z = scale * z
    return z


def coefficient_operator(tables, weights, coef, order):
    """Full Galerkin matrix with pointwise coefficients on a tensor grid (tiny grids only).

    ``tables[t]`` = (B, dB): univariate values and derivatives of direction t
    at its quadrature points; ``weights[t]`` the quadrature weights. Each
    multivariate function B_i (i_1 fastest) and its partial derivatives are
    formed explicitly at every grid point (point index q_1 fastest) as rows
    of a matrix, and the integral is the weighted sum over points:
    order 1: sum_{a,b} G_a diag(w c_ab) G_b^T with G_a = [d_a B_i(q)];
    order 0: G diag(w c) G^T with G = [B_i(q)].
    ``coef`` is (d, d, P) for order 1, (P,) for order 0.
    """
    d = len(tables)
    W = np.ones(1)
    for t in range(d):
        W = np.kron(weights[t], W)

    def rows(a):
        G = np.ones((1, 1))
        for t in range(d):
            B, dB = tables[t]
            G = np.kron(dB if t == a else B, G)
        return G

    if order == 0:
        G = rows(-1)
        return (G * (W * coef)[None, :]) @ G.T
    grads = [rows(a) for a in range(d)]
    A = 0.0
    for a in range(d):
        for b in range(d):
            A = A + (grads[a] * (W * coef[a, b])[None, :]) @ grads[b].T
    return A
