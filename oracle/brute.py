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


def rt_velocity_block_variational(n_el, p, k, c_pen):
    """P_V,k^RT from its variational definition on the parametric cube (eq. precVrt), tiny grids only.

    [P]_ij = a^(e_k B_i, e_k B_j) + sigma^(e_k B_i, e_k B_j) with
    a^(w, v) = int 2 grad^s w : grad^s v over the cube and
    sigma^(w, v) = int over the boundary of 2 [ (c_pen / h) w.v
                   - ((grad^s w) n).v - ((grad^s v) n).w ]
    (Sec. 5, the parametric forms above eq. precVth), over the basis of the
    component k of V_h,0^RT (eq. basisRT_V1): degree p+1, regularity p in
    direction k with its first and last function dropped, degree p,
    regularity p-1 in the other directions (i_1 fastest). Every symmetric
    gradient is formed as a d x d matrix at each Gauss point of the cube and
    of each face (outer normal n = -e_j at eta_j = 0, +e_j at eta_j = 1;
    h = 1/n_el[j] on the faces normal to e_j). Independent of the
    Kronecker-sum factorisation of eq. prec3D_RT, which it checks.
    """
    from .bspline import basis_derivatives, basis_values, element_quadrature, open_uniform_knots

    d = len(n_el)
    npts = p + 2
    tabs = []   # per direction: (knots, degree, keep slice, quadrature points, weights)
    for j in range(d):
        deg, reg = (p + 1, p) if j == k else (p, p - 1)
        knots = open_uniform_knots(n_el[j], deg, reg)
        xq, wq = element_quadrature(n_el[j], npts)
        tabs.append((knots, deg, j == k, xq.ravel(), wq.ravel()))

    def values(j, x):
        knots, deg, drop, _, _ = tabs[j]
        B = basis_values(knots, deg, x)
        dB = basis_derivatives(knots, deg, x)
        return (B[1:-1], dB[1:-1]) if drop else (B, dB)

    def field(pts):
        """Values (nfun, npt) and gradients (nfun, npt, d) of all B_i at the points (each a list per direction)."""
        vals = [values(j, pts[j]) for j in range(d)]
        # multi-indices i_1 fastest, points q_1 fastest: Kronecker products in reversed direction order
        def kron_rows(mats):
            out = np.ones((1, 1))
            for j in range(d):
                out = np.kron(mats[j], out)
            return out
        V = kron_rows([vals[j][0] for j in range(d)])
        G = np.stack([kron_rows([vals[j][1] if j == a else vals[j][0] for j in range(d)]) for a in range(d)], axis=2)
        return V, G

    def sym_grad(G):
        """grad^s of w = e_k B_i for every function and point: (nfun, npt, d, d)."""
        S = np.zeros(G.shape[:2] + (d, d))
        S[:, :, k, :] += 0.5 * G     # row k of grad w is grad B_i
        S[:, :, :, k] += 0.5 * G
        return S

    def weights_of(ws):
        W = np.ones(1)
        for w in ws:
            W = np.kron(w, W)
        return W

    # volume term
    V, G = field([tabs[j][3] for j in range(d)])
    W = weights_of([tabs[j][4] for j in range(d)])
    S = sym_grad(G)
    P = 2.0 * np.einsum("iqab,jqab,q->ij", S, S, W)
    # face terms
    for j in range(d):
        h = 1.0 / n_el[j]
        for side in (0.0, 1.0):
            pts = [tabs[t][3] if t != j else np.array([side]) for t in range(d)]
            ws = [tabs[t][4] if t != j else np.ones(1) for t in range(d)]
            Vf, Gf = field(pts)
            Wf = weights_of(ws)
            Sf = sym_grad(Gf)
            n = np.zeros(d)
            n[j] = 1.0 if side == 1.0 else -1.0
            # w.v = B_i B_j (both along e_k); ((grad^s w) n).v = B_j [ (grad^s w) n ]_k
            Sn = np.einsum("iqab,b->iqa", Sf, n)[:, :, k]      # [(grad^s w_i) n]_k
            pen = (2.0 * c_pen / h) * np.einsum("iq,jq,q->ij", Vf, Vf, Wf)
            cons = 2.0 * (np.einsum("iq,jq,q->ij", Sn, Vf, Wf) + np.einsum("jq,iq,q->ij", Sn, Vf, Wf))
            P += pen - cons
    return P


def stokes_variational_cube(n_el, p):
    """The TH Stokes blocks on the unit cube with G = id, nu = 1 from their forms (Sec. 3), tiny grids only.

    [A_rs]_ij = a(e_r B_i, e_s B_j) = int 2 grad^s(e_r B_i) : grad^s(e_s B_j)
    and [B_r]_lj = b(e_r B_j, Q_l) = -int Q_l div(e_r B_j), over ALL velocity
    functions (degree p+1, regularity p-1) and pressure functions (degree p,
    regularity p-1), i_1 fastest, by tensor Gauss quadrature with every
    symmetric gradient formed as a 3 x 3 matrix at each point. Independent of
    the Kronecker factorisation it checks. Returns (A as a dict (r, s) ->
    matrix, B as a list over r).
    """
    from .bspline import basis_derivatives, basis_values, element_quadrature, open_uniform_knots

    xq, wq = element_quadrature(n_el, p + 3)
    x, w = xq.ravel(), wq.ravel()
    kv = open_uniform_knots(n_el, p + 1, p - 1)
    kq = open_uniform_knots(n_el, p, p - 1)
    V, dV = basis_values(kv, p + 1, x), basis_derivatives(kv, p + 1, x)
    Q = basis_values(kq, p, x)

    def kron3(t1, t2, t3):
        return np.kron(t3, np.kron(t2, t1))   # rows: functions i_1 fastest, columns: points q_1 fastest

    W = kron3(w[None, :], w[None, :], w[None, :]).ravel()
    G = np.stack([kron3(dV, V, V), kron3(V, dV, V), kron3(V, V, dV)], axis=2)   # (nfun, npt, 3)
    QQ = kron3(Q, Q, Q)
    nf, npt = G.shape[:2]

    def symgrad(r):
        S = np.zeros((nf, npt, 3, 3))
        S[:, :, r, :] += 0.5 * G
        S[:, :, :, r] += 0.5 * G
        return S

    Ss = [symgrad(r) for r in range(3)]
    A = {(r, s): 2.0 * np.einsum("iqab,jqab,q->ij", Ss[r], Ss[s], W) for r in range(3) for s in range(3)}
    # div(e_r B_j) = d_r B_j
    Bl = [-(QQ * W[None, :]) @ G[:, :, r].T for r in range(3)]
    return A, Bl
