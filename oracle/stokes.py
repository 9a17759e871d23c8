"""The Taylor-Hood Stokes system on the unit cube (Sec. 3, Sec. 7 'Cube') and its block-diagonal preconditioner.

Test infrastructure only (see ``oracle/__init__``).

With G = id and nu = 1 the forms of Sec. 3 are a(w, v) = int 2 grad^s w :
grad^s v and b(v, q) = -int q div v. For the TH basis phi^r_i = e_r B_i
(velocity degree p+1, regularity p-1; pressure degree p, regularity p-1)
every block is a Kronecker product of univariate integrals:

* A_rr = sum_a (1 + delta_ar) K_a (x) M (x) M ...   (= P_V,r, eq. prec3D_TH),
* A_rs (r != s): [A_rs]_ij = int d_s B_i d_r B_j, the factor C = int b' b
  (derivative on the row function) in direction s, C^T in direction r and M
  in the third,
* B_r: [B_r]_lj = -int q_l d_r B_j, the pressure-velocity factor -D (q times
  b') in direction r and N (q times b) elsewhere.

The unknowns are the velocity coefficients whose functions vanish on the
boundary (first and last univariate function dropped in every direction) and
every pressure coefficient (Sec. 3: no mean-value constraint; the Krylov
solver handles the constant). Boundary data of the driven cavity (Sec. 7):
velocity (1, 0, 0) on the top face eta_3 = 1, (-1, 0, 0) on the bottom face
eta_3 = 0, zero on the lateral faces. Reading (the paper does not say how
the data enters the discrete space): the first velocity component takes the
coefficient +1 (top) or -1 (bottom) on every function of those faces, edge
functions included; every other boundary coefficient is 0. The right-hand
side is minus the system applied to that lifting (f = 0).
"""
import numpy as np
import scipy.sparse as sp

from .bspline import basis_derivatives, basis_values, element_quadrature, open_uniform_knots, space_dim


def univariate(n_el, p):
    """Univariate integrals of the TH spaces over all functions (no boundary function dropped).

    Velocity V: degree p+1, regularity p-1; pressure Q: degree p,
    regularity p-1. Returns KV = int b'b', MV = int b b, CV = int b'_l b_m,
    DQ = int q_l b'_m, NQ = int q_l b_m, MQ = int q q (Gauss rule with p + 3
    points per element, exact for these polynomial degrees).
    """
    npts = p + 3
    xq, wq = element_quadrature(n_el, npts)
    x, w = xq.ravel(), wq.ravel()
    kv = open_uniform_knots(n_el, p + 1, p - 1)
    kq = open_uniform_knots(n_el, p, p - 1)
    BV, dBV = basis_values(kv, p + 1, x), basis_derivatives(kv, p + 1, x)
    BQ = basis_values(kq, p, x)
    W = w[None, :]
    return {"KV": (dBV * W) @ dBV.T, "MV": (BV * W) @ BV.T, "CV": (dBV * W) @ BV.T,
            "DQ": (BQ * W) @ dBV.T, "NQ": (BQ * W) @ BV.T, "MQ": (BQ * W) @ BQ.T}


def _kron3(a1, a2, a3):
    """Operator with direction 1 in the rightmost slot (i_1 fastest): a3 (x) a2 (x) a1."""
    return sp.kron(sp.kron(sp.csr_matrix(a3), sp.csr_matrix(a2)), sp.csr_matrix(a1), format="csr")


class CubeStokes:
    """Assembled TH Stokes matrix on the unit cube with n_el elements per direction, pressure degree p."""

    def __init__(self, n_el, p):
        f = univariate(n_el, p)
        self.n_el, self.p = n_el, p
        m = f["KV"].shape[0]
        self.mV, self.mQ = m, f["MQ"].shape[0]
        inner = np.arange(1, m - 1)
        self.nV = m - 2
        K, M, C = f["KV"], f["MV"], f["CV"]

        def fac(name, rows, cols):
            return f[name][np.ix_(rows, cols)]

        allV = np.arange(m)
        allQ = np.arange(self.mQ)
        # blocks over all velocity functions, restricted afterwards
        full = {}
        for r in range(3):
            for s in range(3):
                if r == s:
                    terms = []
                    for a in range(3):
                        facs = [K if t == a else M for t in range(3)]
                        terms.append((2.0 if a == r else 1.0) * _kron3(*facs))
                    full[r, s] = terms[0] + terms[1] + terms[2]
                else:
                    facs = [M, M, M]
                    facs[s] = C          # d_s on the row function
                    facs[r] = C.T        # d_r on the column function
                    full[r, s] = _kron3(*facs)
        Bfull = []
        for r in range(3):
            facs = [f["NQ"], f["NQ"], f["NQ"]]
            facs[r] = -f["DQ"]
            Bfull.append(_kron3(*facs))
        # interior (unknown) and boundary velocity index sets, i_1 fastest
        idx = np.arange(m ** 3).reshape((m, m, m))   # [i3, i2, i1]
        interior = idx[1:-1, 1:-1, 1:-1].ravel()
        self.interior = interior
        self.A = sp.bmat([[full[r, s][interior][:, interior] for s in range(3)] for r in range(3)], format="csr")
        self.B = sp.hstack([Bfull[r][:, interior] for r in range(3)], format="csr")
        # lifting of the cavity data: component 1 = +1 on the top face, -1 on the bottom face
        g = np.zeros((3, m ** 3))
        g1 = np.zeros((m, m, m))
        g1[-1, :, :] = 1.0
        g1[0, :, :] = -1.0
        g[0] = g1.ravel()
        rhs_u = -np.concatenate([sum(full[r, s] @ g[s] for s in range(3))[interior] for r in range(3)])
        rhs_p = -sum(Bfull[r] @ g[r] for r in range(3))
        self.rhs = np.concatenate([rhs_u, rhs_p])
        self.nu = 3 * self.nV ** 3
        self.nq = self.mQ ** 3
        self.system = sp.bmat([[self.A, self.B.T], [self.B, None]], format="csr")
        self.f = f

    def preconditioner_factors(self):
        """Univariate factors of P_D: per velocity component (Ks, Ms, weights) on the interior functions, and M_Q."""
        K = self.f["KV"][1:-1, 1:-1]
        M = self.f["MV"][1:-1, 1:-1]
        vel = []
        for k in range(3):
            w = np.ones(3)
            w[k] = 2.0
            vel.append(([K] * 3, [M] * 3, w))
        return vel, [self.f["MQ"]] * 3


def block_triangular_inverse(apply_PV_inv, apply_PQ_inv, Bmat, nu):
    """P_T^{-1} of eq. P_T: P_T = [[P_V, B^T], [0, -P_Q]].

    [f; g] -> y = -P_Q^{-1} g, x = P_V^{-1} (f - B^T y).
    """
    def apply(r):
        f, g = r[:nu], r[nu:]
        y = -apply_PQ_inv(g)
        x = apply_PV_inv(f - Bmat.T @ y)
        return np.concatenate([x, y])
    return apply


def constraint_inverse(apply_PV_inv, apply_PQ_inv, Bmat, nu):
    """P_C^{-1} by the factorisation below eq. P_C, applied right to left:

    [I, -P_V^{-1} B^T; 0, I] [I, 0; 0, -P_Q^{-1}] [I, 0; -B, I] [P_V^{-1}, 0; 0, I].
    """
    def apply(r):
        f, g = r[:nu], r[nu:]
        x = apply_PV_inv(f)
        y = g - Bmat @ x
        y = -apply_PQ_inv(y)
        x = x - apply_PV_inv(Bmat.T @ y)
        return np.concatenate([x, y])
    return apply
