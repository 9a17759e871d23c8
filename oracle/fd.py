"""Fast Diagonalization apply (Sec. 5.2, Algorithm 1) and the block preconditioner P_D.

Test infrastructure only (see ``oracle/__init__``).

Index convention (Sec. 2.3, definition of vec): a tensor W of shape
(n_1, ..., n_d) is stored as vec(W) with i_1 fastest, i.e. numpy order='F'.

Reading of a garbled passage: Algorithm 1 writes the transform as
(U_1 (x) U_2 (x) U_3)^T, while the factorization of R just above it, and
eq. prec3D_TH, put direction 3 in the leftmost Kronecker slot
(U_3 (x) U_2 (x) U_1). With i_1 fastest, the matrix of direction k acts on
index i_k, so vec(X x_1 A_1 x_2 A_2 x_3 A_3) = (A_3 (x) A_2 (x) A_1) vec(X);
the oracle uses that ordering. Only tests on sizes and matrices that differ
per direction can tell the two apart, and the tests use such cases.
"""
import numpy as np
import scipy.linalg

from .geneig import generalized_eig


def mode_product(W, Y, k):
    """k-mode product W x_k Y (Sec. 2.3), k counted from 0.

    [W x_k Y]_{..., i_k, ...} = sum_j Y[i_k, j] W[..., j, ...].
    """
    out = np.tensordot(Y, W, axes=([1], [k]))  # new axis first
    return np.moveaxis(out, 0, k)


def unvec(r, shape):
    """vec^{-1}: the i_1-fastest vector back to a tensor (Sec. 2.3)."""
    return np.reshape(np.asarray(r, dtype=np.float64), shape, order="F")


def vec(W):
    """vec with i_1 fastest (Sec. 2.3)."""
    return np.reshape(W, -1, order="F")


class FDFactors:
    """Step 1 of Algorithm 1 for one Kronecker-sum block.

    Holds, per direction i, U_i and the eigenvalues d_i of the pencil
    (K_i, M_i) (eq. eig_dec), and the direction weights w_i of the block
    P = sum_i w_i (M_d (x) .. (x) K_i (x) .. (x) M_1): weight 1 + delta_ik for
    the simple TH velocity block k (eq. prec3D_TH, from T_k = I + e_k e_k^T),
    all ones for the coefficient-aware blocks (Appendix).
    ``K=None`` gives the mass-only block P = M_d (x) .. (x) M_1 (eq. precQ),
    where Lambda is the identity.
    """

    def __init__(self, Ks, Ms, weights=None):
        self.ndim = len(Ms)
        self.n = tuple(M.shape[0] for M in Ms)
        self.mass_only = Ks is None
        self.weights = np.ones(self.ndim) if weights is None else np.asarray(weights, dtype=np.float64)
        self.U = []
        self.d = []
        self.Ks = Ks
        self.Ms = Ms
        for i in range(self.ndim):
            if self.mass_only:
                U, d = generalized_eig(np.zeros_like(Ms[i]), Ms[i])
                d = np.zeros_like(d)
            else:
                U, d = generalized_eig(Ks[i], Ms[i])
            self.U.append(U)
            self.d.append(d)

    def eigenvalue_tensor(self):
        """Lambda = sum_i w_i (I (x) .. (x) D_i (x) .. (x) I) as a tensor (step 3)."""
        if self.mass_only:
            return np.ones(self.n)
        lam = np.zeros(self.n)
        for i in range(self.ndim):
            shape = [1] * self.ndim
            shape[i] = self.n[i]
            lam = lam + self.weights[i] * self.d[i].reshape(shape)
        return lam


def fd_apply(f, r):
    """z = P^{-1} r by Algorithm 1 (steps 2-4) for one block.

    Step 2: t~ = (U_d (x) .. (x) U_1)^T t, i.e. T x_1 U_1^T x_2 U_2^T ...
    Step 3: divide elementwise by Lambda.
    Step 4: q = (U_d (x) .. (x) U_1) q~, i.e. Q~ x_1 U_1 x_2 U_2 ...
    ``r`` is a vector of length prod(n) (i_1 fastest).
    """
    T = unvec(r, f.n)
    for i in range(f.ndim):
        T = mode_product(T, f.U[i].T, i)
    T = T / f.eigenvalue_tensor()
    for i in range(f.ndim):
        T = mode_product(T, f.U[i], i)
    return vec(T)


def apply_operator(f, z):
    """P z by mode products with K_i, M_i (eq. kronvec), without U.

    P = sum_i w_i (M_d (x) .. K_i .. (x) M_1); used to check P P^{-1} r = r.
    """
    Z = unvec(z, f.n)
    if f.mass_only:
        for i in range(f.ndim):
            Z = mode_product(Z, f.Ms[i], i)
        return vec(Z)
    out = np.zeros(f.n)
    for i in range(f.ndim):
        T = Z
        for j in range(f.ndim):
            T = mode_product(T, f.Ks[j] if j == i else f.Ms[j], j)
        out = out + f.weights[i] * T
    return vec(out)


def _banded_lower(M, bw):
    """Lower banded storage of a symmetric matrix for scipy's banded solver."""
    n = M.shape[0]
    ab = np.zeros((bw + 1, n))
    for k in range(bw + 1):
        ab[k, : n - k] = np.diag(M, -k)
    return ab


def mass_solve_banded(Ms, r):
    """z = (M_d (x) .. (x) M_1)^{-1} r through banded solves along each mode.

    This is the paper's route for P_Q (Sec. 5.2, first paragraph): by
    eq. kron_vec_sol the inverse of a Kronecker product is the product of
    the inverses applied mode by mode, and each M_k is banded with
    half-bandwidth equal to its degree, so each mode is a banded
    symmetric positive-definite solve (library routine).
    """
    n = tuple(M.shape[0] for M in Ms)
    Z = unvec(r, n)
    for k, M in enumerate(Ms):
        bw = 0
        for j in range(1, M.shape[0]):
            if np.any(np.diag(M, -j) != 0.0):
                bw = j
        ab = _banded_lower(M, bw)
        Zk = np.moveaxis(Z, k, 0)
        sol = scipy.linalg.solveh_banded(ab, Zk.reshape(n[k], -1), lower=True)
        Z = np.moveaxis(sol.reshape(Zk.shape), 0, k)
    return vec(Z)


def velocity_weights(ndim, k):
    """Direction weights of the simple TH velocity block k (eq. prec3D_TH).

    T_k = I + e_k e_k^T doubles the term with K in direction k.
    """
    w = np.ones(ndim)
    w[k] = 2.0
    return w


def block_apply(vel_factors, pres_Ms, r, pres_scale=None, vel_scales=None):
    """P_D^{-1} r for the block-diagonal preconditioner (eq. P_D).

    r = [u_1; ..; u_d; p] (velocity blocks first, as in the Stokes matrix).
    Velocity block k: FD apply with ``vel_factors[k]``; pressure: the mass
    solve by banded per-mode solves. Optional diagonal scalings give the
    coefficient-aware forms z = D^{-1/2} P^{-1} D^{-1/2} r (Sec. 6), with
    ``*_scale`` holding D^{-1/2}.
    """
    out = []
    off = 0
    for k, f in enumerate(vel_factors):
        N = int(np.prod(f.n))
        rk = r[off:off + N]
        if vel_scales is not None:
            rk = vel_scales[k] * rk
        zk = fd_apply(f, rk)
        if vel_scales is not None:
            zk = vel_scales[k] * zk
        out.append(zk)
        off += N
    NQ = int(np.prod([M.shape[0] for M in pres_Ms]))
    rp = r[off:off + NQ]
    if pres_scale is not None:
        rp = pres_scale * rp
    zp = mass_solve_banded(pres_Ms, rp)
    if pres_scale is not None:
        zp = pres_scale * zp
    out.append(zp)
    if off + NQ != r.size:
        raise ValueError("block vector length does not match the block sizes")
    return np.concatenate(out)
