"""Coefficient-aware blocks of P_D (Sec. 6 and Appendix) from the library's host setup.

Velocity block k: the Kronecker sum of the weighted univariate pairs
(K^k_j[tau^k_j], M^k_j[mu^k_j]) with unit weights (the factor 2 of the simple
block lives inside C_k), scaled by D_V = diag(A_kk) / diag(P_breve_k).
Pressure: the plain mass Kronecker product scaled by D_Q = diag(Q) / diag(P_Q).

The geometry (its Jacobian and the viscosity) is problem data: this module
evaluates it at the library's quadrature points and hands the values to the
library, which computes the coefficient matrices (fd_geometry_coefficients),
their separable approximation (fd_separable_factors), the weighted factors
(fd_assemble_1d) and the operator diagonals (fd_operator_diagonal).
"""
import numpy as np

from . import fd
from .precond import BlockPreconditioner
from .workloads import tensor_points


def _grid(geometry, n_el, npts):
    axes = [fd.quadrature_1d(int(ne), npts)[0].ravel() for ne in n_el]
    eta = tensor_points(axes)
    J = geometry.jacobian(eta)
    nu = geometry.nu(geometry.map(eta))
    return J, nu, [len(a) for a in axes]


def geometry_blocks(problem, geometry, sweeps=20, tol=1e-12):
    """Per block of ``problem``: (Ks, Ms, weights, diag_target) of the coefficient-aware P_D."""
    d, n_el = problem.ndim, problem.n_el
    v = problem.blocks[0].dirs[0]
    vdeg, vreg, vpts = v.degree, v.regularity, v.degree + 1
    J, nu, nq = _grid(geometry, n_el, vpts)
    out = []
    for k in range(d):
        # one coefficient matrix at a time keeps the host memory at d^2 fields
        Ck, _ = fd.geometry_coefficients(J, nu, component=k)
        tau, mu = fd.separable_factors(Ck, nq, sweeps, tol)
        Ks, Ms = [], []
        for j in range(d):
            Ks.append(fd.assemble_1d(n_el[j], vdeg, vreg, True, vpts, tau=tau[j])[0])
            Ms.append(fd.assemble_1d(n_el[j], vdeg, vreg, True, vpts, mu=mu[j])[1])
        dA = fd.operator_diagonal(n_el, vdeg, vreg, True, vpts, Ck, 1)
        del Ck
        out.append((Ks, Ms, np.ones(d), dA))
    del J, nu
    q = problem.blocks[-1].dirs[0]
    qdeg, qreg, qpts = q.degree, q.regularity, q.degree + 1
    Jq, nuq, _ = _grid(geometry, n_el, qpts)
    _, wq = fd.geometry_coefficients(Jq, nuq, matrices=False)
    Ms = [fd.assemble_1d(n_el[j], qdeg, qreg, False, qpts)[1] for j in range(d)]
    dQ = fd.operator_diagonal(n_el, qdeg, qreg, False, qpts, wq, 0)
    out.append((None, Ms, np.ones(d), dQ))
    return out


class GeometryPreconditioner(BlockPreconditioner):
    """P_D with the coefficient-aware blocks z = D^{-1/2} P_breve^{-1} D^{-1/2} r."""

    def __init__(self, problem, geometry, precision="f64", sweeps=20, tol=1e-12, blocks=None):
        blocks = blocks if blocks is not None else geometry_blocks(problem, geometry, sweeps, tol)
        super().__init__(problem, precision,
                         diag_targets=[b[3] for b in blocks],
                         factors=[(b[0], b[1]) for b in blocks],
                         weights=[b[2] for b in blocks])
