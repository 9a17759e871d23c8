"""The oracle's Stokes system on the cube and its P_D-MINRES (Sec. 3, Sec. 4, Sec. 7 'Cube', Table 1).

Pins: the Kronecker-assembled blocks equal those assembled from the forms
a and b by 3D quadrature; with G = id the diagonal blocks of A are the
P_V,k of eq. prec3D_TH; and P_D-MINRES (tolerance 1e-8, zero initial guess)
reproduces the iteration counts of Table 1 (TH, P_D-MINRES) exactly where
the readings of the stopping norm and of the boundary lifting do not matter
(p = 2) and within three iterations elsewhere.
"""
import numpy as np
import pytest

from oracle.fd import FDFactors, fd_apply, mass_solve_banded
from oracle.krylov import minres
from oracle.stokes import CubeStokes


def _pinv(S):
    vel, Mq = S.preconditioner_factors()
    facs = [FDFactors(*v) for v in vel]
    nv = S.nV ** 3

    def apply(r):
        out = np.empty_like(r)
        for k in range(3):
            out[k * nv:(k + 1) * nv] = fd_apply(facs[k], r[k * nv:(k + 1) * nv])
        out[3 * nv:] = mass_solve_banded(Mq, r[3 * nv:])
        return out
    return apply


@pytest.mark.parametrize("n_el,p", [(2, 1), (1, 2)])
def test_kronecker_blocks_equal_forms(n_el, p):
    from oracle.brute import stokes_variational_cube
    from oracle.stokes import _kron3, univariate
    A, Bl = stokes_variational_cube(n_el, p)
    f = univariate(n_el, p)
    K, M, C = f["KV"], f["MV"], f["CV"]
    for r in range(3):
        for s in range(3):
            if r == s:
                P = sum((2.0 if a == r else 1.0) * _kron3(*[K if t == a else M for t in range(3)]) for a in range(3))
            else:
                facs = [M, M, M]
                facs[s] = C
                facs[r] = C.T
                P = _kron3(*facs)
            np.testing.assert_allclose(P.toarray(), A[r, s], rtol=0, atol=1e-12 * np.abs(A[r, r]).max())
        facs = [f["NQ"]] * 3
        facs = list(facs)
        facs[r] = -f["DQ"]
        np.testing.assert_allclose(_kron3(*facs).toarray(), Bl[r], rtol=0, atol=1e-12 * np.abs(Bl[r]).max())


def test_diagonal_blocks_are_the_preconditioner_blocks():
    """G = id, nu = 1: A_kk = P_V,k (Sec. 7: 'In this case ... A_kk = P_V,k')."""
    from oracle.assemble import taylor_hood_velocity_1d
    from oracle.brute import assemble_operator
    from oracle.fd import velocity_weights
    S = CubeStokes(3, 2)
    K, M = taylor_hood_velocity_1d(3, 2)
    nv = S.nV ** 3
    for k in range(3):
        P = assemble_operator([K] * 3, [M] * 3, velocity_weights(3, k)).toarray()
        np.testing.assert_allclose(S.A[k * nv:(k + 1) * nv, k * nv:(k + 1) * nv].toarray(), P,
                                   rtol=0, atol=1e-12 * np.abs(P).max())


def test_minres_solution_solves_the_system():
    S = CubeStokes(3, 2)
    x, it, _ = minres(lambda v: S.system @ v, _pinv(S), S.rhs)
    assert np.linalg.norm(S.rhs - S.system @ x) <= 1e-7 * np.linalg.norm(S.rhs)
    # the discrete velocity is divergence free in the weak sense (B u = -B u_lift part of the rhs)
    u = x[:S.nu]
    assert np.linalg.norm(S.B @ u - S.rhs[S.nu:]) <= 1e-7 * np.linalg.norm(S.rhs)


# Table 1, TH, P_D-MINRES iterations
TABLE1 = {(4, 2): 48, (8, 2): 53, (4, 3): 51, (4, 4): 52, (4, 5): 52}


@pytest.mark.parametrize("n_el,p", [(4, 2), (8, 2), (4, 3)])
def test_minres_iterations_match_table1_exactly(n_el, p):
    S = CubeStokes(n_el, p)
    _, it, _ = minres(lambda v: S.system @ v, _pinv(S), S.rhs)
    assert it == TABLE1[n_el, p]


@pytest.mark.parametrize("n_el,p", [(4, 4), (4, 5)])
def test_minres_iterations_near_table1(n_el, p):
    S = CubeStokes(n_el, p)
    _, it, _ = minres(lambda v: S.system @ v, _pinv(S), S.rhs)
    assert abs(it - TABLE1[n_el, p]) <= 3


def _dense_blocks(S):
    """Dense P_V (block diagonal of A) and P_Q (pressure mass Kronecker product) of a small cube."""
    import scipy.sparse as sp
    from oracle.stokes import _kron3
    nv = S.nV ** 3
    PV = sp.block_diag([S.A[k * nv:(k + 1) * nv, k * nv:(k + 1) * nv] for k in range(3)]).toarray()
    MQ = S.f["MQ"]
    PQ = _kron3(MQ, MQ, MQ).toarray()
    return PV, PQ


def test_block_triangular_and_constraint_inverses_by_brute_force():
    """P_T^{-1} and the factorised P_C^{-1} against dense inverses of the assembled P_T, P_C (eq. P_T, eq. P_C)."""
    from oracle.stokes import block_triangular_inverse, constraint_inverse
    S = CubeStokes(2, 1)
    PV, PQ = _dense_blocks(S)
    B = S.B.toarray()
    nu = S.nu
    PT = np.block([[PV, B.T], [np.zeros((B.shape[0], nu)), -PQ]])
    PC = np.block([[PV, B.T], [B, B @ np.linalg.solve(PV, B.T) - PQ]])
    pv = lambda v: np.linalg.solve(PV, v)
    pq = lambda v: np.linalg.solve(PQ, v)
    rng = np.random.default_rng(3)
    r = rng.standard_normal(PT.shape[0])
    np.testing.assert_allclose(block_triangular_inverse(pv, pq, S.B, nu)(r), np.linalg.solve(PT, r), rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(constraint_inverse(pv, pq, S.B, nu)(r), np.linalg.solve(PC, r), rtol=1e-8, atol=1e-8)


def test_gmres_with_ideal_block_triangular_converges_in_two_steps():
    """With P_V = A and P_Q the Schur complement B A^{-1} B^T, P_T^{-1} A has the minimal polynomial (x - 1)^2
    on the nonsingular part, so GMRES stops after 2 iterations (a property of eq. P_T; pressure constant removed)."""
    from oracle.krylov import gmres
    from oracle.stokes import block_triangular_inverse
    S = CubeStokes(2, 1)
    A = S.A.toarray()
    B = S.B.toarray()
    # drop the pressure constant: a basis of the pressure space orthogonal to the kernel of B^T
    U, sv, Vt = np.linalg.svd(B, full_matrices=False)
    keep = sv > 1e-10 * sv[0]
    Bq = U[:, keep].T @ B
    Sch = Bq @ np.linalg.solve(A, Bq.T)
    nu = S.nu
    K = np.block([[A, Bq.T], [Bq, np.zeros((Bq.shape[0],) * 2)]])
    rhs = np.concatenate([S.rhs[:nu], U[:, keep].T @ S.rhs[nu:]])
    apply = block_triangular_inverse(lambda v: np.linalg.solve(A, v), lambda v: np.linalg.solve(Sch, v), Bq, nu)
    x, it, _ = gmres(lambda v: K @ v, apply, rhs, tol=1e-10)
    assert it <= 2
    assert np.linalg.norm(K @ x - rhs) <= 1e-8 * np.linalg.norm(rhs)


def test_gmres_and_minres_agree_on_the_cube():
    """P_T-GMRES and P_C-GMRES on the cavity reach the MINRES solution (velocity, and pressure up to a constant)."""
    from oracle.fd import FDFactors, fd_apply, mass_solve_banded
    from oracle.krylov import gmres
    from oracle.stokes import block_triangular_inverse, constraint_inverse
    S = CubeStokes(3, 2)
    vel, Mq = S.preconditioner_factors()
    facs = [FDFactors(*v) for v in vel]
    nv = S.nV ** 3

    def pv(r):
        return np.concatenate([fd_apply(facs[k], r[k * nv:(k + 1) * nv]) for k in range(3)])

    xm, _, _ = minres(lambda v: S.system @ v, _pinv(S), S.rhs, tol=1e-10)
    for make in (block_triangular_inverse, constraint_inverse):
        x, it, _ = gmres(lambda v: S.system @ v, make(pv, lambda g: mass_solve_banded(Mq, g), S.B, S.nu), S.rhs,
                         tol=1e-10)
        assert np.linalg.norm(x[:S.nu] - xm[:S.nu]) <= 1e-7 * np.linalg.norm(xm[:S.nu])
        dp = x[S.nu:] - xm[S.nu:]
        assert np.linalg.norm(dp - dp.mean()) <= 1e-6 * np.linalg.norm(xm[S.nu:])
