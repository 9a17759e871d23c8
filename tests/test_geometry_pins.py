"""Pins of the coefficient-aware oracle (Sec. 6 and Appendix) against closed forms,
hand-worked values and brute-force assembly."""
import os

import numpy as np
import pytest

from oracle import brute
from oracle.assemble import pressure_1d, taylor_hood_velocity_1d
from oracle.fd import FDFactors, block_apply, fd_apply, velocity_weights
from oracle.geometry import (GeometryBlocks, _grid_fields, _space_tables, coefficient_matrices,
                             grid_axes, operator_diagonal, pressure_weight, separable_factors,
                             separable_fit)
from paper_1712_00403_amd import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b)


def test_coefficients_hand_worked_2d():
    rows = np.loadtxt(os.path.join(GOLDEN, "geometry_coefficients_2d.txt"))
    J = np.array([[[2.0, 1.0], [0.0, 1.0]]] * len(rows))
    C = coefficient_matrices(J, rows[:, 0])
    for r, row in enumerate(rows):
        assert np.allclose(C[0, r].ravel(), row[1:5], rtol=0, atol=1e-14)
        assert np.allclose(C[1, r].ravel(), row[5:9], rtol=0, atol=1e-14)
    assert np.allclose(pressure_weight(J, rows[:, 0]), rows[:, 9], rtol=1e-15)


def test_coefficients_rotation():
    """J = R orthogonal: J^{-1}J^{-T} = I, |det| = 1, D_k = R^T e_k."""
    a, b = 0.3, -0.7
    Rz = np.array([[np.cos(a), -np.sin(a), 0], [np.sin(a), np.cos(a), 0], [0, 0, 1]])
    Rx = np.array([[1, 0, 0], [0, np.cos(b), -np.sin(b)], [0, np.sin(b), np.cos(b)]])
    R = Rz @ Rx
    C = coefficient_matrices(R[None], np.array([1.0]))
    for k in range(3):
        v = R[k, :]  # R^T e_k
        assert np.allclose(C[k, 0], np.eye(3) + np.outer(v, v), atol=1e-14)
        # R is not symmetric, so using R e_k would differ
        assert not np.allclose(C[k, 0], np.eye(3) + np.outer(R[:, k], R[:, k]), atol=1e-3)


def test_coefficients_axis_scaling():
    L = np.array([2.0, 0.5, 3.0])
    C = coefficient_matrices(np.diag(L)[None], np.array([1.7]))
    for k in range(3):
        want = 1.7 * np.prod(L) * (np.diag(1.0 / L ** 2) + np.diag(np.eye(3)[k]) / L[k] ** 2)
        assert np.allclose(C[k, 0], want, rtol=1e-15, atol=0)


def test_separable_fit_exact_on_separable_field():
    rng = np.random.default_rng(5)
    g = [rng.standard_normal(n) for n in (7, 5, 9)]
    F = g[0][:, None, None] + g[1][None, :, None] + g[2][None, None, :]
    f = separable_fit(F)
    R = F - (f[0][:, None, None] + f[1][None, :, None] + f[2][None, None, :])
    assert np.max(np.abs(R)) < 1e-13


def test_separable_fit_midrange_fixed_point():
    """At convergence every slice of the residual has max = -min (the midrange condition)."""
    rng = np.random.default_rng(6)
    F = rng.standard_normal((6, 7, 5))
    f = separable_fit(F, sweeps=500, tol=1e-15)
    R = F - (f[0][:, None, None] + f[1][None, :, None] + f[2][None, None, :])
    for ax in range(3):
        other = tuple(a for a in range(3) if a != ax)
        assert np.max(np.abs(R.max(axis=other) + R.min(axis=other))) < 1e-9


def test_separable_fit_reaches_best_sup_error_for_xy():
    """x y on a grid containing the corners of [0,1]^2: no g(x)+h(y) is closer than 1/4 in
    max norm (the alternating corner sum of g+h vanishes, that of xy is 1); the iteration
    attains 1/4."""
    x = np.linspace(0.0, 1.0, 11)
    F = np.outer(x, np.linspace(0.0, 1.0, 8))
    f = separable_fit(F)
    R = F - (f[0][:, None] + f[1][None, :])
    assert abs(np.max(np.abs(R)) - 0.25) < 1e-14


def test_separable_factors_exact_products():
    """c_jj = a_j * prod of one-variable factors that agree between entries: recovered exactly."""
    rng = np.random.default_rng(7)
    shape = (6, 4, 5)
    phi = [np.exp(0.3 * rng.standard_normal(n)) for n in shape]     # shared axis factors
    psi = [np.exp(0.3 * rng.standard_normal(n)) for n in shape]     # tau-axis factors
    cdiag = []
    for j in range(3):
        c = np.ones(shape)
        for i in range(3):
            v = psi[i] if i == j else phi[i]
            s = [1, 1, 1]
            s[i] = -1
            c = c * v.reshape(s)
        cdiag.append(c * (1.0 + j))
    tau, mu = separable_factors(cdiag)
    for j in range(3):
        approx = np.ones(shape)
        for i in range(3):
            s = [1, 1, 1]
            s[i] = -1
            approx = approx * (tau[i] if i == j else mu[i]).reshape(s)
        assert np.max(np.abs(approx / cdiag[j] - 1.0)) < 1e-13


def _vel_tables(n_el, p):
    return _space_tables(n_el, p + 1, p - 1, True, p + 2), [w for _, w in grid_axes(n_el, p + 2)]


def _full_A(n_el, p, geometry, k):
    """A_kk by brute-force assembly with the full C_k."""
    tabs, wts = _vel_tables(n_el, p)
    J, nu, shape = _grid_fields(geometry, n_el, p + 2)
    C = coefficient_matrices(J, nu)
    d = len(n_el)
    coef = np.stack([np.stack([C[k, :, a, b] for b in range(d)]) for a in range(d)])
    return brute.coefficient_operator(tabs, wts, coef, 1)


def test_identity_geometry_reduces_to_simple_blocks():
    n_el, p = (3, 4, 2), 2
    gb = GeometryBlocks(n_el, p, workloads.identity_geometry(3))
    vel = [taylor_hood_velocity_1d(n, p) for n in n_el]
    for k in range(3):
        for j in range(3):
            assert np.allclose(gb.tau[k][j], 1.0 + (j == k), rtol=0, atol=1e-14)
            assert np.allclose(gb.mu[k][j], 1.0, rtol=0, atol=1e-14)
            assert np.allclose(gb.vel_K[k][j], (1.0 + (j == k)) * vel[j][0], rtol=0, atol=1e-12)
            assert np.allclose(gb.vel_M[k][j], vel[j][1], rtol=0, atol=1e-14)
        assert np.allclose(gb.vel_scales[k], 1.0, rtol=0, atol=1e-12)
    assert np.allclose(gb.pres_scale, 1.0, rtol=0, atol=1e-12)
    # and the scaled block apply equals the simple one
    r = workloads.residuals(3, 1, 3 * np.prod([v[0].shape[0] for v in vel])
                            + np.prod([pressure_1d(n, p).shape[0] for n in n_el]))[0]
    facs_g = [FDFactors(gb.vel_K[k], gb.vel_M[k]) for k in range(3)]
    facs_s = [FDFactors([v[0] for v in vel], [v[1] for v in vel], velocity_weights(3, k)) for k in range(3)]
    zg = block_apply(facs_g, gb.pres_M, r, pres_scale=gb.pres_scale, vel_scales=gb.vel_scales)
    zs = block_apply(facs_s, [pressure_1d(n, p) for n in n_el], r)
    assert _rel(zg, zs) < 1e-12


def test_axis_scaling_geometry_is_exact():
    """G = diag(L) eta, constant nu: C_k is a constant diagonal, P_breve_k = A_kk and D_V = I."""
    n_el, p = (2, 3, 2), 1
    L = np.diag([1.5, 0.7, 1.2])
    geo = workloads.affine_geometry(L, nu=lambda x: np.full(x.shape[0], 2.5))
    gb = GeometryBlocks(n_el, p, geo)
    for k in range(3):
        A = _full_A(n_el, p, geo, k)
        P = brute.assemble_operator(gb.vel_K[k], gb.vel_M[k]).toarray()
        assert np.max(np.abs(A - P)) < 1e-12 * np.max(np.abs(A))
        assert np.allclose(gb.vel_scales[k], 1.0, rtol=0, atol=1e-12)
        # closed form: K^k_j = c^k_jj K_j with c^k_jj = 2.5 det(L) (1 + delta_jk) / L_j^2
        Ls = np.diag(L)
        for j in range(3):
            cjj = 2.5 * np.prod(Ls) * (1.0 + (j == k)) / Ls[j] ** 2
            K1 = taylor_hood_velocity_1d(n_el[j], p)[0]
            # the constant may sit in tau or be split with mu; the product is fixed
            KM = gb.vel_K[k][j][0, 0] * np.prod([gb.vel_M[k][i][0, 0] for i in range(3) if i != j])
            ref = cjj * K1[0, 0] * np.prod([taylor_hood_velocity_1d(n_el[i], p)[1][0, 0]
                                            for i in range(3) if i != j])
            assert abs(KM / ref - 1.0) < 1e-13


def test_separable_geometry_and_viscosity_are_exact():
    """Axis-separable map and product viscosity: every c^k_jj separates, so P_breve_k = A_kk."""
    n_el, p = (3, 2, 2), 1
    geo = workloads.sine_geometry(3, nu=workloads.separable_viscosity)
    gb = GeometryBlocks(n_el, p, geo)
    for k in range(3):
        A = _full_A(n_el, p, geo, k)
        P = brute.assemble_operator(gb.vel_K[k], gb.vel_M[k]).toarray()
        assert np.max(np.abs(A - P)) < 1e-12 * np.max(np.abs(A))
        assert np.allclose(gb.vel_scales[k], 1.0, rtol=0, atol=1e-12)


@pytest.mark.parametrize("ndim", [2, 3])
def test_operator_diagonal_matches_brute_force(ndim):
    n_el = (3, 2, 2)[:ndim]
    p = 2
    geo = workloads.warped_geometry(ndim, nu=workloads.wavy_viscosity)
    gb = GeometryBlocks(n_el, p, geo)
    for k in range(ndim):
        A = _full_A(n_el, p, geo, k)
        assert np.allclose(A, A.T, atol=1e-13 * np.max(np.abs(A)))
        assert np.min(np.linalg.eigvalsh(A)) > 0
        assert _rel(gb.diagA[k], np.diag(A)) < 1e-13
        # the diagonal of the Kronecker sum of the weighted pairs
        P = brute.assemble_operator(gb.vel_K[k], gb.vel_M[k]).toarray()
        assert _rel(gb.diagP[k], np.diag(P)) < 1e-13
    # pressure: Q with weight nu^{-1} |det J|
    tabs = _space_tables(n_el, p, p - 1, False, p + 1)
    wts = [w for _, w in grid_axes(n_el, p + 1)]
    J, nu, _ = _grid_fields(geo, n_el, p + 1)
    Q = brute.coefficient_operator(tabs, wts, pressure_weight(J, nu), 0)
    assert _rel(gb.diagQ, np.diag(Q)) < 1e-13
    PQ = brute.assemble_operator(None, gb.pres_M).toarray()
    assert _rel(gb.diagPQ, np.diag(PQ)) < 1e-13


def test_geometry_block_apply_matches_brute_force_solve():
    """z = D^{-1/2} P_breve^{-1} D^{-1/2} r by FD against the dense solve of the assembled block."""
    n_el, p = (2, 3, 2), 2
    geo = workloads.warped_geometry(3, nu=workloads.wavy_viscosity)
    gb = GeometryBlocks(n_el, p, geo)
    sizes = [int(np.prod([K.shape[0] for K in gb.vel_K[k]])) for k in range(3)]
    NQ = int(np.prod([M.shape[0] for M in gb.pres_M]))
    r = workloads.residuals(8, 1, sum(sizes) + NQ)[0]
    facs = [FDFactors(gb.vel_K[k], gb.vel_M[k]) for k in range(3)]
    z = block_apply(facs, gb.pres_M, r, pres_scale=gb.pres_scale, vel_scales=gb.vel_scales)
    off = 0
    for k in range(3):
        zk = brute.solve(gb.vel_K[k], gb.vel_M[k], r[off:off + sizes[k]], scale=gb.vel_scales[k])
        assert _rel(z[off:off + sizes[k]], zk) < 1e-12
        off += sizes[k]
    zq = brute.solve(None, gb.pres_M, r[off:], scale=gb.pres_scale)
    assert _rel(z[off:], zq) < 1e-12
    # the scaling is not trivial here
    assert np.max(np.abs(gb.vel_scales[0] - 1.0)) > 1e-3


def test_tensor_grid_order_matches_nested_loops():
    """The oracle's quadrature grid lists points with axis 1 fastest (brute force on a tiny grid)."""
    from oracle.geometry import tensor_grid
    ax = [np.array([0.1, 0.2]), np.array([1.0, 2.0, 3.0]), np.array([7.0, 8.0])]
    expect = [(a, b, c) for c in ax[2] for b in ax[1] for a in ax[0]]
    assert np.array_equal(tensor_grid(ax), np.array(expect))
    assert np.array_equal(tensor_grid(ax[:2]), np.array([(a, b) for b in ax[1] for a in ax[0]]))
