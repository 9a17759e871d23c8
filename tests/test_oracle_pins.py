"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

None of these tests use the HIP library. Each pin is chosen so that a
plausible slip in the oracle (a dropped term, a wrong index or sign, a
transposed operand, a wrong Kronecker ordering) fails at least one of them.
"""
import math

import numpy as np
import pytest
import scipy.linalg

from oracle import brute
from oracle.assemble import assemble_1d, pressure_1d, taylor_hood_velocity_1d
from oracle.bspline import (basis_derivatives, basis_values, element_quadrature,
                            gauss_legendre, open_uniform_knots, space_dim)
from oracle.fd import (FDFactors, apply_operator, block_apply, fd_apply,
                       mass_solve_banded, mode_product, unvec, vec, velocity_weights)
from oracle.geneig import generalized_eig, jacobi_eigh

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


# ---------------------------------------------------------------- knots / spaces

@pytest.mark.parametrize("n_el,p", [(1, 2), (4, 2), (16, 2), (64, 3), (96, 4), (7, 5)])
def test_taylor_hood_dimensions(n_el, p):
    # dim = (degree + 1) + mult * (n_el - 1); velocity: degree p+1, mult 2, minus 2 Dirichlet
    vk = open_uniform_knots(n_el, p + 1, p - 1)
    pk = open_uniform_knots(n_el, p, p - 1)
    assert space_dim(vk, p + 1) - 2 == 2 * n_el + p - 2
    assert space_dim(pk, p) == n_el + p
    K, M = taylor_hood_velocity_1d(n_el, p)
    assert K.shape == M.shape == (2 * n_el + p - 2,) * 2
    assert pressure_1d(n_el, p).shape == (n_el + p,) * 2


def test_config_sizes():
    # 64^3, p=3: 129 velocity and 67 pressure functions per direction
    assert taylor_hood_velocity_1d(64, 3)[0].shape[0] == 129
    assert pressure_1d(64, 3).shape[0] == 67
    assert taylor_hood_velocity_1d(16, 2)[0].shape[0] == 32
    assert pressure_1d(16, 2).shape[0] == 18


@pytest.mark.parametrize("deg,reg,n_el", [(1, 0, 5), (2, 1, 4), (3, 1, 3), (4, 2, 6), (5, 4, 3), (6, 4, 2)])
def test_partition_of_unity_and_support(deg, reg, n_el):
    kn = open_uniform_knots(n_el, deg, reg)
    x = np.linspace(0.0, 1.0, 97)
    B = basis_values(kn, deg, x)
    assert np.allclose(B.sum(axis=0), 1.0, atol=1e-14)
    assert np.all(B >= -1e-15)
    # each B-spline vanishes outside [xi_i, xi_{i+deg+1}]
    for i in range(B.shape[0]):
        out = (x < kn[i]) | (x > kn[i + deg + 1])
        assert np.all(np.abs(B[i, out]) < 1e-15)
    # derivatives of a partition of unity sum to zero
    assert np.allclose(basis_derivatives(kn, deg, x).sum(axis=0), 0.0, atol=1e-11)


@pytest.mark.parametrize("deg,reg,n_el", [(2, 1, 3), (3, 2, 4), (4, 1, 2)])
def test_derivative_matches_finite_difference(deg, reg, n_el):
    kn = open_uniform_knots(n_el, deg, reg)
    # points away from breakpoints
    x = (np.arange(n_el)[:, None] + np.array([0.21, 0.5, 0.77])[None, :]).ravel() / n_el
    h = 1e-6
    fd = (basis_values(kn, deg, x + h) - basis_values(kn, deg, x - h)) / (2 * h)
    assert np.allclose(basis_derivatives(kn, deg, x), fd, atol=1e-6 * n_el)


def test_gauss_legendre_exactness():
    x, w = element_quadrature(3, 4)  # 4 points exact up to degree 7
    for k in range(8):
        assert abs(np.sum(w * x ** k) - 1.0 / (k + 1)) < 1e-15


# ---------------------------------------------------------------- 1D matrices

@pytest.mark.parametrize("n", [1, 2, 3, 5, 6])
def test_single_element_is_bernstein(n):
    """One element: the B-splines are the Bernstein polynomials of degree n.

    Closed forms: int B_i B_j = C(n,i)C(n,j) / ((2n+1) C(2n,i+j)), and with
    B_i' = n (B_{i-1}^{n-1} - B_i^{n-1}), K = n^2 D M^{n-1} D^T.
    """
    def bern_mass(n):
        return np.array([[math.comb(n, i) * math.comb(n, j) / ((2 * n + 1) * math.comb(2 * n, i + j))
                          for j in range(n + 1)] for i in range(n + 1)])
    K, M = assemble_1d(1, n, -1, False)
    assert np.allclose(M, bern_mass(n), rtol=0, atol=1e-15)
    D = np.zeros((n + 1, n))
    for i in range(n + 1):
        if i - 1 >= 0:
            D[i, i - 1] = n
        if i < n:
            D[i, i] = -n
    Kc = D @ bern_mass(n - 1) @ D.T
    assert np.allclose(K, Kc, rtol=0, atol=1e-13 * n * n)


@pytest.mark.parametrize("n_el", [2, 5, 9])
def test_degree1_closed_form_matrices(n_el):
    h = 1.0 / n_el
    K, M = assemble_1d(n_el, 1, 0, True)
    m = n_el - 1
    T = np.diag(np.full(m, 2.0)) - np.diag(np.ones(m - 1), 1) - np.diag(np.ones(m - 1), -1)
    S = np.diag(np.full(m, 4.0)) + np.diag(np.ones(m - 1), 1) + np.diag(np.ones(m - 1), -1)
    assert np.allclose(K, T / h, atol=1e-12)
    assert np.allclose(M, S * h / 6.0, atol=1e-15)


@pytest.mark.parametrize("deg,reg,n_el", [(2, 1, 5), (3, 1, 4), (4, 3, 7), (5, 4, 3)])
def test_full_space_mass_and_stiffness_identities(deg, reg, n_el):
    K, M = assemble_1d(n_el, deg, reg, False)
    kn = open_uniform_knots(n_el, deg, reg)
    assert abs(M.sum() - 1.0) < 1e-14                      # int (sum b)^2 = 1
    assert np.allclose(K @ np.ones(K.shape[0]), 0.0, atol=1e-10)  # constants in the kernel
    # int b_l = (xi_{l+deg+1} - xi_l) / (deg + 1)
    integ = (kn[deg + 1:] - kn[:-deg - 1]) / (deg + 1)
    assert np.allclose(M.sum(axis=1), integ, atol=1e-15)
    # symmetric, banded with half-bandwidth deg
    assert np.allclose(K, K.T) and np.allclose(M, M.T)
    for j in range(deg + 1, K.shape[0]):
        assert np.all(np.diag(K, j) == 0.0) and np.all(np.diag(M, j) == 0.0)


# ---------------------------------------------------------------- eigensolve

def test_jacobi_against_library_eigh():
    rng = np.random.default_rng(11)
    A = rng.standard_normal((23, 23))
    A = A + A.T
    d, V = jacobi_eigh(A)
    assert np.allclose(d, np.linalg.eigvalsh(A), atol=1e-12)
    assert np.allclose(V.T @ V, np.eye(23), atol=1e-13)
    assert np.allclose(A @ V, V * d, atol=1e-12)


@pytest.mark.parametrize("n_el", [4, 9, 32])
def test_degree1_closed_form_eigenpairs(n_el):
    h = 1.0 / n_el
    K, M = assemble_1d(n_el, 1, 0, True)
    U, d = generalized_eig(K, M)
    k = np.arange(1, n_el)
    th = k * np.pi / n_el
    lam = 6.0 * (1.0 - np.cos(th)) / (h * h * (2.0 + np.cos(th)))
    assert np.allclose(d, lam, rtol=1e-13)
    # eigenvectors are discrete sines; compare up to sign after M-normalisation
    j = np.arange(1, n_el)
    for c in range(n_el - 1):
        s = np.sin(j * (c + 1) * np.pi / n_el)
        s = s / np.sqrt(s @ M @ s)
        u = U[:, c]
        assert np.allclose(u * np.sign(u @ s), s, atol=1e-11)


@pytest.mark.parametrize("n_el,p", [(4, 2), (8, 3), (16, 2), (5, 5)])
def test_generalized_eig_properties(n_el, p):
    K, M = taylor_hood_velocity_1d(n_el, p)
    U, d = generalized_eig(K, M)
    n = K.shape[0]
    assert np.allclose(U.T @ M @ U, np.eye(n), atol=1e-13)
    assert np.allclose(U.T @ K @ U, np.diag(d), atol=1e-12 * d.max())
    assert np.allclose(d, scipy.linalg.eigh(K, M, eigvals_only=True), rtol=1e-11)
    # Rayleigh-Ritz: discrete Dirichlet eigenvalues bound (k pi)^2 from above
    assert np.all(d >= (np.arange(1, n + 1) * np.pi) ** 2 * (1 - 1e-12))


def test_first_eigenvalue_converges_to_pi_squared():
    errs = []
    for n_el in (4, 8, 16):
        K, M = taylor_hood_velocity_1d(n_el, 2)
        errs.append(generalized_eig(K, M)[1][0] - np.pi ** 2)
    assert errs[0] > errs[1] > errs[2] > 0 and errs[2] < 1e-6


# ---------------------------------------------------------------- FD apply

def _factors_aniso(ns_el, ps, weights=None, mass_only=False):
    Ks, Ms = [], []
    for n_el, p in zip(ns_el, ps):
        if mass_only:
            Ms.append(pressure_1d(n_el, p))
        else:
            K, M = taylor_hood_velocity_1d(n_el, p)
            Ks.append(K)
            Ms.append(M)
    return (None if mass_only else Ks), Ms


def test_mode_product_definition():
    rng = np.random.default_rng(5)
    W = rng.standard_normal((3, 4, 5))
    Y = rng.standard_normal((6, 4))
    out = mode_product(W, Y, 1)
    assert out.shape == (3, 6, 5)
    i1, i2, i3 = 2, 5, 3
    assert abs(out[i1, i2, i3] - sum(Y[i2, k] * W[i1, k, i3] for k in range(4))) < 1e-13
    # vec ordering: i_1 fastest
    assert vec(W)[1 + 3 * 2 + 12 * 4] == W[1, 2, 4]
    # eq. kronvec with direction 1 rightmost
    A, B, C = rng.standard_normal((3, 3)), rng.standard_normal((4, 4)), rng.standard_normal((5, 5))
    lhs = np.kron(C, np.kron(B, A)) @ vec(W)
    rhs = vec(mode_product(mode_product(mode_product(W, A, 0), B, 1), C, 2))
    assert np.allclose(lhs, rhs, atol=1e-12)


@pytest.mark.parametrize("ns_el,ps,weights", [
    ((2, 3, 4), (1, 2, 3), (1.0, 1.0, 1.0)),
    ((3, 2, 2), (2, 2, 2), (1.0, 2.0, 1.0)),
    ((4, 3, 2), (3, 1, 2), (2.0, 1.0, 1.0)),
    ((3, 4), (2, 3), (1.0, 1.0)),
    ((5, 2), (1, 4), (2.0, 1.0)),
])
def test_fd_equals_brute_force(ns_el, ps, weights):
    Ks, Ms = _factors_aniso(ns_el, ps)
    f = FDFactors(Ks, Ms, np.array(weights))
    rng = np.random.default_rng(7)
    N = int(np.prod(f.n))
    r = rng.standard_normal(N)
    z = fd_apply(f, r)
    zb = brute.solve(Ks, Ms, r, np.array(weights))
    assert np.linalg.norm(z - zb) <= 1e-12 * np.linalg.norm(zb)
    # residual check with the operator applied through K, M mode products
    assert np.linalg.norm(apply_operator(f, z) - r) <= 1e-11 * np.linalg.norm(r)


def test_fd_ordering_is_detected():
    """Swapping the Kronecker slot order must break agreement on anisotropic sizes."""
    Ks, Ms = _factors_aniso((2, 3, 4), (1, 2, 3))
    f = FDFactors(Ks, Ms)
    r = np.random.default_rng(3).standard_normal(int(np.prod(f.n)))
    z = fd_apply(f, r)
    P_wrong = brute.kron_list([Ks[0], Ms[1], Ms[2]]) + brute.kron_list([Ms[0], Ks[1], Ms[2]]) \
        + brute.kron_list([Ms[0], Ms[1], Ks[2]])
    assert P_wrong.shape[0] == z.size
    assert np.linalg.norm(P_wrong @ z - r) > 1e-3 * np.linalg.norm(r)


@pytest.mark.parametrize("ns_el,ps", [((3, 4, 2), (2, 3, 1)), ((4, 5), (2, 2)), ((2, 2, 3), (5, 4, 3))])
def test_mass_solve_routes_agree(ns_el, ps):
    _, Ms = _factors_aniso(ns_el, ps, mass_only=True)
    rng = np.random.default_rng(9)
    N = int(np.prod([M.shape[0] for M in Ms]))
    r = rng.standard_normal(N)
    zb = brute.solve(None, Ms, r)
    z1 = mass_solve_banded(Ms, r)
    z2 = fd_apply(FDFactors(None, Ms), r)
    assert np.linalg.norm(z1 - zb) <= 1e-12 * np.linalg.norm(zb)
    assert np.linalg.norm(z2 - zb) <= 1e-12 * np.linalg.norm(zb)


def test_degree1_fd_closed_form():
    """Degree 1 (piecewise linear) 2D FD is fully closed form: discrete sine transform."""
    n_el = (5, 7)
    Ks, Ms = [], []
    for n in n_el:
        K, M = assemble_1d(n, 1, 0, True)
        Ks.append(K)
        Ms.append(M)
    f = FDFactors(Ks, Ms)
    r = np.random.default_rng(1).standard_normal(int(np.prod(f.n)))
    Us, lams = [], []
    for n in n_el:
        h = 1.0 / n
        k = np.arange(1, n)
        j = np.arange(1, n)
        S = np.sin(np.outer(j, k) * np.pi / n)
        Mh = (np.diag(np.full(n - 1, 4.0)) + np.diag(np.ones(n - 2), 1) + np.diag(np.ones(n - 2), -1)) * h / 6
        S = S / np.sqrt(np.einsum("ik,ij,jk->k", S, Mh, S))
        Us.append(S)
        th = k * np.pi / n
        lams.append(6 * (1 - np.cos(th)) / (h * h * (2 + np.cos(th))))
    R = unvec(r, f.n)
    T = Us[0].T @ R @ Us[1]
    T = T / (lams[0][:, None] + lams[1][None, :])
    z_closed = vec(Us[0] @ T @ Us[1].T)
    assert np.allclose(fd_apply(f, r), z_closed, atol=1e-12 * np.abs(z_closed).max())


def test_block_apply_matches_per_block_brute_force():
    n_el, p = (2, 3, 2), 2
    vel = [taylor_hood_velocity_1d(n, p) for n in n_el]
    Ks = [v[0] for v in vel]
    Ms = [v[1] for v in vel]
    Mp = [pressure_1d(n, p) for n in n_el]
    facs = [FDFactors(Ks, Ms, velocity_weights(3, k)) for k in range(3)]
    NV = int(np.prod([K.shape[0] for K in Ks]))
    NQ = int(np.prod([M.shape[0] for M in Mp]))
    r = np.random.default_rng(4).standard_normal(3 * NV + NQ)
    z = block_apply(facs, Mp, r)
    for k in range(3):
        zk = brute.solve(Ks, Ms, r[k * NV:(k + 1) * NV], velocity_weights(3, k))
        assert np.linalg.norm(z[k * NV:(k + 1) * NV] - zk) <= 1e-12 * np.linalg.norm(zk)
    zq = brute.solve(None, Mp, r[3 * NV:])
    assert np.linalg.norm(z[3 * NV:] - zq) <= 1e-12 * np.linalg.norm(zq)
    # velocity block k of the paper: weight 2 sits on the K of direction k
    P1 = brute.assemble_operator(Ks, Ms, velocity_weights(3, 0)).toarray()
    P1_explicit = (brute.kron_list([Ks[2], Ms[1], Ms[0]]) + brute.kron_list([Ms[2], Ks[1], Ms[0]])
                   + 2 * brute.kron_list([Ms[2], Ms[1], Ks[0]])).toarray()
    assert np.allclose(P1, P1_explicit)


def test_scaled_variant_brute_force():
    Ks, Ms = _factors_aniso((2, 3), (2, 2))
    f = FDFactors(Ks, Ms)
    rng = np.random.default_rng(8)
    N = int(np.prod(f.n))
    s = 0.5 + rng.random(N)
    r = rng.standard_normal(N)
    z = s * fd_apply(f, s * r)
    # P^G = D^{1/2} P D^{1/2} with D^{-1/2} = s
    P = brute.assemble_operator(Ks, Ms).toarray()
    PG = np.diag(1 / s) @ P @ np.diag(1 / s)
    assert np.allclose(PG @ z, r, atol=1e-10 * np.abs(r).max())


# ---------------------------------------------------------------- Raviart-Thomas blocks (Sec. 2.2.2, eq. prec3D_RT)

def test_nitsche_stiffness_degree1_by_hand():
    """K~ of degree-1 hat functions, worked by hand from its definition below eq. prec3D_RT.

    Hats on n_el uniform elements (h = 1/n_el), all functions kept: K = h^-1
    tridiag(-1, 2, -1) with end entries 1. End values: b_1(0) = 1,
    b'_1(0) = -1/h, b'_2(0) = 1/h; b_m(1) = 1, b'_m(1) = 1/h, b'_{m-1}(1) = -1/h.
    So K~_11 = K~_mm = (1 - 2 + 2 C) / h and K~_12 = K~_{m-1,m} = (-1 + 1) / h = 0;
    the interior rows are those of K.
    """
    from oracle.assemble import nitsche_stiffness_1d
    n_el, C = 5, 1.75
    h = 1.0 / n_el
    Kt = nitsche_stiffness_1d(n_el, 1, 0, C)
    m = n_el + 1
    E = (np.diag(np.full(m, 2.0)) - np.diag(np.ones(m - 1), 1) - np.diag(np.ones(m - 1), -1)) / h
    E[0, 0] = E[-1, -1] = (2.0 * C - 1.0) / h
    E[0, 1] = E[1, 0] = E[-1, -2] = E[-2, -1] = 0.0
    np.testing.assert_allclose(Kt, E, rtol=0, atol=1e-12 / h)


@pytest.mark.parametrize("deg,reg,n_el", [(2, 1, 4), (3, 2, 3), (3, 1, 5), (4, 3, 2)])
def test_nitsche_stiffness_quadratic_form_of_polynomials(deg, reg, n_el):
    """u^T K~ u = int u'^2 - 2 (u'(1) u(1) - u'(0) u(0)) + 2 (C/h) (u(1)^2 + u(0)^2) for u in the space.

    The coefficients of u = x^2 - 3x + 2 (in every space of degree >= 2) are
    its L2 projection M c = (int b_l u); the right side is evaluated in
    closed form: int (2x - 3)^2 = 13/3, u(0) = 2, u'(0) = -3, u(1) = 0.
    """
    from oracle.assemble import assemble_1d, nitsche_stiffness_1d
    from oracle.bspline import basis_values, element_quadrature, open_uniform_knots
    C = 3.0
    h = 1.0 / n_el
    knots = open_uniform_knots(n_el, deg, reg)
    xq, wq = element_quadrature(n_el, deg + 3)
    B = basis_values(knots, deg, xq.ravel())
    u = xq.ravel() ** 2 - 3 * xq.ravel() + 2
    _, M = assemble_1d(n_el, deg, reg, False)
    c = np.linalg.solve(M, B @ (wq.ravel() * u))
    Kt = nitsche_stiffness_1d(n_el, deg, reg, C)
    expect = 13.0 / 3.0 - 2.0 * (0.0 - (-3.0) * 2.0) + 2.0 * C / h * (0.0 + 4.0)
    assert c @ Kt @ c == pytest.approx(expect, rel=1e-11)


@pytest.mark.parametrize("n_el,p", [((2, 3, 2), 1), ((2, 2, 3), 2), ((3, 2), 2), ((2, 2, 2), 3)])
def test_rt_kronecker_blocks_equal_variational_definition(n_el, p):
    """eq. prec3D_RT (and its 2D analogue) against the block assembled from a^ + sigma^ (eq. precVrt)."""
    from oracle.assemble import raviart_thomas_velocity_1d, rt_penalty
    from oracle.brute import assemble_operator, rt_velocity_block_variational
    for k in range(len(n_el)):
        Ks, Ms, w = raviart_thomas_velocity_1d(n_el, p, k)
        P = assemble_operator(Ks, Ms, w).toarray()
        V = rt_velocity_block_variational(n_el, p, k, rt_penalty(p))
        np.testing.assert_allclose(P, V, rtol=0, atol=1e-10 * np.abs(V).max())


def test_rt_block_with_misplaced_factors_is_detected():
    """Swapping which directions carry the Nitsche factors (or the weight 2) changes the block."""
    from oracle.assemble import raviart_thomas_velocity_1d, rt_penalty
    from oracle.brute import assemble_operator, rt_velocity_block_variational
    n_el, p, k = (2, 3, 2), 2, 0
    V = rt_velocity_block_variational(n_el, p, k, rt_penalty(p))
    Ks, Ms, w = raviart_thomas_velocity_1d(n_el, p, k)
    w_bad = np.roll(w, 1)
    assert np.abs(assemble_operator(Ks, Ms, w_bad).toarray() - V).max() > 1e-3 * np.abs(V).max()
    V_half_pen = rt_velocity_block_variational(n_el, p, k, 0.5 * rt_penalty(p))
    assert np.abs(V_half_pen - V).max() > 1e-3 * np.abs(V).max()


@pytest.mark.parametrize("n_el,p", [((4, 3, 5), 1), ((3, 4, 2), 2), ((2, 3, 3), 3), ((6, 4), 4)])
def test_rt_fd_equals_brute_force(n_el, p):
    """FD (Algorithm 1) on the RT blocks: anisotropic per-direction spaces, solved exactly."""
    from oracle.assemble import raviart_thomas_velocity_1d
    from oracle.brute import solve
    from oracle.fd import FDFactors, fd_apply
    rng = np.random.default_rng(7)
    for k in range(len(n_el)):
        Ks, Ms, w = raviart_thomas_velocity_1d(n_el, p, k)
        f = FDFactors(Ks, Ms, w)
        r = rng.standard_normal(int(np.prod(f.n)))
        z = fd_apply(f, r)
        zb = solve(Ks, Ms, r, w)
        assert np.linalg.norm(z - zb) / np.linalg.norm(zb) < 1e-11


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_rt_nitsche_factor_is_spd_at_the_experiment_penalty(p):
    """With C_pen = 5 (alpha + 1) the Nitsche factor is positive definite (so Lambda > 0)."""
    from oracle.assemble import nitsche_stiffness_1d, rt_penalty
    for n_el in (1, 2, 8, 33):
        Kt = nitsche_stiffness_1d(n_el, p, p - 1, rt_penalty(p))
        assert np.linalg.eigvalsh(0.5 * (Kt + Kt.T)).min() > 0
