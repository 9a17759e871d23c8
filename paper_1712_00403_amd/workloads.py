"""Seeded synthetic workloads: problem descriptors and random residual draws.

This module holds no arithmetic of the preconditioner. It only names the
discretisations of each workload (number of elements, spline degree,
regularity, boundary treatment, direction weights) and draws the seeded
Gaussian residuals; the sizes n_k of the spaces are computed by whoever
assembles the univariate factors and passed back in.

Conventions (Sec. 7 of the paper): p is the pressure degree, the
regularity is alpha = p - 1, the Taylor-Hood velocity has degree p + 1 with
homogeneous Dirichlet conditions (first and last univariate function
dropped), the pressure space has degree p and no boundary condition.
"""
from dataclasses import dataclass, field
from typing import Callable, List, Optional, Tuple

import numpy as np


@dataclass(frozen=True)
class Factor1D:
    """One univariate space: uniform mesh of [0,1] with n_el elements.

    ``nitsche`` > 0 names the penalty C_pen of a Nitsche-modified stiffness
    factor (the RT blocks' K~ over all functions of the space); 0 for the
    plain stiffness.
    """
    n_el: int
    degree: int
    regularity: int
    dirichlet: bool
    nitsche: float = 0.0


@dataclass(frozen=True)
class BlockSpec:
    """One diagonal block of P_D: per-direction spaces and Kronecker-sum weights.

    ``mass_only`` marks the pressure block P_Q = M_d (x) .. (x) M_1.
    """
    name: str
    dirs: Tuple[Factor1D, ...]
    weights: Tuple[float, ...]
    mass_only: bool


@dataclass(frozen=True)
class Problem:
    """A Taylor-Hood or Raviart-Thomas patch: d velocity blocks then the pressure block."""
    ndim: int
    n_el: Tuple[int, ...]
    p: int
    blocks: Tuple[BlockSpec, ...]


def taylor_hood_problem(n_el, p, unit_weights=False):
    """Blocks of P_D for a TH patch with ``n_el`` elements per direction.

    Velocity block k carries weight 2 on direction k (the simple TH velocity
    block of the paper) unless ``unit_weights`` (plain K(x)M + M(x)K sum).
    """
    n_el = tuple(int(x) for x in n_el)
    d = len(n_el)
    vel = tuple(Factor1D(n_el[i], p + 1, p - 1, True) for i in range(d))
    pres = tuple(Factor1D(n_el[i], p, p - 1, False) for i in range(d))
    blocks = []
    for k in range(d):
        w = tuple(1.0 if (unit_weights or i != k) else 2.0 for i in range(d))
        blocks.append(BlockSpec(f"u{k + 1}", vel, w, False))
    blocks.append(BlockSpec("p", pres, tuple(1.0 for _ in range(d)), True))
    return Problem(d, n_el, p, tuple(blocks))


def raviart_thomas_problem(n_el, p, c_pen=None):
    """Blocks of P_D for an RT patch (Sec. 2.2.2, eq. prec3D_RT) with ``n_el`` elements per direction.

    Velocity block k: direction k has degree p + 1, regularity p (alpha + 1)
    and drops its first and last function (normal component zero on the
    faces normal to e_k), with weight 2; every other direction has degree p,
    regularity p - 1 and all functions, with the Nitsche factor of penalty
    c_pen (default 5 (alpha + 1) = 5 p, the value of the experiments).
    The pressure block is that of TH (degree p, regularity p - 1).
    """
    n_el = tuple(int(x) for x in n_el)
    d = len(n_el)
    c = 5.0 * p if c_pen is None else float(c_pen)
    blocks = []
    for k in range(d):
        dirs = tuple(Factor1D(n_el[j], p + 1, p, True) if j == k else Factor1D(n_el[j], p, p - 1, False, c)
                     for j in range(d))
        blocks.append(BlockSpec(f"u{k + 1}", dirs, tuple(2.0 if j == k else 1.0 for j in range(d)), False))
    pres = tuple(Factor1D(n_el[i], p, p - 1, False) for i in range(d))
    blocks.append(BlockSpec("p", pres, tuple(1.0 for _ in range(d)), True))
    return Problem(d, n_el, p, tuple(blocks))


# Named workloads. Sizes (n_V = 2 n_el + p - 2, n_Q = n_el + p per direction)
# follow from the spaces; they are not stored here.
CONFIGS = {
    # 2D unit square, 16x16 elements, p = 2, unit-weight velocity sums, FP64, 4 residuals.
    "2d_16_p2_4rhs": dict(problem=lambda: taylor_hood_problem((16, 16), 2, unit_weights=True),
                          nrhs=4, seed=0),
    # 3D unit cube, 64^3 elements, p = 3, paper weights, 16 residuals.
    "3d_64_p3_16rhs": dict(problem=lambda: taylor_hood_problem((64, 64, 64), 3), nrhs=16, seed=1),
    # The 2D 16x16 p = 2 patch with 64 residuals for the reduced-precision ladder.
    "2d_16_p2_64rhs": dict(problem=lambda: taylor_hood_problem((16, 16), 2, unit_weights=True),
                           nrhs=64, seed=2),
    # Serving large class: 96^3 elements, p = 4.
    "3d_96_p4_1rhs": dict(problem=lambda: taylor_hood_problem((96, 96, 96), 4), nrhs=1, seed=4),
}


def residuals(seed, nrhs, n_total):
    """nrhs Gaussian residual block vectors of length n_total (FP64, host).

    One draw from numpy's default_rng(seed) in residual-major order.
    """
    rng = np.random.default_rng(seed)
    return rng.standard_normal((int(nrhs), int(n_total)))


def batch_patches(count=256, seed=3):
    """Heterogeneous batch: per patch an anisotropic n_el triple in [8, 48] and p in {2..5}.

    All descriptors are drawn first, in order, from default_rng(seed); the
    residuals of the batch are drawn afterwards from the same generator
    (``batch_residuals``).
    """
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n_el = tuple(int(x) for x in rng.integers(8, 49, 3))
        p = int(rng.choice([2, 3, 4, 5]))
        out.append((n_el, p))
    return out, rng


def batch_residuals(rng, sizes):
    """One Gaussian residual per patch, drawn in patch order after the descriptors."""
    return [rng.standard_normal(int(n)) for n in sizes]


# ---------------------------------------------------------------------------
# Geometries and viscosities for the coefficient-aware blocks. A geometry is
# the parametrisation G of the patch (its map and Jacobian, evaluated at
# parametric points) and the kinematic viscosity nu at physical points. These
# are problem data: the preconditioner only sees their values at quadrature
# points.

@dataclass(frozen=True)
class Geometry:
    """Parametrisation G of the unit square/cube and a viscosity nu(x).

    ``map(eta)`` and ``jacobian(eta)`` take parametric points of shape (P, d);
    ``jacobian`` returns J[p, a, b] = dG_a/deta_b. ``nu(x)`` takes physical
    points (P, d) and returns (P,).
    """
    name: str
    ndim: int
    map: Callable
    jacobian: Callable
    nu: Callable


def _const_nu(c):
    return lambda x: np.full(x.shape[0], float(c))


def identity_geometry(ndim, nu=None):
    """G = id with nu = 1 unless given."""
    return Geometry("identity", ndim, lambda e: np.array(e, dtype=np.float64),
                    lambda e: np.broadcast_to(np.eye(ndim), (e.shape[0], ndim, ndim)).copy(),
                    nu or _const_nu(1.0))


def affine_geometry(A, nu=None):
    """G(eta) = A eta (constant Jacobian A)."""
    A = np.array(A, dtype=np.float64)
    d = A.shape[0]
    return Geometry("affine", d, lambda e: e @ A.T,
                    lambda e: np.broadcast_to(A, (e.shape[0], d, d)).copy(), nu or _const_nu(1.0))


def sine_geometry(ndim, amp=0.1, nu=None):
    """Axis-separable map G(eta)_j = eta_j + amp sin(pi eta_j).

    The Jacobian is diagonal with entries 1 + amp pi cos(pi eta_j) (positive
    for amp < 1/pi). Default viscosity: nu(x) = 1 + 0.5 sin(2 pi x_1) cos(2 pi x_2).
    """
    def jac(e):
        J = np.zeros((e.shape[0], ndim, ndim))
        for j in range(ndim):
            J[:, j, j] = 1.0 + amp * np.pi * np.cos(np.pi * e[:, j])
        return J
    return Geometry("sine", ndim, lambda e: e + amp * np.sin(np.pi * e), jac, nu or wavy_viscosity)


def wavy_viscosity(x):
    """nu(x) = 1 + 0.5 sin(2 pi x_1) cos(2 pi x_2): positive, not separable."""
    return 1.0 + 0.5 * np.sin(2.0 * np.pi * x[:, 0]) * np.cos(2.0 * np.pi * x[:, 1])


def separable_viscosity(x):
    """nu(x) = (1 + x_1^2) exp(x_2) (2 + x_3): a product of one-variable factors."""
    v = (1.0 + x[:, 0] ** 2) * np.exp(x[:, 1])
    if x.shape[1] > 2:
        v = v * (2.0 + x[:, 2])
    return v


def warped_geometry(ndim, nu=None):
    """A curved map with a full, varying Jacobian (off-diagonal coefficients).

    2D: G = (eta_1 + 0.1 eta_2^2, eta_2 + 0.05 sin(pi eta_1));
    3D adds G_3 = eta_3 (1 + 0.1 eta_1).
    """
    def gmap(e):
        x = np.array(e, dtype=np.float64)
        x[:, 0] = e[:, 0] + 0.1 * e[:, 1] ** 2
        x[:, 1] = e[:, 1] + 0.05 * np.sin(np.pi * e[:, 0])
        if ndim == 3:
            x[:, 2] = e[:, 2] * (1.0 + 0.1 * e[:, 0])
        return x

    def jac(e):
        J = np.zeros((e.shape[0], ndim, ndim))
        J[:, 0, 0] = 1.0
        J[:, 0, 1] = 0.2 * e[:, 1]
        J[:, 1, 0] = 0.05 * np.pi * np.cos(np.pi * e[:, 0])
        J[:, 1, 1] = 1.0
        if ndim == 3:
            J[:, 2, 0] = 0.1 * e[:, 2]
            J[:, 2, 2] = 1.0 + 0.1 * e[:, 0]
        return J
    return Geometry("warped", ndim, gmap, jac, nu or _const_nu(1.0))


def tensor_points(axes):
    """All points of the tensor grid of 1D point arrays ``axes``, axis 1 fastest: (P, d)."""
    grids = np.meshgrid(*axes, indexing="ij")
    return np.stack([g.reshape(-1, order="F") for g in grids], axis=1)
