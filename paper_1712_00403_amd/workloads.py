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
from typing import List, Optional, Tuple

import numpy as np


@dataclass(frozen=True)
class Factor1D:
    """One univariate space: uniform mesh of [0,1] with n_el elements."""
    n_el: int
    degree: int
    regularity: int
    dirichlet: bool


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
    """A Taylor-Hood patch: d velocity blocks then the pressure block."""
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


# Named workloads. Sizes (n_V = 2 n_el + p - 2, n_Q = n_el + p per direction)
# follow from the spaces; they are not stored here.
CONFIGS = {
    # 2D unit square, 16x16 elements, p = 2, unit-weight velocity sums, FP64, 4 residuals.
    "c1_2d_16_p2": dict(problem=lambda: taylor_hood_problem((16, 16), 2, unit_weights=True),
                        nrhs=4, seed=0),
    # 3D unit cube, 64^3 elements, p = 3, paper weights, 16 residuals.
    "c2_3d_64_p3": dict(problem=lambda: taylor_hood_problem((64, 64, 64), 3), nrhs=16, seed=1),
    # Config-1 geometry with 64 residuals for the reduced-precision ladder.
    "c3_2d_16_p2": dict(problem=lambda: taylor_hood_problem((16, 16), 2, unit_weights=True),
                        nrhs=64, seed=2),
    # Serving large class: 96^3 elements, p = 4.
    "c5_3d_96_p4": dict(problem=lambda: taylor_hood_problem((96, 96, 96), 4), nrhs=1, seed=4),
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
