"""Host-side checks of libfd that need no GPU: exports, assembly, eigensolve, errors.

The library's own B-spline assembly and FP64 eigensolve are separate code from
the oracle; here both are compared on the CPU.
"""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle.assemble import assemble_1d as oracle_assemble
from oracle.bspline import element_quadrature
from oracle.geneig import generalized_eig

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def fd():
    from paper_1712_00403_amd import fd as _fd
    if not os.path.exists(_fd.LIB_PATH):
        pytest.skip("libfd.so not built")
    return _fd


def test_exports_match_header(fd):
    hdr = open(os.path.join(ROOT, "include", "fd.h")).read()
    declared = set(re.findall(r"\b(fd_[a-z0-9_]+)\s*\(", hdr))
    assert declared == set(fd.EXPORTS)
    L = ctypes.CDLL(fd.LIB_PATH)
    for name in declared:
        assert hasattr(L, name), name


def test_workspace_query_is_zero(fd):
    # every pass after the first runs in place on z: no device workspace per apply
    L = fd.lib()
    for nrhs in (1, 16, 1024):
        assert L.fd_workspace_bytes(None, nrhs) == 0


@pytest.mark.parametrize("n_el,deg,reg,bc", [(16, 3, 1, True), (64, 4, 2, True), (67, 3, 2, False),
                                             (5, 1, 0, True), (9, 6, 4, False), (3, 2, -1, False)])
def test_assembly_matches_oracle(fd, n_el, deg, reg, bc):
    K, M = fd.assemble_1d(n_el, deg, reg, bc)
    Ko, Mo = oracle_assemble(n_el, deg, reg, bc)
    assert K.shape == Ko.shape
    assert np.abs(K - Ko).max() <= 1e-13 * np.abs(Ko).max()
    assert np.abs(M - Mo).max() <= 1e-13 * np.abs(Mo).max()


def test_weighted_assembly_matches_oracle(fd):
    n_el, deg = 7, 4
    xq, _ = element_quadrature(n_el, deg + 1)
    tau = 1.0 + 0.3 * np.sin(3 * xq)
    mu = 2.0 + np.cos(xq)
    K, M = fd.assemble_1d(n_el, deg, deg - 2, True, tau=tau, mu=mu)
    Ko, Mo = oracle_assemble(n_el, deg, deg - 2, True, tau=tau, mu=mu)
    assert np.allclose(K, Ko, rtol=0, atol=1e-13 * np.abs(Ko).max())
    assert np.allclose(M, Mo, rtol=0, atol=1e-13 * np.abs(Mo).max())


def test_quadrature_matches_oracle(fd):
    x, w = fd.quadrature_1d(5, 7)
    xo, wo = element_quadrature(5, 7)
    assert np.allclose(x, xo, atol=1e-15) and np.allclose(w, wo, atol=1e-16)


@pytest.mark.parametrize("n_el,p", [(16, 2), (64, 3), (20, 5)])
def test_factor_properties(fd, n_el, p):
    K, M = fd.assemble_1d(n_el, p + 1, p - 1, True)
    U, d = fd.factor_1d(K, M)
    n = K.shape[0]
    assert np.allclose(U.T @ M @ U, np.eye(n), atol=1e-12)
    assert np.abs(U.T @ K @ U - np.diag(d)).max() <= 1e-12 * d.max()
    Uo, do = generalized_eig(K, M)
    assert np.all(np.abs(d - do) <= 1e-11 * do)


def test_factor_mass_only(fd):
    _, M = fd.assemble_1d(9, 3, 2, False)
    U, d = fd.factor_1d(None, M)
    assert np.all(d == 0.0)
    assert np.allclose(U @ U.T, np.linalg.inv(M), rtol=1e-10, atol=1e-10 * np.abs(np.linalg.inv(M)).max())


def test_factor_errors(fd):
    K, M = fd.assemble_1d(6, 2, 1, True)
    Mbad = M.copy()
    Mbad[0, 0] = -1.0
    with pytest.raises(fd.FDError) as e:
        fd.factor_1d(K, Mbad)
    assert e.value.status == fd.FD_E_NOTSPD
    Kasym = K.copy()
    Kasym[0, 1] += 1e-3
    with pytest.raises(fd.FDError) as e:
        fd.factor_1d(Kasym, M)
    assert e.value.status == fd.FD_E_ARG
    with pytest.raises(fd.FDError) as e:
        fd.assemble_1d(0, 2, 1, True)
    assert e.value.status == fd.FD_E_ARG
    with pytest.raises(fd.FDError) as e:
        fd.assemble_1d(4, 2, 2, True)  # regularity must be < degree
    assert e.value.status == fd.FD_E_ARG


def test_taylor_hood_sizes_from_library(fd):
    # 64^3, p = 3: 129 velocity and 67 pressure functions per direction; 96^3, p = 4: 194 / 100
    assert fd.assemble_1d(64, 4, 2, True)[0].shape[0] == 129
    assert fd.assemble_1d(64, 3, 2, False)[0].shape[0] == 67
    assert fd.assemble_1d(96, 5, 3, True)[0].shape[0] == 194
    assert fd.assemble_1d(96, 4, 3, False)[0].shape[0] == 100


@pytest.mark.parametrize("n_el,deg,reg", [(1, 1, 0), (4, 2, 1), (7, 3, 2), (5, 4, 3), (3, 5, 2), (16, 3, 1)])
def test_nitsche_stiffness_matches_oracle(fd, n_el, deg, reg):
    """The library's K~ of the RT blocks against the oracle's (both from the definition below eq. prec3D_RT)."""
    from oracle.assemble import nitsche_stiffness_1d
    c = 5.0 * (reg + 1)
    K = fd.nitsche_stiffness_1d(n_el, deg, reg, c)
    Ko = nitsche_stiffness_1d(n_el, deg, reg, c)
    np.testing.assert_allclose(K, Ko, rtol=0, atol=1e-12 * np.abs(Ko).max())
    with pytest.raises(fd.FDError):
        fd.nitsche_stiffness_1d(n_el, deg, reg, -1.0)


def test_raviart_thomas_sizes_from_library(fd):
    """RT block sizes: n_el + p - 1 in the component's own direction, n_el + p in the others."""
    from paper_1712_00403_amd import workloads
    from paper_1712_00403_amd.precond import block_factors
    prob = workloads.raviart_thomas_problem((5, 7, 6), 3)
    for k in range(3):
        Ks, Ms = block_factors(prob.blocks[k])
        assert [M.shape[0] for M in Ms] == [n + 3 - 1 if j == k else n + 3 for j, n in enumerate((5, 7, 6))]
        assert [K.shape[0] for K in Ks] == [M.shape[0] for M in Ms]
    _, Mp = block_factors(prob.blocks[3])
    assert [M.shape[0] for M in Mp] == [8, 10, 9]


@pytest.mark.parametrize("n_el,p", [(3, 2), (5, 3), (2, 5)])
def test_mixed_integrals_match_oracle(fd, n_el, p):
    """fd_mixed_1d: the Stokes cube's univariate factors against the oracle's (velocity derivative x value,
    pressure x velocity derivative, pressure x velocity)."""
    from oracle.stokes import univariate
    f = univariate(n_el, p)
    C = fd.mixed_1d(n_el, p + 1, p - 1, 1, p + 1, p - 1, 0)
    D = fd.mixed_1d(n_el, p, p - 1, 0, p + 1, p - 1, 1)
    N = fd.mixed_1d(n_el, p, p - 1, 0, p + 1, p - 1, 0)
    for X, name in ((C, "CV"), (D, "DQ"), (N, "NQ")):
        np.testing.assert_allclose(X, f[name], rtol=0, atol=1e-13 * np.abs(f[name]).max())
    K, M = fd.assemble_1d(n_el, p + 1, p - 1, False)
    np.testing.assert_allclose(fd.mixed_1d(n_el, p + 1, p - 1, 1, p + 1, p - 1, 1), K, rtol=0, atol=1e-12)
    with pytest.raises(fd.FDError):
        fd.mixed_1d(n_el, p, p - 1, 2, p, p - 1, 0)


def test_device_limit_entry_points_without_allocations(fd):
    # (no device here: nothing is held, and setting or clearing the cap always succeeds)
    assert fd.device_bytes_held() == 0
    fd.set_device_limit(1 << 20)
    fd.set_device_limit(0)
    assert fd.device_bytes_held() == 0
