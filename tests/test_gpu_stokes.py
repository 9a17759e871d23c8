"""P_D-MINRES, P_T-GMRES and P_C-GMRES on the driven cavity (Sec. 4, Sec. 7 'Cube'), on the GPU.

The Stokes operator runs matrix-free on the device and every preconditioner
block through the library; the iteration counts must equal the oracle's
(which reproduces Table 1 at p = 2 and (n_el, p) = (4, 3)), and the
solutions must agree with the oracle's (velocity; pressure up to its
constant).
"""
import numpy as np
import pytest

from oracle.fd import FDFactors, fd_apply, mass_solve_banded
from oracle.krylov import gmres as oracle_gmres
from oracle.krylov import minres as oracle_minres
from oracle.stokes import CubeStokes as OracleStokes
from oracle.stokes import block_triangular_inverse, constraint_inverse

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _case(msg):
    print(f"[gpu case] {msg}", flush=True)


_OR = {}


def _oracle(n_el, p, method):
    key = (n_el, p, method)
    if key not in _OR:
        S = OracleStokes(n_el, p)
        vel, Mq = S.preconditioner_factors()
        facs = [FDFactors(*v) for v in vel]
        nv = S.nV ** 3

        def pv(r):
            return np.concatenate([fd_apply(facs[k], r[k * nv:(k + 1) * nv]) for k in range(3)])

        def pq(g):
            return mass_solve_banded(Mq, g)

        A = lambda v: S.system @ v
        if method == "minres":
            res = oracle_minres(A, lambda r: np.concatenate([pv(r[:S.nu]), pq(r[S.nu:])]), S.rhs)
        elif method == "gmres_t":
            res = oracle_gmres(A, block_triangular_inverse(pv, pq, S.B, S.nu), S.rhs)
        else:
            res = oracle_gmres(A, constraint_inverse(pv, pq, S.B, S.nu), S.rhs)
        _OR[key] = (S, res)
    return _OR[key]


def test_operator_and_rhs_match_the_oracle():
    _case("cube Stokes operator and cavity right-hand side against the oracle's assembled system")
    from paper_1712_00403_amd.stokes import CubeStokes
    op = CubeStokes(3, 2)
    S = OracleStokes(3, 2)
    rhs = op.rhs.cpu().numpy()
    assert np.allclose(rhs, S.rhs, rtol=0, atol=1e-12 * np.abs(S.rhs).max())
    x = np.random.default_rng(0).standard_normal(S.system.shape[0])
    y = op.apply(torch.from_numpy(x).cuda()).cpu().numpy()
    ref = S.system @ x
    assert np.linalg.norm(y - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("pressure", ["fd", "banded"])
@pytest.mark.parametrize("n_el,p,paper", [(4, 2, 48), (8, 2, 53), (4, 3, 51)])
def test_pd_minres_iterations_and_solution(n_el, p, paper, pressure):
    _case(f"P_D-MINRES on the cavity n_el={n_el} p={p} pressure route={pressure}")
    from paper_1712_00403_amd.stokes import CavitySolver
    S, (xo, it_o, _) = _oracle(n_el, p, "minres")
    sol = CavitySolver(n_el, p, pressure=pressure)
    x, it, _ = sol.solve("minres")
    print(f"  iterations: GPU {it}, oracle {it_o}, Table 1 {paper}")
    assert it_o == paper
    assert it == it_o
    x = x.cpu().numpy()
    assert np.linalg.norm(x[:S.nu] - xo[:S.nu]) <= 1e-6 * np.linalg.norm(xo[:S.nu])
    sol.close()


@pytest.mark.parametrize("method", ["gmres_t", "gmres_c"])
def test_pt_pc_gmres_iterations_and_solution(method):
    _case(f"{method} on the cavity n_el=4 p=2")
    from paper_1712_00403_amd.stokes import CavitySolver
    S, (xo, it_o, _) = _oracle(4, 2, method)
    sol = CavitySolver(4, 2)
    x, it, _ = sol.solve(method)
    print(f"  iterations: GPU {it}, oracle {it_o}")
    assert abs(it - it_o) <= 1
    x = x.cpu().numpy()
    assert np.linalg.norm(x[:S.nu] - xo[:S.nu]) <= 1e-6 * np.linalg.norm(xo[:S.nu])
    dp = x[S.nu:] - xo[S.nu:]
    assert np.linalg.norm(dp - dp.mean()) <= 1e-5 * np.linalg.norm(xo[S.nu:])
    sol.close()
