"""The Taylor-Hood Stokes system on the unit cube (Sec. 3) and its preconditioned Krylov solves (Sec. 4).

With G = id and nu = 1 every block of the Stokes matrix is a Kronecker
product of univariate factors from the library's host setup
(fd_assemble_1d, fd_mixed_1d); the operator is applied matrix-free on the
device as mode products (library GEMMs), while the preconditioners P_D, P_T
and P_C of Sec. 4 apply their P_V^{-1} and P_Q^{-1} blocks through the FD
library (fd_apply_batched). The driven-cavity data of Sec. 7 (velocity
(1, 0, 0) on the top face, (-1, 0, 0) on the bottom face, zero on the
lateral faces) enter as a lifting: the first velocity component takes
coefficient +1 / -1 on every function of the top / bottom face, edge
functions included, every other boundary coefficient 0; f = 0.

Velocity unknowns are the coefficients of the functions that vanish on the
boundary (i_1 fastest per component); the pressure keeps every coefficient
(no mean-value constraint: the Krylov solver handles the constant).
"""
import numpy as np

from . import fd, krylov, workloads
from .precond import BlockPreconditioner


def _mode(X, F, axis):
    """Mode product along ``axis`` (0: i_1, 1: i_2, 2: i_3) of a tensor stored [i_3, i_2, i_1]."""
    import torch
    if axis == 0:
        return torch.matmul(X, F.T)
    if axis == 1:
        return torch.matmul(F, X)
    n3 = X.shape[0]
    return torch.matmul(F, X.reshape(n3, -1)).reshape(F.shape[0], X.shape[1], X.shape[2])


def _apply3(X, facs):
    """Kronecker product applied to a 3-tensor: facs[a] acts on axis a (direction a + 1)."""
    for a in range(3):
        X = _mode(X, facs[a], a)
    return X


class CubeStokes:
    """TH Stokes operator on the unit cube with n_el elements per direction and pressure degree p."""

    def __init__(self, n_el, p, device="cuda"):
        import torch
        self.n_el, self.p, self.device = n_el, p, torch.device(device)
        dv, rv, dq, rq = p + 1, p - 1, p, p - 1
        K, M = fd.assemble_1d(n_el, dv, rv, False)
        C = fd.mixed_1d(n_el, dv, rv, 1, dv, rv, 0)      # int b'_l b_m
        D = fd.mixed_1d(n_el, dq, rq, 0, dv, rv, 1)      # int q_l b'_m
        Nq = fd.mixed_1d(n_el, dq, rq, 0, dv, rv, 0)     # int q_l b_m
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(self.device)
        self.mV, self.mQ = K.shape[0], D.shape[0]
        self.nV = self.mV - 2
        full = {"K": t(K), "M": t(M), "C": t(C), "D": t(D), "N": t(Nq)}
        inner = slice(1, self.mV - 1)
        self.f_in = {"K": t(K[inner, inner]), "M": t(M[inner, inner]), "C": t(C[inner, inner]),
                     "D": t(D[:, inner]), "N": t(Nq[:, inner])}
        self.nu = 3 * self.nV ** 3
        self.nq = self.mQ ** 3
        self.N = self.nu + self.nq
        # right-hand side: minus the full operator applied to the lifting
        m = self.mV
        g1 = torch.zeros((m, m, m), dtype=torch.float64, device=self.device)
        g1[-1] = 1.0
        g1[0] = -1.0
        zero = torch.zeros_like(g1)
        au, bu = self._blocks(full, [g1, zero, zero])
        rhs_u = [-a[1:-1, 1:-1, 1:-1] for a in au]
        self.rhs = torch.cat([x.reshape(-1) for x in rhs_u] + [-bu.reshape(-1)])

    def _blocks(self, f, us):
        """(A u per component, B u) with the factor set f (interior or full) on velocity tensors us."""
        return self._Au(f, us), self._Bu(f, us)

    @staticmethod
    def _Au(f, us):
        out = []
        for r in range(3):
            acc = None
            for s in range(3):
                if r == s:
                    # A_rr = sum_a (1 + delta_ar) K_a (x) M (x) M (eq. prec3D_TH)
                    for a in range(3):
                        facs = [f["K"] if b == a else f["M"] for b in range(3)]
                        term = _apply3(us[s], facs)
                        if a == r:
                            term = 2.0 * term
                        acc = term if acc is None else acc + term
                else:
                    # [A_rs]_ij = int d_s B_i d_r B_j: C in direction s, C^T in direction r
                    facs = [f["M"], f["M"], f["M"]]
                    facs[s] = f["C"]
                    facs[r] = f["C"].T
                    term = _apply3(us[s], facs)
                    acc = term if acc is None else acc + term
            out.append(acc)
        return out

    @staticmethod
    def _Bu(f, us):
        # [B_r]_lj = -int q_l d_r B_j: -D in direction r, N elsewhere
        bu = None
        for r in range(3):
            facs = [f["N"], f["N"], f["N"]]
            facs[r] = -f["D"]
            term = _apply3(us[r], facs)
            bu = term if bu is None else bu + term
        return bu

    def split(self, x):
        n = self.nV
        us = [x[k * n ** 3:(k + 1) * n ** 3].reshape(n, n, n) for k in range(3)]
        q = self.mQ
        return us, x[self.nu:].reshape(q, q, q)

    def apply(self, x):
        """The Stokes matrix [[A, B^T], [B, 0]] times x (velocity unknowns, then pressure)."""
        import torch
        us, pr = self.split(x)
        au, bu = self._blocks(self.f_in, us)
        f = self.f_in
        for r in range(3):
            facs = [f["N"].T, f["N"].T, f["N"].T]
            facs[r] = -f["D"].T
            au[r] = au[r] + _apply3(pr, facs)
        return torch.cat([a.reshape(-1) for a in au] + [bu.reshape(-1)])

    def apply_B(self, u):
        """B u for the velocity unknowns u."""
        n = self.nV
        us = [u[k * n ** 3:(k + 1) * n ** 3].reshape(n, n, n) for k in range(3)]
        return self._Bu(self.f_in, us).reshape(-1)

    def apply_BT(self, pr):
        import torch
        q = self.mQ
        P = pr.reshape(q, q, q)
        f = self.f_in
        outs = []
        for r in range(3):
            facs = [f["N"].T, f["N"].T, f["N"].T]
            facs[r] = -f["D"].T
            outs.append(_apply3(P, facs).reshape(-1))
        return torch.cat(outs)


class CavitySolver:
    """P_D-MINRES, P_T-GMRES and P_C-GMRES (Sec. 4) for the driven cavity on the cube."""

    def __init__(self, n_el, p, precision="f64", pressure="fd", device="cuda"):
        self.op = CubeStokes(n_el, p, device)
        self.pc = BlockPreconditioner(workloads.taylor_hood_problem((n_el,) * 3, p), precision=precision,
                                      pressure=pressure)
        if self.pc.N != self.op.N:
            raise RuntimeError("preconditioner and operator sizes differ")
        self.precision = precision

    def _io(self, r):
        import torch
        return r.to(torch.float64 if self.pc.io_dtype == "float64" else torch.float32).contiguous()

    def apply_PD_inv(self, r):
        import torch
        return self.pc.apply(self._io(r)).to(torch.float64)

    def _apply_part(self, r, which):
        """P_V^{-1} (which = 'V') or P_Q^{-1} (which = 'Q') of a vector of the part's length."""
        import torch
        nu = self.op.nu
        full = torch.zeros(self.op.N, dtype=r.dtype, device=r.device)
        if which == "V":
            full[:nu] = r
        else:
            full[nu:] = r
        src = self._io(full)
        dst = torch.zeros_like(src)
        works = self.pc.works(src.data_ptr(), dst.data_ptr(), 1)
        works = works[:3] if which == "V" else works[3:]
        fd.apply_batched(works)
        dst = dst.to(torch.float64)
        return dst[:nu] if which == "V" else dst[nu:]

    def apply_PT_inv(self, r):
        """P_T^{-1}: y = -P_Q^{-1} g, x = P_V^{-1} (f - B^T y) (eq. P_T)."""
        import torch
        nu = self.op.nu
        y = -self._apply_part(r[nu:], "Q")
        x = self._apply_part(r[:nu] - self.op.apply_BT(y), "V")
        return torch.cat([x, y])

    def apply_PC_inv(self, r):
        """P_C^{-1} by the factorisation below eq. P_C."""
        import torch
        nu = self.op.nu
        x = self._apply_part(r[:nu], "V")
        y = r[nu:] - self.op.apply_B(x)
        y = -self._apply_part(y, "Q")
        x = x - self._apply_part(self.op.apply_BT(y), "V")
        return torch.cat([x, y])

    def solve(self, method="minres", tol=1e-8, maxiter=1000):
        if method == "minres":
            return krylov.minres(self.op.apply, self.apply_PD_inv, self.op.rhs, tol, maxiter)
        if method == "gmres_t":
            return krylov.gmres(self.op.apply, self.apply_PT_inv, self.op.rhs, tol, maxiter)
        if method == "gmres_c":
            return krylov.gmres(self.op.apply, self.apply_PC_inv, self.op.rhs, tol, maxiter)
        raise ValueError(method)

    def close(self):
        self.pc.close()
