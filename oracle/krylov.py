"""Preconditioned MINRES (Sec. 4, with P_D of eq. P_D) for symmetric indefinite systems.

Test infrastructure only (see ``oracle/__init__``).

The method of Paige and Saunders written from its definition: the Lanczos
process of P^{-1} A in the P-inner product builds an orthonormal basis; the
iterate minimises the P^{-1}-norm of the residual over the Krylov space,
through Givens rotations of the tridiagonal Lanczos matrix. Reading (the
paper gives the tolerance 1e-8 and the zero initial guess, not the norm):
the iteration stops when that residual norm, which the recurrences carry,
falls below tol times its initial value.
"""
import numpy as np


def minres(apply_A, apply_Pinv, b, tol=1e-8, maxiter=1000):
    """Solve A x = b; returns (x, iterations, residual norms (P^{-1}-norm) per iteration)."""
    x = np.zeros_like(b)
    r = b.copy()
    z = apply_Pinv(r)
    beta = np.sqrt(r @ z)
    beta0 = beta
    hist = [beta]
    # Lanczos vectors (unscaled r, preconditioned z), previous directions
    r_old = np.zeros_like(b)
    z_old = np.zeros_like(b)
    w = np.zeros_like(b)
    w_old = np.zeros_like(b)
    beta_old = 0.0
    c_old, s_old = 1.0, 0.0
    c, s = 1.0, 0.0
    eta = beta
    it = 0
    while it < maxiter:
        it += 1
        v = z / beta
        Av = apply_A(v)
        alpha = v @ Av
        r_new = Av - (alpha / beta) * r - (beta / beta_old) * r_old if beta_old > 0 else Av - (alpha / beta) * r
        z_new = apply_Pinv(r_new)
        beta_new = np.sqrt(max(r_new @ z_new, 0.0))
        # QR of the tridiagonal matrix: apply the two previous rotations, then a new one
        delta = c * alpha - c_old * s * beta
        rho2 = s * alpha + c_old * c * beta
        rho3 = s_old * beta
        gamma = np.hypot(delta, beta_new)
        c_new, s_new = delta / gamma, beta_new / gamma
        w_new = (v - rho3 * w_old - rho2 * w) / gamma
        x = x + c_new * eta * w_new
        eta = -s_new * eta
        hist.append(abs(eta))
        if abs(eta) <= tol * beta0:
            break
        r_old, r = r, r_new
        z_old, z = z, z_new
        beta_old, beta = beta, beta_new
        w_old, w = w, w_new
        c_old, s_old, c, s = c, s, c_new, s_new
    return x, it, hist


def gmres(apply_A, apply_Pinv, b, tol=1e-8, maxiter=500):
    """Left-preconditioned GMRES (Saad and Schultz) from its definition, for P_T and P_C (Sec. 4).

    Arnoldi with modified Gram-Schmidt on P^{-1} A from r0 = P^{-1} b; after
    step k the iterate minimises ||beta e_1 - H_k y|| over y (a small dense
    least-squares problem solved by a library routine each step). Stops when
    that minimum, the 2-norm of the preconditioned residual, falls below tol
    times ||P^{-1} b|| (reading: the paper names GMRES and the tolerance, not
    the side of the preconditioner). Returns (x, iterations, history).
    """
    r0 = apply_Pinv(b)
    beta = np.linalg.norm(r0)
    V = [r0 / beta]
    Hcols = []
    hist = [beta]
    y = np.zeros(0)
    for k in range(1, maxiter + 1):
        w = apply_Pinv(apply_A(V[-1]))
        h = np.zeros(k + 1)
        for j in range(k):
            h[j] = V[j] @ w
            w = w - h[j] * V[j]
        h[k] = np.linalg.norm(w)
        Hcols.append(h)
        H = np.zeros((k + 1, k))
        for j, col in enumerate(Hcols):
            H[:j + 2, j] = col
        e1 = np.zeros(k + 1)
        e1[0] = beta
        y = np.linalg.lstsq(H, e1, rcond=None)[0]
        res = np.linalg.norm(e1 - H @ y)
        hist.append(res)
        if res <= tol * beta or h[k] == 0.0:
            break
        V.append(w / h[k])
    x = sum(y[j] * V[j] for j in range(len(y)))
    return x, len(Hcols), hist
