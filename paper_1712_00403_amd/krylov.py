"""Krylov solvers around the preconditioners (Sec. 4): MINRES for P_D, GMRES for P_T and P_C.

Device-resident iterations on torch tensors; the operator and the
preconditioner are callables (the preconditioner's blocks run in the
library's kernels). Both stop on the relative residual in the norm the
method minimises: MINRES the P^{-1}-norm carried by its recurrences,
left-preconditioned GMRES the 2-norm of P^{-1}(b - A x); tolerance 1e-8 and
the zero initial guess are the paper's (Sec. 7).
"""
import math


def minres(apply_A, apply_Pinv, b, tol=1e-8, maxiter=1000):
    """Preconditioned MINRES (Paige-Saunders) for symmetric A and SPD P; returns (x, iterations, history)."""
    import torch
    x = torch.zeros_like(b)
    v_prev = torch.zeros_like(b)      # previous Lanczos vector (unnormalised, A-space)
    r = b.clone()
    z = apply_Pinv(r)
    beta = math.sqrt(max(float(torch.dot(r, z)), 0.0))
    beta0 = beta
    hist = [beta]
    if beta0 == 0.0:
        return x, 0, hist
    d_prev = torch.zeros_like(b)      # search directions of the two previous steps
    d_prev2 = torch.zeros_like(b)
    beta_prev = 0.0
    cs = [1.0, 1.0]                   # rotations of steps k-1 and k-2: (c, s)
    sn = [0.0, 0.0]
    phi = beta
    it = 0
    while it < maxiter:
        it += 1
        q = z / beta                  # P-orthonormal Lanczos vector
        Aq = apply_A(q)
        alpha = float(torch.dot(q, Aq))
        r_next = Aq - (alpha / beta) * r
        if beta_prev > 0.0:
            r_next = r_next - (beta / beta_prev) * v_prev
        z_next = apply_Pinv(r_next)
        beta_next = math.sqrt(max(float(torch.dot(r_next, z_next)), 0.0))
        # new column of the tridiagonal matrix: (beta, alpha, beta_next) rotated by the old rotations
        e2 = sn[1] * beta                          # from the rotation two steps back
        t = cs[1] * beta
        e1 = cs[0] * t + sn[0] * alpha             # from the previous rotation
        g = -sn[0] * t + cs[0] * alpha
        rho = math.hypot(g, beta_next)
        c, s = g / rho, beta_next / rho
        d = (q - e1 * d_prev - e2 * d_prev2) / rho
        x = x + (c * phi) * d
        phi = -s * phi
        hist.append(abs(phi))
        if abs(phi) <= tol * beta0:
            break
        v_prev, r, z = r, r_next, z_next
        beta_prev, beta = beta, beta_next
        d_prev2, d_prev = d_prev, d
        cs = [c, cs[0]]
        sn = [s, sn[0]]
    return x, it, hist


def gmres(apply_A, apply_Pinv, b, tol=1e-8, maxiter=500):
    """Left-preconditioned GMRES without restarts (modified Gram-Schmidt Arnoldi, Givens rotations).

    Solves P^{-1} A x = P^{-1} b; returns (x, iterations, history of the
    preconditioned residual norms).
    """
    import torch
    r0 = apply_Pinv(b)
    nrm0 = float(torch.linalg.vector_norm(r0))
    hist = [nrm0]
    if nrm0 == 0.0:
        return torch.zeros_like(b), 0, hist
    V = [r0 / nrm0]
    H = []                                  # columns of the Hessenberg matrix (after rotations: R)
    cs, sn = [], []
    gvec = [nrm0]
    it = 0
    while it < maxiter:
        w = apply_Pinv(apply_A(V[-1]))
        h = []
        for vj in V:
            hij = float(torch.dot(vj, w))
            w = w - hij * vj
            h.append(hij)
        hnext = float(torch.linalg.vector_norm(w))
        for j in range(len(cs)):           # previous rotations
            a, bb = h[j], h[j + 1]
            h[j] = cs[j] * a + sn[j] * bb
            h[j + 1] = -sn[j] * a + cs[j] * bb
        rho = math.hypot(h[-1], hnext)
        c, s = h[-1] / rho, hnext / rho
        h[-1] = rho
        cs.append(c)
        sn.append(s)
        gvec.append(-s * gvec[-1])
        gvec[-2] = c * gvec[-2]
        H.append(h)
        it += 1
        hist.append(abs(gvec[-1]))
        if abs(gvec[-1]) <= tol * nrm0 or hnext == 0.0:
            break
        V.append(w / hnext)
    # back substitution R y = g
    k = len(H)
    y = [0.0] * k
    for i in range(k - 1, -1, -1):
        acc = gvec[i] - sum(H[j][i] * y[j] for j in range(i + 1, k))
        y[i] = acc / H[i][i]
    x = torch.zeros_like(b)
    for j in range(k):
        x = x + y[j] * V[j]
    return x, it, hist
