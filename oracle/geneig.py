"""Generalized symmetric eigendecomposition K U = M U D with U^T M U = I (Sec. 5.2, eq. eig_dec).

Test infrastructure only (see ``oracle/__init__``).

Route: Cholesky M = L L^T (library routine), C = L^{-1} K L^{-T}, eigenpairs of
the symmetric C by cyclic Jacobi rotations written out here, then U = L^{-T} V.
Then K U = M U D and U^T M U = V^T V = I, which are the two properties the
paper asks of the pencil decomposition.
"""
import numpy as np


def _round_robin_pairs(n):
    """All n(n-1)/2 index pairs, grouped into rounds of disjoint pairs.

    Circle-method tournament schedule on an even number of players (a dummy
    player n is added when n is odd and its games are dropped).
    """
    players = list(range(n + (n % 2)))
    N = len(players)
    rounds = []
    for _ in range(N - 1):
        pairs = []
        for i in range(N // 2):
            a, b = players[i], players[N - 1 - i]
            if a < n and b < n:
                pairs.append((min(a, b), max(a, b)))
        rounds.append(pairs)
        players = [players[0]] + [players[-1]] + players[1:-1]
    return rounds


def jacobi_eigh(C, rel_tol=1e-16, max_sweeps=60):
    """Eigenpairs of a real symmetric matrix by cyclic Jacobi rotations.

    Each rotation zeroes one off-diagonal pair (p, q): with
    theta = (C_qq - C_pp) / (2 C_pq), t = sign(theta)/(|theta| + sqrt(theta^2+1)),
    c = 1/sqrt(t^2+1), s = t c, the plane rotation J(p, q) gives
    (J^T C J)_pq = 0. Rotations on disjoint pairs commute, so each round of
    the tournament schedule applies n/2 of them at once. A pair is left
    alone once |C_pq| <= rel_tol * sqrt(|C_pp C_qq|) (the relative
    threshold that keeps small eigenvalues accurate); sweeps stop when a whole
    sweep leaves every pair alone.
    Returns (eigenvalues ascending, orthonormal eigenvectors as columns).
    """
    A = np.array(C, dtype=np.float64, copy=True)
    n = A.shape[0]
    V = np.eye(n)
    if n == 1:
        return A.diagonal().copy(), V
    rounds = [np.array(r, dtype=np.int64) for r in _round_robin_pairs(n)]
    for _ in range(max_sweeps):
        rotated = False
        for pr in rounds:
            if pr.size == 0:
                continue
            p, q = pr[:, 0], pr[:, 1]
            apq = A[p, q]
            app = A[p, p]
            aqq = A[q, q]
            act = np.abs(apq) > rel_tol * np.sqrt(np.abs(app * aqq))
            if not np.any(act):
                continue
            rotated = True
            with np.errstate(over="ignore", divide="ignore"):
                theta = np.where(act, (aqq - app) / (2.0 * np.where(act, apq, 1.0)), 0.0)
                # sqrt(theta^2 + 1) as hypot so that a huge theta gives t -> 0
                t = np.where(act, np.sign(theta) / (np.abs(theta) + np.hypot(theta, 1.0)), 0.0)
            t = np.where(act & (theta == 0.0), 1.0, t)
            c = 1.0 / np.sqrt(t * t + 1.0)
            s = t * c
            # columns: A <- A J
            Ap, Aq = A[:, p].copy(), A[:, q].copy()
            A[:, p] = c * Ap - s * Aq
            A[:, q] = s * Ap + c * Aq
            # rows: A <- J^T A
            Ap, Aq = A[p, :].copy(), A[q, :].copy()
            A[p, :] = c[:, None] * Ap - s[:, None] * Aq
            A[q, :] = s[:, None] * Ap + c[:, None] * Aq
            Vp, Vq = V[:, p].copy(), V[:, q].copy()
            V[:, p] = c * Vp - s * Vq
            V[:, q] = s * Vp + c * Vq
        if not rotated:
            break
    d = np.diag(A).copy()
    order = np.argsort(d, kind="stable")
    return d[order], V[:, order]


def generalized_eig(K, M):
    """U, d with K U = M U diag(d) and U^T M U = I (eq. eig_dec).

    K symmetric, M symmetric positive definite (Sec. 5.2 asks both SPD).
    Raises numpy.linalg.LinAlgError if M is not positive definite.
    """
    K = 0.5 * (np.asarray(K, dtype=np.float64) + np.asarray(K, dtype=np.float64).T)
    M = 0.5 * (np.asarray(M, dtype=np.float64) + np.asarray(M, dtype=np.float64).T)
    L = np.linalg.cholesky(M)
    Linv_K = np.linalg.solve(L, K)
    C = np.linalg.solve(L, Linv_K.T)
    C = 0.5 * (C + C.T)
    d, V = jacobi_eigh(C)
    U = np.linalg.solve(L.T, V)
    return U, d
