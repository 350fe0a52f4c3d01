"""Dense pencil eigensolver and the exact matrix filter (plain definitions).

* Pencil eigenproblem (eq. IGEVP): A x = lambda B x, B Hermitian positive
  definite.  Cholesky B = L L^H, C = L^-1 A L^-H, cyclic Jacobi on C
  (Hermitian rotations, round-robin ordering), X = L^-H W.  X^H B X = I.
* Exact filter: R_ab(B^-1 A) V = X diag(R_ab(lambda)) X^H B V, because
  B^-1 A = X diag(lambda) X^-1 and X^-1 = X^H B.
* Operator G = Zhat(T(B^-1 A); l1) of eq. (solve): X diag(g(lambda)) X^H B V,
  and its shifted inverses (G + s I)^-1 V by a dense solve.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def _round_robin(n: int):
    """Pairings of a round-robin tournament on n (even) players: n-1 rounds."""
    players = list(range(n))
    rounds = []
    for _ in range(n - 1):
        pairs = [(players[i], players[n - 1 - i]) for i in range(n // 2)]
        rounds.append(pairs)
        players = [players[0]] + [players[-1]] + players[1:-1]
    return rounds


def jacobi_eigh(C, tol: float = 1e-15, max_sweeps: int = 40):
    """Eigen-decomposition of a Hermitian matrix by cyclic Jacobi rotations.

    Each rotation zeroes one off-diagonal pair (p, q): a diagonal phase makes
    C_pq real, then the classical real rotation with t = sign(tau)/(|tau| +
    sqrt(1 + tau^2)), tau = (C_qq - C_pp)/(2|C_pq|).  Disjoint pairs of one
    round-robin round are applied together.  Returns ascending eigenvalues and
    unitary eigenvectors.
    """
    C = np.array(C, dtype=np.complex128 if np.iscomplexobj(C) else np.float64, copy=True)
    n = C.shape[0]
    cplx = np.iscomplexobj(C)
    V = np.eye(n, dtype=C.dtype)
    if n == 1:
        return np.real(np.diag(C)).copy(), V
    m = n + (n % 2)
    rounds = _round_robin(m)
    fro = np.linalg.norm(C)
    for _ in range(max_sweeps):
        off = np.linalg.norm(C - np.diag(np.diag(C)))
        if off <= tol * fro or fro == 0.0:
            break
        for pairs in rounds:
            pq = np.array([(p, q) for (p, q) in pairs if p < n and q < n])
            if pq.size == 0:
                continue
            P = pq[:, 0]
            Q = pq[:, 1]
            cpq = C[P, Q]
            h = np.abs(cpq)
            act = h > 0.0
            if not np.any(act):
                continue
            P, Q, cpq, h = P[act], Q[act], cpq[act], h[act]
            app = np.real(C[P, P])
            aqq = np.real(C[Q, Q])
            tau = (aqq - app) / (2.0 * h)
            big = np.abs(tau) > 1e150
            ts = np.where(big, 1.0, tau)
            t = np.where(big, 0.5 / np.where(big, tau, 1.0), np.where(ts >= 0.0, 1.0, -1.0) / (np.abs(ts) + np.sqrt(1.0 + ts * ts)))
            cs = 1.0 / np.sqrt(1.0 + t * t)
            sn = t * cs
            ph = cpq / h  # e^{i phi}; the sign of C_pq for a real matrix
            # J = diag(1, conj(ph)) @ [[cs, sn], [-sn, cs]]
            j00 = cs
            j01 = sn
            j10 = -sn * np.conj(ph)
            j11 = cs * np.conj(ph)
            # columns: C[:, [p, q]] <- C[:, [p, q]] J
            Cp = C[:, P].copy()
            Cq = C[:, Q].copy()
            C[:, P] = Cp * j00 + Cq * j10
            C[:, Q] = Cp * j01 + Cq * j11
            # rows: C[[p, q], :] <- J^H C[[p, q], :]
            Rp = C[P, :].copy()
            Rq = C[Q, :].copy()
            C[P, :] = np.conj(j00)[:, None] * Rp + np.conj(j10)[:, None] * Rq
            C[Q, :] = np.conj(j01)[:, None] * Rp + np.conj(j11)[:, None] * Rq
            Vp = V[:, P].copy()
            Vq = V[:, Q].copy()
            V[:, P] = Vp * j00 + Vq * j10
            V[:, Q] = Vp * j01 + Vq * j11
    w = np.real(np.diag(C)).copy()
    order = np.argsort(w, kind="stable")
    return w[order], V[:, order]


def pencil_eigh_jacobi(A, B):
    """All eigenpairs of the Hermitian definite pencil by Cholesky + Jacobi."""
    A = np.asarray(A)
    B = np.asarray(B)
    L = np.linalg.cholesky(B)
    Y = sla.solve_triangular(L, A, lower=True)  # L^-1 A
    C = sla.solve_triangular(L, Y.conj().T, lower=True).conj().T  # L^-1 A L^-H
    C = 0.5 * (C + C.conj().T)
    w, W = jacobi_eigh(C)
    X = sla.solve_triangular(L.conj().T, W, lower=False)  # L^-H W
    return w, X


def pencil_eigh_lapack(A, B):
    """LAPACK generalized Hermitian eigensolver (library special case)."""
    return sla.eigh(np.asarray(A), np.asarray(B))


def exact_filter(lam, X, B, V, R):
    """R(B^-1 A) V = X diag(R(lam)) X^H B V for B-orthonormal eigenvectors X."""
    return X @ (np.asarray(R(lam))[:, None] * (X.conj().T @ (B @ V)))


def exact_G(lam, X, B, V, g):
    """G V = X diag(g(lam)) X^H B V with g = Zhat(T(.); l1)."""
    gl = np.real(np.asarray(g(lam)))
    return X @ (gl[:, None] * (X.conj().T @ (B @ V)))


def shifted_solve(lam, X, B, V, g, s):
    """(G + s I)^-1 V = X diag(1/(g(lam)+s)) X^H B V (complex s)."""
    gl = np.real(np.asarray(g(lam)))
    return X @ ((1.0 / (gl + s))[:, None] * (X.conj().T @ (B @ V)))


def count_in(lam, a, b) -> int:
    lam = np.asarray(lam)
    return int(np.sum((lam > a) & (lam < b)))
