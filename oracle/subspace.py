"""Algorithm 1 (subspace iteration with a rational filter) and accuracy metrics.

Algorithm 1: Q orthonormal random; repeat { Y = R_ab(B^-1 A) Q;
A~ = Y^H A Y, B~ = Y^H B Y; solve A~ Q~ = B~ Q~ Lambda~; Q = Y Q~ };
keep the Ritz pairs with a < theta < b.

Reading for a near rank-deficient Y (the paper is silent): Y's columns are
scaled to unit B-norm before the reduced pencil is formed, and the reduced
pencil is solved by LAPACK (a library special case of the plain definition).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .dense import exact_filter


def rel_residuals(A, B, lam, X, normA: float, normB: float):
    """||A x - lam B x||_2 / ((||A|| + |lam| ||B||) ||x||_2) per column."""
    AX = A @ X
    BX = B @ X
    R = AX - BX * lam[None, :]
    return np.linalg.norm(R, axis=0) / ((normA + np.abs(lam) * normB) * np.linalg.norm(X, axis=0))


def e_lambda_x(A, B, lam, X, a: float, b: float) -> float:
    """Relative error e_{Lambda,X} of eq. (relerr)."""
    if X.shape[1] == 0:
        return 0.0
    AX = A @ X
    BX = B @ X
    num = np.linalg.norm(AX - BX * lam[None, :], axis=0)
    den = np.linalg.norm(max(abs(a), abs(b)) * BX, axis=0)
    return float(np.max(num / den))


def b_orthonormality(B, X) -> float:
    """max |X^H B X - I|."""
    G = X.conj().T @ (B @ X)
    return float(np.max(np.abs(G - np.eye(G.shape[0]))))


def inf_norm(M) -> float:
    """||M||_inf = max row sum of |M| (= ||M||_1 for Hermitian M), >= ||M||_2."""
    M = abs(M)
    return float(np.max(np.asarray(M.sum(axis=1)).ravel()))


def norm2_est(M, iters: int = 30, seed: int = 0) -> float:
    """Estimate of ||M||_2 by power iteration on M^H M (iters steps from a
    seeded Gaussian start): sqrt of the Rayleigh quotient of M^H M, a lower
    bound that approaches ||M||_2 from below.  Used to report the residual in
    the 2-norm reading of the spec residual beside the infinity-norm one
    (||M||_2 <= ||M||_inf for Hermitian M)."""
    n = M.shape[1]
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(n)
    if np.iscomplexobj(M.data if hasattr(M, "data") else M):
        x = x + 1j * rng.standard_normal(n)
    x = x / np.linalg.norm(x)
    est = 0.0
    for _ in range(iters):
        y = M @ x
        z = M.conj().T @ y
        est = float(np.sqrt(np.real(np.vdot(x, z))))
        nz = np.linalg.norm(z)
        if nz == 0.0:
            return 0.0
        x = z / nz
    return est


def rayleigh_ritz(A, B, Y, tau_rank: float = 1e-12):
    """Ritz values/vectors of (A, B) on span(Y) (Algorithm 1, lines 4-6).

    Reading for a near rank-deficient Y (the paper is silent): scale Y's
    columns to unit B-norm, eigen-decompose B~ = U S U^H and keep the
    directions with s > tau_rank * max(s); on the B-orthonormal basis
    Z = Y_s U_k S_k^-1/2 solve the standard Hermitian problem Z^H A Z.
    Returns (theta, X, C) with X = Y C B-orthonormal, ascending theta.
    """
    d = np.sqrt(np.real(np.einsum("ij,ij->j", Y.conj(), B @ Y)))
    d[d == 0.0] = 1.0
    Ys = Y / d[None, :]
    At = Ys.conj().T @ (A @ Ys)
    Bt = Ys.conj().T @ (B @ Ys)
    At = 0.5 * (At + At.conj().T)
    Bt = 0.5 * (Bt + Bt.conj().T)
    s, U = np.linalg.eigh(Bt)
    keep = s > tau_rank * s[-1]
    T = U[:, keep] / np.sqrt(s[keep])[None, :]
    Ar = T.conj().T @ At @ T
    Ar = 0.5 * (Ar + Ar.conj().T)
    theta, Wr = np.linalg.eigh(Ar)
    C = (T @ Wr) / d[:, None]
    return theta, Y @ C, C


def alg1_exact(A, B, lam_all, X_all, plan, a, b, Q0, n_iter: int, normA=None, normB=None):
    """Algorithm 1 with the exact matrix filter; returns per-iteration history.

    lam_all, X_all: all eigenpairs of the (small) pencil, B-orthonormal.
    """
    Ad = A
    Bd = B
    normA = inf_norm(A) if normA is None else normA
    normB = inf_norm(B) if normB is None else normB
    Q, _ = np.linalg.qr(Q0)
    hist = []
    for _ in range(n_iter):
        Y = exact_filter(lam_all, X_all, Bd, Q, plan.R)
        theta, Q, _ = rayleigh_ritz(Ad, Bd, Y)
        sel = (theta > a) & (theta < b)
        res = rel_residuals(Ad, Bd, theta[sel], Q[:, sel], normA, normB)
        hist.append({"theta": theta[sel].copy(), "X": Q[:, sel].copy(), "max_res": float(np.max(res)) if res.size else 0.0})
    return hist
