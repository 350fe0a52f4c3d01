"""Large-N oracle: exact counts, windows of eigenvalues, bounds, CPU Alg. 1+2.

* Exact count (Sylvester's law of inertia): n(a, b) = nu(A - bB) - nu(A - aB),
  nu = number of negative pivots of a no-pivot LDL^T in a symmetric
  permutation.  SuperLU with diag_pivot_thresh=0, SymmetricMode and an
  A + A^T minimum-degree ordering; perm_r == perm_c is checked.
* Windows of eigenvalues near a shift: shift-invert Lanczos (scipy/ARPACK,
  a library routine).
* Kato-Temple: |lambda - theta| <= ||r||_{B^-1}^2 / gap for a B-normalised
  Ritz vector with residual r = A x - theta B x.
* CPU Algorithm 2 (hybrid filter): r1 complex SuperLU factors of
  A - sigma_hat_j B (line 5-6), operator G of eq. (solve) (line 7), block
  Arnoldi on G with classical Gram-Schmidt done twice, the shifted block
  Hessenberg least-squares problems of the multi-shift GMRES (line 8, eq.
  solve2) by LAPACK least squares, and the weighted sum (line 9).  Algorithm
  1 wraps it.  This is the reported CPU baseline, not a pin.
"""
from __future__ import annotations

import time

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .subspace import inf_norm, rayleigh_ritz, rel_residuals


def _splu_sym(K):
    return spla.splu(
        sp.csc_matrix(K),
        permc_spec="MMD_AT_PLUS_A",
        diag_pivot_thresh=0.0,
        options={"SymmetricMode": True},
    )


def inertia_neg(A, B, sigma: float) -> int:
    """Number of eigenvalues of (A, B) below sigma (negative pivots of A - sigma B)."""
    lu = _splu_sym(A - sigma * B)
    if not np.array_equal(lu.perm_r, lu.perm_c):
        raise RuntimeError("SuperLU pivoted off the diagonal; inertia not valid")
    d = np.real(lu.U.diagonal())
    return int(np.sum(d < 0.0))


def count_interval(A, B, a: float, b: float) -> int:
    return inertia_neg(A, B, b) - inertia_neg(A, B, a)


def window_near(A, B, sigma0: float, k: int, tol: float = 0.0):
    """The k eigenvalues of (A, B) nearest sigma0 (ascending) and their vectors
    (eigenvalues as the Rayleigh quotients of the returned vectors).

    Shift-invert Lanczos (ARPACK) with (A - sigma0 B)^-1 applied through the
    symmetric-mode minimum-degree SuperLU factorization used for the inertia
    counts (a 3-D stencil needs that ordering to stay within memory and time).
    """
    lu = _splu_sym(sp.csc_matrix(A - sigma0 * B))
    n = A.shape[0]
    dt = np.result_type(A.dtype, B.dtype, np.float64)  # complex Hermitian pencils stay complex
    op = spla.LinearOperator((n, n), matvec=lambda x: lu.solve(np.asarray(x, dtype=dt)), dtype=dt)
    w, X = spla.eigsh(A, k=k, M=B, sigma=sigma0, which="LM", tol=tol, OPinv=op)
    # Rayleigh quotients of the Lanczos vectors: their error is quadratic in the
    # vectors' error, so they stay exact to rounding even when the unpivoted
    # shift-invert solves are only accurate to ~1e-10 (indefinite A - sigma0 B)
    AX, BX = A @ X, B @ X
    w = np.real(np.einsum("ij,ij->j", X.conj(), AX) / np.einsum("ij,ij->j", X.conj(), BX))
    order = np.argsort(w)
    return w[order], X[:, order]


def kato_temple(A, B, theta, X, gap):
    """Kato-Temple bounds ||r||^2_{B^-1} / gap for B-normalised columns of X."""
    Bs = spla.splu(sp.csc_matrix(B))
    out = np.empty(X.shape[1])
    for i in range(X.shape[1]):
        x = X[:, i]
        x = x / np.sqrt(np.real(np.vdot(x, B @ x)))
        r = A @ x - theta[i] * (B @ x)
        out[i] = np.real(np.vdot(r, Bs.solve(r))) / gap
    return out


class HybridFilterCPU:
    """Algorithm 2 on the CPU with SuperLU factors (FP64 / complex128)."""

    def __init__(self, A, B, plan, hermitian_complex: bool = False):
        self.A = sp.csr_matrix(A)
        self.B = sp.csr_matrix(B)
        self.plan = plan
        self.cplx = hermitian_complex or np.iscomplexobj(A.data) or np.iscomplexobj(B.data)
        t0 = time.perf_counter()
        self.lus = [_splu_sym((self.A - s * self.B).astype(np.complex128)) for s in plan.sigma_hat]
        self.t_fact = time.perf_counter() - t0
        self.n_solves = 0

    def apply_G(self, V):
        """G V = M_hat [c0 V + sum_j (w_j K_j^-1 B V + conj(w_j) K_j^-H B V)] (eq. solve)."""
        p = self.plan
        BV = (self.B @ V).astype(np.complex128)
        W = p.c0 * V.astype(np.complex128)
        for lu, wj in zip(self.lus, p.w_hat):
            X = lu.solve(BV)
            self.n_solves += V.shape[1]
            if self.cplx:
                Xh = lu.solve(BV, trans="H")
                self.n_solves += V.shape[1]
                W = W + wj * X + np.conj(wj) * Xh
            else:
                W = W + 2.0 * np.real(wj * X)
        W = p.M_hat * W
        return W if self.cplx else np.real(W)

    def apply(self, V, tol: float = 1e-10, max_iter: int = 200):
        """R_ab(B^-1 A) V by block multi-shift GMRES on G (Algorithm 2, lines 8-9)."""
        p = self.plan
        n, k = V.shape
        Q1, R0 = np.linalg.qr(V)
        basis = [Q1]
        dt = np.complex128 if self.cplx else np.float64
        H = np.zeros(((max_iter + 1) * k, max_iter * k), dtype=dt)
        if self.cplx:
            shifts = np.concatenate([1j * np.sqrt(p.c), -1j * np.sqrt(p.c)])
        else:
            shifts = 1j * np.sqrt(p.c)
        r0n = np.linalg.norm(R0, axis=0)
        Ys = None
        it = 0
        for it in range(1, max_iter + 1):
            W = self.apply_G(basis[-1])
            Vk = np.hstack(basis)
            for _ in range(2):
                h = Vk.conj().T @ W
                W = W - Vk @ h
                H[: it * k, (it - 1) * k : it * k] += h
            Qn, Rn = np.linalg.qr(W)
            H[it * k : (it + 1) * k, (it - 1) * k : it * k] = Rn
            basis.append(Qn)
            Hb = H[: (it + 1) * k, : it * k]
            E = np.zeros(((it + 1) * k, k), dtype=np.complex128)
            E[:k, :] = R0
            Ys = []
            worst = 0.0
            for s in shifts:
                Hs = Hb.astype(np.complex128).copy()
                Hs[np.arange(it * k), np.arange(it * k)] += s
                Y, *_ = np.linalg.lstsq(Hs, E, rcond=None)
                res = np.linalg.norm(E - Hs @ Y, axis=0) / r0n
                worst = max(worst, float(np.max(res)))
                Ys.append(Y)
            # stop when every shift converged, or when the block Krylov space is
            # exhausted (new block numerically zero): then the LS solution is exact
            if worst <= tol or np.linalg.norm(Rn) <= 1e-13 * np.linalg.norm(Hb):
                break
        Vm = np.hstack(basis[:it])
        self.last_iters = it
        if self.cplx:
            out = 0.5 * V.astype(np.complex128)
            r = len(p.c)
            for j in range(r):
                out = out + 0.5 * p.M * 0.5 * p.a[j] * (Vm @ Ys[j] + Vm @ Ys[j + r])
            return out
        C = np.zeros((it * k, k))
        for j in range(len(p.c)):
            C += 0.5 * p.M * p.a[j] * np.real(Ys[j])
        return 0.5 * V + Vm @ C


def zoloeig_cpu(A, B, plan, a, b, Q0, n_iter_max: int = 6, tol_res: float = 1e-8, gmres_tol: float = 1e-10):
    """Algorithm 1 with the CPU hybrid filter; stops when every Ritz pair in
    (a, b) has relative residual <= tol_res.  Returns results and timings."""
    t0 = time.perf_counter()
    filt = HybridFilterCPU(A, B, plan)
    normA = inf_norm(A)
    normB = inf_norm(B)
    Q, _ = np.linalg.qr(Q0)
    t1 = time.perf_counter()
    gm = []
    theta = Xs = None
    res = np.array([])
    for it in range(1, n_iter_max + 1):
        Y = filt.apply(Q, tol=gmres_tol)
        gm.append(filt.last_iters)
        th, X, _ = rayleigh_ritz(A, B, Y)
        sel = (th > a) & (th < b)
        theta, Xs = th[sel], X[:, sel]
        Q = X if X.shape[1] == Q.shape[1] else np.hstack([X, Q[:, : Q.shape[1] - X.shape[1]]])
        res = rel_residuals(A, B, theta, Xs, normA, normB)
        if res.size and np.max(res) <= tol_res:
            break
    t2 = time.perf_counter()
    return {
        "theta": theta,
        "X": Xs,
        "res": res,
        "n_iter": it,
        "n_gmres": gm,
        "n_solv": filt.n_solves,
        "T_fact": filt.t_fact,
        "T_iter": t2 - t1,
        "T_total": t2 - t0,
    }
