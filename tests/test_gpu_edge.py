"""GPU edge cases of zolo_solve against the oracle's dense LAPACK solutions:
a window of degenerate eigenvalue clusters (where eigenvectors are not unique,
so the invariant subspaces are compared by their largest principal angle), and
the top slice of the spectrum (b_+ = +inf), on real and complex Hermitian
pencils.

Bars: exact count, eigenvalues 1e-10 relative, residual 1e-8, B-orthonormality
1e-10; sine of the largest principal angle between the returned subspace and the
exact invariant subspace of (a, b) below 1e-8, and of each cluster's subspace
below 1e-7 (a residual of 1e-10 over the smallest gap between clusters).
"""
import math
import sys

import numpy as np
import pytest

import pencils
from oracle.dense import pencil_eigh_lapack
from oracle.subspace import b_orthonormality, inf_norm, rel_residuals

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
zolo = pytest.importorskip("paper_1701_08935_amd")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return zolo.Context(0)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def sin_max_angle(Xref, X, B):
    """Sine of the largest principal angle between span(X) and span(Xref), both
    B-orthonormal: the B-norm of the part of X outside span(Xref)."""
    Bd = B.toarray()
    L = np.linalg.cholesky(Bd)
    R = X - Xref @ (Xref.conj().T @ (Bd @ X))
    return float(np.linalg.norm(L.conj().T @ R, 2))


def _clusters(lam, rtol=1e-9):
    groups, start = [], 0
    for i in range(1, len(lam) + 1):
        if i == len(lam) or lam[i] - lam[i - 1] > rtol * max(1.0, abs(lam[i])):
            groups.append((start, i))
            start = i
    return groups


def test_degenerate_clusters_by_principal_angles(ctx):
    n = 8
    gp = pencils.grid7(n, v_scale=0.0)
    A, B = gp.scipy()
    lam, Xall = pencil_eigh_lapack(A.toarray(), B.toarray())
    groups = _clusters(lam)
    # a window from the middle of the spectrum holding several clusters, one of them 6-fold
    mid = len(groups) // 2
    g0 = next(i for i in range(mid, len(groups)) if groups[i][1] - groups[i][0] == 6)
    sel = groups[g0 - 2:g0 + 3]
    lo, hi = sel[0][0], sel[-1][1]
    mult = [g[1] - g[0] for g in sel]
    say(f"degenerate grid7 {n}^3, v = 0: window of {hi - lo} eigenvalues in clusters {mult}")
    assert max(mult) >= 3
    am, ap, bm, bp = lam[lo - 1], lam[lo], lam[hi - 1], lam[hi]
    w = {"a": 0.5 * (am + ap), "b": 0.5 * (bm + bp), "a_minus": am, "a_plus": ap, "b_minus": bm, "b_plus": bp}
    P = zolo.Pencil.from_grid(ctx, gp, leaf_size=32)
    k = hi - lo
    opts = zolo.opts_from_window(w, r1=2, r2=0, n_ss=k + 8)
    Q0 = pencils.gaussian_block(gp.n, k + 8, seed=4)
    eig, vec, st, rc = zolo.zolo_solve(ctx, P, w["a"], w["b"], k, opts, Q0=_dev(Q0))
    say(f"  rc={rc} found {len(eig)} iterations {st['n_iter']} resid {st['max_resid']:.2e}")
    assert rc == 0 and len(eig) == k
    assert np.max(np.abs(np.array(eig) - lam[lo:hi]) / np.abs(lam[lo:hi])) < 1e-10
    X = vec.cpu().numpy()
    assert np.max(rel_residuals(A, B, np.array(eig), X, inf_norm(A), inf_norm(B))) < 1e-8
    assert b_orthonormality(B, X) < 1e-10
    s_all = sin_max_angle(Xall[:, lo:hi], X, B)
    say(f"  sin of the largest principal angle to the exact subspace: {s_all:.2e}")
    assert s_all < 1e-8
    # each cluster: the returned columns of that cluster span its invariant subspace
    for g in sel:
        cols = list(range(g[0] - lo, g[1] - lo))
        s_g = sin_max_angle(Xall[:, g[0]:g[1]], X[:, cols], B)
        say(f"  cluster of {g[1] - g[0]} at {lam[g[0]]:.6f}: sin {s_g:.2e}")
        assert s_g < 1e-7


@pytest.mark.parametrize("gen", ["grid7", "grid27p"])
def test_top_slice_b_plus_infinite(ctx, gen):
    gp = pencils.grid7(8) if gen == "grid7" else pencils.grid27p(7, ny=8, nz=6)
    A, B = gp.scipy()
    lam, Xall = pencil_eigh_lapack(A.toarray(), B.toarray())
    N, k = len(lam), 12
    w = {"a": 0.5 * (lam[N - k - 1] + lam[N - k]), "b": lam[-1] + 1.0, "a_minus": lam[N - k - 1],
         "a_plus": lam[N - k], "b_minus": lam[-1], "b_plus": math.inf}
    say(f"top slice {gen} N={N}: {k} largest eigenvalues, b_+ = +inf")
    P = zolo.Pencil.from_grid(ctx, gp, leaf_size=16)
    opts = zolo.opts_from_window(w, r1=2, r2=0, n_ss=k + 8)
    Q0 = pencils.gaussian_block(gp.n, k + 8, seed=6, complex_=gp.is_complex)
    eig, vec, st, rc = zolo.zolo_solve(ctx, P, w["a"], w["b"], k, opts, Q0=_dev(Q0))
    say(f"  rc={rc} found {len(eig)} iterations {st['n_iter']} resid {st['max_resid']:.2e}")
    assert rc == 0 and len(eig) == k
    assert np.max(np.abs(np.array(eig) - lam[N - k:]) / np.abs(lam[N - k:])) < 1e-10
    X = vec.cpu().numpy()
    assert np.max(rel_residuals(A, B, np.array(eig), X, inf_norm(A), inf_norm(B))) < 1e-8
    assert sin_max_angle(Xall[:, N - k:], X, B) < 1e-8
    # the library estimates gaps and count itself for the same top interval
    o2 = zolo.zolo_opts_default()
    o2.a_minus = o2.a_plus = o2.b_minus = o2.b_plus = math.nan
    eig2, vec2, st2, rc2 = zolo.zolo_solve(ctx, P, w["a"], w["b"], k, o2)
    say(f"  estimated gaps: rc={rc2} found {len(eig2)} count {st2['inertia_count']} b_plus {st2['b_plus']}")
    assert rc2 == 0 and len(eig2) == k and st2["inertia_count"] == k
    assert math.isinf(st2["b_plus"])



@pytest.mark.parametrize("case", ["pattern", "real_values", "complex_values", "b_not_positive"])
def test_pencil_rejects_bad_pencils(ctx, case):
    """zolo_pencil_create checks what the method assumes (Sec. 1: A Hermitian,
    B Hermitian positive definite; A and B share one CSR pattern) before
    anything reaches the device: an unsymmetric pattern, unsymmetric real values
    and complex values with A_ij != conj(A_ji) give ZOLO_ENOTHERM; a B with a
    non-positive diagonal entry gives ZOLO_EINVAL."""
    import scipy.sparse as sp

    gp = pencils.grid7(4)
    A, B = gp.scipy()
    A = A.tocsr().astype(np.complex128 if case == "complex_values" else np.float64)
    B = B.tocsr().astype(A.dtype)
    n = gp.n
    want = zolo.ZOLO_ENOTHERM
    if case == "pattern":  # an entry (0, n-1) without its mirror (n-1, 0), in both matrices
        E = sp.csr_matrix(([1.0], ([0], [n - 1])), shape=A.shape)
        A = (A + 0.5 * E).tocsr()
        B = (B + 1e-3 * E).tocsr()
    elif case == "real_values":
        A = A.tolil()
        A[0, 1] = A[0, 1] + 0.25
    elif case == "complex_values":
        A = A.tolil()
        A[0, 1] = A[0, 1] + 0.3j
        A[1, 0] = A[1, 0] + 0.3j  # equal imaginary parts: not conjugate
    else:  # b_not_positive
        B = B.tolil()
        B[3, 3] = -1.0
        want = zolo.ZOLO_EINVAL
    A, B = A.tocsr(), B.tocsr()
    A.sort_indices()
    B.sort_indices()
    assert np.array_equal(A.indptr, B.indptr) and np.array_equal(A.indices, B.indices)
    say(f"bad pencil case {case}")
    with pytest.raises(zolo.ZoloError) as e:
        zolo.Pencil(ctx, A.indptr, A.indices, A.data, B.data)
    say(f"  status {e.value.status}: {e.value}")
    assert e.value.status == want
