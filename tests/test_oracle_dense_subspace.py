"""Pins for oracle.dense, oracle.subspace and oracle.sparse: LAPACK (library
special case), brute force on tiny pencils, invariants of the exact filter,
and Algorithm 1's decay on the 10^3 window."""
import json

import numpy as np
import pytest
import scipy.linalg as sla

import pencils
from oracle.dense import count_in, exact_filter, exact_G, jacobi_eigh, pencil_eigh_jacobi, pencil_eigh_lapack, shifted_solve
from oracle.filt import FilterPlan
from oracle.sparse import HybridFilterCPU, count_interval, inertia_neg, kato_temple, window_near, zoloeig_cpu
from oracle.subspace import alg1_exact, b_orthonormality, e_lambda_x, inf_norm, rayleigh_ritz, rel_residuals

from .conftest import golden


@pytest.mark.parametrize("cplx", [False, True])
def test_jacobi_vs_lapack(cplx):
    g = np.random.Generator(np.random.PCG64(7))
    n = 37
    M = g.standard_normal((n, n)) + (1j * g.standard_normal((n, n)) if cplx else 0)
    C = M + M.conj().T
    w, V = jacobi_eigh(C)
    wr = np.linalg.eigvalsh(C)
    assert np.max(np.abs(w - wr)) < 1e-13 * np.linalg.norm(C)
    assert np.max(np.abs(V.conj().T @ V - np.eye(n))) < 1e-13
    assert np.max(np.abs(C @ V - V * w[None, :])) < 1e-12 * np.linalg.norm(C)


def test_two_by_two_pencil_brute_force():
    # det(A - lam B) = 0 solved as a quadratic
    A = np.array([[2.0, 1.0], [1.0, -1.0]])
    B = np.array([[2.0, 0.5], [0.5, 1.0]])
    a = B[0, 0] * B[1, 1] - B[0, 1] ** 2
    b = -(A[0, 0] * B[1, 1] + A[1, 1] * B[0, 0] - 2 * A[0, 1] * B[0, 1])
    c = A[0, 0] * A[1, 1] - A[0, 1] ** 2
    disc = np.sqrt(b * b - 4 * a * c)
    ref = np.sort([(-b - disc) / (2 * a), (-b + disc) / (2 * a)])
    w, X = pencil_eigh_jacobi(A, B)
    assert np.max(np.abs(w - ref)) < 1e-14
    assert np.max(np.abs(X.T @ B @ X - np.eye(2))) < 1e-14


@pytest.mark.parametrize("maker", [lambda: pencils.grid7(4), lambda: pencils.grid7(5, ny=4, nz=3), lambda: pencils.grid27p(3)])
def test_pencil_jacobi_vs_lapack(maker):
    p = maker()
    A, B = (M.toarray() for M in p.scipy())
    assert np.allclose(A, A.conj().T) and np.allclose(B, B.conj().T)
    w, X = pencil_eigh_jacobi(A, B)
    wr, _ = pencil_eigh_lapack(A, B)
    nA = np.linalg.norm(A, 2)
    assert np.max(np.abs(w - wr)) < 1e-12 * nA
    assert np.max(np.abs(X.conj().T @ B @ X - np.eye(p.n))) < 1e-12
    assert np.max(np.abs(A @ X - (B @ X) * w[None, :])) < 1e-12 * nA
    # B is SPD and the count by inertia equals the dense count
    assert np.min(np.linalg.eigvalsh(B)) > 0
    a, b = float(np.percentile(w, 30)) + 1e-7, float(np.percentile(w, 70)) + 1e-7
    As, Bs = p.scipy()
    assert count_interval(As, Bs, a, b) == count_in(w, a, b)
    assert inertia_neg(As, Bs, a) == int(np.sum(w < a))


def _small_setup(n=8, n_lambda=12, r1=2, r2=3):
    fx = json.load(open(golden(f"window_grid7_{n}.json")))
    p = pencils.grid7(n)
    As, Bs = p.scipy()
    A, B = As.toarray(), Bs.toarray()
    lam, X = pencil_eigh_lapack(A, B)
    f = FilterPlan(fx["a_minus"], fx["a_plus"], fx["b_minus"], fx["b_plus"], r1, r2)
    return fx, p, As, Bs, A, B, lam, X, f


def test_exact_filter_invariants():
    fx, p, As, Bs, A, B, lam, X, f = _small_setup()
    # eigenvectors are invariant: R(B^-1 A) x_i = R(lam_i) x_i
    Y = exact_filter(lam, X, B, X[:, :10], f.R)
    assert np.max(np.abs(Y - X[:, :10] * f.R(lam[:10])[None, :])) < 1e-12
    # definition cross-check: R(B^-1 A) V by a dense matrix function of B^-1 A
    V = pencils.gaussian_block(p.n, 3, seed=5)
    Mx = np.linalg.solve(B, A)
    wv, U = np.linalg.eig(Mx)
    Rm = (U * f.R(np.real(wv))[None, :]) @ np.linalg.inv(U)
    assert np.max(np.abs(np.real(Rm @ V) - exact_filter(lam, X, B, V, f.R))) < 1e-9
    # G and the shifted solves (eq. solve / eq. solve2)
    G = exact_G(lam, X, B, np.eye(p.n), f.g)
    s = 1j * np.sqrt(f.c[0])
    Xs = shifted_solve(lam, X, B, V, f.g, s)
    assert np.max(np.abs((G + s * np.eye(p.n)) @ Xs - V)) < 1e-11
    # projector-like: eigenvalues of R(B^-1 A) lie within delta0 of {0, 1}
    Rl = f.R(lam)
    assert np.all(np.minimum(np.abs(Rl), np.abs(Rl - 1.0)) <= f.delta0 * (1 + 1e-8))
    # in-interval count from the filter values
    assert int(np.sum(Rl > 0.5)) == fx["n_lambda"]


def test_hybrid_cpu_filter_matches_definition():
    fx, p, As, Bs, A, B, lam, X, f = _small_setup()
    V = pencils.gaussian_block(p.n, 16, seed=2)
    V, _ = np.linalg.qr(V)
    hf = HybridFilterCPU(As, Bs, f)
    # G through the factors equals the definition
    G1 = hf.apply_G(V)
    G2 = exact_G(lam, X, B, V, f.g)
    assert np.max(np.abs(G1 - G2)) < 1e-11 * np.max(np.abs(G2))
    Y = hf.apply(V, tol=1e-13)
    Ye = exact_filter(lam, X, B, V, f.R)
    assert np.max(np.abs(Y - Ye)) < 1e-10 * np.max(np.abs(Ye))


def test_hybrid_cpu_filter_complex_pencil():
    p = pencils.grid27p(4)
    As, Bs = p.scipy()
    A, B = As.toarray(), Bs.toarray()
    lam, X = pencil_eigh_lapack(A, B)
    w = pencils.window_from_eigenvalues(lam, 30, 6)
    f = FilterPlan(w["a_minus"], w["a_plus"], w["b_minus"], w["b_plus"], 2, 3)
    V = pencils.gaussian_block(p.n, 10, seed=4, complex_=True)
    hf = HybridFilterCPU(As, Bs, f)
    G1 = hf.apply_G(V)
    G2 = exact_G(lam, X, B, V, f.g)
    assert np.max(np.abs(G1 - G2)) < 1e-11 * np.max(np.abs(G2))
    Y = hf.apply(V, tol=1e-12, max_iter=12)
    Ye = exact_filter(lam, X, B, V, f.R)
    assert np.max(np.abs(Y - Ye)) < 1e-10 * np.max(np.abs(Ye))


def test_alg1_decay_config0():
    fx = json.load(open(golden("window_grid7_10.json")))
    p = pencils.grid7(10)
    As, Bs = p.scipy()
    A, B = As.toarray(), Bs.toarray()
    lam, X = pencil_eigh_lapack(A, B)
    f = FilterPlan(fx["a_minus"], fx["a_plus"], fx["b_minus"], fx["b_plus"], 2, 2)
    Q0 = pencils.gaussian_block(p.n, 24, seed=2)
    h = alg1_exact(As, Bs, lam, X, f, fx["a"], fx["b"], Q0, 3)
    res = [x["max_res"] for x in h]
    # residual decays by roughly delta0-per-iteration (delta0 = 3.2e-4 here)
    assert res[0] < 5e-3 and res[1] < 1e-6 and res[2] < 1e-9
    assert res[1] < 1e-2 * res[0] and res[2] < 1e-2 * res[1]
    th = h[-1]["theta"]
    ref = np.array(fx["eigenvalues"])
    assert th.shape == ref.shape
    assert np.max(np.abs(th - ref) / np.abs(ref)) < 1e-12
    assert b_orthonormality(B, h[-1]["X"]) < 1e-12


def test_cpu_zoloeig_small():
    fx, p, As, Bs, A, B, lam, X, f = _small_setup(8, 12, 2, 5)
    Q0 = pencils.gaussian_block(p.n, 18, seed=2)
    out = zoloeig_cpu(As, Bs, f, fx["a"], fx["b"], Q0)
    ref = np.array(fx["eigenvalues"])
    assert out["theta"].shape == ref.shape
    assert np.max(np.abs(out["theta"] - ref) / np.abs(ref)) < 1e-12
    assert np.max(out["res"]) <= 1e-8
    assert e_lambda_x(As, Bs, out["theta"], out["X"], fx["a"], fx["b"]) < 1e-8
    # Kato-Temple bound holds for the returned Ritz values
    gap = min(fx["a_plus"] - fx["a_minus"], fx["b_plus"] - fx["b_minus"])
    kt = kato_temple(As, Bs, out["theta"], out["X"], gap)
    assert np.all(np.abs(out["theta"] - ref) <= kt + 1e-14 * np.abs(ref))
    # n_solv bookkeeping: r * n_ss * sum(n_gmres) for a real pencil
    assert out["n_solv"] == 2 * 18 * int(np.sum(out["n_gmres"]))


def test_rr_rank_revealing_and_metrics():
    fx, p, As, Bs, A, B, lam, X, f = _small_setup()
    # a rank-deficient block: 4 eigenvectors repeated
    Y = np.hstack([X[:, :4], X[:, :4] * 2.0])
    th, Xr, C = rayleigh_ritz(As, Bs, Y)
    assert th.shape[0] == 4
    assert np.max(np.abs(th - lam[:4])) < 1e-12
    r = rel_residuals(As, Bs, lam[:4], X[:, :4], inf_norm(As), inf_norm(Bs))
    assert np.max(r) < 1e-13
    assert inf_norm(As) >= np.linalg.norm(A, 2) - 1e-12


def test_serving_queries_windows_are_consistent():
    """The serving query generator (input construction only) yields windows whose
    eigengaps are the neighbours of a consecutive run of stored eigenvalues."""
    import json

    import pencils

    from .conftest import golden

    c = json.load(open(golden("serving_clusters.json")))
    qs = pencils.serving_queries(c, 64, rate=10.0, seed=3)
    assert len(qs) == 64 and all(qs[i]["t"] <= qs[i + 1]["t"] for i in range(63))
    for q in qs:
        w = q["window"]
        lam = np.asarray(c["clusters"][f"{q['grid']}:{q['center']}"])
        ev = np.asarray(w["eigenvalues"])
        assert 8 <= w["n_lambda"] == len(ev) <= 128
        assert w["a_minus"] < w["a"] < w["a_plus"] == ev[0] <= ev[-1] == w["b_minus"] < w["b"] < w["b_plus"]
        i = int(np.searchsorted(lam, ev[0]))
        assert np.array_equal(lam[i : i + len(ev)], ev)
        assert lam[i - 1] == w["a_minus"] and lam[i + len(ev)] == w["b_plus"]


def test_window_near_and_inertia_complex_hermitian():
    """Shift-invert Lanczos windows and Sylvester inertia counts on a complex
    Hermitian (Peierls) pencil agree with dense LAPACK (library special case)."""
    gp = pencils.grid27p(5, ny=6, nz=4)
    A, B = gp.scipy()
    lam, _ = pencil_eigh_lapack(A.toarray(), B.toarray())
    w, X = window_near(A.tocsc(), B.tocsc(), 0.3, 12)
    idx = np.argsort(np.abs(lam - 0.3))[:12]
    assert np.max(np.abs(np.sort(lam[idx]) - w)) < 1e-10
    assert np.iscomplexobj(X)
    a, b = -1.0, 1.5
    assert count_interval(A, B, a, b) == count_in(lam, a, b)
