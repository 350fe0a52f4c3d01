"""GPU parity: the HIP path (through the C ABI) against the oracle.

Every test prints the case it is about to run before touching the GPU.
Tolerances: SpMM 1e-13 relative (reordered sums of at most 27 terms);
pole solves 1e-10 relative (kappa(A - sigma B) ~ 1e3-1e4 times FP64 rounding);
operator G and the filter 1e-10/1e-9 relative (G combines r1 solves; the filter
adds the GMRES tolerance 1e-12 used here); eigenpairs: exact count,
eigenvalues 1e-10 relative, residual 1e-8, B-orthonormality 1e-10.
"""
import json
import sys

import numpy as np
import pytest

import pencils
from oracle.dense import exact_filter, exact_G, pencil_eigh_lapack
from oracle.filt import FilterPlan
from oracle.subspace import b_orthonormality, e_lambda_x, inf_norm, norm2_est, rel_residuals

from .conftest import golden

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


def _window(n):
    return json.load(open(golden(f"window_grid7_{n}.json")))


@pytest.mark.parametrize("shape", [(10, 10, 10), (13, 9, 11), (4, 4, 4)])
@pytest.mark.parametrize("p", [24, 13, 1])
def test_spmm_parity(ctx, shape, p):
    say(f"spmm grid {shape} p={p}")
    gp = pencils.grid7(shape[0], ny=shape[1], nz=shape[2])
    A, B = gp.scipy()
    X = pencils.gaussian_block(gp.n, p, seed=11)
    P = zolo.Pencil.from_grid(ctx, gp, leaf_size=16)
    for which, M in ((0, A), (1, B)):
        Y = zolo.zolo_spmm(P, which, _dev(X)).cpu().numpy()
        ref = M @ X
        assert np.max(np.abs(Y - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("n,leaf,use_grid", [(8, 16, True), (10, 64, True), (10, 8, False), (12, 32, True)])
def test_pole_solve_parity(ctx, n, leaf, use_grid):
    say(f"pole solve grid {n}^3 leaf={leaf} grid={use_grid}")
    w = _window(n)
    gp = pencils.grid7(n)
    A, B = gp.scipy()
    co = zolo.zolo_filter_plan(w["a_minus"], w["a_plus"], w["b_minus"], w["b_plus"], 2, 3)
    P = zolo.Pencil.from_grid(ctx, gp, leaf_size=leaf, use_grid=use_grid)
    F = zolo.Factors(ctx, P, co, zolo.ZOLO_PREC_FP64)
    V = pencils.gaussian_block(gp.n, 7, seed=3)
    T = B @ V
    for j in range(2):
        sig = co.sigma_hat_re[j] + 1j * co.sigma_hat_im[j]
        X = zolo.zolo_pole_solve(F, j, _dev(T)).cpu().numpy()
        ref = np.linalg.solve((A - sig * B).toarray(), T.astype(np.complex128))
        err = np.max(np.abs(X - ref)) / np.max(np.abs(ref))
        say(f"  pole {j}: rel err {err:.2e}")
        assert err < 1e-10


def test_pole_solve_mixed_refines_to_fp64(ctx):
    say("pole solve mixed precision grid 10^3")
    n = 10
    w = _window(n)
    gp = pencils.grid7(n)
    A, B = gp.scipy()
    co = zolo.zolo_filter_plan(w["a_minus"], w["a_plus"], w["b_minus"], w["b_plus"], 2, 3)
    P = zolo.Pencil.from_grid(ctx, gp, leaf_size=32)
    F = zolo.Factors(ctx, P, co, zolo.ZOLO_PREC_MIXED)
    V = pencils.gaussian_block(gp.n, 5, seed=4)
    T = B @ V
    sig = co.sigma_hat_re[0] + 1j * co.sigma_hat_im[0]
    X = zolo.zolo_pole_solve(F, 0, _dev(T)).cpu().numpy()
    ref = np.linalg.solve((A - sig * B).toarray(), T.astype(np.complex128))
    err = np.max(np.abs(X - ref)) / np.max(np.abs(ref))
    say(f"  mixed rel err {err:.2e}")
    assert err < 1e-10


@pytest.mark.parametrize("n", [8, 10])
def test_apply_G_and_filter_parity(ctx, n):
    say(f"G and filter grid {n}^3")
    w = _window(n)
    gp = pencils.grid7(n)
    A, B = gp.scipy()
    lam, Xall = pencil_eigh_lapack(A.toarray(), B.toarray())
    for r2 in (2, 5):
        f = FilterPlan(w["a_minus"], w["a_plus"], w["b_minus"], w["b_plus"], 2, r2)
        co = zolo.zolo_filter_plan(w["a_minus"], w["a_plus"], w["b_minus"], w["b_plus"], 2, r2)
        P = zolo.Pencil.from_grid(ctx, gp, leaf_size=32)
        F = zolo.Factors(ctx, P, co, zolo.ZOLO_PREC_FP64)
        V = pencils.gaussian_block(gp.n, 12, seed=5)
        G = zolo.zolo_apply_G(F, _dev(V)).cpu().numpy()
        Gref = exact_G(lam, Xall, B, V, f.g)
        eg = np.max(np.abs(G - Gref)) / np.max(np.abs(Gref))
        say(f"  r2={r2} G rel err {eg:.2e}")
        assert eg < 1e-10
        Y, st = zolo.zolo_filter_apply(F, _dev(V), tol=1e-12, max_iter=60)
        Y = Y.cpu().numpy()
        Yref = exact_filter(lam, Xall, B, V, f.R)
        ey = np.max(np.abs(Y - Yref)) / np.max(np.abs(Yref))
        say(f"  r2={r2} filter rel err {ey:.2e} gmres {st}")
        assert ey < 1e-9


@pytest.mark.parametrize("precision", [0, 1])
def test_solve_window_10(ctx, precision):
    say(f"zolo_solve grid 10^3 window 16 precision={precision}")
    w = _window(10)
    gp = pencils.grid7(10)
    A, B = gp.scipy()
    P = zolo.Pencil.from_grid(ctx, gp, leaf_size=32)
    Q0 = pencils.gaussian_block(gp.n, 24, seed=2)
    opts = zolo.opts_from_window(w, r1=2, r2=0, n_ss=24, precision=precision)
    eig, vec, st, rc = zolo.zolo_solve(ctx, P, w["a"], w["b"], 16, opts, Q0=_dev(Q0))
    say(f"  rc={rc} stats={ {k: st[k] for k in ('n_iter', 'n_gmres_total', 'max_resid', 'b_orth', 'r2', 'n_found')} }")
    assert rc == 0
    ref = np.array(w["eigenvalues"])
    assert len(eig) == 16
    assert np.max(np.abs(np.array(eig) - ref) / np.abs(ref)) < 1e-10
    X = vec.cpu().numpy()
    lam = np.array(eig)
    r = rel_residuals(A, B, lam, X, inf_norm(A), inf_norm(B))
    r2 = rel_residuals(A, B, lam, X, norm2_est(A, iters=300), norm2_est(B, iters=300))
    e = e_lambda_x(A, B, lam, X, w["a"], w["b"])
    bo = b_orthonormality(B, X)
    say(f"  residual inf-norm {np.max(r):.2e}, 2-norm {np.max(r2):.2e}; e_lambda_x {e:.2e} "
        f"(library {st['e_lambda_x']:.2e}); B-orth {bo:.2e} (library {st['b_orth']:.2e})")
    assert np.max(r) < 1e-8 and np.max(r2) < 1e-8
    assert bo < 1e-10
    # the library's own figures, recomputed from the returned vectors by the oracle
    assert st["max_resid"] < 1e-8
    assert abs(st["max_resid"] - np.max(r)) <= 0.05 * np.max(r) + 1e-14
    assert abs(st["e_lambda_x"] - e) <= 0.05 * e + 1e-14
    assert st["b_orth"] <= 1e-10


def test_solve_window_10_large_subspace(ctx):
    """A subspace of 160 for 16 wanted eigenvalues: the 160 x 160 Rayleigh-Ritz
    Gram matrix (200 KB in FP64) does not fit in one workgroup's LDS, so its
    eigensolve runs from global memory, and the filtered block is rank
    deficient, so the rank truncation is exercised too."""
    say("zolo_solve grid 10^3 window 16, subspace 160")
    w = _window(10)
    gp = pencils.grid7(10)
    A, B = gp.scipy()
    P = zolo.Pencil.from_grid(ctx, gp, leaf_size=32)
    Q0 = pencils.gaussian_block(gp.n, 160, seed=4)
    opts = zolo.opts_from_window(w, r1=2, r2=0, n_ss=160)
    eig, vec, st, rc = zolo.zolo_solve(ctx, P, w["a"], w["b"], 16, opts, Q0=_dev(Q0))
    say(f"  rc={rc} stats={ {k: st[k] for k in ('n_iter', 'n_gmres_total', 'max_resid', 'b_orth', 'n_found')} }")
    assert rc == 0
    ref = np.array(w["eigenvalues"])
    assert len(eig) == 16
    assert np.max(np.abs(np.array(eig) - ref) / np.abs(ref)) < 1e-10
    X = vec.cpu().numpy()
    r = np.linalg.norm(A @ X - (B @ X) * np.array(eig)[None, :], axis=0) / (
        (inf_norm(A) + np.abs(eig) * inf_norm(B)) * np.linalg.norm(X, axis=0))
    assert np.max(r) < 1e-8
    assert np.max(np.abs(X.T @ (B @ X) - np.eye(16))) < 1e-10


@pytest.mark.parametrize("gen,shape,p", [("grid7", (13, 9, 11), 1), ("grid7", (13, 9, 11), 130),
                                         ("grid7", (10, 10, 10), 64), ("grid27p", (7, 8, 6), 37),
                                         ("grid27p", (5, 5, 5), 200)])
def test_residuals_parity(ctx, gen, shape, p):
    """zolo_residuals against the oracle's residual definition: random pairs (O(1)
    residuals) and, on grid7 10^3, exact eigenpairs (residuals at rounding level)."""
    say(f"residuals {gen} {shape} p={p}")
    gp = getattr(pencils, gen)(shape[0], ny=shape[1], nz=shape[2])
    A, B = gp.scipy()
    cx = gen == "grid27p"
    P = zolo.Pencil.from_grid(ctx, gp, leaf_size=16)
    X = pencils.gaussian_block(gp.n, p, seed=5, complex_=cx)
    lam = np.random.Generator(np.random.PCG64(6)).uniform(-3.0, 9.0, p)
    nA, nB = inf_norm(A), inf_norm(B)
    got = zolo.zolo_residuals(P, _dev(X), _dev(lam)).cpu().numpy()
    ref = rel_residuals(A, B, lam, X, nA, nB)
    assert np.max(np.abs(got - ref) / ref) < 1e-12
    if shape == (10, 10, 10):
        ev, V = pencil_eigh_lapack(A.toarray(), B.toarray())
        idx = np.arange(100, 100 + p)
        Xe, le = np.ascontiguousarray(V[:, idx]), ev[idx]
        got = zolo.zolo_residuals(P, _dev(Xe), _dev(le)).cpu().numpy()
        ref = rel_residuals(A, B, le, Xe, nA, nB)
        say(f"  exact pairs: max {got.max():.2e} (oracle {ref.max():.2e})")
        assert got.max() < 1e-14 and np.max(np.abs(got - ref)) < 1e-14


def test_result_vector_accessors(ctx):
    """The host copy of the eigenvectors equals the device copy, and the result's own
    device pointer is exported with ld = count."""
    say("result accessors: host copy, device copy, device pointer (grid 10^3)")
    w = _window(10)
    gp = pencils.grid7(10)
    P = zolo.Pencil.from_grid(ctx, gp, leaf_size=32)
    Q0 = _dev(pencils.gaussian_block(gp.n, 24, seed=2))
    opts = zolo.opts_from_window(w, r1=2, r2=0, n_ss=24)
    eig_d, vec_d, _, rc_d = zolo.zolo_solve(ctx, P, w["a"], w["b"], 16, opts, Q0=Q0)
    eig_h, vec_h, _, rc_h = zolo.zolo_solve(ctx, P, w["a"], w["b"], 16, opts, Q0=Q0, host_vectors=True)
    assert rc_d == rc_h == 0 and eig_d == eig_h
    assert isinstance(vec_h, np.ndarray) and np.array_equal(vec_d.cpu().numpy(), vec_h)
    import ctypes

    L = zolo.lib()
    h = ctypes.c_void_p()
    rc = L.zolo_solve(ctx.h, P.h, w["a"], w["b"], 16, ctypes.byref(opts), ctypes.c_void_p(Q0.data_ptr()),
                      zolo._stream(), ctypes.byref(h))
    try:
        assert rc == 0
        ld = ctypes.c_int64(-1)
        ptr = L.zolo_result_device_vectors(h, ctypes.byref(ld))
        assert ptr and ld.value == L.zolo_result_count(h) == 16
    finally:
        L.zolo_result_free(h)


def test_wrong_eigengap_returns_egap(ctx):
    """A stated gap (a_-, a_+) that contains an eigenvalue (a_+ moved past the first
    eigenvalue of the window): the eigenvalue still converges inside (a, b), and the
    call reports ZOLO_EGAP with the results filled."""
    say("EGAP: grid 10^3 window with a_+ moved past the first eigenvalue")
    w = dict(_window(10))
    lam = np.array(w["eigenvalues"])
    w["a_plus"] = 0.5 * (lam[0] + lam[1])
    gp = pencils.grid7(10)
    P = zolo.Pencil.from_grid(ctx, gp, leaf_size=32)
    Q0 = _dev(pencils.gaussian_block(gp.n, 24, seed=2))
    opts = zolo.opts_from_window(w, r1=2, r2=0, n_ss=24, max_subspace_iter=8)
    eig, vec, st, rc = zolo.zolo_solve(ctx, P, w["a"], w["b"], 16, opts, Q0=Q0,
                                       allow=(zolo.ZOLO_EGAP, zolo.ZOLO_ENOCONV))
    say(f"  rc={rc} found={len(eig)} iter={st['n_iter']} resid={st['max_resid']:.2e}")
    assert rc == zolo.ZOLO_EGAP
    assert "eigengap" in zolo.lib().zolo_last_error().decode()
    assert len(eig) == 16 and abs(eig[0] - lam[0]) <= 1e-10 * abs(lam[0])


def test_hbm_budget(ctx):
    """A device-memory budget below what a query needs fails the query with ZOLO_ENOMEM
    (before any allocation beyond it); lifting it lets the same query run."""
    say("HBM budget: grid 10^3 query under a 1 MiB budget, then without a budget")
    w = _window(10)
    gp = pencils.grid7(10)
    P = zolo.Pencil.from_grid(ctx, gp, leaf_size=32)
    opts = zolo.opts_from_window(w, r1=2, r2=0, n_ss=24)
    ctx.set_hbm_budget(1 << 20)
    try:
        with pytest.raises(zolo.ZoloError) as ei:
            zolo.zolo_solve(ctx, P, w["a"], w["b"], 16, opts)
        assert ei.value.status == zolo.ZOLO_ENOMEM and "budget" in str(ei.value)
    finally:
        ctx.set_hbm_budget(0)
    eig, _, _, rc = zolo.zolo_solve(ctx, P, w["a"], w["b"], 16, opts)
    assert rc == 0 and len(eig) == 16


def test_b_not_positive_definite_rejected(ctx):
    say("pencil with a non-positive diagonal entry of B")
    gp = pencils.grid7(4)
    bv = np.array(gp.b_vals, dtype=np.float64)
    d = [e for i in range(gp.n) for e in range(gp.rowptr[i], gp.rowptr[i + 1]) if gp.colind[e] == i]
    bv[d[5]] = -0.5
    with pytest.raises(zolo.ZoloError) as ei:
        zolo.Pencil(ctx, gp.rowptr, gp.colind, gp.a_vals, bv, gp.grid, 16)
    assert ei.value.status == zolo.ZOLO_EINVAL and "positive definite" in str(ei.value)
