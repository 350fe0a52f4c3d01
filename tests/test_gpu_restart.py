"""GPU parity of restarted multi-shift block GMRES (eq. solve2 with collinear
restarts): the filter block with restarts forced well before convergence must
match the oracle's exact filter R(B^-1 A) V on the dense eigendecomposition, as
the unrestarted run does, on real and complex Hermitian pencils; and a full
query with restarts finds the window's eigenpairs.

Tolerance: 1e-9 relative to the largest entry (GMRES to 1e-12 per shift and
column, as in the unrestarted filter tests).
"""
import json
import math
import sys

import numpy as np
import pytest

import pencils
from oracle.dense import exact_filter, pencil_eigh_lapack
from oracle.filt import FilterPlan
from oracle.subspace import inf_norm, rel_residuals

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


def _check_restarted(F, V, Yref, label):
    Y0, st0 = zolo.zolo_filter_apply(F, _dev(V), tol=1e-12, max_iter=200, restart=0)
    e0 = np.max(np.abs(Y0.cpu().numpy() - Yref)) / np.max(np.abs(Yref))
    k = st0["n_gmres"]
    say(f"  {label}: unrestarted {k} steps, rel err {e0:.2e}")
    assert e0 < 1e-9 and st0["restarts"] == 0
    for rs in sorted({max(2, k // 3), max(2, k // 2)}):
        if rs >= k:
            continue
        Y, st = zolo.zolo_filter_apply(F, _dev(V), tol=1e-12, max_iter=400, restart=rs)
        err = np.max(np.abs(Y.cpu().numpy() - Yref)) / np.max(np.abs(Yref))
        say(f"  {label}: restart {rs}: {st['n_gmres']} steps, {st['restarts']} restarts, rel err {err:.2e}")
        assert st["restarts"] >= 1
        assert st["worst_resid"] <= 1e-12
        assert err < 1e-9


@pytest.mark.parametrize("r1,r2", [(1, 3), (2, 4)])
def test_restarted_filter_real(ctx, r1, r2):
    say(f"restarted filter grid7 10^3 r1={r1} r2={r2}")
    w = json.load(open(golden("window_grid7_10.json")))
    gp = pencils.grid7(10)
    A, B = gp.scipy()
    lam, Xall = pencil_eigh_lapack(A.toarray(), B.toarray())
    f = FilterPlan(w["a_minus"], w["a_plus"], w["b_minus"], w["b_plus"], r1, r2)
    co = zolo.zolo_filter_plan(w["a_minus"], w["a_plus"], w["b_minus"], w["b_plus"], r1, r2)
    P = zolo.Pencil.from_grid(ctx, gp, leaf_size=32)
    F = zolo.Factors(ctx, P, co, zolo.ZOLO_PREC_FP64)
    V = pencils.gaussian_block(gp.n, 12, seed=5)
    _check_restarted(F, V, exact_filter(lam, Xall, B, V, f.R), "real")


def test_restarted_filter_complex(ctx):
    say("restarted filter grid27p 7x8x6 (complex Hermitian) r1=1 r2=3")
    gp = pencils.grid27p(7, ny=8, nz=6)
    A, B = gp.scipy()
    lam, Xall = pencil_eigh_lapack(A.toarray(), B.toarray())
    s0, cnt = 40, 12
    am, ap, bm, bp = lam[s0 - 1], lam[s0], lam[s0 + cnt - 1], lam[s0 + cnt]
    f = FilterPlan(am, ap, bm, bp, 1, 3)
    co = zolo.zolo_filter_plan(am, ap, bm, bp, 1, 3)
    P = zolo.Pencil.from_grid(ctx, gp, leaf_size=16)
    F = zolo.Factors(ctx, P, co, zolo.ZOLO_PREC_FP64)
    V = pencils.gaussian_block(gp.n, 9, seed=8, complex_=True)
    _check_restarted(F, V, exact_filter(lam, Xall, B, V, f.R), "complex")


@pytest.mark.parametrize("restart", [3, 5])
def test_solve_with_restarts(ctx, restart):
    say(f"zolo_solve grid7 10^3 window 16, r1=1, gmres_restart={restart}")
    w = json.load(open(golden("window_grid7_10.json")))
    gp = pencils.grid7(10)
    A, B = gp.scipy()
    P = zolo.Pencil.from_grid(ctx, gp, leaf_size=32)
    Q0 = pencils.gaussian_block(gp.n, 24, seed=2)
    opts = zolo.opts_from_window(w, r1=1, r2=0, n_ss=24, gmres_restart=restart, max_gmres_iter=300)
    eig, vec, st, rc = zolo.zolo_solve(ctx, P, w["a"], w["b"], 16, opts, Q0=_dev(Q0))
    say(f"  rc={rc} iterations {st['n_iter']} gmres {st['n_gmres_total']} restarts {st['n_restart']} "
        f"resid {st['max_resid']:.2e}")
    assert rc == 0 and st["n_restart"] >= 1
    ref = np.array(w["eigenvalues"])
    assert len(eig) == 16
    assert np.max(np.abs(np.array(eig) - ref) / np.abs(ref)) < 1e-10
    r = rel_residuals(A, B, np.array(eig), vec.cpu().numpy(), inf_norm(A), inf_norm(B))
    assert np.max(r) < 1e-8
