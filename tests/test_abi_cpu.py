"""CPU-side checks of the C ABI library: it loads, exports every declared
symbol, its host planner agrees with the oracle, its host nested dissection
produces valid orderings, and argument errors come back as status codes."""
import math
import os
import re

import numpy as np
import pytest

import pencils
from oracle.contour import ContourFilter, SingleZolo
from oracle.filt import FilterPlan

from .conftest import ROOT

zolo = pytest.importorskip("paper_1701_08935_amd")


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "zolo.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(zolo_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = zolo.lib()
    names = _declared_symbols()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert L.zolo_version().decode().startswith("zolo")


GAPS = [
    (5.882823443013416, 5.887737557533092, 6.011919794590437, 6.018418278678194),
    (-1.1, -0.9, 0.9, 1.1),
    (-1.05, -0.95, 0.95, 1.05),
    (0.0, 1.0, 2.0, 10.0),
    (-3.0, -2.999, 4.0, 4.5),
    (-math.inf, 0.1, 0.7, 0.7001),
    (0.2, 0.3, 0.9, math.inf),
    (6.0, 6.0 + 1e-7, 6.01, 6.01 + 1e-7),  # l1 ~ 2.5e-11
]


@pytest.mark.parametrize("g", GAPS)
@pytest.mark.parametrize("r1,r2", [(1, 1), (2, 2), (2, 5), (3, 3), (4, 4), (2, 8)])
def test_planner_matches_oracle(g, r1, r2):
    co = zolo.zolo_filter_plan(*g, r1, r2)
    f = FilterPlan(*g, r1, r2)
    assert co.r1 == r1 and co.r2 == r2
    rel = lambda x, y: abs(x - y) / max(abs(y), 1e-300)  # noqa: E731
    assert rel(co.l1, f.l1) < 1e-13
    assert abs(co.l2 - f.l2) < 1e-13
    span = max(abs(x) for x in g if math.isfinite(x)) + 1.0
    assert abs(co.alpha - f.mob.alpha) < 1e-13 * span and abs(co.beta - f.mob.beta) < 1e-13 * span
    # the oracle solves the gap conditions as a 3x3 linear system; its own
    # fourth-condition residual bounds its error at extreme l1
    assert rel(co.gamma, f.mob.gamma) < 1e-12 + 10 * f.mob.check_residual
    assert rel(co.M_hat, f.M_hat) < 1e-12 and abs(co.c0 - f.c0) < 1e-12 * max(1.0, abs(f.c0))
    assert rel(co.M, f.M) < 1e-12
    assert abs(co.delta0 - f.delta0) < 1e-15 + 1e-10 * f.delta0
    sig = np.array(co.sigma_hat_re[:r1]) + 1j * np.array(co.sigma_hat_im[:r1])
    w = np.array(co.w_hat_re[:r1]) + 1j * np.array(co.w_hat_im[:r1])
    slack = 10 * f.mob.check_residual
    assert np.max(np.abs(sig - f.sigma_hat)) < (1e-13 + slack) * span
    assert np.max(np.abs(w - f.w_hat)) < (1e-12 + slack) * max(1.0, np.max(np.abs(f.w_hat)))
    assert np.max(np.abs(np.array(co.c[:r2]) / f.c - 1)) < 1e-12
    assert np.max(np.abs(np.array(co.a[:r2]) - f.a)) < 1e-12
    assert np.max(np.abs(np.array(co.c_hat[:r1]) / f.c_hat - 1)) < 1e-12


def test_planner_auto_r2_and_errors():
    g = GAPS[0]
    co = zolo.zolo_filter_plan(*g, 2, 0, 1e-10)
    assert co.delta0 <= 1e-10
    assert zolo.zolo_filter_plan(*g, 2, co.r2 - 1).delta0 > 1e-10
    for bad in [(1.0, 0.5, 2.0, 3.0), (-math.inf, 0.0, 1.0, math.inf), (0.0, 1.0, 1.0, 2.0)]:
        with pytest.raises(zolo.ZoloError) as e:
            zolo.zolo_filter_plan(*bad, 2, 2)
        assert e.value.status == zolo.ZOLO_EINVAL
    with pytest.raises(zolo.ZoloError):
        zolo.zolo_filter_plan(*g, 0, 2)
    with pytest.raises(zolo.ZoloError):
        zolo.zolo_filter_plan(*g, 2, 99)


def _pole_form(co, x):
    """R(x) = s0 + s1 M_hat [c0 + sum 2 Re(w_hat_j / (x - sigma_hat_j))] from the coefficient set."""
    r = co.r1
    sig = np.array(co.sigma_hat_re[:r]) + 1j * np.array(co.sigma_hat_im[:r])
    w = np.array(co.w_hat_re[:r]) + 1j * np.array(co.w_hat_im[:r])
    g = co.M_hat * (co.c0 + sum(2.0 * np.real(wj / (x - sj)) for sj, wj in zip(sig, w)))
    return 0.5 * (g + 1.0) if co.kind == zolo.ZOLO_FILTER_ZOLO else g


@pytest.mark.parametrize("kind,name", [(zolo.ZOLO_FILTER_TRAPEZOID, "trapezoid"), (zolo.ZOLO_FILTER_GAUSS, "gauss")])
@pytest.mark.parametrize("q", [1, 2, 3, 4, 8, 16])
@pytest.mark.parametrize("ab", [(-1.0, 1.0), (5.8877, 6.0119), (-3.0, 4.0)])
def test_contour_plan_matches_oracle(kind, name, q, ab):
    co = zolo.zolo_filter_plan_kind(kind, *ab, r=q)
    f = ContourFilter(name, *ab, 2 * q)
    assert co.kind == kind and co.r1 == q
    sig = np.array(co.sigma_hat_re[:q]) + 1j * np.array(co.sigma_hat_im[:q])
    order = np.argsort(sig.real)
    ref = np.argsort(f.z.real)
    span = max(abs(ab[0]), abs(ab[1]))
    assert np.max(np.abs(sig[order] - f.z[ref])) < 1e-14 * span
    assert np.all(sig.imag > 0)
    c, rho = 0.5 * (ab[0] + ab[1]), 0.5 * (ab[1] - ab[0])
    x = np.concatenate([np.linspace(ab[0] - 3 * rho, ab[1] + 3 * rho, 997), [c, ab[0] - 10 * rho]])
    assert np.max(np.abs(_pole_form(co, x) - f.R(x))) < 1e-13


@pytest.mark.parametrize("g", GAPS[:5])
@pytest.mark.parametrize("r", [1, 2, 3, 5])
def test_single_zolo_plan_matches_oracle(g, r):
    co = zolo.zolo_filter_plan_kind(zolo.ZOLO_FILTER_ZOLO, 0.5 * (g[0] + g[1]), 0.5 * (g[2] + g[3]), *g, r=r)
    f = SingleZolo(*g, r)
    assert co.kind == zolo.ZOLO_FILTER_ZOLO and co.r1 == r
    lo, hi = g[0] - (g[3] - g[0]), g[3] + (g[3] - g[0])
    x = np.linspace(lo, hi, 1501)
    x = x[np.min(np.abs(x[:, None] - np.array(co.sigma_hat_re[:r])[None, :]), axis=1) > 1e-9 * (hi - lo)]
    assert np.max(np.abs(_pole_form(co, x) - f.R(x))) < 1e-10


def test_filter_plan_kind_errors():
    for args in [(7, -1.0, 1.0), (zolo.ZOLO_FILTER_TRAPEZOID, 1.0, -1.0), (zolo.ZOLO_FILTER_GAUSS, -1.0, 1.0, 0),
                 (zolo.ZOLO_FILTER_GAUSS, -1.0, math.inf)]:
        kind, a, b = args[:3]
        r = args[3] if len(args) > 3 else 4
        with pytest.raises(zolo.ZoloError) as e:
            zolo.zolo_filter_plan_kind(kind, a, b, r=r)
        assert e.value.status == zolo.ZOLO_EINVAL
    with pytest.raises(zolo.ZoloError):
        zolo.zolo_filter_plan_kind(zolo.ZOLO_FILTER_ZOLO, -1.0, 1.0, r=2)  # gaps required


def _check_nd(p, perm, info):
    n = p.n
    assert sorted(perm.tolist()) == list(range(n))
    assert info["fronts"] >= 1 and info["levels"] >= 1
    assert info["panel_entries"] >= p.nnz // 2


@pytest.mark.parametrize("maker", [lambda: pencils.grid7(10), lambda: pencils.grid7(9, ny=5, nz=7),
                                   lambda: pencils.grid27p(6), lambda: pencils.grid7(16)])
def test_symbolic_geometric_and_graph(maker):
    p = maker()
    perm, info = zolo.zolo_symbolic(p.rowptr, p.colind, p.grid, 32)
    _check_nd(p, perm, info)
    perm2, info2 = zolo.zolo_symbolic(p.rowptr, p.colind, None, 32)
    _check_nd(p, perm2, info2)
    # the geometric dissection should not be worse than 3x the generic one in flops
    assert info["flops"] <= 3.0 * info2["flops"]


def test_symbolic_fill_covers_exact_elimination():
    # brute force on a tiny grid: the exact fill of a no-pivot elimination in
    # the returned order must fit in the front structure (panel entries cover
    # every nonzero of L).
    p = pencils.grid7(5)
    perm, info = zolo.zolo_symbolic(p.rowptr, p.colind, p.grid, 8)
    A, _ = p.scipy()
    M = (A.toarray() != 0)[np.ix_(perm, perm)].astype(int)
    n = p.n
    nnzL = 0
    for k in range(n):
        rows = np.nonzero(M[k + 1 :, k])[0] + k + 1
        nnzL += len(rows) + 1
        M[np.ix_(rows, rows)] = 1
    assert info["panel_entries"] >= nnzL


def test_symbolic_rejects_bad_csr():
    p = pencils.grid7(3)
    bad = p.colind.copy()
    bad[3] = 10**6
    with pytest.raises(zolo.ZoloError):
        zolo.zolo_symbolic(p.rowptr, bad, None, 8)
