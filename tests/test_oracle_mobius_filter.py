"""Pins for oracle.mobius and oracle.filt: the four gap conditions, pole
geometry, the printed worked example, infinite gaps, and the scalar filter's
two evaluation routes and its equioscillating error on Omega."""
import json
import math

import numpy as np
import pytest

from oracle.filt import FilterPlan, order_table, select_r2
from oracle.mobius import Mobius

from .conftest import golden

GAPS = [
    (5.882823443013416, 5.887737557533092, 6.011919794590437, 6.018418278678194),  # config-0 window
    (-1.1, -0.9, 0.9, 1.1),
    (0.0, 1.0, 2.0, 10.0),
    (-3.0, -2.999, 4.0, 4.5),
    (-math.inf, 0.1, 0.7, 0.7001),
    (0.2, 0.3, 0.9, math.inf),
]


@pytest.mark.parametrize("g", GAPS)
def test_mobius_conditions(g):
    am, ap, bm, bp = g
    m = Mobius(*g)
    l1 = m.l1
    # T(a_-) = -l1, T(a_+) = l1, T(b_-) = 1, T(b_+) = -1 (reading of eq. req)
    for x, y in [(am, -l1), (ap, l1), (bm, 1.0), (bp, -1.0)]:
        if math.isinf(x):
            assert abs(m.gamma - y) < 1e-14
        else:
            assert abs(m.T(x) - y) < 1e-12 * max(1.0, abs(y) / max(l1, 1e-300)) * max(1.0, abs(y))
    assert m.check_residual < 1e-11
    assert am < m.alpha < ap and bm < m.beta < bp
    assert -1.0 < m.gamma < -l1 or math.isclose(m.gamma, -1.0) or math.isclose(m.gamma, -l1)
    # cross-ratio identity eps = 4 l1 / (1 - l1)^2
    assert abs(m.eps - 4 * l1 / (1 - l1) ** 2) <= 1e-14 * m.eps
    # exterior maps into [-1, -l1], interior into [l1, 1]
    xs_in = np.linspace(ap, bm, 101)
    t_in = m.T(xs_in)
    assert np.all(t_in >= l1 * (1 - 1e-9)) and np.all(t_in <= 1 + 1e-12)
    xs_out = np.concatenate([np.linspace(bp, bp + 50.0, 101)] if not math.isinf(bp) else [np.array([])])
    if not math.isinf(am):
        xs_out = np.concatenate([xs_out, np.linspace(am - 50.0, am, 101)])
    t_out = m.T(xs_out)
    assert np.all(t_out <= -l1 * (1 - 1e-9)) and np.all(t_out >= -1 - 1e-12)


def test_fig4_worked_example():
    fx = json.load(open(golden("fig4_circle.json")))
    # reading: the printed radius matches gaps +-(0.95, 1.05)
    (am, ap), (bm, bp) = fx["reading_gaps"]
    for r1 in (2, 3, 4):
        f = FilterPlan(am, ap, bm, bp, r1, 2)
        center = 0.5 * (f.mob.alpha + f.mob.beta)
        assert abs(center) < 1e-12
        assert np.max(np.abs(np.abs(f.sigma_hat) - fx["printed_radius"])) < 5e-7
        # and the outer poles of the composite sit on the same circle
    # caption's gaps: radius sqrt(b_- b_+)
    (am, ap), (bm, bp) = fx["printed_gaps"]
    f = FilterPlan(am, ap, bm, bp, 3, 3)
    assert np.max(np.abs(np.abs(f.sigma_hat) - math.sqrt(0.9 * 1.1))) < 1e-12


@pytest.mark.parametrize("g", GAPS[:4])
def test_poles_on_circle_diameter_alpha_beta(g):
    f = FilterPlan(*g, 3, 2)
    c = 0.5 * (f.mob.alpha + f.mob.beta)
    rad = 0.5 * (f.mob.beta - f.mob.alpha)
    assert np.max(np.abs(np.abs(f.sigma_hat - c) - rad)) < 1e-12 * max(1.0, abs(c))


@pytest.mark.parametrize("g", GAPS)
@pytest.mark.parametrize("r1,r2", [(2, 2), (2, 4), (3, 3), (1, 3)])
def test_filter_two_routes_and_error(g, r1, r2):
    am, ap, bm, bp = g
    f = FilterPlan(am, ap, bm, bp, r1, r2)
    lo = (am if not math.isinf(am) else ap - 5.0) - 3.0
    hi = (bp if not math.isinf(bp) else bm + 5.0) + 3.0
    xs = np.concatenate([np.linspace(lo, hi, 20001), [ap, bm]])
    xs = xs[np.abs(xs - f.mob.beta) > 1e-9]
    Rp = f.R_product(xs)
    Rc = f.R_pf(xs)
    assert np.max(np.abs(Rc.imag)) < 1e-11
    assert np.max(np.abs(Rc.real - Rp)) < 5e-11
    # error against the rectangle on Omega is bounded by delta0 and reaches it
    om = ((xs <= am) | (xs >= bp) | ((xs >= ap) & (xs <= bm)))
    inside = (xs >= ap) & (xs <= bm)
    err = np.abs(np.where(inside, 1.0, 0.0) - Rp)[om]
    assert np.max(err) <= f.delta0 * (1 + 1e-8) + 1e-14
    # attained at the gap edges: R(a_+) = 1 - delta0, R(b_-) = 1 - delta0
    assert abs(f.R_product(np.array([ap]))[0] - (1 - f.delta0)) < 1e-12
    assert abs(f.R_product(np.array([bm]))[0] - (1 - f.delta0)) < 1e-12
    # constant term and weights reproduce g(x) = Zhat(T(x); l1)
    gx = f.g(xs[::97]).real
    assert np.max(np.abs(gx - f.inner.rescaled(f.mob.T(xs[::97])))) < 1e-11


def test_order_selection_remark():
    g = GAPS[0]
    tab = order_table(Mobius(*g).l1, 5)
    big = tab > 1e-13
    assert np.all((np.diff(tab, axis=0) < 0) | ~big[1:, :]) and np.all((np.diff(tab, axis=1) < 0) | ~big[:, 1:])
    # by Theorem 2 the composite error depends on r1*r2 only
    assert np.allclose(tab, tab.T, rtol=1e-6, atol=1e-15)
    r2 = select_r2(*g, r1=2, eps=1e-10)
    assert FilterPlan(*g, 2, r2).delta0 <= 1e-10 < FilterPlan(*g, 2, r2 - 1).delta0
    # config-0 values: l1 = 4.74e-4, l2 = 0.3998 for r1 = 2
    f = FilterPlan(*g, 2, 2)
    assert abs(f.l1 - 4.7367796e-4) < 1e-10 and abs(f.l2 - 0.39977654) < 1e-7
