"""Pins of the comparison filters (oracle/contour.py): the trapezoidal rule's
closed form 1/(1 + t^p), exact values at the centre, the symmetry of the
Gauss-Legendre filter about the centre, convergence to the indicator, and the
single Zolotarev filter's pole form against its product form and against the
exact error bound delta_1/2 on the region outside the gaps."""
import numpy as np
import pytest

from oracle.contour import ContourFilter, SingleZolo, trapezoid_closed_form


@pytest.mark.parametrize("p", [2, 4, 8, 16, 32])
def test_trapezoid_closed_form(p):
    a, b = 0.3, 1.7
    x = np.linspace(-2.0, 4.0, 2001)
    x = x[(np.abs(x - a) > 1e-3) & (np.abs(x - b) > 1e-3)]
    f = ContourFilter("trapezoid", a, b, p)
    assert np.max(np.abs(f.R(x) - trapezoid_closed_form(x, a, b, p))) < 1e-13


@pytest.mark.parametrize("kind", ["trapezoid", "gauss"])
@pytest.mark.parametrize("p", [4, 8, 16])
def test_contour_centre_and_symmetry(kind, p):
    a, b = -1.0, 3.0
    f = ContourFilter(kind, a, b, p)
    assert abs(f.R(np.array([1.0]))[0] - 1.0) < 1e-14  # the weights sum to 2 pi over the circle
    t = np.array([0.2, 0.7, 1.3, 2.5, 10.0])
    assert np.max(np.abs(f.R(1.0 + 2.0 * t) - f.R(1.0 - 2.0 * t))) < 1e-13


@pytest.mark.parametrize("kind", ["trapezoid", "gauss"])
def test_contour_converges_to_indicator(kind):
    a, b = -1.0, 1.0
    x = np.array([-3.0, -2.0, -0.5, 0.0, 0.5, 2.0, 3.0])
    ind = ((x > a) & (x < b)).astype(float)
    errs = [np.max(np.abs(ContourFilter(kind, a, b, p).R(x) - ind)) for p in (8, 16, 32, 64)]
    assert all(e2 < e1 for e1, e2 in zip(errs, errs[1:]))
    assert errs[-1] < 1e-10


@pytest.mark.parametrize("gap,r", [(1e-2, 2), (1e-2, 4), (1e-6, 3)])
def test_single_zolo_pole_form_and_error(gap, r):
    f = SingleZolo(-1.0 - gap, -1.0 + gap, 1.0 - gap, 1.0 + gap, r)
    x = np.concatenate([np.linspace(-5, -1 - gap, 400), np.linspace(-1 + gap, 1 - gap, 400),
                        np.linspace(1 + gap, 5, 400)])
    # the pole form loses about eps / gap near the gap ends (poles that close to the axis)
    assert np.max(np.abs(f.R(x) - f.R_product(x))) < 1e-16 / gap
    ind = ((x > -1) & (x < 1)).astype(float)
    err = np.max(np.abs(f.R(x) - ind))
    # R = (Zhat + 1)/2 and Zhat maps the gaps' exterior into [-1, -l2] and their interior into
    # [l2, 1], l2 = (1 - delta)/(1 + delta) = lhat with nome q(lhat) = q(l1)^(1/(2r)) (exact, mpmath):
    # the largest error on the region outside the gaps is (1 - lhat)/2, attained at the gap ends
    import mpmath

    mpmath.mp.dps = 40
    lhat = float(mpmath.kfrom(q=mpmath.qfrom(k=mpmath.mpf(f.plan.l1)) ** (mpmath.mpf(1) / (2 * r))))
    assert abs(err - 0.5 * (1.0 - lhat)) <= 1e-9 * max(1.0, 0.5 * (1.0 - lhat)) + 1e-13
