"""Pins for oracle.zolotarev: mpmath coefficients, closed forms, equioscillation,
the exact nome formula for delta, Theorem 2 and the partial-fraction forms."""
import math

import mpmath
import numpy as np
import pytest

from oracle.zolotarev import Zolo, composite, composite_delta

mpmath.mp.dps = 40

CASES = [(1, 0.5), (2, 0.5), (2, 1e-2), (3, 4.7e-4), (4, 1e-2), (2, 1e-6), (3, 2.5e-13), (6, 1e-3)]


def _c_mpmath(r, l):
    l = mpmath.mpf(l)
    m = 1 - l * l
    Kp = mpmath.ellipk(m)
    out = []
    for j in range(1, 2 * r):
        u = j * Kp / (2 * r)
        sn = mpmath.ellipfun("sn", u, m=m)
        cn = mpmath.ellipfun("cn", u, m=m)
        out.append(float(l * l * sn * sn / (cn * cn)))
    return np.array(out)


@pytest.mark.parametrize("r,l", CASES)
def test_coefficients_match_mpmath(r, l):
    z = Zolo(r, l)
    ref = _c_mpmath(r, l)
    assert np.max(np.abs(z.c - ref) / ref) < 1e-13


def test_r1_closed_form():
    # r = 1: c_1 = l, Z_2 = M x/(x^2 + l), maximum at sqrt(l), delta = ((1-sqrt l)/(1+sqrt l))^2
    for l in [0.5, 1e-2, 1e-6, 1e-10]:
        z = Zolo(1, l)
        assert abs(z.c[0] - l) <= 1e-14 * l
        assert abs(z.xeq[1] - math.sqrt(l)) <= 1e-14 * math.sqrt(l)
        d = ((1 - math.sqrt(l)) / (1 + math.sqrt(l))) ** 2
        assert abs(z.delta - d) <= 1e-14
        # M x/(x^2+l) with max 1+delta at sqrt(l)
        assert abs(z(np.sqrt(l)) - (1 + z.delta)) < 1e-14


@pytest.mark.parametrize("r,l", CASES)
def test_equioscillation(r, l):
    z = Zolo(r, l)
    # 1 - Z(x_i) = (-1)^i delta at the 2r+1 points, x_0 = l, x_2r = 1
    vals = 1.0 - z(z.xeq)
    sgn = np.array([(-1) ** i for i in range(2 * r + 1)])
    assert abs(z.xeq[0] - l) <= 1e-15 * l and abs(z.xeq[-1] - 1.0) < 1e-15
    assert np.all(np.diff(z.xeq) > 0)
    assert np.max(np.abs(vals - sgn * z.delta)) < 1e-13
    # brute force: |1 - Z| <= delta on [l, 1] (log-spaced dense sampling)
    xs = np.exp(np.linspace(np.log(l), 0.0, 200001))
    err = np.max(np.abs(1.0 - z(xs)))
    assert err <= z.delta * (1 + 1e-9) + 1e-15
    # odd: Z(-x) = -Z(x)
    assert np.max(np.abs(z(-xs[::1000]) + z(xs[::1000]))) < 1e-15


@pytest.mark.parametrize("r,l", [(1, 0.5), (2, 1e-2), (3, 2.5e-5), (4, 2.5e-13), (2, 4.7e-4)])
def test_delta_exact_nome_formula(r, l):
    # delta(2r, l) = (1 - lh)/(1 + lh), q(lh) = q(l)^(1/(2r)) (Zolotarev / Akhiezer).
    # The paper's printed Goncar bracket does not hold (see DESIGN readings);
    # this exact form replaces it as the closed-form check.
    q = mpmath.qfrom(k=mpmath.mpf(l))
    lh = mpmath.kfrom(q=q ** (mpmath.mpf(1) / (2 * r)))
    d_ref = float((1 - lh) / (1 + lh))
    z = Zolo(r, l)
    assert abs(z.delta - d_ref) <= 1e-12 * d_ref + 1e-16
    # consequently Zhat(l; l) = l_next is the modulus lh
    assert abs(z.l_next - float(lh)) < 1e-12


def test_printed_goncar_bracket_is_not_a_bound():
    # Documents the reading: with rho = exp(pi K(mu')/(4 K(mu))), mu = (1-sqrt l)/(1+sqrt l),
    # the printed 2/(rho^2r + 1) <= delta fails, e.g. l = 0.5, r = 1.
    l, r = 0.5, 1
    mu = (1 - math.sqrt(l)) / (1 + math.sqrt(l))
    Kmu = float(mpmath.ellipk(mu * mu))
    Kmup = float(mpmath.ellipk(1 - mu * mu))
    rho = math.exp(math.pi * Kmup / (4 * Kmu))
    lower = 2 / (rho ** (2 * r) + 1)
    assert Zolo(r, l).delta < lower


@pytest.mark.parametrize("r1,r2,l1", [(2, 2, 1e-3), (3, 3, 1e-3), (2, 3, 4.7e-4), (1, 2, 1e-2), (2, 5, 1e-5)])
def test_theorem2_composition(r1, r2, l1):
    xs = np.exp(np.linspace(np.log(l1), 0.0, 4001))
    S = composite(xs, r1, r2, l1)
    D = Zolo(2 * r1 * r2, l1)(xs)
    assert np.max(np.abs(S - D)) < 2e-12
    assert abs(composite_delta(r1, r2, l1) - Zolo(2 * r1 * r2, l1).delta) < 2e-12


@pytest.mark.parametrize("r,l", CASES)
def test_partial_fractions(r, l):
    z = Zolo(r, l)
    a, b = z.pf_real()
    assert abs(np.sum(a) - 1.0) < 1e-13
    xs = np.concatenate([np.exp(np.linspace(np.log(l), 0.0, 501)), [-0.3, -l, 2.5, 10.0]])
    ref = z(xs)
    assert np.max(np.abs(z.eval_pf_real(xs) - ref)) < 1e-12 * (1 + np.max(np.abs(ref)))
    assert np.max(np.abs(z.eval_pf_complex(xs) - ref)) < 1e-12 * (1 + np.max(np.abs(ref)))
    # residue check: (x^2 + c_{2j-1}) Z(x) at x = i sqrt(c_{2j-1}) equals M x a_j
    for j, cj in enumerate(z.c_odd):
        x = 1j * math.sqrt(cj)
        x2 = x * x
        num = np.prod([x2 + c2 for c2 in z.c_even]) if r > 1 else 1.0
        den = np.prod([x2 + c for i, c in enumerate(z.c_odd) if i != j])
        assert abs(z.M * x * num / den - z.M * x * a[j]) < 1e-10 * abs(z.M * x * a[j]) + 1e-14


def test_proposition2_poles_weights():
    z = Zolo(3, 1e-3)
    alpha, beta, gamma = 0.3, 1.7, -0.4
    sigma, w, const = z.mobius_poles(alpha, beta, gamma)
    xs = np.array([-5.0, -1.0, 0.0, 0.25, 0.9, 1.2, 1.6, 2.0, 7.0])
    T = gamma * (xs - alpha) / (xs - beta)
    ref = z(T)
    got = z.M * const + z.M * np.sum(w[None, :] / (xs[:, None] - sigma[None, :]) + np.conj(w)[None, :] / (xs[:, None] - np.conj(sigma)[None, :]), axis=1)
    assert np.max(np.abs(got.imag)) < 1e-13
    assert np.max(np.abs(got.real - ref)) < 1e-12
    # poles lie on the circle with diameter [alpha, beta]
    assert np.max(np.abs(np.abs(sigma - 0.5 * (alpha + beta)) - 0.5 * abs(beta - alpha))) < 1e-14


def test_six_factorizations_reach_machine_accuracy_at_gap_1e2():
    # Sec. 2.2 after Fig. 3: gaps of 1e-2 around +-1 need few factorizations for
    # machine accuracy.  Rectangle on (-1, 1), gaps (-1.01,-0.99) and (0.99, 1.01).
    from oracle.filt import FilterPlan

    f = FilterPlan(-1.01, -0.99, 0.99, 1.01, 6, 6)
    assert f.delta0 < 1e-15
