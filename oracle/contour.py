"""Comparison filters of the paper's Sec. 2.2 (Figs. 2-3): rational filters from
quadratures of the contour integral (1/(2 pi i)) oint_Gamma dz / (z - x), which is
1 for x inside Gamma and 0 outside, and the single (not composed) Zolotarev
filter.  Test infrastructure (oracle), independent of the GPU library.

Gamma is the circle through a and b: centre c = (a + b)/2, radius rho = (b - a)/2,
z(theta) = c + rho e^{i theta}, dz = i rho e^{i theta} d theta.  A quadrature
{theta_k, omega_k} of theta over [0, 2 pi) gives

    R(x) = sum_k omega_k rho e^{i theta_k} / (2 pi (z_k - x)).

Both rules below place their nodes in conjugate pairs (theta and -theta), so for
real x the lower half-circle adds the conjugates of the upper half's terms:
R(x) = sum over upper nodes of 2 Re(alpha_k / (z_k - x)),
alpha_k = omega_k rho e^{i theta_k} / (2 pi).

* CITZ(p): the trapezoidal rule with p nodes theta_k = pi (2k + 1)/p, weights
  2 pi / p (p even: p/2 upper nodes, i.e. p/2 factorizations for a real pencil).
* CIGQ(p): q = p/2 Gauss-Legendre nodes on the upper half-circle theta in (0, pi)
  (and their mirror images): p poles, p/2 factorizations.
* Zolo(r): the inner function alone, R = (Zhat_2r(T(x); l1) + 1)/2, r
  factorizations (the composite filter with no outer stage).
"""
from __future__ import annotations

import numpy as np

from .filt import FilterPlan


class ContourFilter:
    """Upper-half nodes z_k and weights alpha_k with R(x) = sum 2 Re(alpha_k / (z_k - x))."""

    def __init__(self, kind: str, a: float, b: float, p: int):
        if p < 2 or p % 2:
            raise ValueError("p must be even and >= 2")
        self.kind, self.a, self.b, self.p = kind, float(a), float(b), int(p)
        c, rho = 0.5 * (a + b), 0.5 * (b - a)
        q = p // 2
        if kind == "trapezoid":
            theta = np.pi * (2.0 * np.arange(q) + 1.0) / p  # the upper half of the p nodes
            omega = np.full(q, 2.0 * np.pi / p)
        elif kind == "gauss":
            t, wt = np.polynomial.legendre.leggauss(q)  # on [-1, 1]
            theta = 0.5 * np.pi * (t + 1.0)  # onto (0, pi)
            omega = 0.5 * np.pi * wt
        else:
            raise ValueError(kind)
        self.theta = theta
        self.z = c + rho * np.exp(1j * theta)
        self.alpha = omega * rho * np.exp(1j * theta) / (2.0 * np.pi)

    def R(self, x):
        x = np.asarray(x, dtype=np.complex128)
        s = np.zeros(x.shape, dtype=np.complex128)
        for zk, ak in zip(self.z, self.alpha):
            s = s + 2.0 * np.real(ak / (zk - x))
        return np.real(s)


def trapezoid_closed_form(x, a: float, b: float, p: int):
    """The trapezoidal rule's filter in closed form: 1 / (1 + t^p), t = (x - c)/rho
    (a geometric sum over the p-th roots of -1)."""
    c, rho = 0.5 * (a + b), 0.5 * (b - a)
    t = (np.asarray(x, dtype=np.float64) - c) / rho
    return 1.0 / (1.0 + t**p)


class SingleZolo:
    """Zolo(r): R(x) = (g(x) + 1)/2 with g the inner function of the plan with r1 = r
    (Proposition 2's pole form)."""

    def __init__(self, a_minus, a_plus, b_minus, b_plus, r: int):
        self.plan = FilterPlan(a_minus, a_plus, b_minus, b_plus, r, 1)

    def R(self, x):
        return 0.5 * (np.real(self.plan.g(x)) + 1.0)

    def R_product(self, x):
        """The same from the product form of Zhat_2r (Theorem 1) composed with T."""
        t = self.plan.mob.T(np.asarray(x, dtype=np.float64))
        return 0.5 * (self.plan.inner.rescaled(t) + 1.0)
