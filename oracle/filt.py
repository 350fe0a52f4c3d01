"""Coefficient plan of Algorithm 2 (lines 2-4) and the scalar filter R_ab(x).

R_ab(x) = (Z_2r2(Zhat_2r1(T(x); l1); l2) + 1) / 2          (eq. Rab / eq. R2)

Inner constants (hats, Remark after Proposition 2) come from Zhat_2r1(.; l1)
composed with T (Proposition 2): poles sigma_hat_j, weights w_hat_j and the
constant term c0 = sum_j a_hat_j gamma / (gamma^2 + c_hat_{2j-1}), so that

    g(x) = Zhat(T(x); l1) = M_hat [c0 + sum_j (w_hat_j/(x - sigma_hat_j) + conj(w_hat_j)/(x - conj(sigma_hat_j)))]

(eq. solve, scalar form).  Outer constants come from Z_2r2(.; l2) in the
complex partial-fraction form of Corollary 1 (eq. solve2):

    R = 1/2 + (M/2) sum_j (a_j/2) [1/(g + i sqrt c_j) + 1/(g - i sqrt c_j)].
"""
from __future__ import annotations

import numpy as np

from .mobius import Mobius
from .zolotarev import Zolo


class FilterPlan:
    def __init__(self, a_minus, a_plus, b_minus, b_plus, r1: int, r2: int):
        self.mob = Mobius(a_minus, a_plus, b_minus, b_plus)
        self.r1 = int(r1)
        self.r2 = int(r2)
        self.inner = Zolo(r1, self.mob.l1)
        self.l1 = self.mob.l1
        self.l2 = self.inner.l_next
        self.outer = Zolo(r2, self.l2)
        m = self.mob
        self.sigma_hat, self.w_hat, self.c0 = self.inner.mobius_poles(m.alpha, m.beta, m.gamma)
        self.M_hat = self.inner.Mhat
        self.a_hat, _ = self.inner.pf_real()
        self.c_hat = self.inner.c_odd.copy()
        self.M = self.outer.M
        self.a, _ = self.outer.pf_real()
        self.c = self.outer.c_odd.copy()  # outer shifts are +- i sqrt(c_j)
        self.delta_S = self.outer.delta  # sup |sign - S| on [-1,-l1] u [l1,1]
        self.delta0 = 0.5 * self.delta_S  # sup |S_ab - R_ab| on Omega (Theorem 3)

    # ---- scalar filter, two ways ---------------------------------------
    def R_product(self, x):
        """(S(T(x)) + 1)/2 with product forms throughout (eq. R2)."""
        t = self.mob.T(np.asarray(x, dtype=np.float64))
        return 0.5 * (self.outer(self.inner.rescaled(t)) + 1.0)

    def g(self, x):
        """Inner function g(x) = Zhat(T(x); l1) in pole form (Proposition 2)."""
        x = np.asarray(x, dtype=np.complex128)
        s = np.full(x.shape, self.c0, dtype=np.complex128)
        for sj, wj in zip(self.sigma_hat, self.w_hat):
            s = s + wj / (x - sj) + np.conj(wj) / (x - np.conj(sj))
        return self.M_hat * s

    def R_pf(self, x):
        """Nested partial-fraction route (Algorithm 2, lines 7-9, scalar form)."""
        g = self.g(x)
        s = np.zeros_like(g)
        for aj, cj in zip(self.a, self.c):
            q = 1j * np.sqrt(cj)
            s = s + 0.5 * aj * (1.0 / (g + q) + 1.0 / (g - q))
        return 0.5 + 0.5 * self.M * s

    def R(self, x):
        return np.real(self.R_pf(x))


def select_r2(a_minus, a_plus, b_minus, b_plus, r1: int, eps: float, r2_max: int = 16) -> int:
    """Smallest r2 whose composite error meets eps (Remark after Algorithm 2).

    The composite's sup error on the sign domain is attained at x = l1, so
    delta0 = (1 - S(l1; l1)) / 2 is evaluated for r2 = 1, 2, ... .
    """
    for r2 in range(1, r2_max + 1):
        if FilterPlan(a_minus, a_plus, b_minus, b_plus, r1, r2).delta0 <= eps:
            return r2
    return r2_max


def order_table(l1: float, r_max: int = 6):
    """Small table of delta0 = (1 - S(l1; l1))/2 for (r1, r2) in [1, r_max]^2."""
    out = np.empty((r_max, r_max))
    for r1 in range(1, r_max + 1):
        inner = Zolo(r1, l1)
        for r2 in range(1, r_max + 1):
            outer = Zolo(r2, inner.l_next)
            out[r1 - 1, r2 - 1] = 0.5 * outer.delta
    return out
