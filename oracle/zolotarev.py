"""Zolotarev's best rational approximation of sign(x) and its partial fractions.

Follows Sec. 2.2 of the paper:

* Theorem 1 (eq. ZoloFunc, eq. coef): Z_2r(x; l) = M x prod_{j<r}(x^2+c_2j) /
  prod_{j<=r}(x^2+c_{2j-1}), c_j = l^2 sn^2(jK'/2r; l') / cn^2(jK'/2r; l').
* Equioscillation (after Theorem 1): 1 - Z(x_j) = (-1)^{j+1} delta on 2r+1
  points of [l, 1].  The points are x_i = l / dn(i K'/(2r); l'), i = 0..2r
  (x_0 = l, x_2r = 1); they are not printed in the paper (reading: the
  classical Zolotarev/Akhiezer extremal points).  M is fixed by
  M P(x_0) = 1 - delta and M P(x_1) = 1 + delta, i.e. M = 2/(P(x_0)+P(x_1)).
* eq. rZ: Zhat = Z / max_[l,1] Z = Z / (1 + delta); l2 = Zhat(l; l).
* Theorem 2 (eq. Z): Z_2r2(Zhat_2r1(x; l1); l2) = Z_{(2r1)(2r2)}(x; l1).
* Proposition 1 (eq. pa): Z = M x sum_j a_j / (x^2 + c_{2j-1}).
* Corollary 1 (eq. paRe): Z = (M/2) sum_j a_j (1/(x+i sqrt c) + 1/(x-i sqrt c)).
* Proposition 2: poles sigma_j and weights w_j of Z(T(x)).
"""
from __future__ import annotations

import numpy as np

from .elliptic import ellipk_kc, jacobi_sncndn


class Zolo:
    """Coefficients of Z_2r(x; l) (Theorem 1).

    Attributes: r, l, c (array, c[j-1] = c_j for j = 1..2r-1), M, delta,
    kp (K'), xeq (the 2r+1 equioscillation points, ascending).
    """

    def __init__(self, r: int, l: float):
        if r < 1:
            raise ValueError("r >= 1")
        if not (0.0 < l < 1.0):
            raise ValueError("l in (0,1)")
        self.r = int(r)
        self.l = float(l)
        kp = ellipk_kc(l)  # K' = K(l'), modulus l' = sqrt(1-l^2), complement l
        self.kp = kp
        c = np.empty(2 * r - 1)
        for j in range(1, 2 * r):
            sn, cn, _ = jacobi_sncndn(j * kp / (2 * r), l)
            c[j - 1] = l * l * (sn / cn) ** 2
        self.c = c
        # Equioscillation points x_i = l / dn(i K'/2r; l'), i = 0..2r.
        xeq = np.empty(2 * r + 1)
        for i in range(2 * r + 1):
            _, _, dn = jacobi_sncndn(i * kp / (2 * r), l)
            xeq[i] = l / dn
        self.xeq = xeq
        p0 = self.p(xeq[0])
        p1 = self.p(xeq[1])
        self.M = 2.0 / (p0 + p1)
        self.delta = 1.0 - self.M * p0

    # c_{2j-1}, j = 1..r   and   c_{2j}, j = 1..r-1
    @property
    def c_odd(self) -> np.ndarray:
        return self.c[0::2]

    @property
    def c_even(self) -> np.ndarray:
        return self.c[1::2]

    def p(self, x):
        """P(x) = x prod_{j<r}(x^2+c_2j) / prod_{j<=r}(x^2+c_{2j-1}) (Theorem 1)."""
        x = np.asarray(x)
        x2 = x * x
        num = np.ones_like(x2)
        for c2j in self.c_even:
            num = num * (x2 + c2j)
        den = np.ones_like(x2)
        for c2jm1 in self.c_odd:
            den = den * (x2 + c2jm1)
        return x * num / den

    def __call__(self, x):
        """Z_2r(x; l), product form (eq. ZoloFunc)."""
        return self.M * self.p(x)

    def rescaled(self, x):
        """Zhat_2r(x; l) = Z / max_[l,1] Z = Z / (1 + delta) (eq. rZ)."""
        return self(x) / (1.0 + self.delta)

    @property
    def Mhat(self) -> float:
        return self.M / (1.0 + self.delta)

    @property
    def l_next(self) -> float:
        """Zhat(l; l) = (1 - delta)/(1 + delta): the outer parameter l2 (Theorem 2)."""
        return (1.0 - self.delta) / (1.0 + self.delta)

    # ---- Proposition 1 --------------------------------------------------
    def pf_real(self):
        """(a_j, b_j) of Proposition 1; sum_j a_j == 1."""
        r = self.r
        co = self.c_odd
        ce = self.c_even
        b = np.empty(r - 1)
        for j in range(r - 1):
            prod = 1.0
            for k in range(r - 1):
                if k != j:
                    prod *= (ce[k] - co[j]) / (co[k] - co[j])
            b[j] = (ce[j] - co[j]) * prod
        a = np.empty(r)
        for j in range(r - 1):
            a[j] = b[j] / (co[r - 1] - co[j])
        a[r - 1] = 1.0 - np.sum(a[: r - 1])
        return a, b

    def eval_pf_real(self, x):
        """M x sum_j a_j / (x^2 + c_{2j-1})  (eq. pa)."""
        a, _ = self.pf_real()
        x = np.asarray(x)
        s = np.zeros_like(x, dtype=np.result_type(x, float))
        for aj, cj in zip(a, self.c_odd):
            s = s + aj / (x * x + cj)
        return self.M * x * s

    def eval_pf_complex(self, x):
        """(M/2) sum_j a_j (1/(x + i sqrt c) + 1/(x - i sqrt c))  (Corollary 1)."""
        a, _ = self.pf_real()
        x = np.asarray(x, dtype=np.complex128)
        s = np.zeros_like(x)
        for aj, cj in zip(a, self.c_odd):
            q = 1j * np.sqrt(cj)
            s = s + aj * (1.0 / (x + q) + 1.0 / (x - q))
        return 0.5 * self.M * s

    # ---- Proposition 2 --------------------------------------------------
    def mobius_poles(self, alpha: float, beta: float, gamma: float):
        """Poles sigma_j, weights w_j and constant sum_j a_j gamma/(gamma^2+c)
        of Z(T(x)) with T(x) = gamma (x - alpha)/(x - beta) (Proposition 2).

        Z(T(x)) = M * const + M sum_j (w_j/(x - sigma_j) + conj(w_j)/(x - conj(sigma_j))).
        """
        a, _ = self.pf_real()
        sq = np.sqrt(self.c_odd)
        den = gamma + 1j * sq
        sigma = (gamma * alpha + 1j * sq * beta) / den
        w = a * (sigma - beta) / (2.0 * den)
        const = float(np.sum(a * gamma / (gamma * gamma + self.c_odd)))
        return sigma, w, const


def composite(x, r1: int, r2: int, l1: float):
    """S(x; l1) = Z_2r2(Zhat_2r1(x; l1); l2) with l2 = Zhat_2r1(l1; l1) (eq. S)."""
    inner = Zolo(r1, l1)
    outer = Zolo(r2, inner.l_next)
    return outer(inner.rescaled(x))


def composite_delta(r1: int, r2: int, l1: float) -> float:
    """Error of the composite on [l1, 1]: 1 - S(l1; l1) (Remark after Algorithm 2)."""
    return float(1.0 - composite(np.array(l1), r1, r2, l1))
