"""Moebius map of the eigengap configuration (eq. mo, eq. req).

T(x) = gamma (x - alpha) / (x - beta) must send the two eigengaps onto the
two gaps of sign's domain [-1,-l1] u [l1,1], with alpha in (a_-, a_+) and beta
in (b_-, b_+) (Sec. 2.2).  The four printed conditions T(a_-) = -1,
T(a_+) = 1, T(b_-) = l1, T(b_+) = -l1 cannot hold together with those pole
and zero locations (a real Moebius map is monotone on (-inf, beta)).  Reading
used here (the same R_ab results from either reading, because
Z(l/x; l) = Z(x; l)): keep alpha in (a_-,a_+), beta in (b_-,b_+) and ask

    T(a_-) = -l1,  T(a_+) = l1,  T(b_-) = 1,  T(b_+) = -1,

so [a_+, b_-] -> [l1, 1] (filter ~ 1) and the exterior -> [-1, -l1] (~ 0).

Step 1: Moebius maps preserve cross-ratios, so
    eps = (a_+ - a_-)(b_+ - b_-) / ((b_- - a_+)(b_+ - a_-)) = 4 l1/(1-l1)^2,
    l1  = eps / (sqrt(1+eps) + 1)^2       (cancellation-free root).
Step 2: with l1 known, three of the conditions are linear in
(u1, u2, u3) = (gamma, gamma*alpha, beta):  x u1 - u2 + y u3 = x y  for each
(x, y = T(x)); solved in the shifted, scaled coordinate s = (x - a_+)/(b_- - a_+).
The fourth condition is returned as a residual check.
An infinite endpoint (a_- = -inf or b_+ = +inf) replaces its condition by
T(+-inf) = gamma.
"""
from __future__ import annotations

import math

import numpy as np


class Mobius:
    def __init__(self, a_minus: float, a_plus: float, b_minus: float, b_plus: float):
        am, ap, bm, bp = float(a_minus), float(a_plus), float(b_minus), float(b_plus)
        if math.isinf(am) and math.isinf(bp):
            raise ValueError("at most one infinite gap endpoint")
        if not (am < ap < bm < bp):
            raise ValueError("need a_- < a_+ < b_- < b_+")
        self.gaps = (am, ap, bm, bp)
        W = bm - ap
        # ---- Step 1: cross-ratio ----
        if math.isinf(am):
            eps = (bp - bm) / W
        elif math.isinf(bp):
            eps = (ap - am) / W
        else:
            eps = (ap - am) * (bp - bm) / (W * (bp - am))
        l1 = eps / (math.sqrt(1.0 + eps) + 1.0) ** 2
        self.eps = eps
        self.l1 = l1
        # ---- Step 2: linear solve in s = (x - a_+)/W ----
        s = lambda x: (x - ap) / W  # noqa: E731
        rows = []
        rhs = []
        # Use (a_+, b_-) always, plus one exterior condition; the other is the check.
        use = [(ap, l1), (bm, 1.0)]
        if math.isinf(am):
            rows.append([1.0, 0.0, 0.0])  # gamma = T(-inf) = -l1
            rhs.append(-l1)
            check = (bp, -1.0)
        elif math.isinf(bp):
            rows.append([1.0, 0.0, 0.0])  # gamma = T(+inf) = -1
            rhs.append(-1.0)
            check = (am, -l1)
        else:
            use.append((am, -l1))
            check = (bp, -1.0)
        for x, y in use:
            sx = s(x)
            rows.append([sx, -1.0, y])
            rhs.append(sx * y)
        u = np.linalg.solve(np.array(rows), np.array(rhs))
        gamma = u[0]
        alpha_s = u[1] / gamma
        beta_s = u[2]
        self.gamma = float(gamma)
        self.alpha = float(ap + W * alpha_s)
        self.beta = float(ap + W * beta_s)
        self._alpha_s = alpha_s
        self._beta_s = beta_s
        self._W = W
        xc, yc = check
        self.check_residual = float(abs(self.T(xc) - yc))

    def T(self, x):
        """T(x) = gamma (x - alpha)/(x - beta), evaluated in the scaled coordinate."""
        x = np.asarray(x, dtype=np.result_type(x, float))
        sx = (x - self.gaps[1]) / self._W
        return self.gamma * (sx - self._alpha_s) / (sx - self._beta_s)
