"""Elliptic integrals and Jacobi elliptic functions (FP64, AGM / Landen).

Theorem 1 of the paper needs K' = K(l') and sn, cn(u; l') with modulus
l' = sqrt(1-l^2).  For the tiny l of narrow eigengaps, forming l'^2 = 1 - l^2
throws away the information about l, so every routine here takes the
*complementary* modulus kc (= l) as its input.

* K(k) = pi / (2 AGM(1, k'))            (Gauss; Abramowitz-Stegun 17.6.1)
* sn, cn, dn by the descending Landen / AGM scheme (Abramowitz-Stegun 16.4):
  a_0 = 1, b_0 = k', a_{n+1} = (a_n+b_n)/2, b_{n+1} = sqrt(a_n b_n),
  c_{n+1} = (a_n-b_n)/2; phi_N = 2^N a_N u;
  phi_{n-1} = (phi_n + asin(c_n sin(phi_n) / a_n)) / 2;
  sn = sin phi_0, cn = cos phi_0, dn = cos phi_0 / cos(phi_1 - phi_0).
* For a modulus near 1 (kc < 1/sqrt 2) the same scheme is run for the
  complementary modulus at the imaginary argument i u (Jacobi's imaginary
  transformation, Abramowitz-Stegun 16.20): phi_n = i psi_n stays on the
  imaginary axis, psi_{n-1} = (psi_n + asinh(c_n sinh(psi_n)/a_n)) / 2, and
  sn(u|k) = tanh psi_0, cn(u|k) = sech psi_0, dn(u|k) = sech(psi_1 - psi_0).
  Every step is then well conditioned, so cn keeps full relative accuracy even
  where it is tiny (u near K, reached through the quarter-period shift).
"""
from __future__ import annotations

import numpy as np

_MAX_AGM = 64


def agm(a: float, b: float) -> float:
    """Arithmetic-geometric mean of two positive numbers."""
    a = float(a)
    b = float(b)
    for _ in range(_MAX_AGM):
        if abs(a - b) <= 1e-16 * a:
            break
        a, b = 0.5 * (a + b), np.sqrt(a * b)
    return 0.5 * (a + b)


def ellipk_kc(kc: float) -> float:
    """K(k) for the modulus k whose complement is kc (k^2 + kc^2 = 1).

    The paper's K' = K(l') is ``ellipk_kc(l)`` (Theorem 1).
    """
    if not (0.0 < kc <= 1.0):
        raise ValueError("complementary modulus must lie in (0, 1]")
    return np.pi / (2.0 * agm(1.0, kc))


def _landen_tables(b0: float, c1: float, growth: float = 0.0):
    """a_n and c_n of the AGM started at (1, b0); c1 = (1 - b0)/2 is passed in.

    c_{n+1} = c_n^2 / (4 a_{n+1}) (exact, from a_n^2 - b_n^2 = c_n^2) avoids
    the cancellation of (a_n - b_n)/2.  Iterates until
    c_n * exp(2^n a_n * growth) <= 1e-17 a_n, so that the neglected Landen term
    stays below rounding also for the hyperbolic (imaginary-argument)
    recursion, whose terms grow like exp(psi_n).
    """
    a = [1.0, 0.5 * (1.0 + b0)]
    c = [np.nan, c1]
    for n in range(1, _MAX_AGM):
        if c[-1] == 0.0:
            break
        if np.log(c[-1]) + min((2.0**n) * a[-1] * growth, 700.0) <= np.log(1e-17 * a[-1]):
            break
        cn = c[-1]
        an = a[-1]
        bn = np.sqrt(an * an - cn * cn)
        a.append(0.5 * (an + bn))
        c.append(cn * cn / (4.0 * a[-1]))
    return np.array(a), np.array(c)


def _sncndn_direct(u: float, kc: float, k: float):
    a, c = _landen_tables(kc, 0.5 * (1.0 - kc))
    n = a.shape[0] - 1
    phi = (2.0**n) * a[n] * u
    for j in range(n, 0, -1):
        phi = 0.5 * (phi + np.arcsin(np.clip(c[j] * np.sin(phi) / a[j], -1.0, 1.0)))
    sn = np.sin(phi)
    cn = np.cos(phi)
    dn = np.sqrt(kc * kc + k * k * cn * cn)  # dn^2 = 1 - k^2 sn^2 = k'^2 + k^2 cn^2
    return sn, cn, dn


def _sncndn_imag(v: float, kc: float, k: float):
    """Modulus near 1, 0 <= v <= K/2: Landen for modulus kc at argument i v."""
    a, c = _landen_tables(k, 0.5 * kc * kc / (1.0 + k), growth=v)
    n = a.shape[0] - 1
    psi = (2.0**n) * a[n] * v
    prev = psi
    for j in range(n, 0, -1):
        prev = psi
        psi = 0.5 * (psi + np.arcsinh(c[j] * np.sinh(psi) / a[j]))
    return np.tanh(psi), 1.0 / np.cosh(psi), 1.0 / np.cosh(prev - psi)


def jacobi_sncndn(u, kc: float):
    """sn, cn, dn(u | modulus k) for 0 <= u <= K, complementary modulus kc.

    For a modulus near 1 and u > K/2 the quarter-period shift
    sn(K - v) = cd(v), cn(K - v) = k' sd(v), dn(K - v) = k' nd(v)
    (Abramowitz-Stegun 16.8) keeps the imaginary-argument recursion at
    v <= K/2, away from its pole at v = K.
    """
    if not (0.0 < kc <= 1.0):
        raise ValueError("complementary modulus must lie in (0, 1]")
    uu = np.asarray(u, dtype=np.float64)
    if kc == 1.0:
        return np.sin(uu), np.cos(uu), np.ones_like(uu)
    k = np.sqrt((1.0 - kc) * (1.0 + kc))
    K = ellipk_kc(kc)
    flat = uu.reshape(-1)
    sn = np.empty_like(flat)
    cn = np.empty_like(flat)
    dn = np.empty_like(flat)
    for i, x in enumerate(flat):
        if x < 0.0 or x > K * (1.0 + 1e-15):
            raise ValueError("argument outside [0, K]")
        if kc >= np.sqrt(0.5):
            sn[i], cn[i], dn[i] = _sncndn_direct(x, kc, k)
        elif x <= 0.5 * K:
            sn[i], cn[i], dn[i] = _sncndn_imag(x, kc, k)
        else:
            s, c, d = _sncndn_imag(max(K - x, 0.0), kc, k)
            sn[i], cn[i], dn[i] = c / d, kc * s / d, kc / d
    return sn.reshape(uu.shape), cn.reshape(uu.shape), dn.reshape(uu.shape)
