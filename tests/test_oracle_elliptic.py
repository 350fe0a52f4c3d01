"""Pins for oracle.elliptic: mpmath at 40 digits, identities and special cases."""
import math

import mpmath
import numpy as np
import pytest

from oracle.elliptic import agm, ellipk_kc, jacobi_sncndn

mpmath.mp.dps = 40

KCS = [0.5, 1e-2, 4.7e-4, 1e-6, 1e-10, 2.5e-13]


@pytest.mark.parametrize("kc", KCS)
def test_K_prime_matches_mpmath(kc):
    # K' = K(l') with l'^2 = 1 - l^2 formed in 40-digit arithmetic
    ref = mpmath.ellipk(1 - mpmath.mpf(kc) ** 2)
    got = ellipk_kc(kc)
    assert abs(got - float(ref)) / float(ref) < 1e-14


def test_agm_closed_form():
    # AGM(1, sqrt2) = Gauss' constant reciprocal: 1/G with G = 0.8346268...
    assert abs(agm(1.0, math.sqrt(2.0)) - float(mpmath.agm(1, mpmath.sqrt(2)))) < 1e-15
    assert agm(3.0, 3.0) == 3.0


@pytest.mark.parametrize("kc", [0.9, 0.5, 1e-2, 4.7e-4, 1e-6, 1e-9, 2.5e-13])
@pytest.mark.parametrize("frac", [0.05, 0.2, 0.37, 0.5, 0.8, 0.97, 1.0])
def test_sncndn_match_mpmath(kc, frac):
    K = ellipk_kc(kc)
    u = frac * K
    m = 1 - mpmath.mpf(kc) ** 2
    sn_r = float(mpmath.ellipfun("sn", u, m=m))
    cn_r = float(mpmath.ellipfun("cn", u, m=m))
    dn_r = float(mpmath.ellipfun("dn", u, m=m))
    sn, cn, dn = jacobi_sncndn(u, kc)
    # relative accuracy everywhere on [0, K], including tiny cn near u = K
    tol_rel = 2e-14
    assert abs(sn - sn_r) <= 1e-14 * abs(sn_r)
    assert abs(cn - cn_r) <= tol_rel * abs(cn_r) + 1e-300 + (4e-16 * kc * K if frac == 1.0 else 0.0)
    assert abs(dn - dn_r) <= tol_rel * abs(dn_r)


def test_identities_and_special_cases():
    u = np.linspace(0.0, 1.9, 17)
    sn, cn, dn = jacobi_sncndn(u, 0.3)
    k2 = 1 - 0.3**2
    assert np.max(np.abs(sn**2 + cn**2 - 1)) < 1e-15
    assert np.max(np.abs(dn**2 + k2 * sn**2 - 1)) < 1e-15
    # modulus 0: circular functions
    u = np.linspace(0.0, 2.0, 17)
    sn0, cn0, dn0 = jacobi_sncndn(u, 1.0)
    assert np.allclose(sn0, np.sin(u), atol=0) and np.allclose(dn0, 1.0)
    # modulus -> 1 limit (complement tiny): sn -> tanh, cn, dn -> sech for u << K
    sn1, cn1, dn1 = jacobi_sncndn(np.array([0.1, 0.5, 1.0]), 1e-12)
    assert np.allclose(sn1, np.tanh([0.1, 0.5, 1.0]), rtol=1e-12)
    assert np.allclose(cn1, 1 / np.cosh([0.1, 0.5, 1.0]), rtol=1e-12)
    # quarter period: sn(K) = 1, dn(K) = kc
    K = ellipk_kc(0.2)
    s, c, d = jacobi_sncndn(K, 0.2)
    assert abs(s - 1) < 1e-15 and abs(c) < 1e-7
    assert abs(d - 0.2) < 1e-14
