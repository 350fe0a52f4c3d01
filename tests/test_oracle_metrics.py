"""Pins of the oracle's accuracy metrics on hand-worked pencils.

Every GPU residual, e_{Lambda,X} and B-orthonormality assertion goes through
these functions, so each is checked against numbers worked out by hand here,
on vectors that are NOT eigenvectors (an exact eigenpair gives 0 whatever the
denominator is).  A dropped |lambda| ||B|| term, a missing ||x||, a norm of
B x replaced by one of x, or max(|a|, |b|) replaced by |b| changes every
expected value below.

Residual (the benchmark spec): ||A x - lam B x||_2 / ((||A|| + |lam| ||B||) ||x||_2).
e_{Lambda,X} (eq. relerr, Sec. 3): max_i ||A x_i - B x_i lam_i||_2 /
(max(|a|, |b|) ||B x_i||_2).
"""
import math

import numpy as np
import scipy.sparse as sp

from oracle.subspace import b_orthonormality, e_lambda_x, inf_norm, norm2_est, rel_residuals

# A = [[2, 1], [1, 2]], B = diag(2, 1):  ||A||_inf = 3, ||B||_inf = 2.
A2 = np.array([[2.0, 1.0], [1.0, 2.0]])
B2 = np.diag([2.0, 1.0])


def test_rel_residual_hand_worked_real():
    # x = (1, 1), lam = 1:  A x = (3, 3), B x = (2, 1), r = (1, 2), ||r|| = sqrt 5,
    # ||x|| = sqrt 2, denominator (3 + 1 * 2) sqrt 2  ->  sqrt 5 / (5 sqrt 2) = 1 / sqrt 10
    X = np.array([[1.0], [1.0]])
    r = rel_residuals(A2, B2, np.array([1.0]), X, inf_norm(A2), inf_norm(B2))
    assert abs(r[0] - 1.0 / math.sqrt(10.0)) < 1e-15
    # lam = -2 (the |lam| enters, not lam):  r = (3 + 4, 3 + 2) = (7, 5), ||r|| = sqrt 74,
    # denominator (3 + 2 * 2) sqrt 2 = 7 sqrt 2
    r = rel_residuals(A2, B2, np.array([-2.0]), X, inf_norm(A2), inf_norm(B2))
    assert abs(r[0] - math.sqrt(74.0) / (7.0 * math.sqrt(2.0))) < 1e-15
    # scaling x does not change the residual
    r3 = rel_residuals(A2, B2, np.array([1.0, -2.0]), np.hstack([3.0 * X, -0.5 * X]), 3.0, 2.0)
    assert np.allclose(r3, [1.0 / math.sqrt(10.0), math.sqrt(74.0) / (7.0 * math.sqrt(2.0))], rtol=1e-15, atol=0)


def test_rel_residual_hand_worked_complex_sparse():
    # Hermitian A = [[1, i], [-i, 1]] (||A||_inf = 2), B = I (||B||_inf = 1), x = (1, 0), lam = 1:
    # A x = (1, -i), r = (0, -i), ||r|| = 1, ||x|| = 1, denominator 2 + 1 = 3  ->  1/3
    A = sp.csr_matrix(np.array([[1.0, 1j], [-1j, 1.0]]))
    B = sp.identity(2, format="csr", dtype=np.complex128)
    X = np.array([[1.0 + 0j], [0.0]])
    assert inf_norm(A) == 2.0 and inf_norm(B) == 1.0
    r = rel_residuals(A, B, np.array([1.0]), X, inf_norm(A), inf_norm(B))
    assert abs(r[0] - 1.0 / 3.0) < 1e-15
    # exact eigenpair (eigenvalue 2, vector (1, -i)/sqrt 2 ... A (1, -i) = (1 + 1, -i - i) = 2 (1, -i))
    Xe = np.array([[1.0], [-1j]]) / math.sqrt(2.0)
    assert rel_residuals(A, B, np.array([2.0]), Xe, 2.0, 1.0)[0] < 1e-16


def test_e_lambda_x_hand_worked():
    # x = (1, 1), lam = 1 with A2, B2:  ||r|| = sqrt 5, B x = (2, 1), ||B x|| = sqrt 5.
    # interval (a, b) = (-3, 2): max(|a|, |b|) = 3  ->  e = sqrt 5 / (3 sqrt 5) = 1/3
    X = np.array([[1.0], [1.0]])
    e = e_lambda_x(A2, B2, np.array([1.0]), X, -3.0, 2.0)
    assert abs(e - 1.0 / 3.0) < 1e-15
    # (a, b) = (0.5, 4): max = 4 -> 1/4 ; the maximum over columns is taken
    X2 = np.array([[1.0, 1.0], [1.0, 0.0]])
    # second column x = (1, 0), lam = 2: A x = (2, 1), B x = (2, 0), r = (2 - 4, 1) = (-2, 1),
    # ||r|| = sqrt 5, ||B x|| = 2, e_2 = sqrt 5 / (4 * 2) = 0.2795...
    e2 = e_lambda_x(A2, B2, np.array([1.0, 2.0]), X2, 0.5, 4.0)
    assert abs(e2 - max(0.25, math.sqrt(5.0) / 8.0)) < 1e-15
    assert e_lambda_x(A2, B2, np.array([]), np.zeros((2, 0)), 0.5, 4.0) == 0.0


def test_b_orthonormality_hand_worked():
    # B = diag(4, 1), X = [[0.5, 0.5], [0, 1]]:  X^T B X = [[1, 1], [1, 2]]  ->  max |G - I| = 1
    B = np.diag([4.0, 1.0])
    X = np.array([[0.5, 0.5], [0.0, 1.0]])
    assert abs(b_orthonormality(B, X) - 1.0) < 1e-15
    # complex: X = [[0.5 i], [0]] with B = diag(4, 1): x^H B x = 0.25 * 4 = 1  ->  0
    Xc = np.array([[0.5j], [0.0]])
    assert b_orthonormality(B, Xc) < 1e-16
    # X = I: G = B, max |B - I| = 3
    assert abs(b_orthonormality(B, np.eye(2)) - 3.0) < 1e-15


def test_norm2_estimate():
    # closed form: a diagonal matrix's 2-norm is its largest |entry|
    D = sp.diags([1.0, -7.0, 3.0]).tocsr()
    assert abs(norm2_est(D, iters=60) - 7.0) < 1e-9
    # library special case: LAPACK's 2-norm of a dense symmetric matrix
    rng = np.random.default_rng(5)
    M = rng.standard_normal((40, 40))
    M = M + M.T
    ref = np.linalg.norm(M, 2)
    est = norm2_est(M, iters=400)
    assert est <= ref * (1 + 1e-12) and est >= ref * (1 - 1e-6)
    # never above the infinity norm for Hermitian matrices
    assert est <= inf_norm(M)


def test_norm2_vs_inf_norm_on_stencil_pencils():
    """On the stencil pencils the two readings of ||A||, ||B|| differ by little (10 % at
    8^3, where the Dirichlet boundary lowers the 2-norm most; the gap closes as the
    grid grows), so residuals reported in either norm agree to that factor."""
    import pencils

    gp = pencils.grid7(8)
    A, B = gp.scipy()
    na2, nb2 = norm2_est(A, iters=300), norm2_est(B, iters=300)
    nai, nbi = inf_norm(A), inf_norm(B)
    assert nb2 <= nbi and na2 <= nai
    assert nai / na2 < 1.15 and nbi / nb2 < 1.05
