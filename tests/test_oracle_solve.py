"""Pins of the oracle's linear solve and Pade exponential (section 4.1:
r_km = q_km^{-1} p_km) against hand-worked factors, LAPACK's pivoting,
exact special cases and closed forms of exp."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import solve as osolve

U = 2.0 ** -53


def test_lu_2x2_by_hand():
    LU, piv, info = osolve.lu_pp([[1.0, 2.0], [3.0, 4.0]])
    # row 1 is the pivot: L = [[1, 0], [1/3, 1]], U = [[3, 4], [0, 2 - 4/3]]
    assert list(piv) == [1, 1] and info == 0
    assert LU[0, 0] == 3.0 and LU[0, 1] == 4.0
    assert LU[1, 0] == 1.0 / 3.0
    assert abs(LU[1, 1] - 2.0 / 3.0) <= 2 * U


def test_lu_first_max_on_ties():
    # |-2| = |2| in column 0: the first such row (row 1) is taken
    _, piv, _ = osolve.lu_pp([[1.0, 5.0, 0.0], [-2.0, 1.0, 1.0], [2.0, 0.0, 3.0]])
    assert piv[0] == 1


def test_lu_matches_lapack_pivots_and_factors():
    rng = np.random.default_rng(7)
    for n in (1, 2, 9, 40, 97):
        Q = rng.standard_normal((n, n))
        LU, piv, info = osolve.lu_pp(Q)
        lu_ref, piv_ref = sla.lu_factor(Q)
        assert info == 0
        np.testing.assert_array_equal(piv, piv_ref)
        assert np.max(np.abs(LU - lu_ref)) <= 1e-11 * max(1.0, np.max(np.abs(lu_ref)))


def test_lu_reconstructs_and_bounds_multipliers():
    rng = np.random.default_rng(3)
    n = 60
    Q = rng.standard_normal((n, n)) * np.logspace(0, 3, n)[None, :]
    LU, piv, _ = osolve.lu_pp(Q)
    L = np.tril(LU, -1) + np.eye(n)
    Um = np.triu(LU)
    PQ = Q.copy()
    for k in range(n):
        PQ[[k, piv[k]], :] = PQ[[piv[k], k], :]
    assert np.max(np.abs(L)) <= 1.0                      # partial pivoting
    assert np.linalg.norm(PQ - L @ Um, 1) <= 4 * n * U * np.linalg.norm(Q, 1) * np.max(np.abs(L)) * 8


def test_lu_of_permutation_is_exact():
    n = 7
    perm = [3, 0, 6, 1, 5, 2, 4]
    Q = np.eye(n)[perm]
    B = np.arange(n * 3, dtype=float).reshape(n, 3)
    X, info = osolve.solve(Q, B)
    assert info == 0
    np.testing.assert_array_equal(X, Q.T @ B)


def test_upper_triangular_needs_no_exchange():
    rng = np.random.default_rng(5)
    n = 12
    Q = np.triu(rng.uniform(-1, 1, (n, n))) + np.diag(np.full(n, 4.0))
    LU, piv, info = osolve.lu_pp(Q)
    assert list(piv) == list(range(n)) and info == 0
    np.testing.assert_array_equal(LU, Q)


def test_zero_pivot_reported_first():
    rng = np.random.default_rng(1)
    Q = rng.standard_normal((6, 6))
    Q[:, 2] = 0.0
    Q[:, 4] = 0.0
    _, _, info = osolve.lu_pp(Q)
    assert info == 3


def test_solve_against_numpy():
    rng = np.random.default_rng(11)
    n = 80
    Q = rng.standard_normal((n, n)) + 3 * np.eye(n)
    B = rng.standard_normal((n, 5))
    X, _ = osolve.solve(Q, B)
    ref = np.linalg.solve(Q, B)
    kappa = np.linalg.cond(Q, 1)
    assert np.linalg.norm(X - ref, 1) / np.linalg.norm(ref, 1) <= 10 * n * kappa * U


def test_lower_and_upper_substitution_both_used():
    # a unit-lower-times-upper product with no exchanges: the solve must undo
    # both factors (a dropped forward or back substitution fails)
    Lm = np.array([[1.0, 0, 0], [0.5, 1, 0], [-0.25, 0.5, 1]])
    Um = np.array([[4.0, 1, 2], [0, 2, -1], [0, 0, 1]])
    Q = Lm @ Um
    x = np.array([[1.0], [-2.0], [3.0]])
    X, info = osolve.solve(Q, Q @ x)
    assert info == 0
    np.testing.assert_allclose(X, x, rtol=0, atol=1e-14)


@pytest.mark.parametrize("m", [3, 7, 13])
def test_expm_pade_against_scipy(m):
    rng = np.random.default_rng(20 + m)
    n = 30
    A = rng.standard_normal((n, n))
    A *= 3.0 / np.linalg.norm(A, 1)
    sigma = {3: 7, 7: 4, 13: 0}[m]        # ||X||_1 = 0.023, 0.19, 3
    E = osolve.expm_pade(A, m, sigma)
    ref = sla.expm(A)
    tol = 1e-13 if sigma <= 4 else 5e-13  # rounding grows with each squaring
    assert np.linalg.norm(E - ref, 1) / np.linalg.norm(ref, 1) <= tol


def test_expm_pade_closed_forms():
    d = np.array([-3.0, -0.5, 0.0, 0.25, 2.0])
    E = osolve.expm_pade(np.diag(d), 13, 1)
    np.testing.assert_allclose(np.diag(E), np.exp(d), rtol=4e-15)
    assert np.max(np.abs(E - np.diag(np.diag(E)))) == 0.0
    N = np.array([[0.0, 1.5], [0.0, 0.0]])                  # nilpotent: exp = I + N
    np.testing.assert_allclose(osolve.expm_pade(N, 9, 0), np.eye(2) + N, rtol=0, atol=1e-15)
    Z = np.zeros((4, 4))
    np.testing.assert_array_equal(osolve.expm_pade(Z, 13, 0), np.eye(4))


def test_expm_pade_inverse_pair():
    rng = np.random.default_rng(9)
    A = rng.standard_normal((20, 20))
    A *= 2.0 / np.linalg.norm(A, 1)
    E1 = osolve.expm_pade(A, 13, 0)
    E2 = osolve.expm_pade(-A, 13, 0)
    assert np.linalg.norm(E1 @ E2 - np.eye(20), 1) <= 1e-13
