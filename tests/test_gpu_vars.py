"""GPU parity of Algorithm 2's variable-s branch (ps_expm_vars): the block
size grown on the device's norms equals the oracle's and the closed form of
the Jordan-block cases, and the evaluation with that s matches the
double-double oracle.  Norms are those of the column-major view the library
works on, i.e. of the transpose of each row-major array."""
import math
from fractions import Fraction as F

import numpy as np
import pytest

import oracle
from oracle import coeffs, metrics
from oracle import plan as oplan

from helpers import to_dev, to_np

pytestmark = pytest.mark.gpu

TOL64 = 1e-13
M = 30


@pytest.fixture(scope="module")
def ps():
    import paper_2312_17396_amd as ps
    ps.lib()
    return ps


def _jordan_pairs(n, t, a):
    """block diagonal of n/2 blocks [[-t, a], [0, -t]] (n even)"""
    X = -t * np.eye(n)
    for i in range(0, n, 2):
        X[i, i + 1] = a
    return X


def _margin_ok(X, c):
    """the oracle's growth decisions are not within rounding of a tie"""
    m = len(c) - 1
    s = 1
    while s * s < m:
        s += 1
    nX = metrics.norm1(X)
    if not nX <= s / math.e or s >= m:
        return abs(nX - s / math.e) > 1e-9 * nX
    P = [np.eye(X.shape[0]), X]
    for _ in range(2, s + 1):
        P.append(P[-1] @ X)
    B0 = sum(c[j] * P[j] for j in range(s))
    Y = P[s]
    while True:
        lhs, rhs = metrics.norm1(Y), metrics.norm1(B0) * nX ** s
        if abs(lhs - rhs) <= 1e-9 * max(lhs, rhs):
            return False
        if not (lhs > rhs and s < m):
            return True
        B0 = B0 + c[s] * Y
        s += 1
        Y = X @ Y


# (t, a, s): s from the closed form of the 2 x 2 Jordan block (exact rationals)
JORDAN = [(0.5, 1 / 32, 23), (0.25, 1 / 32, 8), (0.75, 1 / 8, 11), (1.0, 1 / 4, 9), (0.5, 1 / 4, 6)]


@pytest.mark.parametrize("mode", ["fixed", "mixed"])
@pytest.mark.parametrize("t,a,s_exp", JORDAN)
@pytest.mark.parametrize("n,sigma", [(2, 0), (130, 1)])
def test_vars_jordan_closed_form(ps, n, sigma, t, a, s_exp, mode):
    X = _jordan_pairs(n, t, a)
    A = X * 2.0 ** sigma
    c = coeffs.taylor_exp(M)
    assert metrics.variable_s(X.T, c) == s_exp
    E, s, rep = ps.ps_expm_vars(to_dev(A), M, sigma=sigma, mode=mode, report=True)
    assert s == s_exp and rep["s"] == s_exp and rep["r"] == M // s_exp
    Eh, El = oracle.expm_dd(A, c, sigma)
    assert metrics.rel_err_1(to_np(E), Eh, El) <= TOL64
    if mode == "mixed":
        u, nu, tiers = oplan.plan(rep["normB"], rep["normY"], working_tier=0)
        assert tiers[1:] == rep["tier"][1:rep["r"] + 1]


def _shifted(n, t, eps, seed):
    G = np.random.default_rng(seed).standard_normal((n, n))
    return -t * np.eye(n) + G * (eps / metrics.norm1(G.T))


@pytest.mark.parametrize("n,t,eps,seed", [(64, 0.5, 0.05, 1), (200, 0.8, 0.1, 2), (257, 0.3, 0.02, 3),
                                          (100, 1.0, 0.5, 4), (96, 2.5, 0.05, 5)])
def test_vars_dense_matches_oracle(ps, n, t, eps, seed):
    A = _shifted(n, t, eps, seed)
    c = coeffs.taylor_exp(M)
    assert _margin_ok(A.T, c)
    s_o = metrics.variable_s(A.T, c)
    E, s = ps.ps_expm_vars(to_dev(A), M, mode="mixed")
    assert s == s_o
    Eh, El = oracle.expm_dd(A, c, 0)
    assert metrics.rel_err_1(to_np(E), Eh, El) <= TOL64
    # the same s through the fixed-s path agrees with the oracle as well
    E2 = to_np(ps.ps_expm(to_dev(A), M, s=s, mode="mixed"))
    assert metrics.rel_err_1(E2, Eh, El) <= TOL64


def test_vars_grows_to_explicit_powers_for_negative_scalar(ps):
    A = -0.5 * np.eye(70)
    E, s, rep = ps.ps_expm_vars(to_dev(A), M, mode="mixed", report=True)
    assert s == M and rep["r"] == 1 and rep["first_step"] == 0
    np.testing.assert_allclose(np.diag(to_np(E)), math.exp(-0.5), rtol=1e-15)


def test_vars_keeps_default_s_for_large_norm(ps):
    # ||X||_1 = 2.5 > 6/e (kept small: the Taylor sum of a matrix with
    # spectrum near -2.5 loses about e^(2 ||X||) u to cancellation)
    A = _shifted(80, 2.4, 0.1, 9)
    E, s = ps.ps_expm_vars(to_dev(A), M, sigma=0, mode="mixed")
    assert s == 6
    Eh, El = oracle.expm_dd(A, coeffs.taylor_exp(M), 0)
    assert metrics.rel_err_1(to_np(E), Eh, El) <= TOL64


def test_vars_fp32(ps):
    import torch
    A = _jordan_pairs(100, 0.75, 0.125).astype(np.float32).astype(np.float64)
    E, s = ps.ps_expm_vars(to_dev(A, torch.float32), M, mode="mixed")
    assert s == 11
    Eh, El = oracle.expm_dd(A, coeffs.taylor_exp(M), 0)
    assert metrics.rel_err_1(to_np(E).astype(np.float64), Eh, El) <= 8 * 100 * 2.0 ** -24


def test_vars_rejects_bad_arguments(ps):
    A = np.eye(8)
    with pytest.raises(ps.PSError):
        ps.ps_expm_vars(to_dev(A), M, mode="mixed", tier_mask=0, delta=10.0, out=to_dev(np.eye(4)))
    A[3, 2] = np.nan
    with pytest.raises(ps.PSError):
        ps.ps_expm_vars(to_dev(A), M)
