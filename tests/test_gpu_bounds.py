"""Componentwise error bounds of section 2 checked on the GPU path against
the double-double oracle:

  * power lemma: |fl(X^t) - X^t| <= gamma_{(t-1)n} |X|^t.  The library forms
    X_j = X_a X_b (a = ceil(j/2), b = floor(j/2)); the same bound holds since
    gamma_n + gamma_{(a-1)n} + gamma_{(b-1)n} and their products add up to at
    most gamma_{(j-1)n}.  X^t is read out as p(x) = x^t with s = t, where the
    result is the power-table entry itself (B_0 = 0 + 1 * Y, exact).
  * block assembly (the theorem on polynomials of computed powers, eq.
    (xpoly-err)): psi = sum_{j<=t} a_j X^j formed from the computed powers
    satisfies |psi_hat - psi| <= gamma_t |a_0| I
                                + sum_j gamma_{(j-1)(n-1)+t+1} |a_j| |X|^j.
    It is read out as p of degree m = s with c_m = 0: then PS folds
    c_m Y = 0 into B_0 (exactly) and the result is the single block B_0.
gamma_k = k u / (1 - k u), u = 2^-53."""
import numpy as np
import pytest

import oracle

from helpers import to_dev, to_np

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


def gamma(k):
    return k * U / (1.0 - k * U)


@pytest.fixture(scope="module")
def ps():
    import paper_2312_17396_amd as ps
    ps.lib()
    return ps


def _mat(n, seed, scale):
    return np.random.default_rng(seed).standard_normal((n, n)) * (scale / np.sqrt(n))


def _abs_powers(X, t):
    """|X|^1 .. |X|^t in IEEE double (entries rounded up by a relative 1e-12
    slack below, far above their rounding)"""
    Xa = np.abs(X)
    out = [np.eye(X.shape[0]), Xa]
    for _ in range(2, t + 1):
        out.append(out[-1] @ Xa)
    return out


@pytest.mark.parametrize("n,t,seed", [(100, 2, 1), (100, 5, 2), (130, 6, 3), (200, 8, 4), (67, 7, 5)])
def test_power_table_componentwise(ps, n, t, seed):
    X = _mat(n, seed, 1.5)
    coef = [0.0] * t + [1.0]
    P = to_np(ps.ps_eval(to_dev(X), coef, s=t))
    # the library works on the column-major view, i.e. on X^T; p(X^T) = p(X)^T,
    # so the row-major result is X^t itself
    Ph, Pl = oracle.poly_dd(X, coef)
    err = np.abs((P - Ph) - Pl)
    bound = gamma((t - 1) * n) * _abs_powers(X, t)[t] * (1 + 1e-12)
    assert (err <= bound).all(), float(np.max(err / np.maximum(bound, 1e-300)))
    # and the bound is not vacuous: the error is a visible fraction of it
    assert err.max() > 0.0


@pytest.mark.parametrize("n,s,seed,kind", [(100, 4, 6, "taylor"), (150, 6, 7, "taylor"), (96, 5, 8, "mixed"),
                                           (129, 8, 9, "mixed")])
def test_block_assembly_componentwise(ps, n, s, seed, kind):
    X = _mat(n, seed, 1.0)
    t = s - 1                                   # B_0 = sum_{j <= s-1} a_j X^j
    if kind == "taylor":
        from oracle import coeffs
        a = list(coeffs.taylor_exp(t))
    else:
        a = list(np.random.default_rng(seed).uniform(-1.0, 1.0, t + 1))
    P = to_np(ps.ps_eval(to_dev(X), a + [0.0], s=s))   # m = s, c_m = 0
    Ph, Pl = oracle.poly_dd(X, a)
    err = np.abs((P - Ph) - Pl)
    pw = _abs_powers(X, t)
    bound = gamma(t) * abs(a[0]) * np.eye(n)
    for j in range(1, t + 1):
        bound = bound + gamma((j - 1) * (n - 1) + t + 1) * abs(a[j]) * pw[j]
    bound *= 1 + 1e-12
    assert (err <= bound).all(), float(np.max(err / np.maximum(bound, 1e-300)))
