"""Degenerate and extreme arguments of the PS path on the GPU: degree 0 and
1, the largest degree (255, with r = 15 blocks), s = m, one-by-one matrices
and a long squaring chain, each against the double-double oracle (or an
exact value)."""
import numpy as np
import pytest

import oracle
from oracle import coeffs, metrics

from helpers import to_dev, to_np

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


@pytest.fixture(scope="module")
def ps():
    import paper_2312_17396_amd as ps
    ps.lib()
    return ps


def _rand(n, t, seed):
    G = np.random.default_rng(seed).standard_normal((n, n))
    return G * (t / metrics.norm1(G.T))


@pytest.mark.parametrize("mode", ["fixed", "mixed"])
@pytest.mark.parametrize("n", [1, 37, 130])
def test_degree_zero_is_scaled_identity(ps, n, mode):
    A = _rand(n, 2.0, n)
    P = to_np(ps.ps_eval(to_dev(A), [0.375], mode=mode))
    assert np.array_equal(P, 0.375 * np.eye(n))


@pytest.mark.parametrize("mode", ["fixed", "mixed"])
@pytest.mark.parametrize("n", [1, 37, 130])
def test_degree_one(ps, n, mode):
    A = _rand(n, 2.0, 10 + n)
    c = [0.5, -1.25]
    P = to_np(ps.ps_eval(to_dev(A), c, mode=mode))
    Ph, Pl = oracle.poly_dd(A, c)
    # one rounding per entry at most
    assert np.all(np.abs((P - Ph) - Pl) <= U * np.abs(Ph) + 1e-300)


@pytest.mark.parametrize("mode", ["fixed", "mixed"])
def test_largest_degree(ps, mode):
    # m = 255, s = 16: r = 15 blocks; coefficients 2^-k are exact, ||X|| < 1
    n, m = 96, 255
    A = _rand(n, 0.9, 3)
    c = [float(np.ldexp(1.0, -k)) for k in range(m + 1)]
    P, rep = ps.ps_eval(to_dev(A), c, s=16, mode=mode, report=True)
    assert rep["r"] == 15
    Ph, Pl = oracle.poly_dd(A, c)
    assert metrics.rel_err_1(to_np(P), Ph, Pl) <= 1e-13


@pytest.mark.parametrize("mode", ["fixed", "mixed"])
def test_block_size_equal_to_degree(ps, mode):
    # s = m: explicit powers, r = 1 with the trivial last step folded in
    n, m = 70, 9
    A = _rand(n, 1.0, 4)
    c = coeffs.taylor_exp(m)
    P, rep = ps.ps_eval(to_dev(A), c, s=m, mode=mode, report=True)
    assert rep["r"] == 1 and rep["first_step"] == 0
    Ph, Pl = oracle.poly_dd(A, c)
    assert metrics.rel_err_1(to_np(P), Ph, Pl) <= 1e-14


@pytest.mark.parametrize("n,sigma", [(1, 5), (33, 20)])
def test_long_squaring_chain(ps, n, sigma):
    # the squarings amplify the rounding of p(X) by about 2^sigma
    A = _rand(n, 1.0, 5 + n)
    m = 30
    c = coeffs.taylor_exp(m)
    E = to_np(ps.ps_expm(to_dev(A), m, s=6, sigma=sigma, mode="mixed"))
    Eh, El = oracle.expm_dd(A, c, sigma)
    assert metrics.rel_err_1(E, Eh, El) <= 2.0 ** sigma * 4 * n * U
