"""GPU parity of the double-double working precision (ps_expm_dd): against
the double-double oracle on the same polynomial, against exact rational
arithmetic for small inputs with nonzero low parts, and the plan over five
tiers against the oracle's planner."""
from fractions import Fraction as F

import numpy as np
import pytest

import oracle
from oracle import coeffs, metrics
from oracle import plan as oplan

from helpers import DEV

pytestmark = pytest.mark.gpu

U_DD = 2.0 ** -106


@pytest.fixture(scope="module")
def ps():
    import paper_2312_17396_amd as ps
    ps.lib()
    return ps


def _dd_tensor(hi, lo=None):
    import torch
    lo = np.zeros_like(hi) if lo is None else lo
    return torch.tensor(np.stack([hi, lo]), dtype=torch.float64, device=DEV)


def _rand(n, t, seed):
    G = np.random.default_rng(seed).standard_normal((n, n))
    return G * (t / metrics.norm1(G))


def test_square_of_integer_matrix_is_exact(ps):
    # p(x) = x^2: one double-double product.  Entries up to 2^40 make sums of
    # products near 2^88: not representable in double, exact in double-double
    g = np.random.default_rng(3)
    for n in (1, 5, 64, 70, 130):
        A = g.integers(-2 ** 40, 2 ** 40, (n, n)).astype(np.float64)
        E = ps.ps_expm_dd(_dd_tensor(A), 2, s=2, coef=([0.0, 0.0, 1.0], [0.0, 0.0, 0.0])).cpu().numpy()
        Ai = A.astype(np.int64).astype(object)
        exact = Ai @ Ai                                # python integers
        got = np.vectorize(lambda h, l: int(F(h) + F(l)), otypes=[object])(E[0], E[1])
        assert (got == exact).all(), n


@pytest.mark.parametrize("n,m,s,sigma,t", [
    (1, 30, 6, 0, 0.5), (17, 30, 6, 0, 1.0), (64, 30, 6, 2, 3.0), (100, 40, 7, 0, 0.8), (65, 18, 5, 1, 1.5),
])
@pytest.mark.parametrize("mode", ["fixed", "mixed"])
def test_dd_vs_oracle(ps, n, m, s, sigma, t, mode):
    A = _rand(n, t, 100 + n)
    c = coeffs.taylor_exp(m)                     # the oracle's coefficients (doubles)
    Eh, El = oracle.expm_dd(A, c, sigma)
    E, rep = ps.ps_expm_dd(_dd_tensor(A), m, s=s, sigma=sigma, coef=(c, [0.0] * (m + 1)), mode=mode, report=True)
    E = E.cpu().numpy()
    err = metrics.rel_err_dd(E[0], E[1], Eh, El)
    assert err <= 2.0 ** sigma * 64 * n * U_DD, (err, rep["tier"])
    if mode == "mixed" and rep["r"] >= 1:
        u, nu, tiers = oplan.plan(rep["normB"], rep["normY"], working_tier=4)
        assert tiers[1:] == rep["tier"][1:]
        assert rep["tier"][0] == 4


def test_dd_mixed_uses_low_tiers(ps):
    # small ||X||: the plan moves the early Horner products far below double-double
    # (here u_1 ~ 3e-21 is below FP64's 2^-53, so step 1 stays double-double
    # and steps 2..4 go to FP32 and FP8), at the same accuracy
    n, m = 96, 30
    A = _rand(n, 0.25, 9)
    c = coeffs.taylor_exp(m)
    E, rep = ps.ps_expm_dd(_dd_tensor(A), m, s=6, coef=(c, [0.0] * (m + 1)), mode="mixed", report=True)
    steps = rep["tier"][1:rep["first_step"] + 1]
    low = [t for t in steps if t != 4]
    assert len(low) >= 2 and max(low) >= 2, steps
    u, nu, tiers = oplan.plan(rep["normB"], rep["normY"], working_tier=4)
    assert tiers[1:] == rep["tier"][1:]
    Eh, El = oracle.expm_dd(A, c, 0)
    E = E.cpu().numpy()
    assert metrics.rel_err_dd(E[0], E[1], Eh, El) <= 64 * n * U_DD


def test_dd_inputs_with_low_parts_vs_exact_rationals(ps):
    # A = hi + lo with lo ~ 2^-60 hi: p(A) = sum c_k A^k with exact dyadic
    # coefficients, evaluated in exact rational arithmetic
    g = np.random.default_rng(4)
    n, m = 4, 12
    hi = g.standard_normal((n, n)) * 0.3
    lo = hi * np.ldexp(g.uniform(-1, 1, (n, n)), -60)
    ch = [float(np.ldexp(1.0, -k)) for k in range(m + 1)]          # c_k = 2^-k, exact
    cl = [0.0] * (m + 1)
    A = [[F(hi[i, j]) + F(lo[i, j]) for j in range(n)] for i in range(n)]
    P = [[F(0)] * n for _ in range(n)]
    for i in range(n):
        P[i][i] = F(ch[m])
    for k in range(m - 1, -1, -1):                                   # Horner, exact
        P = [[sum(P[i][l] * A[l][j] for l in range(n)) for j in range(n)] for i in range(n)]
        for i in range(n):
            P[i][i] += F(ch[k])
    E = ps.ps_expm_dd(_dd_tensor(hi, lo), m, s=4, coef=(ch, cl)).cpu().numpy()
    err = max(abs(F(E[0, i, j]) + F(E[1, i, j]) - P[i][j]) for i in range(n) for j in range(n))
    scale = max(abs(P[i][j]) for i in range(n) for j in range(n))
    assert float(err / scale) <= 64 * U_DD


def _exact_expm(Aq, cq, sigma):
    """(p(2^-sigma A))^(2^sigma) in exact rational arithmetic (object arrays of
    Fractions), p by Horner's rule with the exact coefficients cq"""
    n = Aq.shape[0]
    X = Aq * F(1, 2 ** sigma)
    I = np.array([[F(int(i == j)) for j in range(n)] for i in range(n)], dtype=object)
    P = I * cq[-1]
    for c in reversed(cq[:-1]):
        P = P.dot(X) + I * c
    for _ in range(sigma):
        P = P.dot(P)
    return P


@pytest.mark.parametrize("n,sigma", [(16, 1), (24, 0)])
@pytest.mark.parametrize("mode", ["fixed", "mixed"])
def test_dd_dyadic_vs_exact_rationals(ps, n, sigma, mode):
    """A reference with more digits than double-double: dyadic inputs with
    nonzero low parts (hi + lo, lo ~ 2^-70 hi) and the Taylor coefficients as
    double-double pairs (dyadic too), so p(2^-sigma A)^(2^sigma)
    is an exact rational; every entry of the GPU result against it."""
    g = np.random.default_rng(40 + n)
    m = 18
    hi = np.ldexp(np.round(g.standard_normal((n, n)) * 2 ** 12), -12) * (1.5 / n)
    lo = np.ldexp(np.round(g.uniform(-1, 1, (n, n)) * 2 ** 20), -20) * np.ldexp(np.abs(hi) + 2 ** -12, -70)
    import math
    ch = [float(F(1, math.factorial(k))) for k in range(m + 1)]           # 1/k! as double-double pairs
    cl = [float(F(1, math.factorial(k)) - F(h)) for k, h in enumerate(ch)]
    Aq = np.array([[F(hi[i, j]) + F(lo[i, j]) for j in range(n)] for i in range(n)], dtype=object)
    cq = [F(a) + F(b) for a, b in zip(ch, cl)]
    P = _exact_expm(Aq, cq, sigma)
    E, rep = ps.ps_expm_dd(_dd_tensor(hi, lo), m, s=5, sigma=sigma, coef=(ch, cl), mode=mode, report=True)
    E = E.cpu().numpy()
    diff = [[abs(F(E[0, i, j]) + F(E[1, i, j]) - P[i, j]) for j in range(n)] for i in range(n)]
    num = max(sum(diff[i][j] for i in range(n)) for j in range(n))
    den = max(sum(abs(P[i, j]) for i in range(n)) for j in range(n))
    err = float(num / den)
    print("dd n=%d sigma=%d %s: rel err %.3e (%.1f u_dd), tiers %s" % (n, sigma, mode, err, err / U_DD, rep["tier"]))
    assert err <= 2.0 ** sigma * 64 * n * U_DD, (err, rep["tier"])


def test_dd_rejects_bad_arguments(ps):
    import torch
    with pytest.raises(ps.PSError):
        ps.ps_expm_dd(torch.zeros(3, 4, 4, dtype=torch.float64, device=DEV), 10)
    with pytest.raises(ps.PSError):
        ps.ps_expm_dd(_dd_tensor(np.eye(4)), 300)
