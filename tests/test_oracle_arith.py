"""Pins of the oracle's double-double arithmetic against exact rational arithmetic.

The oracle's error-free transformations must be exact, and its dd operations
must be accurate to a small multiple of u^2 (u = 2^-53), which is what makes it
a reference with twice the digits of IEEE double (the protocol of the paper's
experiments, section 3.3)."""
from fractions import Fraction as F

import numpy as np
import pytest

import oracle

U = 2.0 ** -53


def _rand_doubles(rng, k, spread=30):
    return rng.standard_normal(k) * np.exp2(rng.integers(-spread, spread, k))


def _dd_rand(rng):
    hi = float(_rand_doubles(rng, 1)[0])
    lo = float(hi * U * rng.uniform(-1, 1))
    s, e = oracle.two_sum(hi, lo)       # normalise so |lo| <= ulp(hi)/2
    return s, e


def test_two_sum_two_prod_exact():
    rng = np.random.default_rng(1)
    a = _rand_doubles(rng, 2000)
    b = _rand_doubles(rng, 2000)
    for x, y in zip(a, b):
        s, e = oracle.two_sum(x, y)
        assert F(s) + F(e) == F(x) + F(y)
        p, q = oracle.two_prod(x, y)
        assert F(p) + F(q) == F(x) * F(y)


@pytest.mark.parametrize("op,bound", [("add", 3.1), ("mul", 5.1), ("mul_d", 2.1)])
def test_dd_ops_accuracy(op, bound):
    rng = np.random.default_rng(2)
    worst = 0.0
    for _ in range(3000):
        a = _dd_rand(rng)
        b = _dd_rand(rng)
        if op == "add":
            r = oracle.dd_add(a, b)
            exact = F(a[0]) + F(a[1]) + F(b[0]) + F(b[1])
        elif op == "mul":
            r = oracle.dd_mul(a, b)
            exact = (F(a[0]) + F(a[1])) * (F(b[0]) + F(b[1]))
        else:
            r = oracle.dd_mul_d(a, b[0])
            exact = (F(a[0]) + F(a[1])) * F(b[0])
        if exact == 0:
            continue
        err = abs((F(r[0]) + F(r[1]) - exact) / exact)
        worst = max(worst, float(err))
    assert worst <= bound * U * U, worst


def test_dd_gemm_vs_exact_rationals():
    rng = np.random.default_rng(3)
    for n in (1, 2, 3, 4):
        Ah = rng.standard_normal((n, n))
        Al = Ah * U * rng.uniform(-1, 1, (n, n))
        Bh = rng.standard_normal((n, n))
        Bl = Bh * U * rng.uniform(-1, 1, (n, n))
        Ch, Cl = oracle.gemm_dd(Ah, Al, Bh, Bl)
        for i in range(n):
            for j in range(n):
                exact = sum((F(Ah[i, l]) + F(Al[i, l])) * (F(Bh[l, j]) + F(Bl[l, j])) for l in range(n))
                scale = sum(abs(Ah[i, l] * Bh[l, j]) for l in range(n))
                err = abs(F(Ch[i, j]) + F(Cl[i, j]) - exact)
                assert float(err) <= 8 * n * U * U * scale


def test_double_times_dd_gemm_vs_exact_rationals():
    rng = np.random.default_rng(4)
    n, k = 4, 3
    X = rng.standard_normal((n, n))
    Vh = rng.standard_normal((n, k))
    Vl = Vh * U * rng.uniform(-1, 1, (n, k))
    c = [0.0, 1.0]               # p(X) V = X V
    Wh, Wl = oracle.poly_apply_dd(X, c, Vh, Vl)
    for i in range(n):
        for j in range(k):
            exact = sum(F(X[i, l]) * (F(Vh[l, j]) + F(Vl[l, j])) for l in range(n))
            scale = sum(abs(X[i, l] * Vh[l, j]) for l in range(n))
            assert float(abs(F(Wh[i, j]) + F(Wl[i, j]) - exact)) <= 8 * n * U * U * scale
