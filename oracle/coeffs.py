"""Polynomial coefficients as exact rationals, rounded once to IEEE double.

TEST INFRASTRUCTURE ONLY (part of the oracle).

  taylor_exp(m)   b_i = 1/i!                      (section 3, start)
  pade_exp(k, m)  numerator p_km and denominator q_km of the [k/m] Pade
                  approximant of exp (section 4.1):
                      p_j = (k+m-j)! k! / ((k+m)! j! (k-j)!)
                      q_j = (-1)^j (k+m-j)! m! / ((k+m)! j! (m-j)!)
                  For k = m, q(x) = p(-x).  Section 2 prints B_0 and B_1 of the
                  [13/13] numerator with s = 4; tests pin those rationals.
  taylor_cos(m)   c_m(Z) = sum_{k=0}^{m} (-1)^k Z^k / (2k)!, a polynomial in
                  Z = X^2 (section 4.2: the cosine approximant has only even
                  powers, so PS runs in X^2).
Python's float(Fraction) is correctly rounded, so each double is the nearest
one to the exact coefficient.
"""
from __future__ import annotations

from fractions import Fraction
from math import factorial


def taylor_exp_exact(m: int):
    return [Fraction(1, factorial(i)) for i in range(m + 1)]


def taylor_exp(m: int):
    return [float(c) for c in taylor_exp_exact(m)]


def pade_exp_exact(k: int, m: int):
    den = factorial(k + m)
    p = [Fraction(factorial(k + m - j) * factorial(k), den * factorial(j) * factorial(k - j)) for j in range(k + 1)]
    q = [Fraction((-1) ** j * factorial(k + m - j) * factorial(m), den * factorial(j) * factorial(m - j))
         for j in range(m + 1)]
    return p, q


def pade_exp(k: int, m: int):
    p, q = pade_exp_exact(k, m)
    return [float(c) for c in p], [float(c) for c in q]


def taylor_cos_exact(m: int):
    return [Fraction((-1) ** k, factorial(2 * k)) for k in range(m + 1)]


def taylor_cos(m: int):
    return [float(c) for c in taylor_cos_exact(m)]
