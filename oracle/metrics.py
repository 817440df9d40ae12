"""Error and cost measures of the paper.

TEST INFRASTRUCTURE ONLY (part of the oracle).

  rel_err_1(P, ref_hi, ref_lo)  the relative error in the 1-norm used
      throughout the experiments (section 3.3):
      ||P - p||_1 / ||p||_1, with the reference p = hi + lo given in dd and the
      difference formed as (P - hi) - lo.
  rel_err_cols(...)  the same measure restricted to a sample of columns.
  cost_saving(D, s, r, d)  the cost ratio of eq. (Cr) read as a saving:
      1 - ((s - 1) D + sum_i d_i) / ((s + r - 1) D), where D is the number of
      decimal digits of the working precision and d_i those of u_i.  This is
      the reading under which all four C_r entries of Table 1 reproduce.
  alpha_m(X, m)  max(||X^d||^(1/d), ||X^(d+1)||^(1/(d+1))) with
      d = floor((1 + sqrt(4m + 5)) / 2)  (section 3.2).
  extra_scaling(normX, s)  l_0 = ceil(log2(e ||X||_1 / s)), the number of
      extra squarings that would force ||X||_1 <= s/e (section 3.2).
  theta_taylor(m, u)  the largest theta with sum_{k>m} theta^k / k! <= u, the
      Taylor truncation error at the scalar alpha_m of eq. (alpha_m-X) with
      the practical estimate xi(X) taken as 1 (50-digit decimal arithmetic,
      bisection).
  auto_sigma(A, m, s, u, norm_guard)  the scaling chosen by the alpha_m
      bound: sigma0 from ||A||_1 <= 2^sigma0 theta_m, alpha_m of
      X0 = 2^-sigma0 A from its powers (repeated multiplication in IEEE
      double), sigma the smallest with 2^-sigma alpha_m(A) <= theta_m; with
      norm_guard also ||2^-sigma A||_1 <= s / e (section 3.2).
  select_degree(A, m_max, u)  the joint choice of (m, s, sigma) by the
      alpha_m bound: candidates m = q^2, q(q+1) <= m_max with PS cost
      (s - 1) + floor(m/s) - [s | m], s = ceil(sqrt(m)); alpha_m(A) from the
      powers of A (repeated multiplication in IEEE double); for each m the
      least sigma with 2^-sigma alpha_m(A) <= theta_m; the least cost plus
      sigma wins, the smaller m on ties (section 3.2).
  variable_s(X, coef)  the block size of Algorithm 2's variable-s branch
      (fix_params = false, section 3.3): s = ceil(sqrt(m)); only when
      ||X||_1 <= s / e, B_0 = sum_{j<s} c_j X^j and Y = X^s, then while
      ||Y||_1 > ||B_0||_1 ||X||_1^s and s < m: B_0 += c_s Y, s += 1,
      Y = X Y (IEEE double, powers by repeated multiplication).
"""
from __future__ import annotations

import math

import numpy as np


def norm1(A) -> float:
    return float(np.max(np.sum(np.abs(np.asarray(A, dtype=np.float64)), axis=0))) if np.size(A) else 0.0


def rel_err_1(P, ref_hi, ref_lo=None) -> float:
    P = np.asarray(P, dtype=np.float64)
    D = P - np.asarray(ref_hi)
    if ref_lo is not None:
        D = D - np.asarray(ref_lo)
    den = norm1(ref_hi)
    num = norm1(D)
    if den == 0.0:
        return 0.0 if num == 0.0 else math.inf
    return num / den


def rel_err_dd(qh, ql, ph, pl) -> float:
    """Relative 1-norm distance between two dd matrices (q - p) / p."""
    D = (np.asarray(qh) - np.asarray(ph)) + (np.asarray(ql) - np.asarray(pl))
    den = norm1(ph)
    return norm1(D) / den if den else (0.0 if norm1(D) == 0 else math.inf)


def rel_err_cols(Pcols, ref_hi, ref_lo=None) -> float:
    """Column-sample version: max_j ||(P - p) e_j||_1 / max_j ||p e_j||_1."""
    return rel_err_1(Pcols, ref_hi, ref_lo)


def cost_saving(D: float, s: int, r: int, d) -> float:
    return 1.0 - ((s - 1) * D + float(sum(d))) / ((s + r - 1) * D)


def alpha_m(X, m: int) -> float:
    X = np.asarray(X, dtype=np.float64)
    d = int(math.floor((1 + math.sqrt(4 * m + 5)) / 2))
    Pd = np.linalg.matrix_power(X, d)
    Pd1 = Pd @ X
    return max(norm1(Pd) ** (1.0 / d), norm1(Pd1) ** (1.0 / (d + 1)))


def extra_scaling(normX: float, s: int) -> int:
    return int(math.ceil(math.log2(math.e * normX / s)))


def _taylor_tail_dec(t, m):
    from decimal import Decimal, localcontext
    with localcontext() as ctx:
        ctx.prec = 50
        t = Decimal(t)
        term = Decimal(1)
        for k in range(1, m + 2):
            term = term * t / k
        total = term
        k = m + 2
        while True:
            term = term * t / k
            total += term
            if term <= total * Decimal("1e-45"):
                return total
            k += 1


def theta_taylor(m: int, u: float) -> float:
    from decimal import Decimal, localcontext
    with localcontext() as ctx:
        ctx.prec = 50
        ud = Decimal(u)
        lo, hi = Decimal(0), Decimal(1)
        while _taylor_tail_dec(hi, m) <= ud:
            hi *= 2
        for _ in range(120):
            mid = (lo + hi) / 2
            if _taylor_tail_dec(mid, m) <= ud:
                lo = mid
            else:
                hi = mid
        return float(lo)


def _smallest_shift(a: float, b: float) -> int:
    """smallest k >= 0 with a <= 2^k b"""
    k = 0
    while a > math.ldexp(b, k):
        k += 1
    return k


def auto_sigma(A, m: int, s: int, u: float, norm_guard: bool = False) -> int:
    A = np.asarray(A, dtype=np.float64)
    th = theta_taylor(m, u)
    nA = norm1(A)
    s0 = _smallest_shift(nA, th)
    X0 = A * math.ldexp(1.0, -s0)
    d = 1
    while (d + 1) * d <= m + 1:
        d += 1
    Pd = np.linalg.matrix_power(X0, d)
    Pd1 = Pd @ X0
    a0 = max(norm1(Pd) ** (1.0 / d), norm1(Pd1) ** (1.0 / (d + 1)))
    sig = min(s0, _smallest_shift(math.ldexp(a0, s0), th))
    if norm_guard:
        sig = max(sig, _smallest_shift(math.e * nA, float(s)))
    return sig


def variable_s(X, coef) -> int:
    X = np.asarray(X, dtype=np.float64)
    c = [float(v) for v in coef]
    m = len(c) - 1
    s = 1
    while s * s < m:
        s += 1
    nX = norm1(X)
    if not (nX <= s / math.e) or s >= m:
        return s
    n = X.shape[0]
    powers = [np.eye(n), X]
    for _ in range(2, s + 1):
        powers.append(powers[-1] @ X)
    B0 = sum(c[j] * powers[j] for j in range(s))
    Y = powers[s]
    while norm1(Y) > norm1(B0) * nX ** s and s < m:
        B0 = B0 + c[s] * Y
        s += 1
        Y = X @ Y
    return s


def _ceil_sqrt(m: int) -> int:
    s = 1
    while s * s < m:
        s += 1
    return s


def select_degree(A, m_max: int, u: float):
    A = np.asarray(A, dtype=np.float64)
    cands = []
    q = 1
    while q * q <= m_max:
        cands.append(q * q)
        if q * (q + 1) <= m_max:
            cands.append(q * (q + 1))
        q += 1
    thetas = [theta_taylor(m, u) for m in cands]
    nA = norm1(A)
    s0 = _smallest_shift(nA, thetas[-1])
    X0 = A * math.ldexp(1.0, -s0)
    dstar = []
    for m in cands:
        d = 1
        while (d + 1) * d <= m + 1:
            d += 1
        dstar.append(d)
    D = max(max(_ceil_sqrt(m), d + 1) for m, d in zip(cands, dstar))
    norms = {1: norm1(X0)}
    P = X0
    for d in range(2, D + 1):
        P = P @ X0
        norms[d] = norm1(P)
    best = None
    for m, d, th in zip(cands, dstar, thetas):
        a0 = max(norms[d] ** (1.0 / d), norms[d + 1] ** (1.0 / (d + 1)))
        sig = _smallest_shift(math.ldexp(a0, s0), th)
        s = _ceil_sqrt(m)
        r = m // s
        cost = (s - 1) + r - (1 if m == s * r else 0) + sig
        if best is None or cost < best[0]:
            best = (cost, m, s, sig)
    return best[1], best[2], best[3]
