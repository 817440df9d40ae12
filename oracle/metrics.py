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
  m_low(D, s, r, d)  the share of the s - 1 + r PS products run in precision
      u^(1/2) or lower (Table 2's M_low), d_i the decimal digits of u_i.
  extra_scaling(normX, s)  l_0 = ceil(log2(e ||X||_1 / s)), the number of
      extra squarings that would force ||X||_1 <= s/e (section 3.2).
  theta_taylor(m, u)  the largest theta with sum_{k>m} theta^k / k! <= u: the
      Taylor truncation threshold at the scalar alpha_m of eq. (alpha_m-X)
      when xi(X) = 1 (50-digit decimal arithmetic, bisection).  Used only for
      the first scaling sigma0 that keeps the powers of X0 = 2^-sigma0 A
      bounded; the acceptance itself uses xi_b0 below.
  taylor_tail(t, m)  sum_{k>m} t^k / k! in 50-digit decimal arithmetic.
  xi_b0(X, s)  the estimate xi(X) of ||e^X||_1 in eq. (alpha_m-X), which the
      paper leaves as "a practical estimate": ||B_0(X)||_1 with
      B_0 = sum_{j<s} X^j / j!, the leading block of the PS form.  Section 3.1
      itself takes B_0(X) as the approximation of e^X (its check of eq.
      (cond-Y)).  Powers by repeated multiplication (Fragment EvalB0), IEEE
      double, coefficients 1/j! correctly rounded.
  accepts(A, sigma, m, s, u, alpha_A)  eq. (alpha_m-X) at X = 2^-sigma A:
      taylor_tail(2^-sigma alpha_m(A), m) <= u xi_b0(X, s).  A non-finite
      xi rejects.  For t = 2^-sigma alpha_m(A) > 800 (then t >= m + 2 for
      every m <= 170, so at least half of the Poisson(t) mass lies above m and
      the tail is at least e^t / 2 > e^799, more than u times the largest
      double) the candidate is rejected without summing the series.
  auto_sigma(A, m, s, u, norm_guard)  the scaling chosen by the alpha_m
      bound: sigma0 from ||A||_1 <= 2^sigma0 theta_m, alpha_m(A) =
      2^sigma0 alpha_m(X0) from the powers of X0 = 2^-sigma0 A (repeated
      multiplication in IEEE double), sigma the least sigma >= 0 that
      `accepts`; with norm_guard also ||2^-sigma A||_1 <= s / e (section 3.2).
  select_degree(A, m_max, u)  the joint choice of (m, s, sigma) by the
      alpha_m bound: candidates m = q^2, q(q+1) <= m_max with PS cost
      (s - 1) + floor(m/s) - [s | m], s = ceil(sqrt(m)); alpha_m(A) from the
      powers of X0 = 2^-sigma0 A (sigma0 from the largest candidate's theta,
      repeated multiplication in IEEE double); for each m the least sigma
      that `accepts` (with that m and s); the least cost plus sigma wins, the
      smaller m on ties.  The cost rule is this build's reading (parity
      unpinned: the paper takes m from its reference algorithm and gives no
      cost rule).
  variable_s(X, coef)  the block size of Algorithm 2's variable-s branch
      (fix_params = false, section 3.3): s = ceil(sqrt(m)); only when
      ||X||_1 <= s / e, B_0 = sum_{j<s} c_j X^j and Y = X^s, then while
      ||Y||_1 > ||B_0||_1 ||X||_1^s and s < m: B_0 += c_s Y, s += 1,
      Y = X Y (IEEE double, powers by repeated multiplication).
"""
from __future__ import annotations

import math

import numpy as np

from .coeffs import taylor_exp


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


def m_low(D: float, s: int, r: int, d) -> float:
    """Table 2's M_low: the share of the s - 1 + r products performed in
    precision u^(1/2) or lower, i.e. with d_i <= D / 2 decimal digits (the
    s - 1 powers run in the working precision)."""
    return sum(1 for x in d if x <= D / 2.0) / float(s - 1 + r)


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


def taylor_tail(t, m: int):
    """sum_{k>m} t^k / k! (t >= 0) as a 50-digit Decimal."""
    return _taylor_tail_dec(t, m)


def xi_b0(X, s: int) -> float:
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    c = taylor_exp(max(s - 1, 0))
    B0 = np.eye(n) * c[0]
    P = np.eye(n)
    with np.errstate(over="ignore", invalid="ignore"):
        for j in range(1, s):
            P = P @ X                       # X^j = X^(j-1) X
            B0 = B0 + c[j] * P
        return norm1(B0)


def accepts(A, sigma: int, m: int, s: int, u: float, alpha_A: float) -> bool:
    from decimal import Decimal
    t = math.ldexp(alpha_A, -sigma)
    if t > 800.0:
        return False
    xi = xi_b0(np.ldexp(np.asarray(A, dtype=np.float64), -sigma), s)
    if not math.isfinite(xi):
        return False
    return taylor_tail(t, m) <= Decimal(u) * Decimal(xi)


def _alpha_scaled(A, m: int, sigma0: int) -> float:
    """alpha_m(A) = 2^sigma0 alpha_m(X0), X0 = 2^-sigma0 A, powers of X0 by
    repeated multiplication"""
    X0 = np.ldexp(np.asarray(A, dtype=np.float64), -sigma0)
    d = 1
    while (d + 1) * d <= m + 1:
        d += 1
    Pd = np.linalg.matrix_power(X0, d)
    Pd1 = Pd @ X0
    a0 = max(norm1(Pd) ** (1.0 / d), norm1(Pd1) ** (1.0 / (d + 1)))
    return math.ldexp(a0, sigma0)


def least_sigma(A, m: int, s: int, u: float, alpha_A: float, sigma_max: int = 1100) -> int:
    """the least sigma >= 0 with accepts(A, sigma, ...)"""
    for sig in range(sigma_max + 1):
        if accepts(A, sig, m, s, u, alpha_A):
            return sig
    raise ValueError("no scaling up to %d meets the bound" % sigma_max)


def auto_sigma(A, m: int, s: int, u: float, norm_guard: bool = False) -> int:
    A = np.asarray(A, dtype=np.float64)
    th = theta_taylor(m, u)
    nA = norm1(A)
    s0 = _smallest_shift(nA, th)
    alpha = _alpha_scaled(A, m, s0)
    sig = least_sigma(A, m, s, u, alpha)
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
    nA = norm1(A)
    s0 = _smallest_shift(nA, theta_taylor(cands[-1], u))
    best = None
    for m in cands:
        s = _ceil_sqrt(m)
        sig = least_sigma(A, m, s, u, _alpha_scaled(A, m, s0))
        r = m // s
        cost = (s - 1) + r - (1 if m == s * r else 0) + sig
        if best is None or cost < best[0]:
            best = (cost, m, s, sig)
    return best[1], best[2], best[3]
