"""Precision choice of the mixed-precision PS scheme, written out from the paper.

TEST INFRASTRUCTURE ONLY (part of the oracle).  Independent of the library's
planner: nothing is shared.

Paper passages followed:
  * Theorem 2.1 and eq. (choose-ui) (section 2): with nu = 1 the product in
    Horner step i may use unit roundoff
        u_i = u * ||B_0|| / (||B_i|| * ||Y||^i),   Y = X^s.
    Algorithms 2 and 3 print a recursive variant with the i-th power of ||Y||
    as well, which unrolls to ||Y||^(i(i+1)/2); that is read as a misprint and
    the closed form above is used.
  * The framework requires u_r >= ... >= u_nu (section 2, summary of the
    framework).  The quantity ||B_i|| ||Y||^i stands for the size of
    everything that step i multiplies, so the oracle uses the running maximum
        u_i = u * ||B_0|| / max_{j >= i} (||B_j|| ||Y||^j),
    which equals the closed form whenever the decay condition (Bi-Xs-bnd)
    holds and is monotone by construction.
  * nu = min{ i : u_i >= delta * u } (delta = 10, section 3.2), else r + 1;
    steps 1..nu-1 run in the working precision (Algorithms 2 and 3).
  * IEEE low-precision variant (section 4.1.1): each u_i is replaced by the
    unit roundoff of the lowest available precision whose unit roundoff does
    not exceed u_i (inclusive).  The tier set here is IEEE double (2^-53),
    single (2^-24), bfloat16 (2^-8) and additionally OCP FP8 E4M3 (2^-4),
    which the paper does not have.
  * Zero norms: when the denominator is zero every later product is exactly
    zero, so any precision is exact and u_i = +inf; when ||B_0|| = 0 but the
    denominator is not, u_i = 0 and the working precision is kept.
Tier codes: 0 = FP64, 1 = FP32, 2 = BF16, 3 = FP8, 4 = double-double (the
working precision of the paper's multi-precision setting, never a lower tier).
"""
from __future__ import annotations

import math

U_TIER = {0: 2.0 ** -53, 1: 2.0 ** -24, 2: 2.0 ** -8, 3: 2.0 ** -4, 4: 2.0 ** -106}   # 4: double-double (working only)
DELTA = 10.0


def block_bounds(s: int, m: int):
    """r and the index ranges of B_0..B_r (eq. (ps))."""
    r = m // s
    ranges = []
    for i in range(r + 1):
        hi = s - 1 if i < r else m - s * r
        ranges.append([s * i + j for j in range(hi + 1)])
    return r, ranges


def choose_u(normB, normY, u_work):
    """u_0..u_r from the block norms ||B_0..B_r|| and ||Y|| (monotone closed form)."""
    r = len(normB) - 1
    u = [u_work] * (r + 1)
    running = 0.0
    for i in range(r, 0, -1):
        term = normB[i] * (normY ** i) if normY > 0 else 0.0
        running = max(running, term)
        if running == 0.0:
            u[i] = math.inf
        else:
            u[i] = u_work * normB[0] / running
    return u


def plan(normB, normY, working_tier=0, allowed=(0, 1, 2, 3), delta=DELTA):
    """Return (u list, nu, tier list) for blocks 0..r.

    tier[0] is always the working tier; tier[i], 1 <= i <= r, is the precision
    of the product P_i Y in Horner step i."""
    u_work = U_TIER[working_tier]
    u = choose_u(normB, normY, u_work)
    r = len(normB) - 1
    nu = r + 1
    for i in range(1, r + 1):
        if u[i] >= delta * u_work:
            nu = i
            break
    tiers = [working_tier] * (r + 1)
    usable = sorted([t for t in allowed if U_TIER[t] >= u_work] + [working_tier])
    for i in range(nu, r + 1):
        best = working_tier
        for t in usable:
            if U_TIER[t] <= u[i] and U_TIER[t] >= U_TIER[best]:
                best = t
        tiers[i] = best
    for i in range(1, nu):
        u[i] = u_work
    return u, nu, tiers


def apriori_norms(coef, s, normX):
    """Coefficient-magnitude estimates ||B_i|| ~ sum_j |c_{si+j}| ||X||^j and
    ||Y|| ~ ||X||^s (upper bounds by submultiplicativity)."""
    m = len(coef) - 1
    r, ranges = block_bounds(s, m)
    nb = []
    for i in range(r + 1):
        nb.append(sum(abs(coef[k]) * normX ** (k - s * i) for k in ranges[i]))
    return nb, normX ** s
