"""Linear solve with a matrix polynomial, and the Pade form of exp.

TEST INFRASTRUCTURE ONLY (part of the oracle; see the package docstring).

Section 4.1 defines the [k/m] Pade approximant as r_km(X) = q_km(X)^{-1}
p_km(X): the PS scheme evaluates p_km and q_km, and the surrounding
scaling-and-squaring algorithm takes the quotient and squares it.  The
quotient is written out here as the textbook solve:

  lu_pp     Gaussian elimination with partial pivoting, PQ = LU.  At step k
            the pivot is the row of largest |entry| in column k at or below
            row k (the first such row on ties), the two rows are exchanged
            over the full width, the multipliers L[i,k] = A[i,k] / A[k,k]
            are stored below the diagonal, and the rank-one update is taken
            on the trailing block.  A zero pivot (the whole column below is
            then zero) is recorded in `info` (1-based, the first one) and the
            step is skipped.
  lu_solve  X = Q^{-1} B: the recorded row exchanges applied to B in order,
            forward substitution with the unit lower factor, back
            substitution with the upper factor.
  expm_pade E = r_m(2^-sigma A)^(2^sigma), r_m = q_m^{-1} p_m with p_m and
            q_m each evaluated by Algorithm 1 in IEEE double, one shared
            block size s (the library's default, ceil(sqrt m), when s = 0).

All arithmetic in IEEE double; numpy row operations stand for the loops of
the elimination, in the textbook order.
"""
from __future__ import annotations

import math

import numpy as np


def lu_pp(Q):
    """Returns (LU, piv, info): LU holds L below the diagonal (unit diagonal
    implied) and U on and above it; piv[k] is the row exchanged with row k
    at step k (0-based); info = 0, or k + 1 for the first zero pivot U[k,k]."""
    A = np.array(Q, dtype=np.float64, copy=True)
    n = A.shape[0]
    if A.shape != (n, n):
        raise ValueError("square matrix expected")
    piv = np.arange(n)
    info = 0
    for k in range(n):
        p = k + int(np.argmax(np.abs(A[k:, k])))
        piv[k] = p
        if p != k:
            A[[k, p], :] = A[[p, k], :]
        d = A[k, k]
        if d == 0.0:
            if info == 0:
                info = k + 1
            continue
        A[k + 1:, k] = A[k + 1:, k] / d
        A[k + 1:, k + 1:] -= np.outer(A[k + 1:, k], A[k, k + 1:])
    return A, piv, info


def lu_solve(LU, piv, B):
    """X with Q X = B from the factors of lu_pp(Q)."""
    X = np.array(B, dtype=np.float64, copy=True)
    n = LU.shape[0]
    if X.ndim != 2 or X.shape[0] != n:
        raise ValueError("B must have n rows")
    for k in range(n):
        p = int(piv[k])
        if p != k:
            X[[k, p], :] = X[[p, k], :]
    for k in range(n):
        X[k + 1:, :] -= np.outer(LU[k + 1:, k], X[k, :])
    for k in range(n - 1, -1, -1):
        X[k, :] = X[k, :] / LU[k, k]
        X[:k, :] -= np.outer(LU[:k, k], X[k, :])
    return X


def solve(Q, B):
    LU, piv, info = lu_pp(Q)
    return lu_solve(LU, piv, B), info


def expm_pade(A, m, sigma, s=0):
    """r_m(2^-sigma A)^(2^sigma) for the diagonal [m/m] Pade approximant."""
    from . import coeffs, ps_f64, gemm_f64
    A = np.asarray(A, dtype=np.float64)
    X = A * (2.0 ** -int(sigma))
    pc, qc = coeffs.pade_exp(m, m)
    if s <= 0:
        s = max(1, math.isqrt(m - 1) + 1) if m > 1 else 1
    P = ps_f64(X, pc, s)
    Qm = ps_f64(X, qc, s)
    R, _ = solve(Qm, P)
    for _ in range(int(sigma)):
        R = gemm_f64(R, R)
    return np.asarray(R)
