"""CPU oracle for matrix polynomials evaluated by the Paterson--Stockmeyer (PS)
scheme (Liu, arXiv 2312.17396).

TEST INFRASTRUCTURE ONLY.  This package is the independent reference that the
GPU library is checked against.  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import it.  It shares no code with the
HIP library (no common kernels, headers, helpers, constants or generators) and
imports nothing from it.

Parts:
  ps_oracle.c  double-double (dd, ~32 significant digits) evaluation of the
               plain definition p(X) = sum_k c_k X^k (section 1, eq. (ps)),
               scaling and squaring (eq. (scal-idea)), Algorithm 1 in dd and in
               IEEE double, explicit powers and Horner in double.
  coeffs.py    exact rational coefficients (Taylor exp, Pade [k/m] of exp,
               Taylor cos) rounded once to double.
  plan.py      the precision choice of section 2 (eq. (choose-ui)) and its
               IEEE-tier rounding (section 4.1.1), written independently of
               the library planner.
  metrics.py   the paper's error measure (section 3.3) and cost ratio (eq. (Cr)).
  solve.py     the quotient r_km = q_km^{-1} p_km of section 4.1 as the textbook
               LU solve with partial pivoting, and exp in the Pade form with
               scaling and squaring.

Parity status: every function here is pinned by tests/test_oracle_*.py against
closed forms, exact integer arithmetic, rational arithmetic, invariants and the
paper's printed numbers (Table 1, the Pade [13/13] blocks of section 2, the
2x2 nonnormal example of section 3.2).  The paper's Ward-matrix numbers of
section 2 do not reproduce under any norm tried, so nothing is pinned to them.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ps_oracle.c")
_LIB = os.path.join(_HERE, "libps_oracle.so")

_CFLAGS = ["-O2", "-mfma", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC", "-Wall"]


def build(force: bool = False) -> str:
    """Compile ps_oracle.c with gcc into libps_oracle.so (next to the source)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *_CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        i = ctypes.c_int
        d = ctypes.c_double
        sig = {
            "orc_two_sum": [d, d, dp],
            "orc_two_prod": [d, d, dp],
            "orc_dd_add": [d, d, d, d, dp],
            "orc_dd_mul": [d, d, d, d, dp],
            "orc_dd_mul_d": [d, d, d, dp],
            "orc_gemm_d_dd": [i, i, dp, dp, dp, dp, dp],
            "orc_gemm_dd": [i, dp, dp, dp, dp, dp, dp],
            "orc_poly_apply_dd": [i, dp, dp, i, i, dp, dp, dp, dp],
            "orc_expm_apply_dd": [i, dp, dp, i, i, i, dp, dp, dp, dp],
            "orc_ps_dd": [i, dp, dp, i, i, dp, dp],
            "orc_gemm_f64": [i, dp, dp, dp],
            "orc_ps_f64": [i, dp, dp, i, i, dp],
            "orc_horner_f64": [i, dp, dp, i, dp],
            "orc_naive_f64": [i, dp, dp, i, dp],
            "orc_expm_ps_f64": [i, dp, dp, i, i, i, dp],
            "orc_set_threads": [i],
            "orc_max_threads": [],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = i if name == "orc_max_threads" else None
        _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _colmajor(A) -> np.ndarray:
    """Copy a square matrix into a Fortran-ordered float64 array."""
    A = np.asarray(A, dtype=np.float64)
    assert A.ndim == 2 and A.shape[0] == A.shape[1]
    return np.asfortranarray(A)


def _coef(coef) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(coef, dtype=np.float64))


def set_threads(t: int) -> None:
    lib().orc_set_threads(int(t))


def max_threads() -> int:
    return int(lib().orc_max_threads())


# --------------------------------------------------------------------------
# scalar dd operations (exposed for the pins against exact rationals)
# --------------------------------------------------------------------------
def _pair(fn, *args):
    out = np.zeros(2)
    fn(*[float(a) for a in args], _p(out))
    return float(out[0]), float(out[1])


def two_sum(a, b):
    return _pair(lib().orc_two_sum, a, b)


def two_prod(a, b):
    return _pair(lib().orc_two_prod, a, b)


def dd_add(a, b):
    return _pair(lib().orc_dd_add, a[0], a[1], b[0], b[1])


def dd_mul(a, b):
    return _pair(lib().orc_dd_mul, a[0], a[1], b[0], b[1])


def dd_mul_d(a, b):
    return _pair(lib().orc_dd_mul_d, a[0], a[1], b)


# --------------------------------------------------------------------------
# matrix routines.  dd results are returned as (hi, lo) numpy arrays in the
# same (square, 2-D) shape as the input.
# --------------------------------------------------------------------------
def gemm_dd(Ah, Al, Bh, Bl):
    Ah, Al, Bh, Bl = map(_colmajor, (Ah, Al, Bh, Bl))
    n = Ah.shape[0]
    Ch = np.zeros((n, n), order="F")
    Cl = np.zeros((n, n), order="F")
    lib().orc_gemm_dd(n, _p(Ah), _p(Al), _p(Bh), _p(Bl), _p(Ch), _p(Cl))
    return Ch, Cl


def poly_dd(X, coef):
    """R1: p(X) = sum_k c_k X^k in dd by the plain definition (section 1)."""
    X = _colmajor(X)
    c = _coef(coef)
    n = X.shape[0]
    Ph = np.zeros((n, n), order="F")
    Pl = np.zeros((n, n), order="F")
    lib().orc_poly_apply_dd(n, _p(X), _p(c), len(c) - 1, n, None, None, _p(Ph), _p(Pl))
    return Ph, Pl


def poly_apply_dd(X, coef, V, Vl=None):
    """p(X) V for an n x k block V (double, or dd when Vl is given)."""
    X = _colmajor(X)
    c = _coef(coef)
    n = X.shape[0]
    V = np.asfortranarray(np.asarray(V, dtype=np.float64).reshape(n, -1))
    k = V.shape[1]
    Vl = None if Vl is None else np.asfortranarray(np.asarray(Vl, dtype=np.float64).reshape(n, k))
    Wh = np.zeros((n, k), order="F")
    Wl = np.zeros((n, k), order="F")
    lib().orc_poly_apply_dd(n, _p(X), _p(c), len(c) - 1, k, _p(V), _p(Vl), _p(Wh), _p(Wl))
    return Wh, Wl


def expm_dd(A, coef, sigma):
    """R3: r(A) = p(2^-sigma A)^(2^sigma) in dd (eq. (scal-idea)); full matrix."""
    A = _colmajor(A)
    c = _coef(coef)
    n = A.shape[0]
    Eh = np.zeros((n, n), order="F")
    El = np.zeros((n, n), order="F")
    lib().orc_expm_apply_dd(n, _p(A), _p(c), len(c) - 1, int(sigma), n, None, None, _p(Eh), _p(El))
    return Eh, El


def expm_apply_dd(A, coef, sigma, V):
    """r(A) V for an n x k block V, by 2^sigma applications of p(2^-sigma A)."""
    A = _colmajor(A)
    c = _coef(coef)
    n = A.shape[0]
    V = np.asfortranarray(np.asarray(V, dtype=np.float64).reshape(n, -1))
    k = V.shape[1]
    Wh = np.zeros((n, k), order="F")
    Wl = np.zeros((n, k), order="F")
    lib().orc_expm_apply_dd(n, _p(A), _p(c), len(c) - 1, int(sigma), k, _p(V), None, _p(Wh), _p(Wl))
    return Wh, Wl


def expm_grad_dd(A, G, coef, sigma, cols=None):
    """R4: gradient of <G, r(A)> with respect to A, r(A) = p(2^-sigma A)^(2^sigma).

    r is a polynomial with real coefficients, so the gradient is the Frechet
    derivative L_r(A^T, G), which is the upper-right n x n block of
    r([[A^T, G], [0, A^T]]) (block upper-triangular argument).  Only the
    requested columns are formed: column j of the gradient is the top half of
    r(Z) e_{n+j}, obtained by 2^sigma applications of p(2^-sigma Z) to e_{n+j}.
    Returns (hi, lo) of shape (n, len(cols))."""
    A = np.asarray(A, dtype=np.float64)
    G = np.asarray(G, dtype=np.float64)
    n = A.shape[0]
    cols = list(range(n)) if cols is None else list(cols)
    Z = np.zeros((2 * n, 2 * n))
    Z[:n, :n] = A.T
    Z[n:, n:] = A.T
    Z[:n, n:] = G
    V = np.zeros((2 * n, len(cols)))
    for t, j in enumerate(cols):
        V[n + j, t] = 1.0
    Wh, Wl = expm_apply_dd(Z, coef, sigma, V)
    return Wh[:n], Wl[:n]


def ps_dd(X, coef, s):
    """Algorithm 1 (PS) carried out in dd."""
    X = _colmajor(X)
    c = _coef(coef)
    n = X.shape[0]
    Ph = np.zeros((n, n), order="F")
    Pl = np.zeros((n, n), order="F")
    lib().orc_ps_dd(n, _p(X), _p(c), len(c) - 1, int(s), _p(Ph), _p(Pl))
    return Ph, Pl


def gemm_f64(A, B):
    A, B = _colmajor(A), _colmajor(B)
    n = A.shape[0]
    C = np.zeros((n, n), order="F")
    lib().orc_gemm_f64(n, _p(A), _p(B), _p(C))
    return C


def ps_f64(X, coef, s):
    """Algorithm 1 (fixed-precision PS) in IEEE double."""
    X = _colmajor(X)
    c = _coef(coef)
    n = X.shape[0]
    P = np.zeros((n, n), order="F")
    lib().orc_ps_f64(n, _p(X), _p(c), len(c) - 1, int(s), _p(P))
    return P


def horner_f64(X, coef):
    X = _colmajor(X)
    c = _coef(coef)
    n = X.shape[0]
    P = np.zeros((n, n), order="F")
    lib().orc_horner_f64(n, _p(X), _p(c), len(c) - 1, _p(P))
    return P


def naive_f64(X, coef):
    X = _colmajor(X)
    c = _coef(coef)
    n = X.shape[0]
    P = np.zeros((n, n), order="F")
    lib().orc_naive_f64(n, _p(X), _p(c), len(c) - 1, _p(P))
    return P


def expm_ps_f64(A, coef, s, sigma):
    """Scaling and squaring around Algorithm 1, all in IEEE double."""
    A = _colmajor(A)
    c = _coef(coef)
    n = A.shape[0]
    E = np.zeros((n, n), order="F")
    lib().orc_expm_ps_f64(n, _p(A), _p(c), len(c) - 1, int(s), int(sigma), _p(E))
    return E


from . import coeffs, plan, metrics, solve  # noqa: E402,F401
