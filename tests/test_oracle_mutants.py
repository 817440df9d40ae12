"""The oracle's pins have teeth: plausible slips are planted in copies of the
oracle (a dropped term, a wrong sign, an index off by one, a transposed
operand, a wrong block boundary, a missing squaring, a wrong tier rule), and
every such copy must fail at least one pin of tests/test_oracle_pins.py,
tests/test_oracle_arith.py or tests/test_oracle_solve.py.

Each mutant is a copy of the whole oracle package in a temporary directory
with one textual change (its C part is recompiled there); the pin files run
against it in a child pytest process whose import path puts the copy first.
The oracle itself is never modified.  A control copy without a change must
pass every pin, so a failure of a mutant is the mutation's doing."""
import concurrent.futures
import os
import shutil
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PIN_FILES = ["test_oracle_pins.py", "test_oracle_arith.py", "test_oracle_solve.py"]

# (label, file in oracle/, exact text, replacement); each text occurs once.
# Mutations that cannot change any result are not listed: e.g. counting the
# folded last Horner step in the degree selector's cost shifts every
# candidate's cost by one, since s divides m for all of q^2 and q(q+1).
MUTANTS = [
    # double-double arithmetic
    ("two_sum drops the error of b", "ps_oracle.c",
     "double e = (a - (s - bb)) + (b - bb);", "double e = (a - (s - bb));"),
    ("fast_two_sum error with the wrong sign", "ps_oracle.c",
     "double e = b - (s - a);", "double e = (s - a) - b;"),
    ("two_prod residual with the wrong sign", "ps_oracle.c",
     "double e = fma(a, b, -p);", "double e = -fma(a, b, -p);"),
    ("dd_add drops the low-part error", "ps_oracle.c",
     "double w = t.lo + v.lo;", "double w = v.lo;"),
    ("dd_mul drops a cross term", "ps_oracle.c",
     "double cl = fma(a.lo, b.hi, t);", "double cl = t;"),
    ("dd_mul_d drops the low part", "ps_oracle.c",
     "double cl = fma(a.lo, b, c.lo);", "double cl = c.lo;"),
    # products
    ("double x dd product with X transposed", "ps_oracle.c",
     "for (int i = 0; i < n; ++i) acc[i] = dd_add(acc[i], dd_mul_d(b, xc[i]));",
     "for (int i = 0; i < n; ++i) acc[i] = dd_add(acc[i], dd_mul_d(b, X[l + (size_t)i * n]));"),
    ("dd product with A transposed", "ps_oracle.c",
     "dd a = { Ah[i + (size_t)l * n], Al[i + (size_t)l * n] };",
     "dd a = { Ah[l + (size_t)i * n], Al[l + (size_t)i * n] };"),
    ("double product with A transposed", "ps_oracle.c",
     "for (int i = 0; i < n; ++i) c[i] += a[i] * b;",
     "for (int i = 0; i < n; ++i) c[i] += A[l + (size_t)i * n] * b;"),
    # the plain definition and scaling and squaring
    ("plain definition drops its last term", "ps_oracle.c",
     "for (int p = 1; p <= m; ++p) {", "for (int p = 1; p < m; ++p) {"),
    ("plain definition with coefficient indices shifted", "ps_oracle.c",
     "s = dd_add(s, dd_mul_d(t, coef[p]));", "s = dd_add(s, dd_mul_d(t, coef[p - 1]));"),
    ("scaling by 2^sigma instead of 2^-sigma", "ps_oracle.c",
     "X[e] = ldexp(A[e], -sigma);   /* exact scaling by 2^-sigma */",
     "X[e] = ldexp(A[e], sigma);   /* exact scaling by 2^-sigma */"),
    ("one squaring missing (full matrix)", "ps_oracle.c",
     "for (int t = 0; t < sigma; ++t) {\n                orc_gemm_dd",
     "for (int t = 1; t < sigma; ++t) {\n                orc_gemm_dd"),
    ("one application too many (column block)", "ps_oracle.c",
     "long reps = 1L << sigma;", "long reps = (1L << sigma) + (sigma > 0);"),
    # Paterson--Stockmeyer (Algorithm 1)
    ("PS in dd: last block one coefficient short", "ps_oracle.c",
     "for (int j = 0; j <= m - s * r; ++j) {\n            dd x",
     "for (int j = 0; j < m - s * r; ++j) {\n            dd x"),
    ("PS in dd: block coefficients shifted", "ps_oracle.c",
     "acc = dd_add(acc, dd_mul_d(x, coef[s * i + j]));",
     "acc = dd_add(acc, dd_mul_d(x, coef[s * i + j + (j == s - 1)]));"),
    ("PS in dd: Horner in X^(s-1)", "ps_oracle.c",
     "orc_gemm_dd(n, Xh + (size_t)s * nn, Xl + (size_t)s * nn, Ph, Pl, Qh, Ql);",
     "orc_gemm_dd(n, Xh + (size_t)(s - 1) * nn, Xl + (size_t)(s - 1) * nn, Ph, Pl, Qh, Ql);"),
    ("PS in double: block subtracted", "ps_oracle.c",
     "P[e] = acc + Q[e];", "P[e] = acc - Q[e];"),
    ("PS in double: last block one coefficient short", "ps_oracle.c",
     "for (int j = 0; j <= m - s * r; ++j) acc += coef[s * r + j] * Xp[j * nn + e];",
     "for (int j = 0; j < m - s * r; ++j) acc += coef[s * r + j] * Xp[j * nn + e];"),
    ("Horner in double: identity terms shifted", "ps_oracle.c",
     "P[e] = Q[e] + (((e % n) == (e / n)) ? coef[k] : 0.0);",
     "P[e] = Q[e] + (((e % n) == (e / n)) ? coef[k + 1] : 0.0);"),
    ("explicit powers drop the last term", "ps_oracle.c",
     "for (int k = 1; k <= m; ++k) {\n        orc_gemm_f64(n, T, X, U);",
     "for (int k = 1; k < m; ++k) {\n        orc_gemm_f64(n, T, X, U);"),
    ("double scaling and squaring: one squaring missing", "ps_oracle.c",
     "for (int t = 0; t < sigma; ++t) {\n        orc_gemm_f64(n, E, E, Q);",
     "for (int t = 1; t < sigma; ++t) {\n        orc_gemm_f64(n, E, E, Q);"),
    # coefficients
    ("Taylor exp: 1/(i+1)! instead of 1/i!", "coeffs.py",
     "return [Fraction(1, factorial(i)) for i in range(m + 1)]",
     "return [Fraction(1, factorial(i + 1)) for i in range(m + 1)]"),
    ("Pade denominator without the alternating sign", "coeffs.py",
     "q = [Fraction((-1) ** j * factorial(k + m - j)", "q = [Fraction(factorial(k + m - j)"),
    ("Pade numerator with m and k swapped", "coeffs.py",
     "factorial(k), den * factorial(j) * factorial(k - j)) for j in range(k + 1)]",
     "factorial(m), den * factorial(j) * factorial(m - j)) for j in range(k + 1)]"),
    ("Taylor cos: (2k+1)! instead of (2k)!", "coeffs.py",
     "return [Fraction((-1) ** k, factorial(2 * k)) for k in range(m + 1)]",
     "return [Fraction((-1) ** k, factorial(2 * k + 1)) for k in range(m + 1)]"),
    # planner (eq. (choose-ui), section 4.1.1)
    ("planner: ||Y||^(i+1) instead of ||Y||^i", "plan.py",
     "term = normB[i] * (normY ** i) if normY > 0 else 0.0",
     "term = normB[i] * (normY ** (i + 1)) if normY > 0 else 0.0"),
    ("planner: no running maximum", "plan.py",
     "running = max(running, term)", "running = term"),
    ("planner: numerator without ||B_0||", "plan.py",
     "u[i] = u_work * normB[0] / running", "u[i] = u_work / running"),
    ("planner: strict tier comparison", "plan.py",
     "if U_TIER[t] <= u[i] and U_TIER[t] >= U_TIER[best]:",
     "if U_TIER[t] < u[i] and U_TIER[t] >= U_TIER[best]:"),
    ("planner: nu ignores delta", "plan.py",
     "if u[i] >= delta * u_work:", "if u[i] >= u_work:"),
    ("block boundaries: blocks of s + 1 terms", "plan.py",
     "hi = s - 1 if i < r else m - s * r", "hi = s if i < r else m - s * r"),
    ("a-priori norms: ||X||^k instead of ||X||^(k - si)", "plan.py",
     "nb.append(sum(abs(coef[k]) * normX ** (k - s * i) for k in ranges[i]))",
     "nb.append(sum(abs(coef[k]) * normX ** k for k in ranges[i]))"),
    # metrics and the automatic choices (section 3)
    ("1-norm over rows instead of columns", "metrics.py",
     "np.abs(np.asarray(A, dtype=np.float64)), axis=0)", "np.abs(np.asarray(A, dtype=np.float64)), axis=1)"),
    ("cost ratio (eq. (Cr)) with s products for the powers", "metrics.py",
     "return 1.0 - ((s - 1) * D + float(sum(d))) / ((s + r - 1) * D)",
     "return 1.0 - (s * D + float(sum(d))) / ((s + r - 1) * D)"),
    ("theta_m: Taylor tail from degree m instead of m + 1", "metrics.py",
     "for k in range(1, m + 2):\n            term = term * t / k",
     "for k in range(1, m + 1):\n            term = term * t / k"),
    ("alpha_m: the second power's root taken as a d-th root", "metrics.py",
     "return max(norm1(Pd) ** (1.0 / d), norm1(Pd1) ** (1.0 / (d + 1)))",
     "return max(norm1(Pd) ** (1.0 / d), norm1(Pd1) ** (1.0 / d))"),
    ("alpha_m: d* one too small", "metrics.py",
     "d = int(math.floor((1 + math.sqrt(4 * m + 5)) / 2))", "d = int(math.floor((1 + math.sqrt(4 * m + 5)) / 2)) - 1"),
    ("automatic sigma: the 1-norm choice kept", "metrics.py",
     "sig = least_sigma(A, m, s, u, alpha)", "sig = s0"),
    ("alpha_m acceptance with xi(X) = 1 (an absolute tolerance)", "metrics.py",
     "return taylor_tail(t, m) <= Decimal(u) * Decimal(xi)", "return taylor_tail(t, m) <= Decimal(u)"),
    ("xi: B_0 with the power X^s as well", "metrics.py",
     "for j in range(1, s):\n            P = P @ X", "for j in range(1, s + 1):\n            P = P @ X"),
    ("xi: B_0 of the unscaled matrix", "metrics.py",
     "xi = xi_b0(np.ldexp(np.asarray(A, dtype=np.float64), -sigma), s)",
     "xi = xi_b0(np.asarray(A, dtype=np.float64), s)"),
    ("alpha_m(A) not rescaled by 2^sigma0", "metrics.py",
     "return math.ldexp(a0, sigma0)", "return a0"),
    ("shift search: a < 2^k b instead of a <= 2^k b", "metrics.py",
     "while a > math.ldexp(b, k):", "while a >= math.ldexp(b, k):"),
    ("variable s: growth test against ||X||^(s+1)", "metrics.py",
     "while norm1(Y) > norm1(B0) * nX ** s and s < m:", "while norm1(Y) > norm1(B0) * nX ** (s + 1) and s < m:"),
    ("variable s: B_0 grows by c_(s-1) Y", "metrics.py",
     "B0 = B0 + c[s] * Y", "B0 = B0 + c[s - 1] * Y"),
    ("degree selection: ties go to the larger degree", "metrics.py",
     "if best is None or cost < best[0]:", "if best is None or cost <= best[0]:"),
    ("degree selection: q(q+1) candidates left out", "metrics.py",
     "cands.append(q * (q + 1))", "pass"),
    # the adjoint (block upper-triangular argument)
    # linear solve and the Pade form
    ("LU pivot by signed value instead of magnitude", "solve.py",
     "p = k + int(np.argmax(np.abs(A[k:, k])))", "p = k + int(np.argmax(A[k:, k]))"),
    ("LU exchanges only the trailing columns", "solve.py",
     "A[[k, p], :] = A[[p, k], :]", "A[[k, p], k:] = A[[p, k], k:]"),
    ("LU multipliers not divided by the pivot", "solve.py",
     "A[k + 1:, k] = A[k + 1:, k] / d", "A[k + 1:, k] = A[k + 1:, k]"),
    ("LU update with the wrong sign", "solve.py",
     "A[k + 1:, k + 1:] -= np.outer(A[k + 1:, k], A[k, k + 1:])",
     "A[k + 1:, k + 1:] += np.outer(A[k + 1:, k], A[k, k + 1:])"),
    ("LU zero pivot recorded 0-based", "solve.py", "info = k + 1", "info = k"),
    ("solve skips the row exchanges", "solve.py", "            X[[k, p], :] = X[[p, k], :]", "            pass"),
    ("back substitution without the division", "solve.py",
     "X[k, :] = X[k, :] / LU[k, k]", "X[k, :] = X[k, :]"),
    ("forward substitution with the transposed factor", "solve.py",
     "X[k + 1:, :] -= np.outer(LU[k + 1:, k], X[k, :])", "X[k + 1:, :] -= np.outer(LU[k, k + 1:], X[k, :])"),
    ("Pade exp as p q^-1 with q and p swapped", "solve.py", "R, _ = solve(Qm, P)", "R, _ = solve(P, Qm)"),
    ("Pade exp: one squaring missing", "solve.py", "for _ in range(int(sigma)):", "for _ in range(int(sigma) - 1):"),
    ("gradient oracle without the transposes", "__init__.py",
     "Z[:n, :n] = A.T\n    Z[n:, n:] = A.T", "Z[:n, :n] = A\n    Z[n:, n:] = A"),
    ("gradient oracle with G transposed", "__init__.py",
     "Z[:n, n:] = G", "Z[:n, n:] = G.T"),
]


def _make_copy(base, label, fname, old, new):
    """A copy of the oracle package (and of the pin files) under base/label."""
    d = os.path.join(base, label)
    shutil.copytree(os.path.join(ROOT, "oracle"), os.path.join(d, "oracle"),
                    ignore=shutil.ignore_patterns("__pycache__", "*.so", "*.tmp*"))
    os.makedirs(os.path.join(d, "tests"))
    for f in PIN_FILES + ["conftest.py"]:
        shutil.copy(os.path.join(ROOT, "tests", f), os.path.join(d, "tests", f))
    shutil.copytree(os.path.join(ROOT, "tests", "golden"), os.path.join(d, "tests", "golden"))
    if fname is not None:
        p = os.path.join(d, "oracle", fname)
        src = open(p).read()
        assert src.count(old) == 1, (label, src.count(old))
        open(p, "w").write(src.replace(old, new))
    if fname != "ps_oracle.c":
        # the C part is unchanged: reuse the oracle's build
        import oracle
        shutil.copy(oracle.build(), os.path.join(d, "oracle", "libps_oracle.so"))
    return d


def _run_pins(d):
    env = dict(os.environ, OMP_NUM_THREADS="2", PYTHONPATH=ROOT, PYTHONDONTWRITEBYTECODE="1")
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu"]
    cmd += [os.path.join("tests", f) for f in PIN_FILES]
    r = subprocess.run(cmd, cwd=d, env=env, capture_output=True, text=True, timeout=600)
    return r.returncode, r.stdout[-2000:] + r.stderr[-2000:]


def test_every_planted_mistake_fails_a_pin():
    with tempfile.TemporaryDirectory(prefix="oracle_mutants_") as base:
        jobs = [("control", None, None, None)] + [("m%02d" % k, f, o, n) for k, (_, f, o, n) in enumerate(MUTANTS)]
        dirs = {lab: _make_copy(base, lab, f, o, n) for lab, f, o, n in jobs}
        with concurrent.futures.ThreadPoolExecutor(max_workers=4) as ex:
            res = dict(zip(dirs, ex.map(_run_pins, dirs.values())))
    rc, out = res.pop("control")
    assert rc == 0, "the unmodified copy must pass every pin:\n" + out
    survivors = [MUTANTS[int(lab[1:])][0] for lab, (rc, out) in res.items() if rc != 1]
    assert not survivors, "planted mistakes that no pin catches: %s" % survivors
