"""Pins of the oracle against what the paper and the mathematics fix.

Each check is chosen so that a plausible slip in the oracle (a dropped term, a
wrong sign or index, a transposed operand, a wrong block boundary in the PS
split, a missing squaring) fails at least one of them."""
import math
import os
from fractions import Fraction as F

import numpy as np
import pytest

import oracle
from oracle import coeffs, metrics
from oracle import plan as oplan

GOLD = os.path.join(os.path.dirname(__file__), "golden")
U = 2.0 ** -53


# ---------------------------------------------------------------- helpers
def fmat(A):
    return [[F(float(x)) for x in row] for row in np.asarray(A)]


def fmul(A, B):
    n, k, p = len(A), len(B), len(B[0])
    return [[sum(A[i][l] * B[l][j] for l in range(k)) for j in range(p)] for i in range(n)]


def fpoly(X, c):
    """sum_k c_k X^k with exact rationals (brute force)."""
    n = len(X)
    T = [[F(int(i == j)) for j in range(n)] for i in range(n)]
    S = [[F(c[0]) * T[i][j] for j in range(n)] for i in range(n)]
    for k in range(1, len(c)):
        T = fmul(T, X)
        S = [[S[i][j] + F(c[k]) * T[i][j] for j in range(n)] for i in range(n)]
    return S


def as_float(Fm):
    return np.array([[float(x) for x in row] for row in Fm])


def dd_close(hi, lo, exact, rtol):
    n = len(exact)
    scale = max(max(abs(x) for x in row) for row in exact) or F(1)
    for i in range(n):
        for j in range(len(exact[0])):
            err = abs(F(float(hi[i, j])) + F(float(lo[i, j])) - exact[i][j])
            assert err <= F(rtol) * scale, (i, j, float(err), float(scale))


def rand_normed(rng, n, t=1.0):
    G = rng.standard_normal((n, n))
    return G * (t / metrics.norm1(G))


# ------------------------------------------------- P1: exactness on integers
@pytest.mark.parametrize("seed", range(6))
def test_integer_inputs_all_routes_bitwise(seed):
    """Integer X in {-2..2}, integer c_k, n <= 4, m <= 8: every intermediate is an
    integer below 2^53, so Algorithm 1 (any s), Horner, explicit powers and the
    dd routes must all equal the exact integer polynomial bitwise."""
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(1, 5))
    m = int(rng.integers(0, 9))
    X = rng.integers(-2, 3, (n, n)).astype(np.float64)
    c = rng.integers(-5, 6, m + 1).astype(np.float64)
    exact = as_float(fpoly(fmat(X), c))
    assert np.all(np.abs(exact) < 2 ** 53)
    for s in range(1, max(m, 1) + 1):
        assert np.array_equal(oracle.ps_f64(X, c, s), exact), ("ps_f64", s)
        h, l = oracle.ps_dd(X, c, s)
        assert np.array_equal(h, exact) and not np.any(l), ("ps_dd", s)
    assert np.array_equal(oracle.horner_f64(X, c), exact)
    assert np.array_equal(oracle.naive_f64(X, c), exact)
    h, l = oracle.poly_dd(X, c)
    assert np.array_equal(h, exact) and not np.any(l)


# ---------------------------------------------- P2: diagonal closed form
def test_diagonal_closed_form():
    rng = np.random.default_rng(7)
    d = rng.uniform(-3, 3, 5)
    c = coeffs.taylor_exp(20)
    h, l = oracle.poly_dd(np.diag(d), c)
    exact = [[F(0)] * 5 for _ in range(5)]
    for i in range(5):
        exact[i][i] = sum(F(ck) * F(float(d[i])) ** k for k, ck in enumerate(c))
    dd_close(h, l, exact, 1e-30)
    # scaling and squaring on a diagonal: diag(p(d_i / 2^sigma)^(2^sigma))
    sigma = 3
    h, l = oracle.expm_dd(np.diag(d), c, sigma)
    for i in range(5):
        x = F(float(d[i])) / 2 ** sigma
        exact[i][i] = sum(F(ck) * x ** k for k, ck in enumerate(c)) ** (2 ** sigma)
    dd_close(h, l, exact, 1e-29)


# ---------------------------------------------- P3: triangular invariant
def test_upper_triangular_stays_triangular():
    rng = np.random.default_rng(8)
    n = 24
    T = np.triu(rng.standard_normal((n, n))) / 4
    c = coeffs.taylor_exp(16)
    for P in (oracle.ps_f64(T, c, 4), oracle.poly_dd(T, c)[0], oracle.ps_dd(T, c, 4)[0],
              oracle.expm_dd(T, c, 2)[0]):
        assert not np.any(np.tril(P, -1))
    h, l = oracle.poly_dd(T, c)
    for i in range(n):
        ex = sum(F(ck) * F(float(T[i, i])) ** k for k, ck in enumerate(c))
        assert abs(F(float(h[i, i])) + F(float(l[i, i])) - ex) <= F(1e-30) * abs(ex)


# ---------------------------------------------- P4: nilpotent / Jordan
@pytest.mark.parametrize("n", [1, 2, 5, 9])
def test_jordan_block_taylor_is_exact_exponential(n):
    """For J = J_n(0), J^n = 0, so the Taylor polynomial of degree m >= n-1 is
    e^J with its coefficients: the Toeplitz matrix with c_j = fl(1/j!) on
    superdiagonal j.  Every entry is a single product c_j * 1, so the result is
    exact (lo part zero)."""
    J = np.diag(np.ones(n - 1), 1) if n > 1 else np.zeros((1, 1))
    c = coeffs.taylor_exp(max(n - 1, 0) + 3)
    h, l = oracle.poly_dd(J, c)
    exact = [[F(c[j - i]) if j >= i else F(0) for j in range(n)] for i in range(n)]
    dd_close(h, l, exact, 0.0)
    assert not np.any(l)
    # and c_j is the double nearest to 1/j!
    for j in range(n):
        assert abs(F(c[j]) - F(1, math.factorial(j))) <= F(1, math.factorial(j)) * F(2.0 ** -53)
    # PS with s = n: Y = J^n = 0 so p = B_0 (section 2, the nilpotent remark)
    if n > 1:
        h2, l2 = oracle.ps_dd(J, c, n)
        dd_close(h2, l2, exact, 0.0)


def test_strictly_upper_random_nilpotent():
    rng = np.random.default_rng(9)
    n = 5
    N = np.triu(rng.integers(-3, 4, (n, n)), 1).astype(float)
    c = coeffs.taylor_exp(8)
    h, l = oracle.poly_dd(N, c)
    exact = fpoly(fmat(N), c[:n])          # N^n = 0: terms beyond n-1 vanish
    dd_close(h, l, exact, 1e-30)


# ---------------------------------------------- P5: rotation generator
@pytest.mark.parametrize("theta", [0.3, 1.0, 2.5])
def test_rotation_generator_gives_truncated_cos_sin(theta):
    m = 18
    X = np.array([[0.0, -theta], [theta, 0.0]])
    c = coeffs.taylor_exp(m)
    h, l = oracle.poly_dd(X, c)
    t = F(theta)
    # truncated scalar cos / sin series with the same (double) coefficients
    C = sum((-1) ** (k // 2) * F(c[k]) * t ** k for k in range(0, m + 1, 2))
    S = sum((-1) ** ((k - 1) // 2) * F(c[k]) * t ** k for k in range(1, m + 1, 2))
    dd_close(h, l, [[C, -S], [S, C]], 1e-31)
    # with a long series the matrix tends to the rotation by theta
    h, _ = oracle.poly_dd(X, coeffs.taylor_exp(40))
    assert abs(h[0, 0] - math.cos(theta)) < 4e-16 and abs(h[1, 0] - math.sin(theta)) < 4e-16


def test_cos_in_square_argument():
    """X = theta [[0,1],[1,0]] has X^2 = theta^2 I, so c_m(X^2) = c_m(theta^2) I."""
    theta = 1.3
    X = theta * np.array([[0.0, 1.0], [1.0, 0.0]])
    Z = oracle.gemm_f64(X, X)
    c = coeffs.taylor_cos(12)
    h, l = oracle.poly_dd(Z, c)
    z = F(float(Z[0, 0]))
    val = sum(F(ck) * z ** k for k, ck in enumerate(c))
    dd_close(h, l, [[val, F(0)], [F(0), val]], 1e-31)
    assert abs(float(val) - math.cos(theta)) < 1e-15


# ---------------------------------------------- P6: group / commutation
def test_exp_times_exp_minus_is_identity():
    rng = np.random.default_rng(10)
    n = 16
    A = rand_normed(rng, n, 4.0)
    # truncation is far below u at ||X|| = 1; what remains is the rounding of the
    # coefficients c_k = fl(1/k!) themselves (relative u each), so the product
    # is I to a few u, while a dropped or wrong term would leave O(1/k!).
    c = coeffs.taylor_exp(40)
    Eh, El = oracle.expm_dd(A, c, 2)
    Fh, Fl = oracle.expm_dd(-A, c, 2)
    Ph, Pl = oracle.gemm_dd(Eh, El, Fh, Fl)
    R = (Ph - np.eye(n)) + Pl
    assert metrics.norm1(R) < 16 * U


def test_polynomial_commutes_with_argument():
    rng = np.random.default_rng(11)
    n = 20
    A = rand_normed(rng, n, 2.0)
    h, l = oracle.poly_dd(A, coeffs.taylor_exp(25))
    Z = np.zeros((n, n))
    AP = oracle.gemm_dd(A, Z, h, l)
    PA = oracle.gemm_dd(h, l, A, Z)
    D = (AP[0] - PA[0]) + (AP[1] - PA[1])
    assert metrics.norm1(D) < 1e-29 * metrics.norm1(A) * metrics.norm1(h)


# ---------------------------------------------- P14: route consistency
@pytest.mark.parametrize("n,m,s", [(33, 30, 6), (64, 16, 4), (70, 13, 4), (40, 18, 5), (17, 7, 3)])
def test_ps_dd_matches_plain_definition(n, m, s):
    rng = np.random.default_rng(12 + n)
    X = rand_normed(rng, n, 1.0)
    c = coeffs.taylor_exp(m)
    ph, pl = oracle.poly_dd(X, c)
    qh, ql = oracle.ps_dd(X, c, s)
    assert metrics.rel_err_dd(qh, ql, ph, pl) < 1e-28


def test_column_apply_matches_full_matrix():
    rng = np.random.default_rng(13)
    n, sigma = 48, 3
    A = rand_normed(rng, n, 8.0)
    c = coeffs.taylor_exp(18)
    Eh, El = oracle.expm_dd(A, c, sigma)
    cols = [0, 7, 47]
    V = np.eye(n)[:, cols]
    Wh, Wl = oracle.expm_apply_dd(A, c, sigma, V)
    assert metrics.rel_err_dd(Wh, Wl, Eh[:, cols], El[:, cols]) < 1e-27


def test_fp64_ps_close_to_dd():
    rng = np.random.default_rng(14)
    n = 64
    X = rand_normed(rng, n, 1.0)
    c = coeffs.taylor_exp(16)
    h, l = oracle.poly_dd(X, c)
    e = metrics.rel_err_1(oracle.ps_f64(X, c, 4), h, l)
    assert 0 < e < n * 4 * U


def test_fp64_scaling_and_squaring_on_a_diagonal():
    # the double route of eq. (scal-idea): on a diagonal matrix every entry is
    # the scalar r(d) = p(2^-sigma d)^(2^sigma), and the Taylor polynomial of
    # degree 30 is e^x to double precision for |x| <= 1
    d = np.array([0.5, -1.0, 3.0, 7.5, -6.0])
    c = coeffs.taylor_exp(30)
    for sigma in (2, 3):
        E = oracle.expm_ps_f64(np.diag(d), c, 6, sigma)
        assert np.array_equal(E - np.diag(np.diag(E)), np.zeros_like(E))
        assert np.allclose(np.diag(E), np.exp(d), rtol=1e-13, atol=0), sigma


# ---------------------------------------------- P7: Pade coefficients
def test_pade_defining_property_and_small_cases():
    # section 4.1: p_km / q_km is the [k/m] Pade approximant of e^x, so
    # q(x) e^x - p(x) = O(x^(k+m+1)) with a non-zero coefficient at k+m+1
    for k, m in [(0, 1), (1, 0), (2, 1), (1, 2), (3, 5), (6, 2), (13, 13)]:
        p, q = coeffs.pade_exp_exact(k, m)
        assert len(p) == k + 1 and len(q) == m + 1 and p[0] == 1 and q[0] == 1
        ex = [F(1, math.factorial(j)) for j in range(k + m + 2)]
        prod = [sum(q[i] * ex[d - i] for i in range(min(d, m) + 1)) for d in range(k + m + 2)]
        for d in range(k + m + 1):
            assert prod[d] == (p[d] if d <= k else 0), (k, m, d)
        assert prod[k + m + 1] != 0
    # textbook forms: [2/1] = (1 + 2x/3 + x^2/6) / (1 - x/3), [1/2] = (1 + x/3) / (1 - 2x/3 + x^2/6)
    assert coeffs.pade_exp_exact(2, 1) == ([1, F(2, 3), F(1, 6)], [1, F(-1, 3)])
    assert coeffs.pade_exp_exact(1, 2) == ([1, F(1, 3)], [1, F(-2, 3), F(1, 6)])


def test_pade13_blocks_match_paper():
    p, q = coeffs.pade_exp_exact(13, 13)
    rows = [ln.split() for ln in open(os.path.join(GOLD, "pade13_blocks.txt")) if ln.strip() and ln[0] != "#"]
    assert len(rows) == 8
    for idx, num, den in rows:
        assert p[int(idx)] == F(int(num), int(den))
    # q_mm(x) = p_mm(-x)
    assert all(q[j] == (-1) ** j * p[j] for j in range(14))
    # general formula sanity: [1/1] is (1 + x/2)/(1 - x/2)
    p1, q1 = coeffs.pade_exp_exact(1, 1)
    assert p1 == [1, F(1, 2)] and q1 == [1, F(-1, 2)]


def test_taylor_cos_coefficients():
    c = coeffs.taylor_cos_exact(4)
    assert c == [1, F(-1, 2), F(1, 24), F(-1, 720), F(1, 40320)]
    assert coeffs.taylor_exp(3) == [1.0, 1.0, 0.5, 1.0 / 6.0]


# ---------------------------------------------- P8: alpha_m example
def test_nonnormal_example_numbers():
    g = {}
    for ln in open(os.path.join(GOLD, "nonnormal_2x2.txt")):
        if ln.strip() and ln[0] != "#":
            k, v, tol = ln.split()
            g[k] = (float(v), float(tol))
    A = np.array([[-0.1, 1e6], [0.0, -0.1]])
    X = A / 2
    nx = metrics.norm1(X)
    assert abs(nx - g["norm1_X"][0]) <= g["norm1_X"][1]
    assert abs(metrics.alpha_m(X, 42) - g["alpha_m"][0]) <= g["alpha_m"][1]
    s = math.ceil(math.sqrt(42))
    assert s == 7
    assert metrics.extra_scaling(nx, s) == int(g["l0"][0])
    # the scaling the paper's Taylor-based algorithm chooses at u = 1e-64, m = 42:
    # X = A/2 is accepted, i.e. one squaring (with xi(X) = 1 the bound would ask
    # for two: the relative acceptance needs the estimate of ||e^X||_1 ~ 4.8e5)
    m, u = int(g["m"][0]), g["u"][0]
    assert metrics.auto_sigma(A, m, s, u) == int(g["l"][0])
    assert metrics.xi_b0(X, s) == pytest.approx(math.exp(-0.05) * (1 + 5e5), rel=1e-4)


# ---------------------------------------------- P9: cost model
def test_table1_cost_ratio_and_block_counts():
    for ln in open(os.path.join(GOLD, "table1_cauchy100.txt")):
        if not ln.strip() or ln[0] == "#":
            continue
        head, tail = ln.split("|")
        D, m, s, r, cr = head.split()
        d = [int(x) for x in tail.split()]
        D, m, s, r = int(D), int(m), int(s), int(r)
        assert s == math.ceil(math.sqrt(m)) and r == m // s and len(d) == r
        assert abs(100 * metrics.cost_saving(D, s, r, d) - float(cr)) < 0.05
        # precisions decrease along the Horner chain (u_r >= ... >= u_1)
        assert all(d[i] >= d[i + 1] for i in range(r - 1))


def test_m_low_from_table1_within_table2s_range():
    # Table 2 prints M_low between 22% and 27% for every class and size, and
    # section 3.3.1 says about a fifth of the products of Table 1's runs use
    # precision u^(1/2) or lower: Table 1's digits give 3/12, 4/15, 5/19, 6/26
    want = {32: (3, 12), 64: (4, 15), 128: (5, 19), 256: (6, 26)}
    for ln in open(os.path.join(GOLD, "table1_cauchy100.txt")):
        if not ln.strip() or ln[0] == "#":
            continue
        head, tail = ln.split("|")
        D, m, s, r, _ = head.split()
        d = [int(x) for x in tail.split()]
        D, s, r = int(D), int(s), int(r)
        ml = metrics.m_low(D, s, r, d)
        k, tot = want[D]
        assert ml == k / tot
        assert 0.22 <= ml <= 0.27
    # the boundary is inclusive (u_i = u^(1/2) counts) and the powers never do
    assert metrics.m_low(32, 3, 2, [16, 17]) == 1 / 4
    assert metrics.m_low(32, 3, 2, [1, 1]) == 2 / 4


def test_table2_saving():
    g = dict((ln.split()[0], float(ln.split()[1])) for ln in open(os.path.join(GOLD, "table2_runtime.txt"))
             if ln.strip() and ln[0] != "#")
    assert abs(100 * (1 - g["T_tot"] / g["T_fix"]) - g["saving_percent"]) < 0.05


# ---------------------------------------------- oracle planner
def test_planner_hand_cases():
    # strong decay: B norms 1, 1e-3, 1e-7; ||Y|| = 1e-2
    u, nu, t = oplan.plan([1.0, 1e-3, 1e-7], 1e-2, working_tier=0)
    # u_1 = 2^-53 / max(1e-5, 1e-11) = 1.1e-11 -> still FP64 (needs >= 2^-24)
    # u_2 = 2^-53 / 1e-11 = 1.1e-5 -> FP32
    assert nu == 1 and t == [0, 0, 1]
    # Y = 0 (nilpotent of index <= s): every product is exactly zero
    u, nu, t = oplan.plan([2.0, 1.0, 1.0], 0.0)
    assert nu == 1 and t == [0, 3, 3]
    # B_0 = 0: keep the working precision everywhere
    u, nu, t = oplan.plan([0.0, 1.0, 1.0], 0.5)
    assert nu == 3 and t == [0, 0, 0]
    # no decay: fixed-precision PS is recovered
    u, nu, t = oplan.plan([1.0, 1.0, 1.0], 2.0)
    assert nu == 3 and t == [0, 0, 0]
    # FP32 working precision with bf16/fp8 tiers; inclusive comparison at the threshold
    u, nu, t = oplan.plan([1.0, 2.0 ** -20 / 2.0 ** -4, 1e-30], 2.0 ** -0, working_tier=1)
    assert t[1] == 2 and t[2] == 3
    # monotone: a large late block pulls earlier u_i down
    u, nu, t = oplan.plan([1.0, 1e-12, 1e-3], 1e-1)
    assert u[1] <= u[2]


def test_planner_exact_values():
    # eq. (choose-ui) with powers of two, so every u_i is exact:
    # ||B|| = (4, 2^-10, 2^-20), ||Y|| = 2^-3: the denominators are 2^-13 and
    # 2^-26, u_1 = 4u 2^13 and u_2 = 4u 2^26 (u = 2^-53)
    u, nu, t = oplan.plan([4.0, 2.0 ** -10, 2.0 ** -20], 2.0 ** -3)
    assert u == [2.0 ** -53, 2.0 ** -38, 2.0 ** -25] and nu == 1 and t == [0, 0, 0]
    # nu and delta (section 3.2): u_1 = 4u < 10u keeps step 1 in the working
    # precision; u_2 = 2^30 u = 2^-23 >= 2^-24 moves step 2 to FP32
    u, nu, t = oplan.plan([1.0, 2.0 ** -2, 2.0 ** -30], 1.0)
    assert nu == 2 and u == [2.0 ** -53, 2.0 ** -53, 2.0 ** -23] and t == [0, 0, 1]
    # with delta = 1 the same u_1 = 4u starts the lower tiers at step 1
    u, nu, t = oplan.plan([1.0, 2.0 ** -2, 2.0 ** -30], 1.0, delta=1.0)
    assert nu == 1 and t == [0, 0, 1]


def test_block_bounds_partition_the_coefficients():
    # eq. (ps): B_i takes c_{si}..c_{si+s-1} for i < r and c_{sr}..c_m last
    assert oplan.block_bounds(4, 10) == (2, [[0, 1, 2, 3], [4, 5, 6, 7], [8, 9, 10]])
    assert oplan.block_bounds(3, 9) == (3, [[0, 1, 2], [3, 4, 5], [6, 7, 8], [9]])
    for s, m in [(1, 5), (5, 5), (6, 30), (7, 40), (16, 255)]:
        r, ranges = oplan.block_bounds(s, m)
        assert r == m // s and sum(ranges, []) == list(range(m + 1))


def test_norm1_is_the_largest_column_sum():
    # section 3.3 measures errors in the 1-norm: maximum absolute column sum
    assert metrics.norm1([[1.0, -2.0], [3.0, 4.0]]) == 6.0
    assert metrics.norm1(np.array([[1.0, 5.0, 0.0], [-2.0, 0.0, 0.0]])) == 5.0
    assert metrics.norm1(np.zeros((0, 0))) == 0.0


def test_apriori_norms_bound_block_norms():
    rng = np.random.default_rng(15)
    n, m, s = 30, 18, 5
    X = rand_normed(rng, n, 0.7)
    c = coeffs.taylor_exp(m)
    r, ranges = oplan.block_bounds(s, m)
    assert r == 3 and ranges[-1] == [15, 16, 17, 18]
    nb, ny = oplan.apriori_norms(c, s, metrics.norm1(X))
    powers = [np.eye(n)]
    for _ in range(s):
        powers.append(powers[-1] @ X)
    for i in range(r + 1):
        B = sum(c[k] * powers[k - s * i] for k in ranges[i])
        assert metrics.norm1(B) <= nb[i] * (1 + 1e-12)
    assert metrics.norm1(powers[s]) <= ny * (1 + 1e-12)


# ---------------------------------------------- R4: gradient oracle
def _fadd(A, B, a=1, b=1):
    return [[a * A[i][j] + b * B[i][j] for j in range(len(A[0]))] for i in range(len(A))]


def _fr(A, c, sigma):
    X = [[x / 2 ** sigma for x in row] for row in A]
    R = fpoly(X, c)
    for _ in range(sigma):
        R = fmul(R, R)
    return R


@pytest.mark.parametrize("sigma", [0, 1, 2])
def test_gradient_oracle_matches_derivative_definition(sigma):
    """<grad, E> must equal d/dh <G, r(A + hE)> at h = 0.  The derivative is
    taken from its definition by an exact rational central difference with
    h = 1e-30 (remainder O(h^2)), independent of the block-triangular identity
    the oracle uses."""
    rng = np.random.default_rng(20 + sigma)
    n = 3
    A = rng.standard_normal((n, n)) / 2
    G = rng.standard_normal((n, n))
    E = rng.standard_normal((n, n))
    c = coeffs.taylor_exp(5)
    gh, gl = oracle.expm_grad_dd(A, G, c, sigma)
    got = sum(F(float(gh[i, j])) * F(float(E[i, j])) + F(float(gl[i, j])) * F(float(E[i, j]))
              for i in range(n) for j in range(n))
    h = F(1, 10 ** 30)
    Af, Ef, Gf = fmat(A), fmat(E), fmat(G)
    Rp = _fr(_fadd(Af, Ef, 1, h), c, sigma)
    Rm = _fr(_fadd(Af, Ef, 1, -h), c, sigma)
    want = sum(Gf[i][j] * (Rp[i][j] - Rm[i][j]) for i in range(n) for j in range(n)) / (2 * h)
    assert abs(got - want) <= F(1e-28) * (abs(want) + 1)


def test_gradient_oracle_polynomial_closed_form():
    """p(X) = X^2: the gradient of <G, X^2> is G X^T + X^T G."""
    rng = np.random.default_rng(23)
    n = 5
    X = rng.standard_normal((n, n))
    G = rng.standard_normal((n, n))
    gh, gl = oracle.expm_grad_dd(X, G, [0.0, 0.0, 1.0], 0, cols=[1, 4])
    want = (G @ X.T + X.T @ G)[:, [1, 4]]
    assert np.max(np.abs(gh + gl - want)) < 1e-14 * np.max(np.abs(want))


# ---------------------------------------------- P10: truncation threshold of the alpha_m bound
@pytest.mark.parametrize("u", [2.0 ** -53, 2.0 ** -24])
def test_theta_taylor_closed_forms_and_bounds(u):
    # m = 0: the tail is e^t - 1, so theta_0 = log1p(u) exactly
    assert abs(metrics.theta_taylor(0, u) - math.log1p(u)) <= 1e-14 * u
    # m = 1: e^t - 1 - t = u, theta_1 = sqrt(2u) (1 - sqrt(2u)/6 + O(u))
    r = math.sqrt(2 * u)
    assert abs(metrics.theta_taylor(1, u) / r - (1 - r / 6)) <= 4 * r * r
    # all m: t^(m+1)/(m+1)! <= tail(t) <= t^(m+1)/(m+1)! / (1 - t/(m+2)) for t < m+2
    for m in (2, 5, 10, 18, 30, 60, 100, 170):
        th = metrics.theta_taylor(m, u)
        lead = math.exp((math.lgamma(m + 2) + math.log(u)) / (m + 1))   # ((m+1)! u)^(1/(m+1))
        assert th <= lead * (1 + 1e-12)
        if lead < m + 2:
            assert th >= lead * (1 - lead / (m + 2)) ** (1.0 / (m + 1)) * (1 - 1e-12)
    ths = [metrics.theta_taylor(m, u) for m in range(0, 40)]
    assert all(a < b for a, b in zip(ths, ths[1:]))


def test_alpha_m_closed_forms():
    # eq. (alpha_m-X): alpha_m(X) = max(||X^d||^(1/d), ||X^(d+1)||^(1/(d+1))) with
    # d the largest integer such that d (d - 1) <= m + 1
    for m in (12, 30, 42):
        d = 1
        while (d + 1) * d <= m + 1:
            d += 1
        for t in (0.5, 2.0, 3.0):
            assert metrics.alpha_m(t * np.eye(3), m) == pytest.approx(t, rel=1e-15)
        # Jordan block [[a, b], [0, a]]: ||X^k||_1 = a^k + k a^(k-1) b
        a, b = 0.75, 0.5
        ex = max((a ** d + d * a ** (d - 1) * b) ** (1.0 / d),
                 (a ** (d + 1) + (d + 1) * a ** d * b) ** (1.0 / (d + 1)))
        assert metrics.alpha_m(np.array([[a, b], [0.0, a]]), m) == pytest.approx(ex, rel=1e-14)
        # nilpotent of index 2
        assert metrics.alpha_m(np.array([[0.0, 5.0], [0.0, 0.0]]), m) == 0.0


def test_smallest_shift_is_inclusive():
    # sigma is the least k >= 0 with a <= 2^k b (the scaled norm may reach theta)
    assert metrics._smallest_shift(4.0, 1.0) == 2
    assert metrics._smallest_shift(4.0 + 2.0 ** -50, 1.0) == 3
    assert metrics._smallest_shift(1.0, 1.0) == 0 and metrics._smallest_shift(0.25, 1.0) == 0


def test_auto_sigma_on_the_nonnormal_example():
    # A = [[-0.1, 1e6], [0, -0.1]] (eq. (nonnormal-mat-A)): ||A||_1 ~ 1e6 asks for
    # 19 halvings, while alpha_m(A) = 2 alpha_m(A/2) ~ 1.3 (pinned above) is
    # below theta_30 ~ 3.78: the alpha_m bound needs no scaling at all
    A = np.array([[-0.1, 1e6], [0.0, -0.1]])
    u = 2.0 ** -53
    th = metrics.theta_taylor(30, u)
    assert metrics.auto_sigma(A, 30, 6, u) == 0
    assert math.ldexp(th, 18) < metrics.norm1(A) <= math.ldexp(th, 19)
    # the norm guard forces ||X||_1 <= s/e: l_0 = ceil(log2(e ||A||_1 / 6)) = 19
    assert metrics.auto_sigma(A, 30, 6, u, norm_guard=True) == math.ceil(math.log2(math.e * metrics.norm1(A) / 6))
    # a normal matrix: alpha_m = ||A||_1 for a diagonal one, so sigma = sigma0
    D = np.diag([-9.0, 3.0, 1.0])
    assert metrics.auto_sigma(D, 30, 6, u) == math.ceil(math.log2(9.0 / th))


def _tail_bounds(t, m):
    """exact rational bounds lo <= sum_{k>m} t^k / k! <= hi for the double t >= 0:
    a partial sum, and the partial sum plus the geometric bound of the rest"""
    t = F(t)
    term = F(1)
    for k in range(1, m + 2):
        term = term * t / k
    lo = F(0)
    k = m + 1
    while True:
        lo += term
        k += 1
        term = term * t / k
        if k > t + 1 and term < lo * F(1, 10 ** 40):
            break
    return lo, lo + term / (1 - t / (k + 1))


def _taylor_partial(x, s):
    """sum_{j<s} x^j / j! exactly (x a double)"""
    x = F(x)
    return sum(x ** j / math.factorial(j) for j in range(s))


def test_xi_b0_closed_forms():
    # diagonal: B_0(D) = diag(T(d_i)), T the degree-(s-1) Taylor sum
    d = [-2.25, 0.75, 0.5, -0.125]
    for s in (1, 2, 4, 6, 7):
        want = max(abs(_taylor_partial(x, s)) for x in d)
        assert metrics.xi_b0(np.diag(d), s) == pytest.approx(float(want), rel=1e-14)
    # Jordan block [[a, b], [0, a]]: X^j = a^j I + j a^(j-1) b N, so
    # B_0 = T(a) I + b T'(a) N and ||B_0||_1 = |T(a)| + |b| |T'(a)|
    for a, b, s in ((-0.05, 5e5, 7), (0.5, -3.0, 4), (-1.5, 0.25, 6)):
        T = _taylor_partial(a, s)
        Tp = sum(F(j) * F(a) ** (j - 1) / math.factorial(j) for j in range(1, s))
        want = max(abs(T), abs(T) + abs(F(b)) * abs(Tp))
        X = np.array([[a, b], [0.0, a]])
        assert metrics.xi_b0(X, s) == pytest.approx(float(want), rel=1e-13)


@pytest.mark.parametrize("d,m,s,u", [([-9.0, 3.0, 1.0], 30, 6, U), ([6.0, -0.5], 30, 6, U),
                                     ([-40.0, -3.0], 18, 5, 2.0 ** -24), ([2.5, 1.25, -0.75], 16, 4, U),
                                     ([100.0, -100.0, 1.0], 42, 7, 1e-64)])
def test_auto_sigma_is_the_least_accepted_scaling(d, m, s, u):
    # diagonal D: alpha_m(D) = max|d_i| and xi(2^-k D) = max_i |T(2^-k d_i)|, so the
    # acceptance test of eq. (alpha_m-X) can be decided in exact rationals: the
    # chosen k passes with the tail's upper bound and every smaller k fails with
    # its lower bound (the cases are far from ties)
    D = np.diag(d)
    sig = metrics.auto_sigma(D, m, s, u)
    a = max(abs(x) for x in d)

    def passes(k, bound):
        lo, hi = _tail_bounds(math.ldexp(a, -k), m)
        xi = max(abs(_taylor_partial(math.ldexp(x, -k), s)) for x in d)
        return (hi if bound == "hi" else lo) <= F(u) * xi

    assert passes(sig, "hi")
    for k in range(sig):
        assert not passes(k, "lo"), k


# --------------------------------------------------------------------------
# Algorithm 2's variable-s branch (fix_params = false, section 3.3)
# --------------------------------------------------------------------------
def _jordan_s(t, a, m):
    """The branch's s for X = [[-t, a], [0, -t]] (t, a > 0) in exact rational
    arithmetic from the closed forms X^k = (-t)^k I + k (-t)^(k-1) a N:
    ||X^k||_1 = t^k + k t^(k-1) a, ||X||_1 = t + a, and
    ||B_0||_1 = |sum_{j<s} c_j (-t)^j| + a |sum_{0<j<s} c_j j (-t)^(j-1)|."""
    c = [F(1, math.factorial(k)) for k in range(m + 1)]
    s = 1
    while s * s < m:
        s += 1
    nX = t + a
    if not (nX <= F(s) / F(math.e)) or s >= m:
        return s

    def nB0(s):
        S = sum(c[j] * (-t) ** j for j in range(s))
        Sp = sum(c[j] * j * (-t) ** (j - 1) for j in range(1, s))
        return abs(S) + a * abs(Sp)
    while t ** s + s * t ** (s - 1) * a > nB0(s) * nX ** s and s < m:
        s += 1
    return s


@pytest.mark.parametrize("t,a", [(F(1, 2), F(1, 32)), (F(1, 4), F(1, 32)), (F(3, 4), F(1, 8)), (F(1), F(1, 4)),
                                 (F(1, 2), F(1, 4)), (F(1, 4), F(1, 64)),
                                 # growth that stops part-way (s = 20 and s = 7), where the
                                 # norm of the growing B_0 decides the stop
                                 (F(17, 16), F(1, 8)), (F(9, 8), F(3, 8))])
def test_variable_s_on_jordan_blocks(t, a):
    m = 30
    X = np.array([[-float(t), float(a)], [0.0, -float(t)]])
    assert metrics.variable_s(X, coeffs.taylor_exp(m)) == _jordan_s(t, a, m)


def test_variable_s_special_cases():
    m = 30
    c = coeffs.taylor_exp(m)
    # -tI, 0 < t <= 1: every partial sum of e^-t lies in (0, 1) while
    # ||X^s|| = ||X||^s, so s grows to m (explicit powers)
    assert metrics.variable_s(-0.5 * np.eye(5), c) == m
    # tI, t > 0: ||B_0|| > 1 = ||X^s|| / ||X||^s, so s stays at ceil(sqrt(m))
    assert metrics.variable_s(0.5 * np.eye(5), c) == 6
    # nilpotent of order 2: Y = X^s = 0
    assert metrics.variable_s(np.array([[0.0, 2.0], [0.0, 0.0]]), c) == 6
    # ||X||_1 > s/e: the branch does not run
    assert metrics.variable_s(-3.0 * np.eye(5), c) == 6
    # small degrees: m = 4 grows from 2 to 4; m = 2 and m = 1 start at s = m
    assert metrics.variable_s(-0.5 * np.eye(3), coeffs.taylor_exp(4)) == 4
    assert metrics.variable_s(-0.5 * np.eye(3), coeffs.taylor_exp(2)) == 2
    assert metrics.variable_s(-0.5 * np.eye(3), coeffs.taylor_exp(1)) == 1


# --------------------------------------------------------------------------
# joint choice of the Taylor degree and the scaling (section 3.2)
# --------------------------------------------------------------------------
def _alpha_brute(A, m):
    """alpha_m from eq. (alpha_m-X) with d* found by enumeration and powers
    by numpy.linalg.matrix_power"""
    d = max(k for k in range(1, m + 3) if k * (k - 1) <= m + 1)
    return max(metrics.norm1(np.linalg.matrix_power(A, d)) ** (1.0 / d),
               metrics.norm1(np.linalg.matrix_power(A, d + 1)) ** (1.0 / (d + 1)))


def _cost_brute(m):
    s = math.isqrt(m - 1) + 1 if m > 1 else 1          # ceil(sqrt(m))
    r = m // s
    return (s - 1) + r - (1 if m == s * r else 0)


def test_select_degree_zero_and_nilpotent():
    u = 2.0 ** -53
    # alpha_m = 0: no scaling, and the cheapest candidate m = 1 (p_1(X) = I + X,
    # which is e^A exactly when A^2 = 0)
    assert metrics.select_degree(np.zeros((4, 4)), 42, u) == (1, 1, 0)
    assert metrics.select_degree(np.array([[0.0, 5.0], [0.0, 0.0]]), 42, u) == (1, 1, 0)


def _accepts_brute(A, k, m, u):
    """eq. (alpha_m-X) at X = 2^-k A with alpha_m and B_0 from numpy's
    matrix_power and the tail's exact rational bounds; None when the two
    bounds disagree (a near-tie)"""
    X = np.ldexp(A, -k)
    s = math.isqrt(m - 1) + 1 if m > 1 else 1
    a = _alpha_brute(X, m)
    xi = metrics.norm1(sum(np.linalg.matrix_power(X, j) / math.factorial(j) for j in range(s)))
    lo, hi = _tail_bounds(a, m)
    if hi <= F(u) * F(xi):
        return True
    if lo > F(u) * F(xi):
        return False
    return None


@pytest.mark.parametrize("t,seed", [(0.01, 1), (0.3, 2), (1.0, 3), (8.0, 4), (64.0, 5), (1e3, 6)])
def test_select_degree_is_the_cheapest_admissible_choice(t, seed):
    u = 2.0 ** -53
    G = np.random.default_rng(seed).standard_normal((12, 12))
    A = G * (t / metrics.norm1(G))
    m, s, sig = metrics.select_degree(A, 42, u)
    assert s == (math.isqrt(m - 1) + 1 if m > 1 else 1)
    # the bound holds at the chosen pair, and one squaring fewer fails it
    assert _accepts_brute(A, sig, m, u) is True
    if sig > 0:
        assert _accepts_brute(A, sig - 1, m, u) is False
    # no candidate is cheaper at its own least admissible scaling
    best = _cost_brute(m) + sig
    for q in range(1, 7):
        for mc in (q * q, q * (q + 1)):
            if mc > 42:
                continue
            sc = 0
            while True:
                ok = _accepts_brute(A, sc, mc, u)
                assert ok is not None, (mc, sc)
                if ok:
                    break
                sc += 1
            assert _cost_brute(mc) + sc >= best, (mc, sc, m, sig)
            if _cost_brute(mc) + sc == best:
                assert mc >= m                      # ties go to the smaller degree


def test_select_degree_scales_by_one_squaring():
    # once every candidate needs scaling, doubling A adds exactly one squaring
    u = 2.0 ** -53
    G = np.random.default_rng(9).standard_normal((10, 10))
    A = G * (20.0 / metrics.norm1(G))
    m, s, sig = metrics.select_degree(A, 42, u)
    assert sig >= 1
    assert metrics.select_degree(2 * A, 42, u) == (m, s, sig + 1)
