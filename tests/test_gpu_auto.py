"""GPU parity of the automatic scaling (ps_expm_auto): the scaling chosen by
the alpha_m bound equals the oracle's choice, and the result matches the
double-double oracle at that scaling.  Norms are those of the column-major
view the library works on, i.e. of the transpose of each row-major array."""
import math

import numpy as np
import pytest

import oracle
from oracle import coeffs, metrics

from helpers import to_dev, to_np

pytestmark = pytest.mark.gpu

TOL64 = 1e-13
M, S = 30, 6


@pytest.fixture(scope="module")
def ps():
    import paper_2312_17396_amd as ps
    ps.lib()
    return ps


def _dense(n, t, seed):
    G = np.random.default_rng(seed).standard_normal((n, n))
    return G * (t / metrics.norm1(G.T))


def _cases():
    g = np.random.default_rng(7)
    tri = np.triu(g.standard_normal((100, 100)), 1) * 4.0 - 0.5 * np.eye(100)   # nonnormal: alpha_m << ||A||_1
    h = np.random.default_rng(5)
    shifted = -12.0 * np.eye(50) + h.standard_normal((50, 50)) / math.sqrt(50)   # ||e^X|| far from 1
    pos = np.abs(h.standard_normal((40, 40))) * 0.5                               # ||e^X|| well above 1
    return [
        ("dense64_t0.5", _dense(64, 0.5, 1)),
        ("dense64_t5", _dense(64, 5.0, 2)),
        ("dense200_t60", _dense(200, 60.0, 3)),
        ("nonnormal_2x2", np.array([[-0.1, 1e6], [0.0, -0.1]]).T),   # column-major view = the paper's A
        ("triangular100", tri),
        ("shifted_neg50", shifted),
        ("positive40", pos),
    ]


def test_acceptance_is_relative_to_xi(ps):
    # eq. (alpha_m-X) accepts X when the Taylor tail at alpha_m(X) is at most
    # u xi(X), xi(X) an estimate of ||e^X||_1: on these matrices that takes
    # one squaring fewer than the absolute test (xi = 1) would
    u = 2.0 ** -53
    for name, A in _cases()[4:]:
        th = metrics.theta_taylor(M, u)
        At = A.T
        s0 = metrics._smallest_shift(metrics.norm1(At), th)
        sig_abs = min(s0, metrics._smallest_shift(metrics._alpha_scaled(At, M, s0), th))
        _, sig = ps.ps_expm_auto(to_dev(A), M, s=S)
        assert sig == metrics.auto_sigma(At, M, S, u) == sig_abs - 1, name


@pytest.mark.parametrize("mode", ["fixed", "mixed"])
@pytest.mark.parametrize("name,A", _cases(), ids=[c[0] for c in _cases()])
def test_auto_sigma_and_accuracy(ps, name, A, mode):
    u = 2.0 ** -53
    sig_o = metrics.auto_sigma(A.T, M, S, u)
    E, sig = ps.ps_expm_auto(to_dev(A), M, s=S, mode=mode)
    assert sig == sig_o, (name, sig, sig_o)
    Eh, El = oracle.expm_dd(A, coeffs.taylor_exp(M), sig)
    err = metrics.rel_err_1(to_np(E), Eh, El)
    # equal accuracy: the 1e-13 target, or twice the error of the oracle's
    # own IEEE double Algorithm 1 with the same (m, s, sigma) where that
    # misses it (||e^X|| far below e^||X||: the Taylor sum cancels)
    tol = max(TOL64, 2 * metrics.rel_err_1(oracle.expm_ps_f64(A, coeffs.taylor_exp(M), S, sig), Eh, El))
    assert err <= tol, (name, sig, err, tol)
    # the same evaluation through the explicit-sigma path agrees to rounding
    E2 = to_np(ps.ps_expm(to_dev(A), M, s=S, sigma=sig, mode=mode))
    assert metrics.rel_err_1(E2, Eh, El) <= tol


def test_auto_sigma_alpha_below_norm(ps):
    # the paper's example: ||A||_1 ~ 1e6 would take 19 halvings, alpha_m none
    A = np.array([[-0.1, 1e6], [0.0, -0.1]]).T
    u = 2.0 ** -53
    c = coeffs.taylor_exp(M)
    E0, sig = ps.ps_expm_auto(to_dev(A), M, s=S)
    assert sig == 0
    Eh, El = oracle.expm_dd(A, c, 0)
    err0 = metrics.rel_err_1(to_np(E0), Eh, El)
    assert err0 <= TOL64
    # the norm guard (||X||_1 <= s/e) takes the 19 squarings, and the squaring
    # phase amplifies the rounding errors (section 3.2): still within the
    # 2^sigma growth of the squarings, but far less accurate than sigma = 0
    E, sig_g = ps.ps_expm_auto(to_dev(A), M, s=S, norm_guard=True)
    assert sig_g == metrics.auto_sigma(A.T, M, S, u, norm_guard=True) == 19
    Eh, El = oracle.expm_dd(A, c, sig_g)
    err_g = metrics.rel_err_1(to_np(E), Eh, El)
    assert err_g <= 2.0 ** sig_g * 4 * u
    assert err_g > 10 * err0


def test_auto_sigma_fp32(ps):
    import torch
    A = _dense(128, 6.0, 11).astype(np.float32).astype(np.float64)
    u = 2.0 ** -24
    sig_o = metrics.auto_sigma(A.T, M, S, u)
    E, sig = ps.ps_expm_auto(to_dev(A, torch.float32), M, s=S, mode="mixed")
    assert sig == sig_o
    Eh, El = oracle.expm_dd(A, coeffs.taylor_exp(M), sig)
    assert metrics.rel_err_1(to_np(E).astype(np.float64), Eh, El) <= 2.0 ** sig * 8 * 128 * u


def test_auto_rejects_nonfinite(ps):
    A = np.eye(8)
    A[3, 2] = np.inf
    with pytest.raises(ps.PSError):
        ps.ps_expm_auto(to_dev(A), M, s=S)


# --------------------------------------------------------------------------
# joint choice of the degree and the scaling (ps_expm_select)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("mode", ["fixed", "mixed"])
@pytest.mark.parametrize("name,A", _cases(), ids=[c[0] for c in _cases()])
def test_select_matches_oracle_and_accuracy(ps, name, A, mode):
    u = 2.0 ** -53
    m_o, s_o, sig_o = metrics.select_degree(A.T, 42, u)
    E, (m, s, sig) = ps.ps_expm_select(to_dev(A), 42, mode=mode)
    assert (m, s, sig) == (m_o, s_o, sig_o), name
    c = coeffs.taylor_exp(m)
    Eh, El = oracle.expm_dd(A, c, sig)
    tol = max(TOL64, 2 * metrics.rel_err_1(oracle.expm_ps_f64(A, c, s, sig), Eh, El))
    assert metrics.rel_err_1(to_np(E), Eh, El) <= tol, (name, m, sig)


def test_select_nilpotent_is_exact(ps):
    A = np.zeros((70, 70))
    A[np.arange(0, 70, 2), np.arange(1, 70, 2)] = 3.0          # A^2 = 0: e^A = I + A
    E, ch = ps.ps_expm_select(to_dev(A), 42)
    assert ch == (1, 1, 0)
    assert np.array_equal(to_np(E), np.eye(70) + A)


def test_select_fp32_and_doubling(ps):
    import torch
    A = _dense(96, 20.0, 12).astype(np.float32).astype(np.float64)
    u = 2.0 ** -24
    E, ch = ps.ps_expm_select(to_dev(A, torch.float32), 42, mode="mixed")
    assert ch == metrics.select_degree(A.T, 42, u)
    Eh, El = oracle.expm_dd(A, coeffs.taylor_exp(ch[0]), ch[2])
    assert metrics.rel_err_1(to_np(E).astype(np.float64), Eh, El) <= 2.0 ** ch[2] * 8 * 96 * u
    # every candidate needs scaling here, so doubling A adds one squaring
    _, ch2 = ps.ps_expm_select(to_dev(2 * A, torch.float32), 42, mode="mixed")
    assert ch2 == (ch[0], ch[1], ch[2] + 1)
