"""GPU parity of the a-priori planning rule (opts.rule = PS_RULE_APRIORI):
the denominators of eq. (choose-ui) bounded by sum |c_k| ||X||^k instead of
the assembled blocks' norms, ||B_0|| still the block norm.  The plan must
equal the oracle's plan on the oracle's a-priori norms built from the
reported ||X||_1, the result must meet the FP64 tolerance, and the rule may
only keep products at higher precision than the block-norm rule."""
import math

import numpy as np
import pytest

import oracle
from oracle import coeffs, metrics
from oracle import plan as oplan

from helpers import to_dev, to_np

pytestmark = pytest.mark.gpu

M, S = 30, 6


@pytest.fixture(scope="module")
def ps():
    import paper_2312_17396_amd as ps
    ps.lib()
    return ps


def _dense(n, t, seed):
    G = np.random.default_rng(seed).standard_normal((n, n))
    return G * (t / metrics.norm1(G.T))


@pytest.mark.parametrize("n,t,sigma", [(200, 0.1, 0), (200, 1.0, 0), (130, 8.0, 3), (64, 0.5, 0), (300, 64.0, 6)])
def test_apriori_plan_and_accuracy(ps, n, t, sigma):
    A = _dense(n, t, 7 + n)
    c = coeffs.taylor_exp(M)
    E, rep = ps.ps_expm(to_dev(A), M, s=S, sigma=sigma, mode="mixed", rule="apriori", report=True)
    nX = metrics.norm1(A.T) * 2.0 ** -sigma            # column-major view, X = 2^-sigma A
    assert abs(rep["normX"] - nX) <= 1e-13 * nX
    nb, ny = oplan.apriori_norms(c, S, rep["normX"])
    nb[0] = rep["normB"][0]
    u, nu, tiers = oplan.plan(nb, ny, working_tier=0)
    assert tiers[1:] == rep["tier"][1:], (tiers, rep["tier"])
    Eh, El = oracle.expm_dd(A, c, sigma)
    assert metrics.rel_err_1(to_np(E), Eh, El) <= 1e-13
    # never lower than the block-norm plan (the a-priori bound is an upper bound)
    _, rb = ps.ps_expm(to_dev(A), M, s=S, sigma=sigma, mode="mixed", report=True)
    first = rep["first_step"]
    for ta, tb in zip(rep["tier"][1:first + 1], rb["tier"][1:first + 1]):
        assert oplan.U_TIER[ta] <= oplan.U_TIER[tb]


def test_apriori_keeps_more_fp64_on_the_dense_set(ps):
    # ||A||_1 = 1, m = 30, s = 6: the block norms of a random dense matrix sit
    # far below the coefficient bounds, so the rules differ on this input
    A = _dense(512, 1.0, 3)
    _, ra = ps.ps_expm(to_dev(A), M, s=S, mode="mixed", rule="apriori", report=True)
    _, rb = ps.ps_expm(to_dev(A), M, s=S, mode="mixed", report=True)
    first = ra["first_step"]
    ua = [oplan.U_TIER[x] for x in ra["tier"][1:first + 1]]
    ub = [oplan.U_TIER[x] for x in rb["tier"][1:first + 1]]
    assert all(x <= y for x, y in zip(ua, ub)) and ua != ub, (ra["tier"], rb["tier"])


def test_apriori_batched_equals_single_path(ps):
    g = np.random.default_rng(11)
    mats = [_dense(int(n), float(t), 50 + k) for k, (n, t) in enumerate(zip(g.integers(1, 33, 6) * 8,
                                                                          g.uniform(0.05, 4.0, 6)))]
    sig = [max(0, math.ceil(math.log2(metrics.norm1(A.T)))) for A in mats]
    E, reps = ps.ps_expm_batched([to_dev(A) for A in mats], 18, s=4, sigma=sig, mode="mixed", rule="apriori",
                                 report=True)
    for A, Eb, rb, sg in zip(mats, E, reps, sig):
        Es, rs = ps.ps_expm(to_dev(A), 18, s=4, sigma=sg, mode="mixed", rule="apriori", report=True)
        assert rb["tier"][1:rs["first_step"] + 1] == rs["tier"][1:rs["first_step"] + 1]
        assert np.array_equal(to_np(Eb), to_np(Es))


def test_apriori_rejected_by_dd_path(ps):
    import torch
    T = torch.zeros(2, 8, 8, dtype=torch.float64, device="cuda:0")
    o, _k = ps._opts("mixed", rule="apriori")
    nbytes = ps.dd_workspace(8, 10)
    with pytest.raises(ps.PSError):
        ps._check(ps.lib().ps_expm_dd(8, T.data_ptr(), 8, None, 10, 0, 0, torch.empty_like(T).data_ptr(), 8,
                                      ps.ctypes.byref(o), None, nbytes[1], nbytes[2], ps._stream_ptr(T.device)))
