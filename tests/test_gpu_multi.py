"""GPU parity of several polynomials sharing one power table (ps_eval_multi):
the Pade [13/13] numerator and denominator of exp (section 4.1) and the
Taylor cosine evaluated as a polynomial in A^2 (section 4.2)."""
import numpy as np
import pytest

import oracle
from oracle import coeffs, metrics
from paper_2312_17396_amd import inputs

from helpers import relerr_cols, sample_cols, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ps():
    import paper_2312_17396_amd as ps
    ps.lib()
    return ps


def _even(c):
    """coefficients of c(A^2) as a polynomial in A"""
    out = [0.0] * (2 * len(c) - 1)
    for k, ck in enumerate(c):
        out[2 * k] = ck
    return out


@pytest.mark.parametrize("mode", ["fixed", "mixed"])
@pytest.mark.parametrize("n", [3, 90, 200])
def test_pade_pair_and_cos_small(ps, mode, n):
    g = np.random.default_rng(n)
    Q = inputs.haar_orthogonal(n, g)
    A = (Q * g.uniform(-2, 2, n)[None, :]) @ Q.T
    p, q = coeffs.pade_exp(13, 13)
    (P, Qm), reps = ps.ps_eval_multi(to_dev(A), [p, q], s=4, mode=mode, report=True)
    for got, cc in ((P, p), (Qm, q)):
        h, l = oracle.poly_dd(A, cc)
        assert metrics.rel_err_1(to_np(got), h, l) <= 1e-13
    cc = coeffs.taylor_cos(12)
    (C,), rep = ps.ps_eval_multi(to_dev(A), [cc], s=4, square_arg=True, mode=mode, report=True)
    h, l = oracle.poly_dd(A, _even(cc))
    assert metrics.rel_err_1(to_np(C), h, l) <= 1e-13
    # q(X) = p(-X)
    P2 = ps.ps_eval(to_dev(-A), p, s=4, mode=mode)
    assert np.allclose(to_np(P2), to_np(Qm), rtol=0, atol=1e-13 * np.abs(to_np(Qm)).max())


@pytest.mark.parametrize("nonnormal", [False, True])
def test_orthosim_2048(ps, nonnormal):
    """n = 2048 FP64: Pade [13/13] p and q from one power table (s = 4) and
    Taylor cos of degree 12 in A^2 (s = 4), plain and mixed, sampled columns
    against the oracle."""
    A = inputs.orthosim_2048(nonnormal=nonnormal)
    n = A.shape[0]
    cols = sample_cols(n, 4, seed=int(nonnormal))
    V = np.eye(n)[:, cols]
    p, q = coeffs.pade_exp(13, 13)
    cc = coeffs.taylor_cos(12)
    refs = [oracle.poly_apply_dd(A, p, V), oracle.poly_apply_dd(A, q, V), oracle.poly_apply_dd(A, _even(cc), V)]
    At = to_dev(A)
    for mode in ("fixed", "mixed"):
        (P, Qm), reps = ps.ps_eval_multi(At, [p, q], s=4, mode=mode, report=True)
        (C,), crep = ps.ps_eval_multi(At, [cc], s=4, square_arg=True, mode=mode, report=True)
        for got, (wh, wl), name in ((P, refs[0], "p"), (Qm, refs[1], "q"), (C, refs[2], "cos")):
            err = relerr_cols(to_np(got)[:, cols], wh, wl)
            print("nonnormal=%s %s %s err=%.3e" % (nonnormal, mode, name, err))
            assert err <= 1e-13, (mode, name, err)
