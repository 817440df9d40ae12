"""GPU parity of the hand-written adjoint (ps_expm_backward) against the
oracle's block-triangular gradient, central finite differences and the
dot-product identity, and of the autograd wrapper."""
import numpy as np
import pytest

import oracle
from oracle import coeffs, metrics

from helpers import U32, U64, sample_cols, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ps():
    import paper_2312_17396_amd as ps
    ps.lib()
    return ps


def _rand(n, t, seed):
    g = np.random.default_rng(seed)
    G = g.standard_normal((n, n))
    return G * (t / metrics.norm1(G))


@pytest.mark.parametrize("n,m,s,sigma,t", [
    (1, 6, 2, 0, 0.5), (17, 18, 5, 2, 3.0), (40, 8, 2, 1, 1.5), (64, 12, 1, 0, 0.7), (70, 9, 9, 1, 1.0),
    (100, 30, 6, 3, 6.0), (130, 13, 4, 0, 1.0),
])
def test_gradient_fp64_vs_block_triangular_oracle(ps, n, m, s, sigma, t):
    A = _rand(n, t, 10 + n)
    G = np.random.default_rng(20 + n).standard_normal((n, n))
    c = coeffs.taylor_exp(m)
    gh, gl = oracle.expm_grad_dd(A, G, c, sigma)
    for rec in (False, True):
        gA = to_np(ps.ps_expm_backward(to_dev(A), to_dev(G), m, s=s, sigma=sigma, recompute=rec))
        err = metrics.rel_err_1(gA, gh, gl)
        assert err <= 1e-12, (rec, err)
    a = to_np(ps.ps_expm_backward(to_dev(A), to_dev(G), m, s=s, sigma=sigma, recompute=False))
    b = to_np(ps.ps_expm_backward(to_dev(A), to_dev(G), m, s=s, sigma=sigma, recompute=True))
    assert np.array_equal(a, b)   # same products in the same order


def test_dot_product_identity_with_forward_derivative(ps):
    """<gradA, E> = <G, L_r(A, E)>, with L_r(A, E) the upper-right block of
    r([[A, E], [0, A]]) from the oracle (forward-mode derivative)."""
    n, m, s, sigma = 30, 18, 5, 2
    A = _rand(n, 3.0, 5)
    g = np.random.default_rng(6)
    G, E = g.standard_normal((n, n)), g.standard_normal((n, n))
    c = coeffs.taylor_exp(m)
    gA = to_np(ps.ps_expm_backward(to_dev(A), to_dev(G), m, s=s, sigma=sigma))
    Z = np.block([[A, E], [np.zeros((n, n)), A]])
    Wh, Wl = oracle.expm_apply_dd(Z, c, sigma, np.eye(2 * n)[:, n:])
    L = (Wh + Wl)[:n]
    lhs = float(np.sum(gA * E))
    rhs = float(np.sum(G * L))
    assert abs(lhs - rhs) <= 1e-12 * abs(rhs)


def test_gradient_vs_central_differences_fp64(ps):
    n, m, s, sigma = 48, 18, 5, 2
    A = _rand(n, 3.0, 7)
    g = np.random.default_rng(8)
    G = g.standard_normal((n, n))
    gA = to_np(ps.ps_expm_backward(to_dev(A), to_dev(G), m, s=s, sigma=sigma))
    c = coeffs.taylor_exp(m)
    h = 1e-3
    for k in range(3):
        E = g.standard_normal((n, n))
        E /= metrics.norm1(E)            # unit direction: h E is a small step, truncation O(h^2)
        fd = (np.sum(G * oracle.expm_ps_f64(A + h * E, c, s, sigma)) -
              np.sum(G * oracle.expm_ps_f64(A - h * E, c, s, sigma))) / (2 * h)
        an = float(np.sum(gA * E))
        assert abs(fd - an) <= 1e-5 * abs(an), (fd, an)


def test_autograd_function(ps):
    import torch
    n = 5
    A = torch.tensor(_rand(n, 1.0, 9), dtype=torch.float64, device="cuda:0", requires_grad=True)
    f = lambda X: ps.expm(X, 10, s=3, sigma=1, mode="fixed")
    assert torch.autograd.gradcheck(f, (A,), eps=1e-6, atol=1e-8, rtol=1e-6)
    G = torch.randn(n, n, dtype=torch.float64, device="cuda:0")
    (ps.expm(A, 10, s=3, sigma=1, mode="mixed") * G).sum().backward()
    want = ps.ps_expm_backward(A.detach(), G, 10, s=3, sigma=1, mode="mixed")
    assert torch.equal(A.grad, want)


# ---------------------------------------------------------------- mixed tiers
def _tiers(ps, A, m, s, sigma, **kw):
    """The forward plan's tiers of Horner steps 1..first_step."""
    _, rep = ps.ps_expm(to_dev(A), m, s=s, sigma=sigma, mode="mixed", report=True, **kw)
    return rep["tier"][1:rep["first_step"] + 1]


@pytest.mark.parametrize("n,m,s,sigma,t", [
    (17, 18, 5, 2, 3.0), (64, 30, 6, 0, 0.25), (100, 30, 6, 3, 6.0), (130, 16, 4, 0, 0.5), (70, 40, 7, 1, 1.0),
])
def test_gradient_mixed_fp64_vs_oracle(ps, n, m, s, sigma, t):
    """Reverse Horner step i in forward step i's tier: the gradient stays
    within the FP64 target's tolerance of the block-triangular oracle."""
    A = _rand(n, t, 40 + n)
    G = np.random.default_rng(50 + n).standard_normal((n, n))
    c = coeffs.taylor_exp(m)
    gh, gl = oracle.expm_grad_dd(A, G, c, sigma)
    tiers = _tiers(ps, A, m, s, sigma)
    fixed = to_np(ps.ps_expm_backward(to_dev(A), to_dev(G), m, s=s, sigma=sigma))
    out = []
    for rec in (False, True):
        gA = to_np(ps.ps_expm_backward(to_dev(A), to_dev(G), m, s=s, sigma=sigma, recompute=rec, mode="mixed"))
        err = metrics.rel_err_1(gA, gh, gl)
        print("n=%d tiers %s mixed grad rel err %.3e (fixed %.3e)" % (n, tiers, err, metrics.rel_err_1(fixed, gh, gl)))
        assert err <= 1e-12, (rec, tiers, err)
        out.append(gA)
    assert np.array_equal(out[0], out[1])
    # the tiered products ran: any lower tier changes the bits
    if any(tt != 0 for tt in tiers):
        assert not np.array_equal(out[0], fixed)


def test_gradient_mixed_uses_low_tiers(ps):
    """A small ||X||: the plan takes later steps down to BF16/FP8."""
    n, m, s, sigma = 96, 30, 6, 0
    A = _rand(n, 0.1, 3)
    assert max(_tiers(ps, A, m, s, sigma)) >= 2


def test_gradient_mixed_with_only_the_working_tier_is_the_fixed_gradient(ps):
    n, m, s, sigma = 80, 18, 5, 1
    A = _rand(n, 2.0, 11)
    G = np.random.default_rng(12).standard_normal((n, n))
    a = to_np(ps.ps_expm_backward(to_dev(A), to_dev(G), m, s=s, sigma=sigma))
    b = to_np(ps.ps_expm_backward(to_dev(A), to_dev(G), m, s=s, sigma=sigma, mode="mixed", tier_mask=1))
    assert np.array_equal(a, b)


def test_gradient_forced_tiers(ps):
    """Every reverse Horner product forced into one tier (the forward plan
    overridden) on p(x) = sum_{k<=16} x^k with ||A||_1 = 1, where every block
    weighs about the same, so a wrong product would show at O(1): the error
    grows with the tier's unit roundoff and stays within a few of them."""
    n, m, s, sigma = 72, 16, 4, 0
    A = _rand(n, 1.0, 21)
    G = np.random.default_rng(22).standard_normal((n, n))
    c = [1.0] * (m + 1)
    gh, gl = oracle.expm_grad_dd(A, G, c, sigma)
    e64 = metrics.rel_err_1(to_np(ps.ps_expm_backward(to_dev(A), to_dev(G), m, s=s, sigma=sigma, coef=c)), gh, gl)
    errs = [e64]
    for tier, u in ((1, 2.0 ** -24), (2, 2.0 ** -8), (3, 2.0 ** -4)):
        ov = [0] + [tier] * (m // s)
        gA = to_np(ps.ps_expm_backward(to_dev(A), to_dev(G), m, s=s, sigma=sigma, coef=c, mode="mixed",
                                       tier_override=ov))
        err = metrics.rel_err_1(gA, gh, gl)
        print("forced tier %d: grad rel err %.3e (%.3g u), FP64 %.3e" % (tier, err, err / u, e64))
        assert err <= 4 * u, (tier, err)
        errs.append(err)
    # each lower tier moves the result further from the oracle
    assert 10 * errs[0] < errs[1] < errs[2] < errs[3], errs


def test_grad_batch_512_fp32(ps):
    """64 FP32 matrices of order 512 with N(0,1)/sqrt(n) entries, upstream
    gradients N(0,1), Taylor m = 18, s = 5, sigma = ceil(log2 ||A||_1):
    two sampled matrices against the block-triangular oracle on sampled
    columns, and one central difference (h = 1e-3, FP64 oracle forward)."""
    import torch
    from paper_2312_17396_amd import inputs
    A, G = inputs.grad_batch_512()
    norms = [metrics.norm1(a) for a in A]
    sigma = inputs.squarings_for(max(norms))
    At = torch.tensor(A, device="cuda:0")
    Gt = torch.tensor(G, device="cuda:0")
    gA = to_np(ps.ps_expm_backward(At, Gt, 18, s=5, sigma=sigma))
    gM = to_np(ps.ps_expm_backward(At, Gt, 18, s=5, sigma=sigma, mode="mixed"))
    assert np.all(np.isfinite(gA)) and np.all(np.isfinite(gM))
    c32 = [float(np.float32(x)) for x in coeffs.taylor_exp(18)]
    for b in (0, 37):
        Ab = A[b].astype(np.float64)
        Gb = G[b].astype(np.float64)
        cols = sample_cols(512, 3, seed=b)
        gh, gl = oracle.expm_grad_dd(Ab, Gb, c32, sigma, cols=cols)
        errs = []
        for g in (gA, gM):
            D = (g[b][:, cols] - gh) - gl
            errs.append(float(np.max(np.sum(np.abs(D), 0)) / np.max(np.sum(np.abs(gh), 0))))
        print("b=%d sigma=%d grad rel err fixed %.3e mixed %.3e" % (b, sigma, errs[0], errs[1]))
        # the backward tolerance 1e-5 for FP32, and equal accuracy with the
        # tiers in both passes
        assert errs[0] <= 1e-5, errs
        assert errs[1] <= max(1e-5, 2 * errs[0]), errs
    g = np.random.default_rng(1)
    E = g.standard_normal((512, 512))
    E /= metrics.norm1(E)
    h = 1e-3
    Ab, Gb = A[0].astype(np.float64), G[0].astype(np.float64)
    fd = (np.sum(Gb * oracle.expm_ps_f64(Ab + h * E, c32, 5, sigma)) -
          np.sum(Gb * oracle.expm_ps_f64(Ab - h * E, c32, 5, sigma))) / (2 * h)
    an = float(np.sum(gA[0] * E))
    assert abs(fd - an) <= 1e-4 * abs(an), (fd, an)
