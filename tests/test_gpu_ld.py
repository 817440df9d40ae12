"""Leading dimensions larger than the order, and batch strides larger than
one matrix, through the C ABI.  Each input's padding holds NaN (a kernel that
read it into a result would show it) and each output's padding a sentinel that
must survive.  Every result equals, bit for bit, the same call on the
contiguous matrix (ld = n): the entry points read and write only the n x n
part, whether the tiles take the whole-tile vector loads (n a multiple of 64
and ld even) or the guarded loads (ld odd or n ragged)."""
import ctypes

import numpy as np
import pytest

from oracle import coeffs

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
SENT = 12345.0


@pytest.fixture(scope="module")
def ps():
    import paper_2312_17396_amd as ps
    ps.lib()
    return ps


def _tdt(dt):
    import torch
    return torch.float64 if dt == "f64" else torch.float32


def _mat(n, t, seed):
    G = np.random.default_rng(seed).standard_normal((n, n))
    return G * (t / np.abs(G).sum(axis=0).max())


def _buf(mats, ld, stride, dt, fill):
    """one flat device buffer holding column-major matrices with leading
    dimension ld at element offsets b * stride; everything else is `fill`"""
    import torch
    n = mats[0].shape[0]
    T = torch.full((len(mats) * stride,), fill, dtype=_tdt(dt), device=DEV)
    for b, M in enumerate(mats):
        v = T[b * stride: b * stride + n * ld].view(n, ld)
        v[:, :n] = torch.tensor(np.ascontiguousarray(M.T), dtype=_tdt(dt))
    return T


def _get(T, b, n, ld, stride):
    return T[b * stride: b * stride + n * ld].view(n, ld)[:, :n]


def _padding_intact(T, nb, n, ld, stride):
    import torch
    mask = torch.ones_like(T, dtype=torch.bool)
    for b in range(nb):
        mask[b * stride: b * stride + n * ld].view(n, ld)[:, :n] = False
    return bool((T[mask] == SENT).all())


def _ws(ps, nbytes):
    return ps._workspace(nbytes, DEV)


def _p(T):
    return ctypes.c_void_p(T.data_ptr())


def _ok(ps, st):
    assert st == 0, ps.lib().ps_last_error().decode()


CASES = [(128, 130, "f64"), (128, 131, "f64"), (100, 103, "f64"), (576, 578, "f64"),
         (128, 132, "f32"), (128, 129, "f32"), (100, 102, "f32")]


@pytest.mark.parametrize("n,ld,dt", CASES)
def test_expm_ld(ps, n, ld, dt):
    import torch
    L = ps.lib()
    m, s, sigma = 18, 5, 2
    M = _mat(n, 3.0, n + ld)
    code = 0 if dt == "f64" else 1
    o, _k = ps._opts("mixed")
    nb = ctypes.c_size_t()
    _ok(ps, L.ps_workspace_size(code, n, m, s, sigma, ctypes.byref(nb)))
    outs = []
    for lda, lde in ((n, n), (ld, ld + 1)):
        A = _buf([M], lda, lda * n, dt, float("nan") if lda > n else 0.0)
        E = _buf([np.zeros((n, n))], lde, lde * n, dt, SENT)
        ws, wsp, wsb = _ws(ps, nb.value)
        _ok(ps, L.ps_expm(code, n, _p(A), lda, None, m, s, sigma, _p(E), lde, ctypes.byref(o), None, wsp, wsb,
                          ps._stream_ptr(DEV)))
        torch.cuda.synchronize()
        assert _padding_intact(E, 1, n, lde, lde * n)
        outs.append(_get(E, 0, n, lde, lde * n).clone())
    assert torch.equal(outs[0], outs[1])
    assert bool(torch.isfinite(outs[0]).all())


@pytest.mark.parametrize("n,ld,dt", [(128, 131, "f64"), (100, 102, "f32")])
def test_strided_batched_ld_and_stride(ps, n, ld, dt):
    import torch
    L = ps.lib()
    m, s, sigma, nbat = 18, 4, 1, 3
    mats = [_mat(n, 2.0 + b, 7 * b + n) for b in range(nbat)]
    code = 0 if dt == "f64" else 1
    o, _k = ps._opts("mixed")
    nb = ctypes.c_size_t()
    _ok(ps, L.ps_workspace_size_strided(code, nbat, n, m, s, sigma, ctypes.byref(nb)))
    outs = []
    for lda, sa, lde, se in ((n, n * n, n, n * n), (ld, ld * n + 37, ld + 1, (ld + 1) * n + 11)):
        A = _buf(mats, lda, sa, dt, float("nan") if lda > n else 0.0)
        E = _buf([np.zeros((n, n))] * nbat, lde, se, dt, SENT)
        ws, wsp, wsb = _ws(ps, nb.value)
        _ok(ps, L.ps_expm_strided_batched(code, nbat, n, _p(A), lda, sa, None, m, s, sigma, _p(E), lde, se,
                                          ctypes.byref(o), None, wsp, wsb, ps._stream_ptr(DEV)))
        torch.cuda.synchronize()
        assert _padding_intact(E, nbat, n, lde, se)
        outs.append([_get(E, b, n, lde, se).clone() for b in range(nbat)])
    for b in range(nbat):
        assert torch.equal(outs[0][b], outs[1][b]), b


def test_uneven_batched_ld(ps):
    import torch
    L = ps.lib()
    ns = [40, 64, 100, 8]
    m = 18
    mats = [_mat(n, 1.5, n) for n in ns]
    k = len(ns)
    o, _k = ps._opts("mixed")
    n_arr = (ctypes.c_int32 * k)(*ns)
    sg = (ctypes.c_int32 * k)(0, 1, 2, 0)
    nb = ctypes.c_size_t()
    _ok(ps, L.ps_workspace_size_batched(0, k, n_arr, m, None, ctypes.byref(nb)))
    res = []
    for pad in (0, 1):
        As, Es, lda, lde = [], [], [], []
        for b, n in enumerate(ns):
            la, le = (n + 3 * pad, n + 2 * pad + (b & 1) * pad)
            As.append(_buf([mats[b]], la, la * n, "f64", float("nan") if pad else 0.0))
            Es.append(_buf([np.zeros((n, n))], le, le * n, "f64", SENT))
            lda.append(la)
            lde.append(le)
        ws, wsp, wsb = _ws(ps, nb.value)
        _ok(ps, L.ps_expm_batched(0, k, n_arr, (ctypes.c_void_p * k)(*[a.data_ptr() for a in As]),
                                  (ctypes.c_int64 * k)(*lda), None, m, None, sg,
                                  (ctypes.c_void_p * k)(*[e.data_ptr() for e in Es]), (ctypes.c_int64 * k)(*lde),
                                  ctypes.byref(o), None, wsp, wsb, ps._stream_ptr(DEV)))
        torch.cuda.synchronize()
        for b, n in enumerate(ns):
            assert _padding_intact(Es[b], 1, n, lde[b], lde[b] * n)
        res.append([_get(Es[b], 0, n, lde[b], lde[b] * n).clone() for b, n in enumerate(ns)])
    for b in range(k):
        assert torch.equal(res[0][b], res[1][b]), ns[b]


@pytest.mark.parametrize("n", [128, 100])
def test_eval_multi_ld(ps, n):
    import torch
    L = ps.lib()
    p, q = coeffs.pade_exp(13, 13)
    M = _mat(n, 2.0, n)
    o, _k = ps._opts("mixed")
    degs = (ctypes.c_int * 2)(13, 13)
    nb = ctypes.c_size_t()
    _ok(ps, L.ps_workspace_size_multi(0, n, 2, degs, 4, 0, ctypes.byref(nb)))
    cp, cq = ps._darr(p), ps._darr(q)
    cptrs = (ctypes.POINTER(ctypes.c_double) * 2)(ctypes.cast(cp, ctypes.POINTER(ctypes.c_double)),
                                                  ctypes.cast(cq, ctypes.POINTER(ctypes.c_double)))
    res = []
    for lda, ldp in ((n, (n, n)), (n + 3, (n + 2, n + 5))):
        A = _buf([M], lda, lda * n, "f64", float("nan") if lda > n else 0.0)
        Ps = [_buf([np.zeros((n, n))], l, l * n, "f64", SENT) for l in ldp]
        ws, wsp, wsb = _ws(ps, nb.value)
        _ok(ps, L.ps_eval_multi(0, n, _p(A), lda, 2, cptrs, degs, 4, 0,
                                (ctypes.c_void_p * 2)(*[t.data_ptr() for t in Ps]), (ctypes.c_int64 * 2)(*ldp),
                                ctypes.byref(o), None, wsp, wsb, ps._stream_ptr(DEV)))
        torch.cuda.synchronize()
        for t, l in zip(Ps, ldp):
            assert _padding_intact(t, 1, n, l, l * n)
        res.append([_get(t, 0, n, l, l * n).clone() for t, l in zip(Ps, ldp)])
    assert torch.equal(res[0][0], res[1][0]) and torch.equal(res[0][1], res[1][1])


@pytest.mark.parametrize("n", [128, 100])
def test_solve_and_pade_ld(ps, n):
    import torch
    L = ps.lib()
    rng = np.random.default_rng(n)
    Q = rng.standard_normal((n, n)) + n ** 0.5 * np.eye(n)
    P = rng.standard_normal((n, n))
    nb = ctypes.c_size_t()
    _ok(ps, L.ps_workspace_size_solve(0, n, ctypes.byref(nb)))
    res = []
    for ldq, ldp in ((n, n), (n + 3, n + 2)):
        Qd = _buf([Q], ldq, ldq * n, "f64", SENT)        # in/out: its padding must survive too
        Pd = _buf([P], ldp, ldp * n, "f64", SENT)
        piv = torch.full((n,), -7, dtype=torch.int32, device=DEV)
        info = ctypes.c_int(-1)
        ws, wsp, wsb = _ws(ps, nb.value)
        _ok(ps, L.ps_solve(0, n, _p(Qd), ldq, n, _p(Pd), ldp, _p(piv), ctypes.byref(info), wsp, wsb,
                           ps._stream_ptr(DEV)))
        torch.cuda.synchronize()
        assert info.value == 0
        assert _padding_intact(Qd, 1, n, ldq, ldq * n) and _padding_intact(Pd, 1, n, ldp, ldp * n)
        res.append((_get(Qd, 0, n, ldq, ldq * n).clone(), _get(Pd, 0, n, ldp, ldp * n).clone(), piv.clone()))
    for a, b in zip(res[0], res[1]):
        assert torch.equal(a, b)
    # exp in the Pade form
    M = _mat(n, 4.0, n + 1)
    o, _k = ps._opts("mixed")
    _ok(ps, L.ps_workspace_size_pade(0, n, 13, 4, 2, ctypes.byref(nb)))
    outs = []
    for lda, lde in ((n, n), (n + 2, n + 3)):
        A = _buf([M], lda, lda * n, "f64", float("nan") if lda > n else 0.0)
        E = _buf([np.zeros((n, n))], lde, lde * n, "f64", SENT)
        ws, wsp, wsb = _ws(ps, nb.value)
        _ok(ps, L.ps_expm_pade(0, n, _p(A), lda, 13, 4, 2, _p(E), lde, ctypes.byref(o), None, wsp, wsb,
                               ps._stream_ptr(DEV)))
        torch.cuda.synchronize()
        assert _padding_intact(E, 1, n, lde, lde * n)
        outs.append(_get(E, 0, n, lde, lde * n).clone())
    assert torch.equal(outs[0], outs[1])


@pytest.mark.parametrize("recompute", [0, 1])
def test_backward_ld_and_stride(ps, recompute):
    import torch
    L = ps.lib()
    n, m, s, sigma, nbat = 128, 18, 5, 2, 2
    mats = [_mat(n, 3.0, 40 + b) for b in range(nbat)]
    Gs = [np.random.default_rng(50 + b).standard_normal((n, n)) for b in range(nbat)]
    o, _k = ps._opts("mixed")
    nb = ctypes.c_size_t()
    _ok(ps, L.ps_workspace_size_backward(0, nbat, n, m, s, sigma, recompute, ctypes.byref(nb)))
    res = []
    for pad in (0, 1):
        la, lg, lo = n + 3 * pad, n + 2 * pad, n + 1 * pad
        sa, sg, so = la * n + 5 * pad, lg * n + 64 * pad, lo * n + 3 * pad
        A = _buf(mats, la, sa, "f64", float("nan") if pad else 0.0)
        G = _buf(Gs, lg, sg, "f64", float("nan") if pad else 0.0)
        gA = _buf([np.zeros((n, n))] * nbat, lo, so, "f64", SENT)
        ws, wsp, wsb = _ws(ps, nb.value)
        _ok(ps, L.ps_expm_backward(0, nbat, n, _p(A), la, sa, _p(G), lg, sg, None, m, s, sigma, _p(gA), lo, so,
                                   recompute, ctypes.byref(o), wsp, wsb, ps._stream_ptr(DEV)))
        torch.cuda.synchronize()
        assert _padding_intact(gA, nbat, n, lo, so)
        res.append([_get(gA, b, n, lo, so).clone() for b in range(nbat)])
    for b in range(nbat):
        assert torch.equal(res[0][b], res[1][b]), b
