"""The no-allocation entry point ps_expm_noalloc, called through the C ABI:
its results equal ps_expm's (same kernels, same workspace layout, so the same
bits) on two calls in a row, the second with a smaller input, for FP64 and
FP32 and both modes; sizes beyond the static scratch are rejected before any
device work, and the output is then left untouched."""
import ctypes

import numpy as np
import pytest

from helpers import to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ps():
    import paper_2312_17396_amd as ps
    ps.lib()
    return ps


def _dense(n, t, seed, dtype=np.float64):
    G = np.random.default_rng(seed).standard_normal((n, n))
    return (G * (t / np.abs(G).sum(axis=1).max())).astype(dtype)


def _noalloc(ps, A, m, s, sigma, mode, out=None):
    import torch
    n = A.shape[0]
    E = torch.full_like(A, float("nan")) if out is None else out
    o, _k = ps._opts(mode)
    rep = ps.ps_report()
    st = ps.lib().ps_expm_noalloc(ps._dtype_code(A), n, ctypes.c_void_p(A.data_ptr()), n, None, m, s, sigma,
                                  ctypes.c_void_p(E.data_ptr()), n, ctypes.byref(o), ctypes.byref(rep),
                                  ps._stream_ptr(A.device))
    return st, E, rep.to_dict()


@pytest.mark.parametrize("mode", ["fixed", "mixed"])
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_noalloc_equals_ps_expm_twice_shrinking(ps, mode, dt):
    import torch
    tdt = torch.float64 if dt == "f64" else torch.float32
    cases = [(1024 if dt == "f64" else 700, 30, 6, 3, 8.0, 1), (130, 16, 4, 1, 2.0, 2)]
    for n, m, s, sigma, t, seed in cases:          # second call: a smaller input
        A = to_dev(_dense(n, t, seed), tdt)
        st, E, rep = _noalloc(ps, A, m, s, sigma, mode)
        assert st == 0, ps.lib().ps_last_error().decode()
        E_ref, rep_ref = ps.ps_expm(A, m, s=s, sigma=sigma, mode=mode, report=True)
        torch.cuda.synchronize()
        assert torch.equal(E, E_ref), (n, m, s, sigma)
        assert rep["tier"] == rep_ref["tier"] and rep["normB"] == rep_ref["normB"]


def test_noalloc_rejects_sizes_beyond_the_scratch(ps):
    import torch
    A = torch.zeros((2048, 2048), dtype=torch.float64, device="cuda:0")
    st, E, _ = _noalloc(ps, A, 30, 6, 2, "mixed")
    torch.cuda.synchronize()
    assert st == -3                                  # PS_ERR_WORKSPACE
    assert "scratch" in ps.lib().ps_last_error().decode()
    assert bool(torch.isnan(E).all())                # nothing was written
    # the binding raises, and a fitting call afterwards still works
    with pytest.raises(ps.PSError):
        ps.ps_expm_noalloc(A, 30, s=6, sigma=2)
    B = to_dev(_dense(64, 1.0, 3))
    assert torch.equal(ps.ps_expm_noalloc(B, 16, s=4), ps.ps_expm(B, 16, s=4))
