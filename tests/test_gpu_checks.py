"""opts.check_finite on the device: finite inputs give the same bits as
without the check; a NaN or infinity in an input is reported as
PS_ERR_NONFINITE before anything is evaluated (the output keeps its previous
contents); a result that overflows is reported after the evaluation.  Also the
report's modelled cost (C_r as a saving, M_low) against ps_model_cost."""
import numpy as np
import pytest

from oracle import coeffs

from helpers import to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ps():
    import paper_2312_17396_amd as ps
    ps.lib()
    return ps


def _mat(n, t, seed):
    G = np.random.default_rng(seed).standard_normal((n, n))
    return G * (t / np.abs(G).sum(axis=1).max())


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_check_finite_same_bits_and_rejects(ps, dt):
    import torch
    tdt = torch.float64 if dt == "f64" else torch.float32
    A = to_dev(_mat(200, 3.0, 1), tdt)
    E0 = ps.ps_expm(A, 18, s=5, sigma=2, mode="mixed")
    E1 = ps.ps_expm(A, 18, s=5, sigma=2, mode="mixed", check_finite=True)
    assert torch.equal(E0, E1)
    for bad in (float("nan"), float("inf"), -float("inf")):
        B = A.clone()
        B[17, 3] = bad
        out = torch.full_like(A, 7.0)
        with pytest.raises(ps.PSError, match="non-finite"):
            ps.ps_expm(B, 18, s=5, sigma=2, mode="mixed", check_finite=True, out=out)
        torch.cuda.synchronize()
        assert bool((out == 7.0).all())          # nothing was evaluated
        # without the check the NaN propagates
        assert not bool(torch.isfinite(ps.ps_expm(B, 18, s=5, sigma=2, mode="mixed")).all())


def test_check_finite_result_overflow(ps):
    import torch
    A = to_dev(720.0 * np.eye(64))                # e^720 overflows double
    with pytest.raises(ps.PSError, match="result"):
        ps.ps_expm(A, 18, s=5, sigma=10, check_finite=True)
    E = ps.ps_expm(to_dev(700.0 * np.eye(64)), 18, s=5, sigma=10, check_finite=True)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(E).all())


def test_check_finite_other_entry_points(ps):
    import torch
    A = _mat(96, 2.0, 2)
    A[5, 70] = np.nan
    with pytest.raises(ps.PSError, match="non-finite"):
        ps.ps_eval(to_dev(A), coeffs.taylor_exp(12), s=4, mode="mixed", check_finite=True)
    with pytest.raises(ps.PSError, match="non-finite"):
        ps.ps_expm_noalloc(to_dev(A), 12, s=4, check_finite=True)
    L = ps.lib()
    # strided batch: the second matrix holds the NaN
    Ab = torch.stack([to_dev(_mat(96, 2.0, 3)), to_dev(A)])
    import ctypes
    o, _k = ps._opts("mixed", check_finite=True)
    nb = ctypes.c_size_t()
    assert L.ps_workspace_size_strided(0, 2, 96, 12, 4, 1, ctypes.byref(nb)) == 0
    ws, wsp, wsb = ps._workspace(nb.value, "cuda:0")
    Eb = torch.empty_like(Ab)
    st = L.ps_expm_strided_batched(0, 2, 96, Ab.data_ptr(), 96, 96 * 96, None, 12, 4, 1, Eb.data_ptr(), 96,
                                   96 * 96, ctypes.byref(o), None, wsp, wsb, ps._stream_ptr("cuda:0"))
    assert st == -4 and b"input matrix 1" in L.ps_last_error()
    # Pade exp and automatic scaling
    assert L.ps_workspace_size_pade(0, 96, 13, 4, 1, ctypes.byref(nb)) == 0
    ws, wsp, wsb = ps._workspace(nb.value, "cuda:0")
    Ad = to_dev(A)
    E = torch.empty_like(Ad)
    st = L.ps_expm_pade(0, 96, Ad.data_ptr(), 96, 13, 4, 1, E.data_ptr(), 96, ctypes.byref(o), None, wsp, wsb,
                        ps._stream_ptr("cuda:0"))
    assert st == -4
    p, q = coeffs.pade_exp(13, 13)
    outs = ps.ps_eval_multi(to_dev(_mat(96, 2.0, 4)), [p, q], s=4, mode="mixed")
    assert all(bool(torch.isfinite(t).all()) for t in outs)


def test_report_cost_model(ps):
    A = to_dev(_mat(576, 1.0, 5))
    _, rep = ps.ps_expm(A, 30, s=6, sigma=0, mode="mixed", report=True)
    cr, ml = ps.model_cost(rep["tier"], 6)
    assert rep["cost_saving"] == cr and rep["m_low"] == ml
    # some products below FP64: a positive saving; fixed mode: none
    assert cr > 0 and ml > 0
    _, rep0 = ps.ps_expm(A, 30, s=6, sigma=0, mode="fixed", report=True)
    assert rep0["cost_saving"] == 0.0 and rep0["m_low"] == 0.0
