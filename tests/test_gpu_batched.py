"""GPU parity of the batched path (many matrices of uneven order, one launch
per phase for all of them) against the single-matrix path and the CPU oracle, and of its
captured hipGraph against eager calls."""
import numpy as np
import pytest

import oracle
from oracle import coeffs, metrics
from oracle import plan as oplan
from paper_2312_17396_amd import inputs

from helpers import U32, relerr_cols, sample_cols, to_dev, to_np

pytestmark = pytest.mark.gpu

SIZES = [1, 7, 8, 16, 33, 64, 65, 100, 130, 200, 256]


@pytest.fixture(scope="module")
def ps():
    import paper_2312_17396_amd as ps
    ps.lib()
    return ps


def _mats(seed, sizes, dtype):
    import torch
    g = np.random.default_rng(seed)
    out, ts = [], []
    for n in sizes:
        t = float(g.uniform(0.05, 4.0))
        G = g.standard_normal((n, n))
        A = G * (t / metrics.norm1(G))
        if dtype == torch.float32:
            A = A.astype(np.float32).astype(np.float64)
        out.append(A)
        ts.append(t)
    return out, ts


@pytest.mark.parametrize("mode", ["fixed", "mixed"])
def test_batched_fp64_matches_oracle_and_single_path(ps, mode):
    import torch
    mats, ts = _mats(1, SIZES, torch.float64)
    sig = [inputs.squarings_for(t) for t in ts]
    E, reps = ps.ps_expm_batched([to_dev(A) for A in mats], 18, s=None, sigma=sig, mode=mode, report=True)
    c = coeffs.taylor_exp(18)
    for A, e, sg, rp in zip(mats, E, sig, reps):
        n = A.shape[0]
        Eh, El = oracle.expm_dd(A, c, sg)
        err = metrics.rel_err_1(to_np(e), Eh, El)
        assert err <= 1e-13, (n, err, rp)
        assert rp["s"] in (4, 5)
        # same kernels, same s: the grid path returns the same bits
        e1 = ps.ps_expm(to_dev(A), 18, s=rp["s"], sigma=sg, mode=mode)
        assert np.array_equal(to_np(e1), to_np(e)), n


def test_batched_fp32_equal_accuracy(ps):
    import torch
    mats, ts = _mats(2, SIZES, torch.float32)
    sig = [inputs.squarings_for(t) for t in ts]
    c32 = [float(np.float32(x)) for x in coeffs.taylor_exp(18)]
    dev = [to_dev(A, torch.float32) for A in mats]
    Ef = ps.ps_expm_batched(dev, 18, sigma=sig, mode="fixed")
    Em = ps.ps_expm_batched(dev, 18, sigma=sig, mode="mixed")
    for A, ef, em, sg in zip(mats, Ef, Em, sig):
        Eh, El = oracle.expm_dd(A, c32, sg)
        e_f = metrics.rel_err_1(to_np(ef), Eh, El)
        e_m = metrics.rel_err_1(to_np(em), Eh, El)
        assert e_f <= 2 ** sg * 4 * A.shape[0] * U32
        assert e_m <= max(1e-6, 2 * e_f), (A.shape[0], e_f, e_m)


def test_batched_graph_replays_match_eager(ps):
    import torch
    mats, ts = _mats(3, SIZES * 3, torch.float32)
    sig = [inputs.squarings_for(t) for t in ts]
    dev = [to_dev(A, torch.float32) for A in mats]
    eager = [to_np(e) for e in ps.ps_expm_batched(dev, 18, sigma=sig, mode="mixed")]
    gr = ps.BatchedGraph(dev, 18, sigma=sig, mode="mixed")
    for rep in range(4):
        outs = gr.launch()
        torch.cuda.synchronize()
        # eager work between replays
        _ = ps.ps_expm_batched(dev[:5], 18, sigma=sig[:5], mode="fixed")
        torch.cuda.synchronize()
        for a, b in zip(outs, eager):
            assert np.array_equal(to_np(a), b), rep
    gr.close()


def test_uneven_4096_batch_fp32(ps):
    """The 4096-matrix uneven batch (n in {8, ..., 256}, ||A||_1 ~ U[0.05, 4],
    Taylor m = 18, FP32, s chosen per matrix), plain and mixed: every result
    finite; on every 8th matrix (512 of them; all columns for n <= 64, eight
    sampled columns above) the plain evaluation within 2^sigma 4 n u32 of the
    oracle and the mixed one at equal accuracy, max(1e-6, 2 err_plain)."""
    import torch
    mats, ts = inputs.batch_uneven()
    sig = [inputs.squarings_for(t) for t in ts]
    dev = [torch.tensor(A, dtype=torch.float32, device="cuda:0") for A in mats]
    Ef = ps.ps_expm_batched(dev, 18, sigma=sig, mode="fixed")
    Em, reps = ps.ps_expm_batched(dev, 18, sigma=sig, mode="mixed", report=True)
    torch.cuda.synchronize()
    assert all(bool(torch.isfinite(e).all()) for e in Em + Ef)
    c32 = [float(np.float32(x)) for x in coeffs.taylor_exp(18)]
    checked, worst = 0, 0.0
    for b in range(0, len(mats), 8):
        A = mats[b].astype(np.float32).astype(np.float64)
        n = A.shape[0]
        cols = list(range(n)) if n <= 64 else sample_cols(n, 8, seed=int(b))
        Wh, Wl = oracle.expm_apply_dd(A, c32, sig[b], np.eye(n)[:, cols])
        e_f = relerr_cols(to_np(Ef[b])[:, cols], Wh, Wl)
        e_m = relerr_cols(to_np(Em[b])[:, cols], Wh, Wl)
        assert e_f <= 2 ** sig[b] * 4 * n * U32, (b, n, e_f)
        assert e_m <= max(1e-6, 2 * e_f), (b, n, sig[b], e_f, e_m, reps[b])
        checked += 1
        worst = max(worst, e_m)
    assert checked == 512
    print("uneven batch: %d matrices checked, worst mixed error %.2e" % (checked, worst))
