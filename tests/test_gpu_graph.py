"""hipGraph capture of single-matrix evaluations: ps_expm issues no host
synchronisation, allocation or memset on its stream (the workspace is the
caller's), so a step of several evaluations forked over streams can be
captured once and replayed.  Every replay, with eager work and
synchronisations in between, must equal the eager result bitwise, and the
eager result must match the double-double oracle."""
import numpy as np
import pytest

import oracle
from oracle import coeffs, metrics

from helpers import to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ps():
    import paper_2312_17396_amd as ps
    ps.lib()
    return ps


def _dense(n, t, seed):
    G = np.random.default_rng(seed).standard_normal((n, n))
    return G * (t / metrics.norm1(G.T))


@pytest.mark.parametrize("mode", ["fixed", "mixed"])
def test_forked_graph_replays_match_eager(ps, mode):
    import torch
    dev = torch.device("cuda:0")
    m, s = 30, 6
    cases = [(200, 0.5, 0), (130, 5.0, 3), (64, 1.0, 0), (257, 30.0, 5)]
    mats = [to_dev(_dense(n, t, 40 + k)) for k, (n, t, _) in enumerate(cases)]
    sig = [c[2] for c in cases]
    outs = [torch.empty_like(a) for a in mats]
    wss = [ps.expm_workspace(a, m, s, sg) for a, sg in zip(mats, sig)]
    streams = [torch.cuda.Stream(device=dev) for _ in mats]

    def eager():
        for a, o, w, sg in zip(mats, outs, wss, sig):
            ps.ps_expm(a, m, s=s, sigma=sg, mode=mode, out=o, workspace=w)

    def forked():
        cur = torch.cuda.current_stream(dev)
        for st in streams:
            st.wait_stream(cur)
        for a, o, w, sg, st in zip(mats, outs, wss, sig, streams):
            with torch.cuda.stream(st):
                ps.ps_expm(a, m, s=s, sigma=sg, mode=mode, out=o, workspace=w)
        for st in streams:
            cur.wait_stream(st)

    eager()
    torch.cuda.synchronize()
    ref = [o.clone() for o in outs]
    c = coeffs.taylor_exp(m)
    for (n, t, sg), A, E in zip(cases, mats, ref):
        Eh, El = oracle.expm_dd(to_np(A), c, sg)
        assert metrics.rel_err_1(to_np(E), Eh, El) <= 1e-13, (n, t, sg)
    side = torch.cuda.Stream(device=dev)
    side.wait_stream(torch.cuda.current_stream(dev))
    with torch.cuda.stream(side):
        forked()
    torch.cuda.current_stream(dev).wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        forked()
    for _ in range(4):
        for o in outs:
            o.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        for o, r in zip(outs, ref):
            assert torch.equal(o, r)
        eager()                      # eager work between the replays
        torch.cuda.synchronize()
    del g
