"""The size-class schedule tuner of the uneven batch: every schedule (the
one-branch default, the tuned one, and a forced one branch per class) gives
the same bits, eagerly and as a replayed graph; the tuned schedule lands in
the cache under this batch's key and survives a JSON round trip."""
import json

import numpy as np
import pytest

from oracle import metrics
from paper_2312_17396_amd import inputs

from helpers import to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ps():
    import paper_2312_17396_amd as ps
    ps.lib()
    return ps


def _batch(count=384, seed=3):
    import torch
    g = np.random.default_rng(seed)
    mats, sig = [], []
    for k in range(count):
        n = int(8 * g.integers(1, 33))
        t = float(g.uniform(0.05, 4.0))
        G = g.standard_normal((n, n))
        mats.append(torch.tensor(G * (t / metrics.norm1(G)), dtype=torch.float32, device="cuda:0"))
        sig.append(inputs.squarings_for(t))
    return mats, sig


@pytest.mark.parametrize("mode", ["fixed", "mixed"])
def test_schedules_give_the_same_bits(ps, mode, tmp_path):
    import torch
    mats, sig = _batch()
    ps.autotune_clear()
    ref = [to_np(e) for e in ps.ps_expm_batched(mats, 18, sigma=sig, mode=mode)]
    res = ps.batched_tune(mats, 18, sigma=sig, mode=mode, reps=2)
    assert len(res["ms"]) == 8 and all(t > 0 for t in res["ms"])   # four classes: 2^3 groupings
    found, groups = ps.autotune_lookup(mats, 18)
    assert found and groups == res["groups"]
    tuned = ps.ps_expm_batched(mats, 18, sigma=sig, mode=mode)
    for a, b in zip(tuned, ref):
        assert np.array_equal(to_np(a), b)
    # one branch per class, forced through the cache file
    path = tmp_path / "c.json"
    ps.autotune_save(path)
    d = json.loads(path.read_text())
    for e in d["entries"]:
        e["groups"] = [0, 1, 2, 3]
    path.write_text(json.dumps(d))
    ps.autotune_clear()
    ps.autotune_load(path)
    assert ps.autotune_lookup(mats, 18) == (True, [0, 1, 2, 3])
    four = ps.ps_expm_batched(mats, 18, sigma=sig, mode=mode)
    g = ps.BatchedGraph(mats, 18, sigma=sig, mode=mode)
    for rep in range(3):
        outs = g.launch()
        torch.cuda.synchronize()
        _ = ps.ps_expm_batched(mats[:7], 18, sigma=sig[:7], mode="fixed")   # eager work between replays
        torch.cuda.synchronize()
        for a, b, c in zip(four, outs, ref):
            assert np.array_equal(to_np(a), c) and np.array_equal(to_np(b), c), rep
    g.close()
    ps.autotune_clear()
