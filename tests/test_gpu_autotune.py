"""The size-class schedule tuner of the uneven batch: every schedule (the
one-branch default, the tuned one, a forced one branch per class, and the
orders up to 64 evaluated whole by one workgroup per matrix) gives the same
bits, eagerly and as a replayed graph; the tuned schedule lands in the cache
under this batch's key and survives a JSON round trip."""
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
    # four classes: 2^3 groupings, and the 4 that give class 1 a branch of its
    # own again with that class on the one-workgroup kernel
    assert len(res["ms"]) == 12 and all(t > 0 for t in res["ms"])
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


def _key(mats, m):
    """the cache key of a batch (device architecture, dtype, degree, order of
    magnitude of each size class's matrix count)"""
    import torch
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    cnt = [0] * 5
    for a in mats:
        cnt[(a.shape[0] + 63) // 64] += 1
    dt = "f64" if mats[0].dtype == torch.float64 else "f32"
    return "%s|%s|m%d|%s" % (arch, dt, m, ",".join(str(c.bit_length()) for c in cnt[1:]))


def _force(ps, tmp_path, mats, m, groups, whole64):
    path = tmp_path / "force.json"
    path.write_text(json.dumps({"ps_autotune": 1, "entries": [
        {"key": _key(mats, m), "groups": groups, "whole64": whole64}]}))
    ps.autotune_clear()
    ps.autotune_load(path)
    assert ps.autotune_lookup(mats, m, whole64=True) == (True, groups, whole64)


@pytest.mark.parametrize("dtype", ["float32", "float64"])
@pytest.mark.parametrize("mode", ["fixed", "mixed"])
def test_whole64_gives_the_same_bits(ps, dtype, mode, tmp_path):
    """Orders 1..64 (one padded tile) evaluated whole by one workgroup per
    matrix: every phase in one launch, the same tile routines in the same
    order, so the same bits as the per-phase launches, for fixed and chosen
    block sizes (s = 1 included) and 0..3 squarings; alone, next to a class of
    larger orders in its own branch, and as replayed graphs."""
    import torch
    g = np.random.default_rng(11)
    tdt = getattr(torch, dtype)
    orders = [1, 2, 3, 7, 8, 9, 16, 31, 32, 33, 47, 63, 64]
    mats, sig, sv = [], [], []
    for k in range(3 * len(orders)):
        n = orders[k % len(orders)]
        t = float(g.uniform(0.05, 4.0))
        G = g.standard_normal((n, n))
        mats.append(torch.tensor(G * (t / metrics.norm1(G)), dtype=tdt, device="cuda:0"))
        sig.append(int(k % 4))
        sv.append([0, 1, 2, 4, 5][k % 5])
    ps.autotune_clear()
    ref = [to_np(e) for e in ps.ps_expm_batched(mats, 18, s=sv, sigma=sig, mode=mode)]
    _force(ps, tmp_path, mats, 18, [0, 0, 0, 0], 1)
    whole = ps.ps_expm_batched(mats, 18, s=sv, sigma=sig, mode=mode)
    for k, (a, b) in enumerate(zip(whole, ref)):
        assert np.array_equal(to_np(a), b), (k, mats[k].shape[0], sv[k], sig[k])
    gr = ps.BatchedGraph(mats, 18, s=sv, sigma=sig, mode=mode)
    for rep in range(3):
        outs = gr.launch()
        torch.cuda.synchronize()
        _ = ps.ps_expm_batched(mats[:5], 18, sigma=sig[:5], mode="fixed")   # eager work between replays
        torch.cuda.synchronize()
        for a, b in zip(outs, ref):
            assert np.array_equal(to_np(a), b), rep
    gr.close()
    # next to a class of orders 193..256 on the per-phase launches, in its own branch
    big = [torch.tensor(g.standard_normal((n, n)) / n, dtype=tdt, device="cuda:0") for n in (200, 256, 250)]
    mix, msig, ms = mats + big, sig + [1, 0, 2], sv + [0, 0, 0]
    ps.autotune_clear()
    ref2 = [to_np(e) for e in ps.ps_expm_batched(mix, 18, s=ms, sigma=msig, mode=mode)]
    _force(ps, tmp_path, mix, 18, [0, 1, 1, 1], 1)
    res2 = ps.ps_expm_batched(mix, 18, s=ms, sigma=msig, mode=mode)
    for a, b in zip(res2, ref2):
        assert np.array_equal(to_np(a), b)
    # and in the same branch as that class (the one-workgroup launch first)
    _force(ps, tmp_path, mix, 18, [0, 0, 0, 0], 1)
    res3 = ps.ps_expm_batched(mix, 18, s=ms, sigma=msig, mode=mode)
    for a, b in zip(res3, ref2):
        assert np.array_equal(to_np(a), b)
    ps.autotune_clear()
