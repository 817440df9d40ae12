"""CPU checks of the C-ABI library: it loads, exports every entry point that
include/ps.h declares, its host-only helpers agree with the oracle, and
argument validation rejects bad calls before any device work (no kernel is
launched in this file)."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from oracle import coeffs
from oracle import plan as oplan

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def ps():
    import paper_2312_17396_amd as ps
    if not os.path.exists(ps.LIBPATH):
        from paper_2312_17396_amd import build
        build.build()
    ps.lib()
    return ps


def declared_functions():
    src = open(os.path.join(ROOT, "include", "ps.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ps_[a-z0-9_]+)\s*\(", src)))


def test_header_symbols_exported(ps):
    names = declared_functions()
    assert len(names) >= 20
    L = ctypes.CDLL(ps.LIBPATH)
    for nm in names:
        assert hasattr(L, nm), nm
    assert set(names) == set(ps.exported_symbols())


def test_builtin_coefficients_match_exact_rationals(ps):
    assert ps.coef_taylor_exp(170) == coeffs.taylor_exp(170)
    assert ps.coef_taylor_cos(40) == coeffs.taylor_cos(40)
    for d in range(0, 31):
        p, q = ps.coef_pade_exp(d)
        P, Q = coeffs.pade_exp(d, d)
        assert p == P and q == Q, d


def test_host_planner_matches_oracle_planner(ps):
    rng = np.random.default_rng(5)
    for trial in range(400):
        r = int(rng.integers(0, 8))
        nb = list(np.exp(rng.uniform(-40, 3, r + 1)))
        if trial % 17 == 0:
            nb[0] = 0.0
        ny = float(np.exp(rng.uniform(-30, 2))) if trial % 13 else 0.0
        for wt in (0, 1, 2):   # dtype codes: FP64, FP32, double-double (working tier 4)
            mask = int(rng.integers(0, 16))
            allowed = [t for t in range(4) if (mask >> t) & 1] if mask else [0, 1, 2, 3]
            t_lib, u_lib, nu_lib = ps.ps_plan(nb, ny, dtype=wt, mode="mixed", tier_mask=mask)
            u_o, nu_o, t_o = oplan.plan(nb, ny, working_tier=4 if wt == 2 else wt, allowed=allowed)
            assert t_lib == t_o and nu_lib == nu_o, (nb, ny, wt, mask)
            assert np.allclose(u_lib, u_o, rtol=1e-15, atol=0) or all(
                (a == b) for a, b in zip(u_lib, u_o))


def test_fixed_mode_plan_is_working_precision(ps):
    t, u, nu = ps.ps_plan([1.0, 1e-9, 1e-20], 1e-3, mode="fixed")
    assert t == [0, 0, 0] and nu == 3


def test_workspace_sizes(ps):
    sz = ctypes.c_size_t()
    L = ps.lib()
    assert L.ps_workspace_size(0, 1024, 30, 6, 6, ctypes.byref(sz)) == 0
    n = 1024
    assert sz.value >= (5 + 5 + 2) * n * n * 8
    assert sz.value % 256 == 0
    small = ctypes.c_size_t()
    assert L.ps_workspace_size(1, 64, 16, 4, 0, ctypes.byref(small)) == 0
    assert 0 < small.value < sz.value


@pytest.mark.parametrize("args,code", [
    (dict(n=0), -1), (dict(m=-1), -1), (dict(s=7, m=5), -1), (dict(sigma=-1), -1), (dict(sigma=501), -1),
    (dict(lda=3, n=4), -1), (dict(dtype=7), -1), (dict(A=0), -1), (dict(alias=True), -2),
    (dict(ws_small=True), -3), (dict(ws_misaligned=True), -3), (dict(m=300), -1),
])
def test_argument_validation_before_device_work(ps, args, code):
    L = ps.lib()
    n = args.get("n", 4)
    m = args.get("m", 6)
    s = args.get("s", 0)
    sigma = args.get("sigma", 0)
    lda = args.get("lda", n)
    dtype = args.get("dtype", 0)
    A = args.get("A", 0x10000000)
    E = A if args.get("alias") else 0x20000000
    need = ctypes.c_size_t(1 << 30)
    ws = 0x40000010 if args.get("ws_misaligned") else 0x40000000
    wsb = 16 if args.get("ws_small") else (1 << 30)
    st = L.ps_expm(dtype, n, A, lda, None, m, s, sigma, E, n, None, None, ws, wsb, None)
    assert st == code, (st, L.ps_last_error())
    assert L.ps_last_error()


def test_unimplemented_entry_points_report_unsupported(ps):
    L = ps.lib()
    assert L.ps_batched_launch(None, None) in (-1, -5)


def test_theta_taylor_host_matches_oracle():
    from oracle import metrics
    import paper_2312_17396_amd as ps
    for dt, u in (("f64", 2.0 ** -53), ("f32", 2.0 ** -24)):
        for m in (0, 1, 2, 5, 10, 18, 30, 45, 60, 100, 170):
            a, b = ps.theta_taylor(m, dt), metrics.theta_taylor(m, u)
            assert abs(a - b) <= 1e-12 * b, (dt, m, a, b)
    with pytest.raises(ps.PSError):
        ps.theta_taylor(171)


def test_rule_names_checked_on_the_host():
    import paper_2312_17396_amd as ps
    o, _ = ps._opts("mixed", rule="apriori")
    assert o.rule == 1
    o, _ = ps._opts("mixed")
    assert o.rule == 0
    with pytest.raises(ps.PSError):
        ps._opts("mixed", rule="nonsense")


@pytest.mark.parametrize("args,code", [
    (dict(n=0), -1), (dict(n=9000), -5), (dict(dtype=2), -5), (dict(Q=0), -1), (dict(ldq=3, n=4), -1),
    (dict(nrhs=-1), -1), (dict(P=0), -1), (dict(ldp=2, n=4), -1), (dict(alias=True), -2),
    (dict(ws_small=True), -3), (dict(ws_misaligned=True), -3), (dict(piv_alias=True), -2),
])
def test_solve_argument_validation(ps, args, code):
    L = ps.lib()
    n = args.get("n", 4)
    Q = args.get("Q", 0x10000000)
    P = Q if args.get("alias") else args.get("P", 0x20000000)
    ws = 0x40000010 if args.get("ws_misaligned") else 0x40000000
    wsb = 16 if args.get("ws_small") else (1 << 30)
    piv = 0x40000000 if args.get("piv_alias") else 0x50000000
    st = L.ps_solve(args.get("dtype", 0), n, Q, args.get("ldq", n), args.get("nrhs", 3), P, args.get("ldp", n),
                    piv, None, ws, wsb, None)
    assert st == code, (st, L.ps_last_error())
    assert L.ps_last_error()


@pytest.mark.parametrize("args,code", [
    (dict(m=0), -1), (dict(m=61), -1), (dict(sigma=-1), -1), (dict(dtype=2), -5), (dict(n=9000), -5),
    (dict(alias=True), -2), (dict(ws_small=True), -3), (dict(A=0), -1), (dict(s=9, m=6), -1),
])
def test_expm_pade_argument_validation(ps, args, code):
    L = ps.lib()
    n = args.get("n", 4)
    A = args.get("A", 0x10000000)
    E = A if args.get("alias") and A else 0x20000000
    wsb = 16 if args.get("ws_small") else (1 << 34)
    st = L.ps_expm_pade(args.get("dtype", 0), n, A, n, args.get("m", 13), args.get("s", 0), args.get("sigma", 0),
                        E, n, None, None, 0x400000000, wsb, None)
    assert st == code, (st, L.ps_last_error())
    assert L.ps_last_error()


def test_solve_and_pade_workspace_sizes(ps):
    L = ps.lib()
    sz = ctypes.c_size_t()
    assert L.ps_workspace_size_solve(0, 2048, ctypes.byref(sz)) == 0
    assert sz.value >= 2048 * 4 and sz.value % 256 == 0
    multi, pade = ctypes.c_size_t(), ctypes.c_size_t()
    deg = (ctypes.c_int * 2)(13, 13)
    assert L.ps_workspace_size_multi(0, 2048, 2, deg, 4, 0, ctypes.byref(multi)) == 0
    assert L.ps_workspace_size_pade(0, 2048, 13, 4, 2, ctypes.byref(pade)) == 0
    assert pade.value >= multi.value + 2 * 2048 * 2048 * 8 + sz.value


def test_model_cost_matches_oracle(ps):
    """ps_model_cost (the report's C_r and M_low) against the oracle's
    cost_saving and m_low with d_i the digits of each tier's unit roundoff."""
    from oracle import metrics
    import math
    rng = np.random.default_rng(3)
    for dt, work in (("f64", 0), ("f32", 1), ("dd", 4)):
        lowest = 1 if work == 0 else (2 if work == 1 else 0)
        for trial in range(200):
            s = int(rng.integers(1, 14))
            r = int(rng.integers(0, 13))
            tiers = [work] + [int(t) for t in rng.integers(lowest, 4, r)] if work != 4 else \
                [4] + [int(t) for t in rng.choice([0, 1, 2, 3, 4], r)]
            if work != 4:
                tiers = [work] + [max(t, work) if rng.random() < 0.8 else work for t in tiers[1:]]
            cr, ml = ps.model_cost(tiers, s, dt)
            D = -math.log10(oplan.U_TIER[work])
            d = [-math.log10(oplan.U_TIER[t]) for t in tiers[1:]]
            if s - 1 + r == 0:
                assert cr == 0.0 and ml == 0.0
                continue
            assert cr == pytest.approx(metrics.cost_saving(D, s, r, d), abs=1e-12)
            assert ml == pytest.approx(metrics.m_low(D, s, r, d), abs=1e-15)
    # every product in the working precision saves nothing
    assert ps.model_cost([0, 0, 0, 0], 6) == (0.0, 0.0)
    with pytest.raises(ps.PSError):
        ps.model_cost([0, 7], 2)


def test_nonfinite_status_and_unsupported_paths(ps):
    L = ps.lib()
    assert L.ps_strerror(-4).decode().startswith("non-finite")
    o, _ = ps._opts("mixed", check_finite=True)
    assert o.check_finite == 1
    # check_finite is refused by the entry points that do not scan, before any device work
    st = L.ps_expm_backward(0, 1, 8, 0x10000000, 8, 64, 0x20000000, 8, 64, None, 6, 0, 0, 0x30000000, 8, 64, 0,
                            ctypes.byref(o), 0x40000000, 1 << 30, None)
    assert st == -5 and b"check_finite" in L.ps_last_error()
    n = (ctypes.c_int32 * 1)(8)
    ptrs = (ctypes.c_void_p * 1)(0x10000000)
    outs = (ctypes.c_void_p * 1)(0x20000000)
    ld = (ctypes.c_int64 * 1)(8)
    sg = (ctypes.c_int32 * 1)(0)
    st = L.ps_expm_batched(1, 1, n, ptrs, ld, None, 6, None, sg, outs, ld, ctypes.byref(o), None, 0x40000000,
                           1 << 30, None)
    assert st == -5 and b"check_finite" in L.ps_last_error()
    st = L.ps_expm_dd(8, 0x10000000, 8, None, 6, 0, 0, 0x20000000, 8, ctypes.byref(o), None, 0x40000000, 1 << 30,
                      None)
    assert st == -5 and b"check_finite" in L.ps_last_error()


def test_backward_batched_validation(ps):
    L = ps.lib()
    k = 2
    n = (ctypes.c_int32 * k)(8, 16)
    ld = (ctypes.c_int64 * k)(8, 16)
    A = (ctypes.c_void_p * k)(0x10000000, 0x10100000)
    G = (ctypes.c_void_p * k)(0x20000000, 0x20100000)
    O = (ctypes.c_void_p * k)(0x30000000, 0x10100000)        # the second output is the second input
    sz = ctypes.c_size_t()
    assert L.ps_workspace_size_backward_batched(0, k, n, 18, None, None, 0, ctypes.byref(sz)) == 0
    one = [ctypes.c_size_t(), ctypes.c_size_t()]
    for b, nb in enumerate((8, 16)):
        assert L.ps_workspace_size_backward(0, 1, nb, 18, 0, 0, 0, ctypes.byref(one[b])) == 0
    assert sz.value == sum((x.value + 255) // 256 * 256 for x in one)
    st = L.ps_expm_backward_batched(0, k, n, A, ld, G, ld, None, 18, None, None, O, ld, 0, None, 0x40000000,
                                    sz.value, None)
    assert st == -2, L.ps_last_error()
    O2 = (ctypes.c_void_p * k)(0x30000000, 0x30100000)
    assert L.ps_expm_backward_batched(0, k, n, A, ld, G, ld, None, 18, None, None, O2, ld, 0, None, 0x40000000,
                                      16, None) == -3
    bad = (ctypes.c_int64 * k)(8, 15)
    assert L.ps_expm_backward_batched(0, k, n, A, bad, G, ld, None, 18, None, None, O2, ld, 0, None, 0x40000000,
                                      sz.value, None) == -1


def test_eval_batched_requires_coefficients(ps):
    L = ps.lib()
    n = (ctypes.c_int32 * 1)(4)
    st = L.ps_eval_batched(0, 1, n, (ctypes.c_void_p * 1)(0x1000), (ctypes.c_int64 * 1)(4), None, 4, None,
                           (ctypes.c_void_p * 1)(0x2000), (ctypes.c_int64 * 1)(4), None, None, 0x40000000, 1 << 30,
                           None)
    assert st == -1 and b"coef" in L.ps_last_error()


def test_autotune_cache_roundtrip(ps, tmp_path):
    """The schedule cache on the host: a JSON file loaded, looked up, saved and
    loaded again; malformed files refused.  The key's architecture part comes
    from the device (on a machine without one it reads 'unknown')."""
    import torch
    ps.autotune_clear()
    mats = [torch.zeros(n, n) for n in (8, 100, 250, 250)]
    found, groups = ps.autotune_lookup(mats, 18)
    assert not found and groups == [0, 0, 0, 0]
    # write an entry under the key this process computes: find it by saving one
    L = ps.lib()
    n = (ctypes.c_int32 * 4)(8, 100, 250, 250)
    arch = "unknown"
    if torch.cuda.is_available():
        arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    key = "%s|f32|m18|1,1,0,2" % arch            # classes 1, 2 and 4 with 1, 1 and 2 matrices
    p = tmp_path / "cache.json"
    p.write_text('{"ps_autotune": 1, "entries": [{"key": "%s", "groups": [0, 1, 1, 2]}]}' % key)
    ps.autotune_load(p)
    found, groups = ps.autotune_lookup(mats, 18)
    assert found and groups == [0, 1, 1, 2]
    q = tmp_path / "saved.json"
    ps.autotune_save(q)
    ps.autotune_clear()
    assert not ps.autotune_lookup(mats, 18)[0]
    ps.autotune_load(q)
    assert ps.autotune_lookup(mats, 18) == (True, [0, 1, 1, 2])
    assert not ps.autotune_lookup(mats, 16)[0]    # another degree: another key
    bad = tmp_path / "bad.json"
    bad.write_text('{"something": 1}')
    with pytest.raises(ps.PSError):
        ps.autotune_load(bad)
    bad.write_text('{"ps_autotune": 1, "entries": [{"key": "x", "groups": [0, 9, 0, 0]}]}')
    with pytest.raises(ps.PSError):
        ps.autotune_load(bad)
    with pytest.raises(ps.PSError):
        ps.autotune_load(tmp_path / "missing.json")
    ps.autotune_clear()


def test_autotune_cache_whole64(ps, tmp_path):
    """The class-1 kernel choice in the cache file: read per entry (an entry
    without it reads as per-phase launches, even when the next entry has it),
    kept by a save/load round trip, and out-of-range values refused."""
    import torch
    ps.autotune_clear()
    arch = "unknown"
    if torch.cuda.is_available():
        arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    a = [torch.zeros(n, n) for n in (8, 40, 250)]          # classes 1 and 4
    b = [torch.zeros(n, n) for n in (8, 100)]              # classes 1 and 2
    ka = "%s|f32|m18|2,0,0,1" % arch
    kb = "%s|f32|m18|1,1,0,0" % arch
    p = tmp_path / "cache.json"
    p.write_text('{"ps_autotune": 1, "entries": [{"key": "%s", "groups": [0, 0, 0, 1]},\n'
                 ' {"key": "%s", "groups": [0, 1, 0, 0], "whole64": 1}]}' % (ka, kb))
    ps.autotune_load(p)
    assert ps.autotune_lookup(a, 18, whole64=True) == (True, [0, 0, 0, 1], 0)
    assert ps.autotune_lookup(b, 18, whole64=True) == (True, [0, 1, 0, 0], 1)
    assert ps.autotune_lookup(b, 18) == (True, [0, 1, 0, 0])
    q = tmp_path / "saved.json"
    ps.autotune_save(q)
    assert '"whole64": 1' in q.read_text() and '"whole64": 0' in q.read_text()
    ps.autotune_clear()
    ps.autotune_load(q)
    assert ps.autotune_lookup(b, 18, whole64=True) == (True, [0, 1, 0, 0], 1)
    assert ps.autotune_lookup(a, 18, whole64=True) == (True, [0, 0, 0, 1], 0)
    bad = tmp_path / "bad.json"
    bad.write_text('{"ps_autotune": 1, "entries": [{"key": "x", "groups": [0, 1, 0, 0], "whole64": 2}]}')
    with pytest.raises(ps.PSError):
        ps.autotune_load(bad)
    ps.autotune_clear()
