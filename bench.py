#!/usr/bin/env python3
"""Throughput of the PS hot path on one MI355X: exp(A) by scaling and squaring
around Taylor PS (m = 30, s = 6) on dense n = 1024 FP64 matrices with
||A||_1 in {0.1, 1, 8, 64} (sigma = 0, 0, 3, 6), mixed-precision tiers vs
plain FP64 PS on the same GPU.

One step = one evaluation of each of the four matrices (4 evals), inputs
resident in HBM.  `value` = evals/s of the mixed-precision path.

Also reported:
  plain       the same workload with every product in FP64 (Algorithm 1)
  accuracy    relative 1-norm distance mixed vs plain (full matrices, GPU)
  roofline    the dominant kernel, k_gemm<double>, the FP64 MFMA tile kernel of
              the squarings (one n^3 product per launch): algorithmic 2 n^3
              flops over its average launch duration, from hipEvent pairs around
              the squaring phase (library profile mode, on the launch stream),
              for K steps of the plain evaluation run right after the timed
              region; roofline_power_levels gives the same per product for the
              power-table launches (k_gemm_group, the same tile routine)
  cpu_baseline  the CPU oracle's plain FP64 Algorithm 1 + squarings
              (OpenMP, all host cores, median of three runs, CPU model stated)
              on one evaluation of each matrix, plus the GPU result's error
              against the dd oracle on sampled columns; the batched extra's
              accuracy gate is computed in this leg too
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N = 1024
M = 30
S = 6
PEAK_FP64_MFMA = 78.6   # TFLOP/s, MI355X dense FP64 matrix
# dense MFMA peaks per tier (FP64, FP32, BF16, FP8) in flop/s and HBM bytes/s
TIER_PEAK = {0: 78.6e12, 1: 157.3e12, 2: 2.5e15, 3: 5.0e15}
HBM_BW = 8.0e12
TIER_BYTES = {0: 8.0, 1: 4.0, 2: 2.0, 3: 1.0 + 1.0 / 32}   # per element, FP8 with its E8M0 scales


def step_ideal_s(rep, sigma, mixed):
    """Ideal time of one evaluation at nominal peaks: sum over its steps of
    max(flops / peak(tier), algorithmic bytes / HBM bandwidth); and the
    MFMA-only part, sum of flops / peak(tier)."""
    n2, F = float(N) * N, 2.0 * N ** 3
    gemm64 = max(F / TIER_PEAK[0], 3 * 8 * n2 / HBM_BW)
    # power products per tier from the report (mixed mode may form Y = X^s by
    # an FP32 product, and again in FP64 when the plan keeps a product there)
    steps = [rep["tier"][i] for i in range(1, rep["first_step"] + 1)]
    pow64 = rep["gemms"][0] - sigma - sum(1 for t in steps if t == 0)
    pow32 = rep["gemms"][1] - sum(1 for t in steps if t == 1)
    gemm32 = max(F / TIER_PEAK[1], (2 * 8 + 4) * n2 / HBM_BW)
    t = pow64 * gemm64 + pow32 * gemm32 + sigma * gemm64                     # powers, squarings
    mf = (pow64 + sigma) * F / TIER_PEAK[0] + pow32 * F / TIER_PEAK[1]
    copies = sum(TIER_BYTES[k] for k in (1, 2, 3)) if mixed else 0.0
    fs = rep["first_step"]
    t += (S * 8 + (fs + 1) * 8 + copies) * n2 / HBM_BW                           # block assembly
    tiers = rep["tier"]
    t += (8 + TIER_BYTES[tiers[fs]]) * n2 / HBM_BW                              # B_first into step format
    for i in range(fs, 0, -1):
        ti, to = tiers[i], tiers[i - 1]
        byts = (2 * TIER_BYTES[ti] + 8 + TIER_BYTES[to]) * n2                   # P_i, Y, B_{i-1}, P_{i-1}
        t += max(F / TIER_PEAK[ti], byts / HBM_BW)
        mf += F / TIER_PEAK[ti]
    return t, mf


EXTRAS = ("latency", "sizes", "batched", "pade_cos", "grad", "auto", "select", "vars", "dd")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", choices=["mixed", "plain", "both"], default="both",
                    help="restrict the timed modes (profiling runs)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the secondary workloads (batched, Pade/cos, adjoint)")
    ap.add_argument("--extra", default=",".join(EXTRAS),
                    help="comma-separated subset of the secondary workloads: " + ",".join(EXTRAS))
    ap.add_argument("--schedule", choices=["graph", "sequential"], default="graph",
                    help="graph: the step's four evaluations forked over four streams in one replayed hipGraph; "
                         "sequential: eager calls on one stream (kernels never overlap; used for kernel traces)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run three 256 MiB device-to-device copies (known traffic, for counter scaling)")
    ap.add_argument("--summarize", nargs="+", metavar="ARG",
                    help="write a profile summary under profiles/ from rocprofv3 CSV output instead of running: "
                         "'stats OUT DIR', 'traffic OUT DIR_FETCH DIR_WRITE' or 'mfma OUT DIR' "
                         "(the header lines come from --note, one per use)")
    ap.add_argument("--note", action="append", default=[],
                    help="a header line of the summary (the workload, the command that made the CSVs)")
    return ap.parse_args()


# ---------------------------------------------------------------------------
# profile summaries (rocprofv3 CSV -> short text under profiles/)
# ---------------------------------------------------------------------------
SRC_FILES = ("ps_kernels.hip", "ps_device.h", "ps_batched.hip", "ps_dd.hip", "ps_solve.hip", "ps_api.cpp",
             "ps_backward.cpp")


def source_hashes():
    import hashlib
    csrc = os.path.join(ROOT, "paper_2312_17396_amd", "csrc")
    return {f: hashlib.sha256(open(os.path.join(csrc, f), "rb").read()).hexdigest() for f in SRC_FILES}


def _csvs(d, suffix):
    import glob
    out = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not out:
        raise SystemExit("no *%s under %s" % (suffix, d))
    return out


def _short(name, w=72):
    return name if len(name) <= w else name[:w]


def _header(notes, what):
    h = source_hashes()
    lines = ["# " + n for n in notes]
    lines.append("# " + what)
    lines.append("# source sha256 (first 16 hex digits): " +
                 ", ".join("%s %s" % (f, h[f][:16]) for f in SRC_FILES))
    return lines


def summarize(args):
    import csv
    kind, out = args.summarize[0], args.summarize[1]
    path = os.path.join(ROOT, "profiles", out)
    if kind == "stats":
        rows = []
        for f in _csvs(args.summarize[2], "kernel_stats.csv"):
            rows += list(csv.DictReader(open(f)))
        rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
        tot = sum(float(r["TotalDurationNs"]) for r in rows)
        lines = _header(args.note, "rocprofv3 --kernel-trace --stats: per-kernel durations")
        lines.append("%-72s %6s %11s %9s %9s %9s %6s" % ("kernel", "calls", "total_ms", "avg_us", "min_us", "max_us",
                                                       "pct"))
        for r in rows:
            lines.append("%-72s %6s %11.3f %9.2f %9.2f %9.2f %6.2f" % (
                _short(r["Name"]), r["Calls"], float(r["TotalDurationNs"]) / 1e6, float(r["AverageNs"]) / 1e3,
                float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3, 100.0 * float(r["TotalDurationNs"]) / tot))
    elif kind in ("traffic", "mfma"):
        def per_kernel(d):
            acc = {}
            for f in _csvs(d, "counter_collection.csv"):
                for r in csv.DictReader(open(f)):
                    k = (r["Kernel_Name"], r["Counter_Name"])
                    v = acc.setdefault(k, {})
                    v[r.get("Dispatch_Id", r.get("Correlation_Id"))] = float(r["Counter_Value"])
            return {k: (len(v), sum(v.values()) / len(v), max(v.values())) for k, v in acc.items()}
        if kind == "mfma":
            pk = per_kernel(args.summarize[2])
            names = sorted({k[0] for k in pk})
            lines = _header(args.note, "rocprofv3 --pmc MfmaUtil MfmaFlopsF64: averages over dispatches "
                                       "(MfmaUtil = MFMA-busy cycles / (active cycles x SIMDs) in percent; "
                                       "MfmaFlopsF64 = F64 MFMA ops x 512)")
            lines.append("%-72s %6s %11s %16s" % ("kernel", "calls", "MfmaUtil_%", "F64_GFLOP/launch"))
            for nm in names:
                u = pk.get((nm, "MfmaUtil"))
                fl = pk.get((nm, "MfmaFlopsF64"))
                if not u:
                    continue
                lines.append("%-72s %6d %11.1f %16.3f" % (_short(nm), u[0], u[1], (fl[1] / 1e9) if fl else 0.0))
        else:
            pf = per_kernel(args.summarize[2])
            pw = per_kernel(args.summarize[3])
            # calibration: the 256 MiB device copies (largest written bytes among the copy kernels)
            cal = [k[0] for k in pw if k[1] == "WRITE_SIZE" and ("copy" in k[0].lower() or "Copy" in k[0])]
            if not cal:
                raise SystemExit("no copy kernel in the WRITE_SIZE run: take it with --calib-copy")
            ck = max(cal, key=lambda nm: pw[(nm, "WRITE_SIZE")][2])
            kib = 256 * 1024.0
            f_cal, w_cal = pf[(ck, "FETCH_SIZE")][2], pw[(ck, "WRITE_SIZE")][2]
            fs, wsc = kib / f_cal, kib / w_cal
            lines = _header(args.note, "rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE (KiB per dispatch), "
                                       "one run each, scaled by a 256 MiB device copy")
            lines.append("# calibration: the copy reads %.1f KiB fetched, %.1f KiB written -> scale fetch x%.3f, "
                         "write x%.3f" % (f_cal, w_cal, fs, wsc))
            lines.append("%-72s %6s %11s %11s %15s" % ("kernel", "calls", "fetch_MiB", "write_MiB", "hbm_MiB/launch"))
            names = sorted({k[0] for k in pf if k[1] == "FETCH_SIZE"} & {k[0] for k in pw if k[1] == "WRITE_SIZE"})
            gemm = None
            for nm in names:
                if nm == ck:
                    continue
                fm = pf[(nm, "FETCH_SIZE")][1] * fs / 1024.0
                wm = pw[(nm, "WRITE_SIZE")][1] * wsc / 1024.0
                lines.append("%-72s %6d %11.2f %11.2f %15.2f" % (_short(nm), pf[(nm, "FETCH_SIZE")][0], fm, wm, fm + wm))
                if nm.startswith("void psk::k_gemm<double, false, false>"):
                    gemm = (fm, wm)
            if gemm is not None:
                h = source_hashes()
                rec = {"kernel": "k_gemm<double,false,false> n=1024",
                       "kernel_source_sha256": h["ps_kernels.hip"], "device_header_sha256": h["ps_device.h"],
                       "hbm_bytes_per_launch": int(round((gemm[0] + gemm[1]) * 1024 * 1024)),
                       "fetch_MiB": round(gemm[0], 3), "write_MiB": round(gemm[1], 3),
                       "fetch_scale": round(fs, 4), "write_scale": round(wsc, 4),
                       "algorithmic_bytes_per_launch": 3 * N * N * 8}
                with open(os.path.join(ROOT, "profiles", "traffic_gemm_f64_n1024.json"), "w") as fh:
                    json.dump(rec, fh, indent=1)
                    fh.write("\n")
    else:
        raise SystemExit("--summarize: stats, traffic or mfma")
    with open(path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("wrote", path)


def gemm_count(sigma):
    r = M // S
    horner = r - 1 if M % S == 0 else r
    return (S - 1) + horner + sigma


def load_traffic():
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    counter summary, if it was taken on the current kernel source."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic_gemm_f64_n1024.json")
    csrc = os.path.join(ROOT, "paper_2312_17396_amd", "csrc")
    try:
        rec = json.load(open(path))
        h1 = hashlib.sha256(open(os.path.join(csrc, "ps_kernels.hip"), "rb").read()).hexdigest()
        h2 = hashlib.sha256(open(os.path.join(csrc, "ps_device.h"), "rb").read()).hexdigest()
        if rec.get("kernel_source_sha256") != h1 or rec.get("device_header_sha256") != h2:
            return None
        return rec.get("hbm_bytes_per_launch")
    except Exception:
        return None


def main():
    args = parse()
    if args.summarize:
        summarize(args)
        return
    if args.gpus != 1:
        print("bench.py: runs on one GPU only (no multi-GPU path is implemented); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2312_17396_amd as ps
    from paper_2312_17396_amd import inputs

    ps.lib()
    dev = torch.device("cuda:0")
    norms = list(inputs.DENSE_NORMS)
    sigmas = [inputs.squarings_for(t) for t in norms]
    mats = [torch.tensor(inputs.dense_1024(t), dtype=torch.float64, device=dev) for t in norms]
    outs = [torch.empty_like(a) for a in mats]
    wss = [ps.expm_workspace(a, M, S, sg) for a, sg in zip(mats, sigmas)]
    flops_per_step = sum(gemm_count(sg) * 2.0 * N ** 3 for sg in sigmas)

    def step(mode, profile=False):
        reps = []
        for a, o, w, sg in zip(mats, outs, wss, sigmas):
            r = ps.ps_expm(a, M, s=S, sigma=sg, mode=mode, out=o, workspace=w, profile=profile)
            if profile:
                reps.append(r[1])
        return reps

    streams = [torch.cuda.Stream(device=dev) for _ in mats]   # default priority

    # the forked step issues the evaluations longest first (most products,
    # i.e. most squarings), so that the longest chain starts first: the
    # runtime starts a graph's independent branches one after another
    order = sorted(range(len(mats)), key=lambda i: (-gemm_count(sigmas[i]), i))

    def step_forked(mode):
        """the four evaluations on four streams (they are independent), joined"""
        cur = torch.cuda.current_stream(dev)
        for st in streams:
            st.wait_stream(cur)
        for i, st in zip(order, streams):
            with torch.cuda.stream(st):
                ps.ps_expm(mats[i], M, s=S, sigma=sigmas[i], mode=mode, out=outs[i], workspace=wss[i])
        for st in streams:
            cur.wait_stream(st)

    def capture(mode):
        """one hipGraph of the forked step; its replays are checked against the
        eager results (with eager work and synchronisations between them)"""
        step(mode)
        torch.cuda.synchronize()
        ref = [o.clone() for o in outs]
        side = torch.cuda.Stream(device=dev)
        side.wait_stream(torch.cuda.current_stream(dev))
        with torch.cuda.stream(side):
            step_forked(mode)
        torch.cuda.current_stream(dev).wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            step_forked(mode)
        for _ in range(2):
            for o in outs:
                o.zero_()
            g.replay()
            torch.cuda.synchronize()
            if not all(torch.equal(o, r) for o, r in zip(outs, ref)):
                raise RuntimeError("graph replay differs from the eager evaluation")
            step(mode)
            torch.cuda.synchronize()
        return g

    def run_timed(fn, per_step=None):
        """wall-clock mean over K steps; per_step (a list) also receives each
        step's duration from a pair of events on the current stream"""
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.steps)] if per_step is not None else None
        t0 = time.perf_counter()
        for k in range(args.steps):
            if evs:
                evs[k][0].record()
            fn()
            if evs:
                evs[k][1].record()
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / args.steps
        if evs:
            per_step.extend(a.elapsed_time(b) for a, b in evs)
        return t

    eager = {}
    step_ms = {}

    def timed(mode):
        step_ms[mode] = []
        if args.schedule == "sequential":
            eager[mode] = run_timed(lambda: step(mode), step_ms[mode])
            return eager[mode]
        eager[mode] = run_timed(lambda: step(mode))
        g = capture(mode)
        t = run_timed(g.replay, step_ms[mode])
        del g
        return t

    def stats(v):
        v = sorted(v)
        q = lambda f: v[min(len(v) - 1, int(round(f * (len(v) - 1))))]
        return {"median": round(q(0.5), 4), "p10": round(q(0.1), 4), "p90": round(q(0.9), 4)}

    if args.calib_copy:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    res = {}
    modes = ["plain", "mixed"] if args.only == "both" else [args.only]
    for mode in modes:
        res[mode] = timed("fixed" if mode == "plain" else "mixed")

    # tiers and accuracy (outside the timed region)
    plans = []
    errs = []
    ideal = {"plain": 0.0, "mixed": 0.0}
    mfma_only = {"plain": 0.0, "mixed": 0.0}
    for a, sg in zip(mats, sigmas):
        em, rp = ps.ps_expm(a, M, s=S, sigma=sg, mode="mixed", report=True)
        ef, rf = ps.ps_expm(a, M, s=S, sigma=sg, mode="fixed", report=True)
        for mode, rr, mixed in (("mixed", rp, True), ("plain", rf, False)):
            ti, tm = step_ideal_s(rr, sg, mixed)
            ideal[mode] += ti
            mfma_only[mode] += tm
        plans.append([ps.TIER_NAMES[t] for t in rp["tier"][1:rp["first_step"] + 1]])
        d = torch.linalg.matrix_norm(em - ef, ord=1).item() / torch.linalg.matrix_norm(ef, ord=1).item()
        errs.append(d)

    # roofline of the dominant kernel: FP64 GEMM (power table + squarings),
    # timed on the plain evaluation, whose power products are all FP64 (the
    # mixed one forms Y = X^s by an FP32 product when its plan allows)
    prof_mode = "fixed"
    sq_ms, sq_n, pw_ms, pw_n = 0.0, 0, 0.0, 0
    for _ in range(args.steps):
        for r, sg in zip(step(prof_mode, profile=True), sigmas):
            pw_ms += r["ms"]["power"]
            pw_n += S - 1
            sq_ms += r["ms"]["square"]
            sq_n += sg
    sq_avg = sq_ms / max(sq_n, 1)            # ms per k_gemm launch (one product each)
    achieved = 2.0 * N ** 3 / (sq_avg * 1e-3) / 1e12
    roofline = {"kernel": "k_gemm<double> (the squarings: one n^3 FP64 product per launch; 64x64 tiles, "
                          "MFMA 16x16x4)", "bound": "mfma",
                "achieved": round(achieved, 2), "peak": PEAK_FP64_MFMA, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP64_MFMA, 4), "avg_us_per_launch": round(sq_avg * 1e3, 2),
                "launches_timed": sq_n, "traffic": load_traffic()}
    pw_avg = pw_ms / max(pw_n, 1)            # ms per product of the power-table levels
    roofline_power = {"kernel": "k_gemm_group<double> (power table X^2..X^6: one launch per level of "
                                "ceil(log2 j), one or two products; same tile routine)",
                      "achieved": round(2.0 * N ** 3 / (pw_avg * 1e-3) / 1e12, 2), "peak": PEAK_FP64_MFMA,
                      "unit": "TFLOP/s", "frac": round(2.0 * N ** 3 / (pw_avg * 1e-3) / 1e12 / PEAK_FP64_MFMA, 4),
                      "avg_us_per_product": round(pw_avg * 1e3, 2)}

    main_mode = "mixed" if "mixed" in res else "plain"
    t_step = res[main_mode]
    value = len(mats) / t_step
    out = {
        "metric": "p(A) evals/s at fixed rel. error vs FP64 oracle, mixed vs FP64 PS",
        "value": round(value, 2),
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_step * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "expm_taylor_dense_1024", "n": N, "m": M, "s": S, "norms_1": norms,
                   "sigma": sigmas, "mode": main_mode, "evals_per_step": len(mats)},
        "tflops": round(flops_per_step / t_step / 1e12, 3),
        "tiers": plans,
        "rel_diff_mixed_vs_plain": [float("%.3e" % e) for e in errs],
        "roofline": roofline,
        "roofline_power_levels": roofline_power,
        "step_roofline": {mode: {"ideal_ms": round(ideal[mode] * 1e3, 4), "measured_ms": round(res[mode] * 1e3, 4),
                                 "frac": round(ideal[mode] / res[mode], 4),
                                 "mfma_only_frac": round(mfma_only[mode] / res[mode], 4)} for mode in res},
        "step_ms_events": {("plain" if k == "fixed" else k): stats(v) for k, v in step_ms.items()},
    }
    out["schedule"] = ("one hipGraph per step: the four evaluations forked over four streams "
                       "(default priority) and joined; replays checked bitwise against eager calls"
                       if args.schedule == "graph" else "eager sequential calls on one stream")
    out["eager_sequential"] = {("plain" if mode == "fixed" else mode): {"ms_per_step": round(t * 1e3, 4),
                                                                        "evals_per_s": round(len(mats) / t, 2)}
                               for mode, t in eager.items()}
    if "plain" in res and "mixed" in res:
        out["plain"] = {"evals_per_s": round(len(mats) / res["plain"], 2),
                        "ms_per_step": round(res["plain"] * 1e3, 4),
                        "tflops": round(flops_per_step / res["plain"] / 1e12, 3)}
        out["speedup_mixed_vs_plain"] = round(res["plain"] / res["mixed"], 4)

    if not args.no_extra:
        which = set(x for x in args.extra.split(",") if x)
        if not which <= set(EXTRAS):
            sys.exit("unknown --extra entries: %s" % ",".join(sorted(which - set(EXTRAS))))
        out["extra"] = extra_workloads(ps, inputs, torch, which)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(mats, outs_mixed=[ps.ps_expm(a, M, s=S, sigma=sg, mode="mixed")
                                                             for a, sg in zip(mats, sigmas)],
                                           norms=norms, sigmas=sigmas)
        worst = max(out["cpu_baseline"]["gpu_mixed_rel_err_vs_dd_oracle_sampled_cols"])
        out["accuracy_gate"] = {"tol": 1e-13, "max_rel_err_vs_dd_oracle": worst, "ok": worst <= 1e-13,
                                "note": "mixed results, sampled columns, 1-norm relative error"}
        bx = out.get("extra", {}).get("batched_uneven_4096")
        if bx is not None and "_gate_samples" in bx:
            bx["accuracy_gate"] = batched_gate(bx.pop("_gate_samples"))
            if not bx["accuracy_gate"]["ok"]:
                bx.pop("speedup_graph_vs_loop", None)
                bx.pop("speedup_mixed_vs_fixed", None)
    bx = out.get("extra", {}).get("batched_uneven_4096")
    if bx is not None and "_gate_samples" in bx:
        bx.pop("_gate_samples")
        bx["accuracy_gate"] = {"ok": None, "note": "not computed: the oracle leg was skipped (--no-cpu-baseline)"}
    print(json.dumps(out))


def _time(fn, reps, torch):
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def extra_workloads(ps, inputs, torch, which=EXTRAS):
    """Secondary workloads of the hot path (each a few seconds):
    latency   one 64x64 FP64 matrix, ||A||_1 = 1, Taylor m = 16, s = 4, no
              scaling: microseconds per evaluation, as a stream of ps_expm
              calls, as one ps_expm call captured into a hipGraph and
              replayed, and as one replayed hipGraph of the batched path with
              one matrix;
    sizes     one N(0,1) matrix with ||A||_1 = 1 (m = 30, s = 6, no scaling) at
              n = 512, 2048, 4096: mixed vs plain ms per evaluation and the FP64
              GEMM tile kernel's TFLOP/s (library profile mode, hipEvents);
    batched   4096 matrices, n uniform in {8..256}, ||A||_1 ~ U[0.05, 4], Taylor
              m = 18, s chosen per matrix, FP32: the per-phase launches of the whole
              batch replayed from one hipGraph (one branch, then the size-class
              schedule chosen by ps_batched_tune), each size class alone, and a
              loop of single-matrix calls; accuracy gate in the oracle leg;
    pade_cos  n = 2048 FP64, A = Q diag(lambda) Q^T: Pade [13/13] p and q from one
              power table (s = 4), exp as q^-1 p (the LU solve on the device;
              its time is the difference to the pair), and Taylor cos of degree
              12 in A^2 (s = 4);
    grad      64 FP32 matrices of order 512: forward + hand-written adjoint;
    auto      the dense n = 1024 set with the scaling chosen by the alpha_m bound
              (ps_expm_auto) instead of ceil(log2 ||A||_1);
    select    the dense n = 1024 set with the Taylor degree (<= 42) and the scaling
              chosen together by the alpha_m bound (ps_expm_select);
    vars      n = 1024, A = -0.5 I + E with ||E||_1 = 0.05, Taylor m = 30, sigma = 0:
              Algorithm 2's variable-s branch (ps_expm_vars) against s = 6;
    dd        n = 1024, ||A||_1 = 1, Taylor m = 30 (theta_30 = 1.16 at u = 2^-106,
              so no scaling), s = 6, double-double working precision: every
              product in double-double vs the planned tiers below it."""
    import numpy as np
    res = {}
    dev = torch.device("cuda:0")
    # ---- latency of the small case
    if "latency" in which:
        A1 = torch.tensor(inputs.single_64(), device=dev)
        E1 = torch.empty_like(A1)
        ws1 = ps.expm_workspace(A1, 16, 4, 0)
        out = {"n": 64, "m": 16, "s": 4, "sigma": 0, "dtype": "f64"}
        for mode in ("fixed", "mixed"):
            tc = _time(lambda: ps.ps_expm(A1, 16, s=4, mode=mode, out=E1, workspace=ws1), 200, torch)
            g = ps.BatchedGraph([A1], 16, s=[4], sigma=[0], mode=mode)
            tg = _time(g.launch, 200, torch)
            g.close()
            # one ps_expm call captured into a hipGraph and replayed, checked
            # bitwise against the eager call
            ps.ps_expm(A1, 16, s=4, mode=mode, out=E1, workspace=ws1)
            torch.cuda.synchronize()
            ref1 = E1.clone()
            side = torch.cuda.Stream(device=dev)
            side.wait_stream(torch.cuda.current_stream(dev))
            with torch.cuda.stream(side):
                ps.ps_expm(A1, 16, s=4, mode=mode, out=E1, workspace=ws1)
            torch.cuda.current_stream(dev).wait_stream(side)
            torch.cuda.synchronize()
            g1 = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g1):
                ps.ps_expm(A1, 16, s=4, mode=mode, out=E1, workspace=ws1)
            E1.zero_()
            g1.replay()
            torch.cuda.synchronize()
            if not torch.equal(E1, ref1):
                raise RuntimeError("graph replay of the 64 x 64 case differs from the eager call")
            t1 = _time(g1.replay, 200, torch)
            del g1
            out[mode] = {"us_per_eval_calls": round(tc * 1e6, 2), "us_per_eval_graph": round(tg * 1e6, 2),
                         "us_per_eval_call_graph": round(t1 * 1e6, 2)}
        res["latency_single_64"] = out
        del A1, E1, ws1
    # ---- other orders
    if "sizes" in which:
        out = {}
        for n in (512, 2048, 4096):
            An = torch.tensor(inputs.dense_1024(1.0, n=n), device=dev)
            En = torch.empty_like(An)
            wsn = ps.expm_workspace(An, M, S, 0)
            row = {}
            for mode in ("fixed", "mixed"):
                tt = _time(lambda: ps.ps_expm(An, M, s=S, mode=mode, out=En, workspace=wsn), 5, torch)
                row["plain" if mode == "fixed" else mode] = {"ms": round(tt * 1e3, 3)}
            gm = 0.0
            for _ in range(3):
                _, rp = ps.ps_expm(An, M, s=S, mode="mixed", out=En, workspace=wsn, profile=True)
                gm += rp["ms"]["power"] / 3
            tf = (S - 1) * 2.0 * n ** 3 / (gm * 1e-3) / 1e12
            row["speedup_mixed_vs_plain"] = round(row["plain"]["ms"] / row["mixed"]["ms"], 3)
            row["gemm_f64_tflops"] = round(tf, 2)
            row["gemm_f64_frac"] = round(tf / PEAK_FP64_MFMA, 4)
            out["n%d" % n] = row
            del An, En, wsn
        res["sizes_taylor_exp"] = out
    # ---- batched
    if "batched" in which:
        mats, ts = inputs.batch_uneven()
        sig = [inputs.squarings_for(t) for t in ts]
        A = [torch.tensor(a, dtype=torch.float32, device=dev) for a in mats]
        gemms = lambda n, sg: 2.0 * n ** 3 * (3 + 4 + sg)   # s = 4/5: 7 products + squarings
        flops = sum(gemms(a.shape[0], sg) for a, sg in zip(mats, sig))
        out = {"matrices": len(A), "m": 18, "dtype": "f32"}
        ps.autotune_clear()
        for mode in ("fixed", "mixed"):
            g = ps.BatchedGraph(A, 18, sigma=sig, mode=mode)
            t = _time(g.launch, 5, torch)
            g.close()
            tune = ps.batched_tune(A, 18, sigma=sig, mode=mode, reps=3)
            g = ps.BatchedGraph(A, 18, sigma=sig, mode=mode)      # the tuned schedule, from the cache
            tt = _time(g.launch, 5, torch)
            g.close()
            out[mode] = {"ms": round(tt * 1e3, 3), "evals_per_s": round(len(A) / tt, 1),
                         "tflops_credited": round(flops / tt / 1e12, 2),
                         "frac_fp32_mfma_credited": round(flops / tt / 157.3e12, 4),
                         "one_branch_ms": round(t * 1e3, 3),
                         "tuned_schedule": {"branch_of_class": tune["groups"], "whole64": tune["whole64"],
                                            "candidate_ms": tune["ms"]}}
        out["speedup_mixed_vs_fixed"] = round(out["fixed"]["ms"] / out["mixed"]["ms"], 3)
        # per size class (padded order 64 k): the class alone as a batch, mixed
        classes = {}
        for i, a in enumerate(mats):
            classes.setdefault(64 * ((a.shape[0] + 63) // 64), []).append(i)
        per = {}
        for npad in sorted(classes):
            idx = classes[npad]
            g = ps.BatchedGraph([A[i] for i in idx], 18, sigma=[sig[i] for i in idx], mode="mixed")
            tc = _time(g.launch, 5, torch)
            g.close()
            fc = sum(gemms(mats[i].shape[0], sig[i]) for i in idx)
            per["n<=%d" % npad] = {"matrices": len(idx), "ms": round(tc * 1e3, 3),
                                   "tflops_credited": round(fc / tc / 1e12, 2),
                                   "frac_fp32_mfma_credited": round(fc / tc / 157.3e12, 4)}
            if npad == 64:   # the per-phase launches against one workgroup per matrix (tuner candidates 0, 1)
                t64 = ps.batched_tune([A[i] for i in idx], 18, sigma=[sig[i] for i in idx], mode="mixed", reps=5)
                per["n<=64"]["phases_vs_one_workgroup_ms"] = t64["ms"][:2]
                ps.autotune_clear()
        out["per_class_mixed"] = per
        sub = list(range(0, len(A), 8))          # per-matrix loop on every 8th matrix, scaled
        wsl = [ps.expm_workspace(A[i], 18, 0, sig[i]) for i in sub]
        outs = [torch.empty_like(A[i]) for i in sub]

        def loop():
            for k, i in enumerate(sub):
                ps.ps_expm(A[i], 18, s=0, sigma=sig[i], mode="mixed", out=outs[k], workspace=wsl[k])
        t = _time(loop, 1, torch) * len(A) / len(sub)
        out["per_matrix_loop_mixed"] = {"ms": round(t * 1e3, 2), "evals_per_s": round(len(A) / t, 1),
                                        "note": "loop of ps_expm calls timed on every 8th matrix, scaled"}
        out["speedup_graph_vs_loop"] = round(t / (out["mixed"]["ms"] * 1e-3), 2)
        # results kept for the accuracy gate (computed in the oracle leg):
        # every 128th matrix, mixed and plain, two columns each
        gs = []
        Ef = ps.ps_expm_batched(A, 18, sigma=sig, mode="fixed")
        Em = ps.ps_expm_batched(A, 18, sigma=sig, mode="mixed")
        for i in range(0, len(A), 128):
            n = A[i].shape[0]
            cols = [0, n // 2]
            gs.append((mats[i], sig[i], cols, Em[i][:, cols].double().cpu().numpy(),
                       Ef[i][:, cols].double().cpu().numpy()))
        out["_gate_samples"] = gs
        ps.autotune_clear()
        res["batched_uneven_4096"] = out
        del A, outs, wsl, Ef, Em
    # ---- Pade pair and cos at n = 2048
    if "pade_cos" in which:
        Aq = torch.tensor(inputs.orthosim_2048(), dtype=torch.float64, device=dev)
        p, q = ps.coef_pade_exp(13)
        c = ps.coef_taylor_cos(12)
        out = {"n": 2048, "dtype": "f64"}
        for mode in ("fixed", "mixed"):
            tp = _time(lambda: ps.ps_eval_multi(Aq, [p, q], s=4, mode=mode), 5, torch)
            tc = _time(lambda: ps.ps_eval_multi(Aq, [c], s=4, square_arg=True, mode=mode), 5, torch)
            wse = ps.pade_workspace(Aq, 13, 4, 0)
            Ee = torch.empty_like(Aq)
            te = _time(lambda: ps.ps_expm_pade(Aq, 13, s=4, sigma=0, mode=mode, out=Ee, workspace=wse), 5, torch)
            out[mode] = {"pade_pair_ms": round(tp * 1e3, 3), "pade_tflops_credited": round(9 * 2 * 2048 ** 3 / tp / 1e12, 2),
                         "cos_ms": round(tc * 1e3, 3), "cos_tflops_credited": round(6 * 2 * 2048 ** 3 / tc / 1e12, 2),
                         "expm_pade_ms": round(te * 1e3, 3),
                         "solve_ms_by_difference": round((te - tp) * 1e3, 3),
                         "solve_tflops_credited": round((2 / 3 + 2) * 2048 ** 3 / max(te - tp, 1e-9) / 1e12, 2)}
            del wse, Ee
        res["pade_cos_2048"] = out
        del Aq
    # ---- adjoint batch
    if "grad" in which:
        An, Gn = inputs.grad_batch_512()
        At = torch.tensor(An, device=dev)
        Gt = torch.tensor(Gn, device=dev)
        sigma = inputs.squarings_for(max(float(x) for x in torch.linalg.matrix_norm(At.double(), ord=1).cpu()))
        tf = _time(lambda: ps.ps_expm_strided_batched(At, 18, s=5, sigma=sigma, mode="mixed"), 3, torch)
        tb = _time(lambda: ps.ps_expm_backward(At, Gt, 18, s=5, sigma=sigma), 3, torch)
        tbm = _time(lambda: ps.ps_expm_backward(At, Gt, 18, s=5, sigma=sigma, mode="mixed"), 3, torch)
        rep = ps.ps_expm_strided_batched(At[:1], 18, s=5, sigma=sigma, mode="mixed", report=True)[1][0]
        gem_f = 4 + 3 + sigma
        fl = 64 * (gem_f + 2 * gem_f) * 2 * 512 ** 3   # the backward's forward recomputation + reverse pass
        res["grad_batch_512"] = {"batch": 64, "n": 512, "sigma": sigma, "dtype": "f32",
                                 "forward_ms": round(tf * 1e3, 3),
                                 "backward_ms": round(tb * 1e3, 3),
                                 "backward_tflops_credited": round(fl / tb / 1e12, 2),
                                 "backward_mixed_ms": round(tbm * 1e3, 3),
                                 "backward_mixed_tflops_credited": round(fl / tbm / 1e12, 2),
                                 "tiers_matrix_0": [ps.TIER_NAMES[t] for t in rep["tier"][1:rep["first_step"] + 1]],
                                 "note": "forward: mixed tiers; backward: working precision, and with the reverse "
                                         "Horner products in the forward plan's tiers (backward_mixed)"}
        del At, Gt
    # ---- automatic scaling (alpha_m bound) on the dense n = 1024 set
    if "auto" in which:
        mats = [torch.tensor(inputs.dense_1024(t), device=dev) for t in inputs.DENSE_NORMS]
        wsa = [ps.auto_workspace(a, M, S) for a in mats]
        outs = [torch.empty_like(a) for a in mats]
        sig = [ps.ps_expm_auto(a, M, s=S, mode="mixed", out=o, workspace=w)[1] for a, o, w in zip(mats, outs, wsa)]

        def auto_step():
            for a, o, w in zip(mats, outs, wsa):
                ps.ps_expm_auto(a, M, s=S, mode="mixed", out=o, workspace=w)
        ta = _time(auto_step, 5, torch)
        res["expm_auto_dense_1024"] = {"sigma_chosen": sig, "sigma_fixed_rule": [inputs.squarings_for(t) for t in inputs.DENSE_NORMS],
                                       "ms_per_step": round(ta * 1e3, 3), "evals_per_s": round(len(mats) / ta, 1),
                                       "note": "mixed tiers; includes the two norm read-backs of each call"}
        del mats, outs, wsa
    # ---- joint choice of degree and scaling
    if "select" in which:
        mats = [torch.tensor(inputs.dense_1024(t), device=dev) for t in inputs.DENSE_NORMS]
        wsl = [ps.select_workspace(a, 42) for a in mats]
        outs = [torch.empty_like(a) for a in mats]
        chosen = [ps.ps_expm_select(a, 42, mode="mixed", out=o, workspace=w)[1] for a, o, w in zip(mats, outs, wsl)]

        def select_step():
            for a, o, w in zip(mats, outs, wsl):
                ps.ps_expm_select(a, 42, mode="mixed", out=o, workspace=w)
        tsel = _time(select_step, 5, torch)
        res["expm_select_dense_1024"] = {"m_max": 42, "chosen_m_s_sigma": [list(c) for c in chosen],
                                         "ms_per_step": round(tsel * 1e3, 3),
                                         "evals_per_s": round(len(mats) / tsel, 1),
                                         "note": "mixed tiers, eager sequential calls; two norm read-backs per call"}
        del mats, outs, wsl
    # ---- variable block size (Algorithm 2, fix_params = false)
    if "vars" in which:
        Av = torch.tensor(inputs.shifted_1024(), device=dev)
        Ev = torch.empty_like(Av)
        wsv = ps.vars_workspace(Av, M, 0)
        wsf = ps.expm_workspace(Av, M, S, 0)
        _, s_var, rep_v = ps.ps_expm_vars(Av, M, mode="mixed", out=Ev, workspace=wsv, report=True)
        _, rep_f = ps.ps_expm(Av, M, s=S, mode="mixed", out=Ev, workspace=wsf, report=True)
        tv = _time(lambda: ps.ps_expm_vars(Av, M, mode="mixed", out=Ev, workspace=wsv), 5, torch)
        tf = _time(lambda: ps.ps_expm(Av, M, s=S, mode="mixed", out=Ev, workspace=wsf), 5, torch)
        res["expm_vars_shifted_1024"] = {
            "n": 1024, "m": M, "sigma": 0,
            "variable_s": {"s": s_var, "ms": round(tv * 1e3, 3),
                           "tiers": [ps.TIER_NAMES[x] for x in rep_v["tier"][:rep_v["first_step"] + 1]]},
            "fixed_s": {"s": S, "ms": round(tf * 1e3, 3),
                        "tiers": [ps.TIER_NAMES[x] for x in rep_f["tier"][:rep_f["first_step"] + 1]]},
            "note": "mixed tiers; the variable-s call includes one norm read-back per growth step"}
        del Av, Ev, wsv, wsf
    # ---- double-double working precision
    if "dd" in which:
        Ad = inputs.dense_1024(1.0)
        Td = torch.tensor(np.stack([Ad, np.zeros_like(Ad)]), dtype=torch.float64, device=dev)
        wsd = ps.dd_workspace(1024, 30, 6, 0)
        Ed = torch.empty_like(Td)
        out = {"n": 1024, "m": 30, "s": 6, "sigma": 0, "dtype": "dd"}
        for mode in ("fixed", "mixed"):
            _, rep = ps.ps_expm_dd(Td, 30, s=6, mode=mode, out=Ed, workspace=wsd, report=True)
            t = _time(lambda: ps.ps_expm_dd(Td, 30, s=6, mode=mode, out=Ed, workspace=wsd), 3, torch)
            out[mode] = {"ms": round(t * 1e3, 3), "tiers": [ps.TIER_NAMES[x] for x in rep["tier"][:rep["first_step"] + 1]]}
        out["speedup_mixed_vs_fixed"] = round(out["fixed"]["ms"] / out["mixed"]["ms"], 3)
        res["expm_dd_1024"] = out
    return res


def batched_gate(samples):
    """Accuracy gate of the uneven FP32 batch (part of the oracle leg): on the
    sampled matrices and columns, the mixed results within max(1e-6, 2 err_plain)
    of the oracle (the equal-accuracy rule of the FP32 target)."""
    import numpy as np

    import oracle
    from oracle import coeffs
    c32 = [float(np.float32(x)) for x in coeffs.taylor_exp(18)]
    worst, ok = 0.0, True
    for A, sg, cols, em, ef in samples:
        A = A.astype(np.float32).astype(np.float64)
        wh, wl = oracle.expm_apply_dd(A, c32, sg, np.eye(A.shape[0])[:, cols])
        err = lambda e: float(np.max(np.sum(np.abs((e - wh) - wl), 0)) / np.max(np.sum(np.abs(wh), 0)))
        e_m, e_f = err(em), err(ef)
        worst = max(worst, e_m)
        ok = ok and e_m <= max(1e-6, 2 * e_f)
    return {"rule": "err_mixed <= max(1e-6, 2 err_plain) per matrix", "matrices": len(samples),
            "max_rel_err_mixed": float("%.3e" % worst), "ok": ok,
            "note": "every 128th matrix, two columns each, against the oracle's dd evaluation"}


def cpu_baseline(mats, outs_mixed, norms, sigmas):
    """The oracle's plain FP64 Algorithm 1 + squarings on the host cores (one
    evaluation of each matrix), and the GPU result against the dd oracle on
    sampled columns."""
    import numpy as np

    import oracle
    from oracle import coeffs

    threads = min(os.cpu_count() or 1, 16)
    oracle.set_threads(threads)
    c = coeffs.taylor_exp(M)
    A_np = [a.cpu().numpy() for a in mats]
    runs = []
    for _ in range(3):                       # median of three runs
        t0 = time.perf_counter()
        for A, sg in zip(A_np, sigmas):
            oracle.expm_ps_f64(A, c, S, sg)
        runs.append(time.perf_counter() - t0)
    dt = sorted(runs)[1]
    errs = []
    for A, sg, e in zip(A_np, sigmas, outs_mixed):
        cols = [0, N // 2 + 1]
        V = np.eye(N)[:, cols]
        wh, wl = oracle.expm_apply_dd(A, c, sg, V)
        got = e.cpu().numpy()[:, cols]
        d = (got - wh) - wl
        errs.append(float(np.max(np.sum(np.abs(d), 0)) / np.max(np.sum(np.abs(wh), 0))))
    # one core: the sigma = 0 matrix alone
    oracle.set_threads(1)
    t1 = time.perf_counter()
    oracle.expm_ps_f64(A_np[1], c, S, sigmas[1])
    d1 = time.perf_counter() - t1
    oracle.set_threads(threads)
    cpu = "unknown"
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                cpu = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": round(len(A_np) / dt, 4), "unit": "evals/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu,
            "sample": "one evaluation of each of the 4 dense n=1024 matrices by the oracle's FP64 "
                      "Algorithm 1 + squarings; median of 3 runs (%s s)" % ", ".join("%.2f" % r for r in runs),
            "single_core": {"value": round(1.0 / d1, 4), "unit": "evals/s",
                            "sample": "the ||A||_1 = 1 matrix (sigma = 0) once on one thread (%.1f s)" % d1},
            "gpu_mixed_rel_err_vs_dd_oracle_sampled_cols": [float("%.3e" % e) for e in errs]}


if __name__ == "__main__":
    main()
