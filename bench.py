#!/usr/bin/env python3
"""Benchmark of the hardware-fitted linear run-time model on one MI355X.

Timed step: one batched pass of the counter + FP64 prediction (libpm's
six counter kernels) over the batched-sweep workload -- 4096 tiled/naive
matmul, stencil and transpose variants whose main iteration domains hold
2^U(16,30) points, extents not multiples of the tile -- with the variants
already resident in HBM.  Reported `value`: variants counted and predicted
per second.

Also reported, outside the timed region:
  * the plain per-variant path (one synchronous pm_count call per variant,
    host in / host out) and the batched/plain ratio;
  * the model itself: the instructive suite measured (4 warm-ups, 26 timed
    runs, minimum) and fitted (relative-error least squares), then the test
    suite measured and predicted: geometric-mean relative error;
  * per-kernel HIP-event times of the counter over the timed steps and the
    roofline of the dominant kernel;
  * the CPU oracle (simulated execution) on a bounded sample of the same
    workload, extrapolated by its event rate.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--skip-model]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12  # bytes/s, MI355X HBM3E


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def domain_points(v):
    """Points of the variant's main iteration domain."""
    f = v["family"]
    if f == "matmul":
        return v["n"] * v["m"] * v["l"]
    if f in ("stencil", "transpose"):
        return v["n"] * v["n"]
    if f == "nbody":
        return v["n"] * v["n"]
    return v.get("n", 0)


# Issue peak of plain vector ALU work: 256 CUs x 4 SIMDs x 16 lanes per
# clock at 2.4 GHz = 3.93e13 lane operations/s (a wave64 instruction takes
# four clocks on a 16-lane SIMD).
ALU_PEAK = 256 * 4 * 16 * 2.4e9
KERNEL_SOURCES = ("include/pm.h", "paper_1604_04997_amd/csrc/desc.h",
                  "paper_1604_04997_amd/csrc/counter.h",
                  "paper_1604_04997_amd/csrc/counter.hip")
PMC_SUMMARY = "profiles/counter_batched4096_pmc.txt"
COPY_BYTES = 2 * (1 << 26) * 4  # the calibration copy: 2^26 fp32 read + written


def source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_pmc():
    """Per-dispatch hardware counters of the counter kernels on the batched
    workload, from the committed rocprofv3 summary, or None when the kernel
    sources have changed since it was taken."""
    path = os.path.join(ROOT, PMC_SUMMARY)
    if not os.path.exists(path):
        return None
    rows, h = {}, None
    for line in open(path):
        if line.startswith("# kernel sources sha256/16:"):
            h = line.split(":")[1].strip()
        if line.startswith("#") or not line.strip():
            continue
        name, rest = line.split(" grid=", 1)
        kv = dict(x.split("=") for x in ("grid=" + rest).split())
        kv = {k: float(x) for k, x in kv.items()}
        name = name.split("::")[-1].split("<")[0]
        if name not in rows or kv["grid"] > rows[name]["grid"]:
            rows[name] = kv
    if h != source_hash():
        return None
    return rows


def counter_roofline(phase, ms, nv):
    """Roofline of the dominant counter kernel.  Its work is integer
    bookkeeping (descriptor expansion, closed-form counts, count vector),
    bounded by the vector ALU: achieved = live VALU lane operations per launch
    (rocprofv3 SQ_THREAD_CYCLES_VALU per dispatch: VALU instructions times
    the lanes active in each) / the launch's live HIP-event duration, against
    256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz.  traffic = FETCH_SIZE and
    WRITE_SIZE per dispatch, each scaled by what it reads for a copy of known
    size."""
    kern = "k_" + phase
    roof = {"kernel": kern, "bound": "alu", "achieved": None, "peak": round(ALU_PEAK / 1e12, 2),
            "unit": "TOP/s (live int lane-ops)", "frac": None, "traffic": None,
            "launch_ms": round(ms, 4), "variants_per_launch": nv,
            "variants_per_s_in_kernel": round(nv / (ms * 1e-3), 1)}
    pmc = read_pmc()
    if not pmc or kern not in pmc:
        roof["note"] = "no counter summary for the current kernel sources"
        return roof
    r = pmc[kern]
    live = r["SQ_THREAD_CYCLES_VALU"]
    ach = live / (ms * 1e-3)
    roof.update({"achieved": round(ach / 1e12, 3), "frac": round(ach / ALU_PEAK, 4),
                 "live_lane_ops_per_launch": live,
                 "active_lanes_per_valu_instr": round(live / r["SQ_INSTS_VALU"], 1),
                 "issue_frac_64_lanes": round(r["SQ_INSTS_VALU"] * 64 / (ms * 1e-3) / ALU_PEAK, 4),
                 "valu_instr_per_variant": round(r["SQ_INSTS_VALU"] / nv, 1)})
    cal = pmc.get("k_stream")
    if cal and "FETCH_SIZE" in r and "WRITE_SIZE" in r:
        fs = (COPY_BYTES / 2) / (cal["FETCH_SIZE"] * 1024)
        ws = (COPY_BYTES / 2) / (cal["WRITE_SIZE"] * 1024)
        roof["traffic"] = round((r["FETCH_SIZE"] * fs + r["WRITE_SIZE"] * ws) * 1024)
        roof["traffic_scale"] = {"fetch": round(fs, 3), "write": round(ws, 3)}
        # algorithmic bytes: variants in (88 B), count vectors (PM_NCOUNT
        # int64), predictions (8 B) and statuses (4 B) out
        import ctypes
        import paper_1604_04997_amd as P
        roof["algorithmic_bytes"] = nv * (ctypes.sizeof(P.Variant) + 8 * P.PM_NCOUNT + 8 + 4)
    return roof


def measure_suite(ctx, P, variants, warmup=4, reps=26):
    """Minimum of `reps` timed runs after `warmup` (Sec. 4.2) per variant;
    also which ones fall below twice the context's launch floor."""
    import torch
    T, low = [], []
    for i, v in enumerate(variants):
        ts, _ = P.device_buffers(v, v.get("seed", i), fast=True)
        r = ctx.measure_until(v, ts, warmup=warmup, reps=reps)
        assert r["status"] == 0
        T.append(r["t_min"])
        low.append(r["below_floor"])
        del ts
        if i % 25 == 0:
            log("  measured %d/%d (%s: %.3g ms)" % (i + 1, len(variants), v["family"],
                                                    r["t_min"] * 1e3))
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return np.array(T), np.array(low, dtype=bool)


def geomean(e):
    return float(math.exp(np.mean(np.log(np.maximum(np.asarray(e, dtype=np.float64), 1e-12)))))


def c1_phase(ctx, P):
    """The plain method on the tiny suite (4 fp32 stream loads at lane
    stride 1/2/4/8, 2 fp32 FMA loops): 4 untimed and 10 timed runs each,
    counts on the GPU, the 3-feature fit [global bytes, fp32 FMAs,
    work-groups] in FP64 (pm_fit), predictions through pm_predict; the
    geometric mean of the relative errors of the six."""
    from synth import suite_tiny
    vs = suite_tiny()
    T, low = measure_suite(ctx, P, vs, warmup=4, reps=10)
    cnt = ctx.count_raw(vs)
    m, cond, resid, rank = P.fit(cnt, T, "p3")
    pred = ctx.predict(m, vs)
    err = np.abs(pred - T) / T
    return {"geomean": float("%.3g" % geomean(err)), "rank": rank, "cond": float("%.3g" % cond),
            "alpha": [float("%.4g" % a) for a in P.model_alpha(m)],
            "ms_measured": [round(t * 1e3, 5) for t in T],
            "ms_predicted": [round(float(t) * 1e3, 5) for t in pred],
            "below_launch_floor": int(low.sum())}


def model_phase(ctx, P, proj_list=("p12", "full", "ext", "bank")):
    from synth import suite_instructive, suite_test
    # the paper's instructive suite, plus grids smaller than the GPU holds at
    # once, which only the extension projection is fitted on
    meas = suite_instructive(extended=True)
    test = suite_test()
    log("model: measuring %d instructive variants" % len(meas))
    Tm, low_m = measure_suite(ctx, P, meas)
    cm = ctx.count_raw(meas)
    log("model: measuring %d test variants" % len(test))
    Tt, low_t = measure_suite(ctx, P, test)
    out = {}
    models = {}
    for proj in proj_list:
        rows = [i for i, v in enumerate(meas)
                if proj in ("ext", "bank") or not v.get("extension")]
        sub = (P.Counts * len(rows))(*[cm[i] for i in rows])
        m, cond, resid, rank = P.fit(sub, Tm[rows], proj)
        pred = ctx.predict(m, test)  # counted and predicted on the GPU
        err = np.abs(pred - Tt) / Tt
        fam = {}
        for f in ("finite_difference", "skinny_mm", "nbody", "convolution",
                  "matmul", "transpose"):
            e = [err[i] for i, v in enumerate(test) if v["kernel"] == f]
            fam[f] = round(float(math.exp(np.mean(np.log(np.maximum(e, 1e-12))))), 4)
        paper4 = [err[i] for i, v in enumerate(test) if v["kernel"] in
                  ("finite_difference", "skinny_mm", "nbody", "convolution")]
        gm = float(math.exp(np.mean(np.log(np.maximum(err, 1e-12)))))
        fit_err = float(math.exp(np.mean(np.log(np.maximum(np.abs(resid), 1e-12)))))
        table = {}
        for i, v in enumerate(test):
            if v["kernel"] in ("finite_difference", "skinny_mm", "nbody", "convolution") \
                    and v.get("dtype", "f32") == "f32":
                size = v["m"] if v["kernel"] == "skinny_mm" else v["n"]
                table.setdefault(v["kernel"], []).append(
                    [size, round(Tt[i] * 1e3, 4), round(float(pred[i]) * 1e3, 4)])
        # work-group size sensitivity: error by tile (work-group T x T) and
        # by n-body block size
        by_wg = {}
        for i, v in enumerate(test):
            wg = v.get("T", v.get("wg"))
            if wg:
                by_wg.setdefault("%s.%d" % (v["kernel"], wg), []).append(err[i])
        by_wg = {k: round(float(math.exp(np.mean(np.log(np.maximum(e, 1e-12))))), 4)
                 for k, e in sorted(by_wg.items())}
        out[proj] = {"geomean": round(gm, 4), "per_kernel": fam, "per_work_group": by_wg,
                     "table1_ms_actual_predicted": table,
                     "geomean_paper_test_kernels": round(float(math.exp(np.mean(np.log(
                         np.maximum(paper4, 1e-12))))), 4), "rank": rank,
                     "cond": float("%.3g" % cond), "fit_geomean": round(fit_err, 4)}
        models[proj] = m
    out["below_launch_floor"] = {
        "instructive": int(low_m.sum()), "test": int(low_t.sum()),
        "instructive_families": sorted({v["family"] for v, f in zip(meas, low_m) if f}),
        "test_kernels": sorted({v["kernel"] for v, f in zip(test, low_t) if f})}
    return out, models, (meas, Tm, test, Tt)


def wg_phase(ctx, P, models, fitdata, proj_list=("ext", "p12")):
    """Work-group size sensitivity (Sec. 5): the measurement kernels and
    the n-body test kernel at 128, 256 and 512 work-items per group, total
    work fixed.  Per kernel, the spread of measured and of predicted run
    time over the sizes (largest / smallest - 1); per size, the geometric
    mean relative error of the fitted model and its rank among the sizes
    (1 = most accurate); and the test suite's error when the model is
    fitted, as in the paper, on the measurement kernels at every size
    rather than at 256 alone."""
    from synth import WG_SIZES, suite_wg
    vs = suite_wg()
    log("work-group sizes: measuring %d variants" % len(vs))
    T, low = measure_suite(ctx, P, vs)
    cw = ctx.count_raw(vs)
    meas, Tm, test, Tt = fitdata
    cm = ctx.count_raw(meas)
    bases = sorted({v["base"] for v in vs})
    of = {b: [i for i, v in enumerate(vs) if v["base"] == b] for b in bases}

    def spread(t):
        sp = np.array([max(t[i] for i in of[b]) / min(t[i] for i in of[b]) - 1 for b in bases])
        worst = bases[int(np.argmax(sp))]
        v = vs[of[worst][0]]
        return {"median": round(float(np.median(sp)), 4), "max": round(float(sp.max()), 4),
                "under_30pct": round(float(np.mean(sp < 0.3)), 4),
                "largest": "%s.%s" % (v["family"], v.get("op", v.get("dtype", "")))}

    out = {"variants": len(vs), "kernels": len(bases), "sizes": list(WG_SIZES),
           "below_launch_floor": int(low.sum()), "runtime_spread": spread(T)}
    wrows = [i for i, v in enumerate(vs) if v["family"] != "nbody"]
    for proj in proj_list:
        if proj not in models:
            continue
        pred = ctx.predict(models[proj], vs)
        err = np.abs(pred - T) / T
        by = {wg: geomean([err[i] for i, v in enumerate(vs) if v["wg"] == wg]) for wg in WG_SIZES}
        order = sorted(WG_SIZES, key=lambda w: by[w])
        nb = {wg: geomean([err[i] for i, v in enumerate(vs) if v["wg"] == wg and
                           v["family"] == "nbody"]) for wg in WG_SIZES}
        rows = [i for i, v in enumerate(meas) if proj in ("ext", "bank") or not v.get("extension")]
        sub = (P.Counts * (len(rows) + len(wrows)))(*([cm[i] for i in rows] +
                                                      [cw[i] for i in wrows]))
        m2, _, _, _ = P.fit(sub, np.concatenate([Tm[rows], T[wrows]]), proj)
        e1 = np.abs(ctx.predict(models[proj], test) - Tt) / Tt
        e2 = np.abs(ctx.predict(m2, test) - Tt) / Tt
        out[proj] = {"geomean_by_wg": {str(w): round(by[w], 4) for w in WG_SIZES},
                     "wg256_rank": order.index(256) + 1,
                     "nbody_geomean_by_wg": {str(w): round(nb[w], 4) for w in WG_SIZES},
                     "predicted_spread": spread(pred),
                     "test_geomean_fit_wg256": round(geomean(e1), 4),
                     "test_geomean_fit_all_wg": round(geomean(e2), 4)}
    return out


def c4_phase(ctx, P, vs, pred, per_family=8):
    """Model ranking of the batched sweep: every variant's FP64 prediction
    comes from the counted pass; per family the `per_family` variants with
    the highest predicted rate (domain points per predicted second, the
    autotuning objective) are measured (4 untimed + 26 timed runs, minimum).
    Reported per family: the rank correlation of predicted and measured rate
    among them, whether the predicted-best is the measured-best, and the
    geometric-mean relative error of their predictions.  The top variants'
    predicted rates lie close together, so the same is reported for
    `per_family` variants spread evenly over the family's predicted-rate
    ranking (its first, last and evenly spaced ranks between)."""
    import torch

    def measure(sel):
        T = []
        for i in sel:
            ts, _ = P.device_buffers(vs[i], vs[i].get("seed", i), fast=True)
            r = ctx.measure_until(vs[i], ts, warmup=4, reps=26)
            assert r["status"] == 0
            T.append(r["t_min"])
            del ts
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        return np.array(T)

    def agree(sel, T, rate):
        pr = np.array([rate[i] for i in sel])
        mr = np.array([domain_points(vs[i]) for i in sel]) / T
        rp, rm = np.argsort(np.argsort(-pr)), np.argsort(np.argsort(-mr))
        e = np.abs(np.array([pred[i] for i in sel]) - T) / T
        rows = [[vs[i].get("op", vs[i].get("dtype")), vs[i].get("T"), int(domain_points(vs[i])),
                 round(float(pred[i]) * 1e3, 4), round(float(t) * 1e3, 4)]
                for i, t in zip(sel, T)]
        return float(np.corrcoef(rp, rm)[0, 1]), bool(rm[0] == 0), e, rows

    out, errs, serrs = {}, [], []
    for fam in ("matmul", "stencil", "transpose"):
        idx = [i for i, v in enumerate(vs) if v["family"] == fam]
        rate = {i: domain_points(vs[i]) / pred[i] for i in idx}
        order = sorted(idx, key=lambda i: -rate[i])
        top = order[:per_family]
        rho, best, e, rows = agree(top, measure(top), rate)
        errs += list(e)
        spread = [order[int(k)] for k in np.linspace(0, len(order) - 1, per_family).round()]
        srho, _, se, srows = agree(spread, measure(spread), rate)
        serrs += list(se)
        out[fam] = {"spearman": round(rho, 4), "predicted_best_is_measured_best": best,
                    "geomean_rel_err": round(geomean(e), 4), "measured": rows,
                    "spread_spearman": round(srho, 4),
                    "spread_geomean_rel_err": round(geomean(se), 4), "spread_measured": srows}
    fams = ("matmul", "stencil", "transpose")
    out["geomean_rel_err"] = round(geomean(errs), 4)
    out["mean_spearman"] = round(float(np.mean([out[f]["spearman"] for f in fams])), 4)
    out["spread_geomean_rel_err"] = round(geomean(serrs), 4)
    out["spread_mean_spearman"] = round(float(np.mean([out[f]["spread_spearman"]
                                                       for f in fams])), 4)
    out["note"] = ("measured rows: op (stencil: dtype), tile, domain points, predicted ms, "
                   "measured ms")
    return out


def qpoly_phase(ctx, P, vs, counts, reps=20):
    """Counts as quasi-polynomials of the size (Sec. 3.2, re-evaluated
    cheaply, Sec. 2): for every single-size configuration of the sweep
    (stencil and transpose by op, dtype and tile) the counts are derived
    once from the batched counter (period = the tile, from n = 64), then
    every such sweep variant is evaluated on the host (pm_qpoly_eval_many)
    and compared with the GPU's counts of the timed pass."""
    groups = {}
    for i, v in enumerate(vs):
        if v["family"] in ("stencil", "transpose"):
            groups.setdefault((v["family"], v.get("op"), v.get("dtype"), v["T"]), []).append(i)
    t0 = time.perf_counter()
    qps = {}
    for key, idx in groups.items():
        d = {k: x for k, x in vs[idx[0]].items() if k != "seed"}
        d["n"] = 0
        qps[key] = ctx.qpoly_derive(d, fields=1, scale=1, period=key[3], x0=64)
    t_derive = time.perf_counter() - t0
    xs = {key: [vs[i]["n"] for i in idx] for key, idx in groups.items()}
    best = 1e9
    for _ in range(reps):
        t1 = time.perf_counter()
        outs = {key: P.qpoly_eval_many(qps[key], xs[key]) for key in groups}
        best = min(best, time.perf_counter() - t1)
    n = sum(len(idx) for idx in groups.values())
    mism = 0
    for key, idx in groups.items():
        ev = P.counts_numpy(outs[key])
        mism += int((ev != counts[idx]).any(axis=1).sum())
    assert mism == 0, "%d quasi-polynomial evaluations differ from the counter" % mism
    return {"configurations": len(groups), "variants": n,
            "derivation_s": round(t_derive, 4),
            "derivation_variants_counted": int(sum(6 * k[3] for k in groups)),
            "eval_per_s": round(n / best, 1), "us_per_eval": round(best / n * 1e6, 3),
            "equal_to_counter": n - mism}


def suite_roofline(ctx, P):
    """Unit-stride stream kernels against the 8 TB/s HBM peak (1 GiB+
    working sets, far past the 256 MB last-level cache) and FMA loops
    against the vector FP32 / FP64 peaks."""
    res = {"stream": [], "fma": []}
    for op, mult in (("load", 1), ("copy", 2)):
        for dt, esz in (("f32", 4), ("f64", 8)):
            for vec, U in ((1, 1), (1, 4), (1, 8), (1, 16), (4 if dt == "f32" else 2, 1),
                           (4 if dt == "f32" else 2, 4)):
                for nt in (False, True):
                    elems = (1 << 28) if dt == "f32" else (1 << 27)
                    v = dict(family="stream", op=op, dtype=dt, n=elems // (vec * U), wg=256,
                             s=1, gs=1, vec=vec, U=U, streaming=nt)
                    ts, _ = P.device_buffers(v, 11, fast=True)
                    t, _ = ctx.measure(v, ts, warmup=3, reps=20)
                    del ts
                    gbs = mult * elems * esz / t
                    res["stream"].append({"op": op, "dtype": dt, "vec": vec, "U": U,
                                          "streaming_hint": nt,
                                          "bytes": mult * elems * esz,
                                          "ms": round(t * 1e3, 4), "GB/s": round(gbs / 1e9, 1),
                                          "frac_8TBs": round(gbs / HBM_PEAK, 4)})
    for op in ("load", "copy"):
        best = max((r for r in res["stream"] if r["op"] == op), key=lambda r: r["frac_8TBs"])
        res["best_" + op] = {k: best[k] for k in ("dtype", "vec", "U", "streaming_hint",
                                                   "GB/s", "frac_8TBs")}
        # the 32-bit access class alone (fp32, one element per access)
        b4 = max((r for r in res["stream"] if r["op"] == op and r["dtype"] == "f32"
                  and r["vec"] == 1), key=lambda r: r["frac_8TBs"])
        res["best_%s_4B" % op] = {k: b4[k] for k in ("U", "streaming_hint", "GB/s",
                                                     "frac_8TBs")}
    for dt, peak_pub in (("f32", 157.3e12), ("f64", 78.6e12)):
        v = dict(family="fma", dtype=dt, n=1 << 24, wg=256, F=1024, K=16)
        ts, _ = P.device_buffers(v, 12, fast=True)
        t, _ = ctx.measure(v, ts, warmup=3, reps=20)
        del ts
        fl = 2.0 * 1024 * (1 << 24) / t
        res["fma"].append({"dtype": dt, "TFLOP/s": round(fl / 1e12, 2),
                           "frac_published_peak": round(fl / peak_pub, 4)})
    import torch
    torch.cuda.empty_cache()
    return res


def host_cpu():
    """CPU model and logical CPU count of the host (for the record)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count() or 1


def cpu_baseline(workload, gpu_counts, names, budget_s=15.0, par_budget_s=8.0,
                 max_threads=16):
    """Simulated-execution oracle on a bounded random sample of the workload:
    variants in random order until ~budget_s of oracle time; its event rate
    (events = sum of a variant's count vector) extrapolates the whole
    workload.  Then the same oracle on every core the host offers (threads
    calling the C oracle, which runs without the interpreter lock; at most
    max_threads) for ~par_budget_s of wall time, reported beside it.  Every
    oracle result is compared with the GPU's count vector of the same
    variant; a mismatch fails the run."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle import count as OC
    rng = np.random.default_rng(42)
    order = rng.permutation(len(workload))
    ev_all = gpu_counts.sum(axis=1).astype(np.float64)
    t_used, ev_used, done = 0.0, 0.0, 0

    def check(i, got):
        want = {names[k]: int(x) for k, x in enumerate(gpu_counts[i]) if x}
        if got != want:
            raise AssertionError("oracle and GPU counts differ for variant %d: %s" %
                                 (i, workload[i]))

    for i in order:
        if ev_all[i] > 3e8:  # one oracle call must stay a few seconds
            continue
        t0 = time.perf_counter()
        got = OC.count(workload[i])
        t_used += time.perf_counter() - t0
        check(i, got)
        ev_used += ev_all[i]
        done += 1
        if t_used > budget_s:
            break
    rate = ev_used / t_used
    est = ev_all.sum() / rate
    model, ncpu = host_cpu()
    res = {"value": round(len(workload) / est, 4), "unit": "variants/s",
           "cores": 1, "kind": "oracle",
           "sample": "%d of %d workload variants (random order, those under "
                     "3e8 events), %.1f s, %.3g events/s; value = 4096 / "
                     "(all variants' events / that rate); every sampled count "
                     "vector equal to the GPU's; host: %s, %d logical CPUs"
                     % (done, len(workload), t_used, rate, model, ncpu),
           "sample_variants_per_s": round(done / t_used, 3), "checked_vs_gpu": done}
    # all cores: the next variants of the same order, one per thread
    nthr = max(1, min(ncpu, max_threads))
    rest = [i for i in order if ev_all[i] <= 3e8][done:]
    ev_par, n_par = 0.0, 0
    t0 = time.perf_counter()
    with ThreadPoolExecutor(nthr) as ex:
        pending = []
        it = iter(rest)
        for _ in range(nthr):
            i = next(it, None)
            if i is not None:
                pending.append((i, ex.submit(OC.count, workload[i])))
        while pending:
            i, fu = pending.pop(0)
            check(i, fu.result())
            ev_par += ev_all[i]
            n_par += 1
            if time.perf_counter() - t0 < par_budget_s:
                j = next(it, None)
                if j is not None:
                    pending.append((j, ex.submit(OC.count, workload[j])))
    wall = time.perf_counter() - t0
    if n_par and wall > 0:
        prate = ev_par / wall
        res["all_cores"] = {
            "value": round(len(workload) / (ev_all.sum() / prate), 4), "unit": "variants/s",
            "cores": nthr,
            "sample": "%d further variants on %d threads, %.1f s wall, %.3g events/s"
                      % (n_par, nthr, wall, prate), "checked_vs_gpu": n_par}
    return res


def output_oracle_timing(ctx, P, n=2048, max_threads=16):
    """The output oracle of the matmul test kernel (NumPy, FP64) timed on the
    host with its BLAS pinned to one thread and to every core (at most
    max_threads), beside the GPU's tiled fp32 kernel of the same size
    (minimum of 26 timed runs)."""
    from threadpoolctl import threadpool_limits
    from oracle import outputs as O
    from synth import uniform
    A = uniform(11, n * n).reshape(n, n)
    B = uniform(12, n * n).reshape(n, n)
    flop = 2.0 * n ** 3
    out = {"kernel": "C = A B, n = m = l = %d: NumPy FP64 (the oracle) vs the tiled fp32 "
                     "kernel (T = 16)" % n}
    _, ncpu = host_cpu()
    for key, thr in (("1_thread", 1), ("all_cores", max(1, min(ncpu, max_threads)))):
        with threadpool_limits(limits=thr):
            O.matmul(A, B)  # warm
            best = 1e9
            for _ in range(3):
                t0 = time.perf_counter()
                O.matmul(A, B)
                best = min(best, time.perf_counter() - t0)
        out["oracle_gflops_" + key] = round(flop / best / 1e9, 1)
        out["threads_" + key] = thr
    v = dict(family="matmul", op="tiled", n=n, m=n, l=n, T=16)
    ts, _ = P.device_buffers(v, 13, fast=True)
    r = ctx.measure_until(v, ts, warmup=4, reps=26)
    del ts
    out["gpu_gflops"] = round(flop / r["t_min"] / 1e9, 1)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=64)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--skip-model", action="store_true")
    ap.add_argument("--plain-sample", type=int, default=1024)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--autotune-problems", type=int, default=8)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed steps, copy 2^26 fp32 once (a kernel of "
                         "known traffic for scaling hardware byte counters)")
    ap.add_argument("--suite-roofline-only", action="store_true",
                    help="only the stream and FMA roofline measurements (one JSON "
                         "line of them; for profiling those kernels)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the counter's work is per variant and "
              "independent, so a multi-GPU run would shard the variant list; "
              "this build runs and reports --gpus 1 only", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1604_04997_amd as P
    from synth import suite_batched

    assert torch.cuda.is_available(), "no GPU"
    dev = torch.cuda.get_device_properties(0)
    log("device:", dev.name, "CUs:", dev.multi_processor_count)
    ctx = P.Context(0, hbm_budget=128 << 30)
    if args.suite_roofline_only:
        print(json.dumps(suite_roofline(ctx, P)), flush=True)
        return

    # launch overhead first (Sec. 4.2): the empty kernel's minimum time;
    # measurements below twice it are flagged
    floor = ctx.launch_floor()
    log("launch floor: %.2f us" % (floor * 1e6))

    # ------------------------------------------------------------- model --
    model_info, models, c1, wgs = None, {}, None, None
    if not args.skip_model:
        c1 = c1_phase(ctx, P)
        log("tiny plain-method suite:", json.dumps(c1))
        model_info, models, fitdata = model_phase(ctx, P)
        log("model:", json.dumps(model_info))
        wgs = wg_phase(ctx, P, models, fitdata)
        log("work-group sizes:", json.dumps(wgs))
    # prediction: the paper's property list with its named extensions
    m = models.get("ext") or P.model_struct("ext", [1e-12] * 157)

    # ------------------------------------------------------ batched step --
    vs = suite_batched(4096)
    nv = len(vs)
    va = P.variant_array(vs)
    d_v = torch.frombuffer(bytearray(bytes(memoryview(va).cast("B"))), dtype=torch.uint8).cuda()
    d_c = torch.zeros((nv, P.PM_NCOUNT), dtype=torch.int64, device="cuda")
    d_t = torch.zeros(nv, dtype=torch.float64, device="cuda")
    d_s = torch.zeros(nv, dtype=torch.int32, device="cuda")
    bm_bytes = sum(P.bitmap_bytes(v) for v in vs)
    ctx.reserve(nv, bm_bytes)
    stream = torch.cuda.current_stream().cuda_stream

    # one batch enqueued per step, its arguments marshalled once
    step = ctx.count_device_call(d_v.data_ptr(), nv, d_c.data_ptr(), m, d_t.data_ptr(),
                                 d_s.data_ptr(), stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    assert int((d_s != 0).sum()) == 0, "variants failed: %s" % d_s.unique()
    # the counter's own schedule, tuned on this workload before the timed steps
    from paper_1604_04997_amd import autotune as AT
    default_sched = ctx.schedule()
    # every candidate timed (the reference), then the schedule the counter's
    # own fitted model ranks first, which the timed steps use
    best_timed, sched_table = AT.tune_counter(ctx, step)
    sched, sched_model = AT.tune_counter_model(ctx, step)
    torch.cuda.synchronize()
    assert int((d_s != 0).sum()) == 0
    t_all = {(c["inblock_items"], c["tail_wgs_per_cu"]): t for c, t in sched_table}
    sched_model["exhaustive_best"] = best_timed
    sched_model["exhaustive_best_ms"] = round(min(t_all.values()), 4)
    sched_model["chosen_ms_in_exhaustive"] = round(
        t_all[(sched["inblock_items"], sched["tail_wgs_per_cu"])], 4)
    log("counter schedule: model chose %s (default %s, fastest timed %s); %s" % (
        sched, default_sched, best_timed, json.dumps(sched_model)))
    # the timed steps carry HIP events (taken by the kernel's dispatch) around
    # the expansion kernel of one step in eight: the dominant kernel's live
    # duration for the roofline, at an eighth of the events' cost per step
    ctx.profile(2)
    ctx.profile_sample(8)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    build_ms = ctx.profile_read()[0]["build"]
    ctx.profile(False)
    ctx.profile_sample(1)
    stats = ctx.batch_stats()
    assert int((d_s != 0).sum()) == 0
    ms_step = (t1 - t0) * 1e3 / args.steps
    value = nv / ((t1 - t0) / args.steps)
    counts = d_c.cpu().numpy()
    points = float(sum(domain_points(v) for v in vs))
    # per-phase breakdown from extra, untimed steps with events around every phase
    ctx.profile(1)
    for _ in range(min(args.steps, 20)):
        step()
    phase_ms, nb = ctx.profile_read()
    ctx.profile(False)
    log("batched: %.3f ms/step, %.0f variants/s; expansion kernel %.4f ms; phases "
        "(events around each) %s" % (ms_step, value, build_ms, phase_ms))

    if args.copy_calibration:
        cv = dict(family="stream", op="copy", dtype="f32", n=1 << 26, wg=256, s=1,
                  gs=1, vec=1, U=1)
        cts, _ = P.device_buffers(cv, 3, fast=True)
        ctx.launch(cv, cts)
        torch.cuda.synchronize()
        del cts

    qpoly = qpoly_phase(ctx, P, vs, counts)
    log("quasi-polynomials:", json.dumps(qpoly))

    c4 = None
    if models:
        log("model ranking of the sweep: measuring the top-8 per family")
        c4 = c4_phase(ctx, P, vs, d_t.cpu().numpy())
        log("sweep ranking:", json.dumps(c4))

    # -------------------------------------------------------- plain path --
    ns = min(args.plain_sample, nv)
    rng = np.random.default_rng(1)
    idx = rng.permutation(nv)[:ns]
    one = [P.variant_array([vs[i]]) for i in idx]
    for a in one[:8]:
        ctx.count_raw(a)
    tp0 = time.perf_counter()
    for a in one:
        ctx.count_raw(a)
    tp1 = time.perf_counter()
    plain = ns / (tp1 - tp0)
    t_call = (tp1 - tp0) / ns
    log("plain: %.0f variants/s (%.1f us per call, %d-variant sample)" % (plain, t_call * 1e6, ns))
    # the whole sweep through the host-memory call (variants in, count
    # vectors out over PCIe): one pm_count of 4096 variants, best of three
    va_host = P.variant_array(vs)
    t_host = []
    for _ in range(3):
        th0 = time.perf_counter()
        ctx.count_raw(va_host)
        t_host.append(time.perf_counter() - th0)
    host_batched = nv / min(t_host)
    log("batched through host memory: %.0f variants/s (%.3f ms per call)" % (
        host_batched, min(t_host) * 1e3))

    # ---------------------------------------------------------- autotune --
    tune = None
    if models and args.autotune_problems > 0:
        from paper_1604_04997_amd import autotune
        probs, seen = [], set()
        for fam in ("matmul", "stencil", "transpose"):
            k = 0
            for v in vs:
                if v["family"] != fam or domain_points(v) > (1 << 27):
                    continue
                key = autotune.problem_key(v)
                if key in seen:
                    continue
                seen.add(key)
                probs.append({x: y for x, y in v.items() if x not in ("op", "T", "seed")})
                k += 1
                if k >= args.autotune_problems:
                    break
        log("autotune: %d problems, every configuration measured" % len(probs))
        res = autotune.rank_and_measure(ctx, m, probs, measure_all=True)
        tune = autotune.summary(res)
        tune["per_problem"] = [
            {"problem": r["problem"],
             "configs": ["%s/%s" % (c.get("op", ""), c.get("T", c.get("wg", ""))) for c in r["configs"]],
             "predicted_ms": [round(x * 1e3, 5) for x in r["predicted"]],
             "measured_ms": [round(x * 1e3, 5) for x in r["measured"]]} for r in res]
        tune["per_family"] = {}
        for fam in ("matmul", "stencil", "transpose"):
            rr = [r for r in res if r["problem"]["family"] == fam]
            if rr:
                tune["per_family"][fam] = autotune.summary(rr)
        log("autotune:", json.dumps({k: x for k, x in tune.items() if k != "per_problem"}))

    # ----------------------------------------------------------- serving --
    serving = None
    if args.serve_seconds > 0:
        from paper_1604_04997_amd import serve
        from synth import serving_trace
        trace = serving_trace(rate=2000.0, duration=args.serve_seconds)
        srv = serve.Server(ctx, m)
        _, st_b = srv.run(trace)
        _, st_p = serve.run_plain(ctx, m, trace)
        # a rate at which requests overlap and batches form
        fast = serving_trace(rate=20000.0, duration=min(args.serve_seconds, 2.0), seed=11)
        _, f_b = srv.run(fast)
        _, f_p = serve.run_plain(ctx, m, fast)
        # capacity: the same requests all queued at once
        _, cap_b = srv.run(trace, realtime=False)
        _, cap_p = serve.run_plain(ctx, m, trace, realtime=False)
        rnd = lambda d: {k: (round(x, 4) if isinstance(x, float) else x)  # noqa: E731
                         for k, x in d.items()}
        serving = {"requests": len(trace), "rate_per_s": 2000.0,
                   "batched": rnd(st_b), "plain": rnd(st_p),
                   "requests_20k": len(fast), "batched_20k": rnd(f_b), "plain_20k": rnd(f_p),
                   "saturated_batched": rnd(cap_b), "saturated_plain": rnd(cap_p)}
        log("serving:", json.dumps(serving))

    # ---------------------------------------------------------- roofline --
    roof = counter_roofline("build", build_ms, nv)
    log("roofline:", json.dumps(roof))

    # ------------------------------------------------- suite rooflines --
    suite_roof = None
    if not args.skip_model:
        suite_roof = suite_roofline(ctx, P)
        log("suite roofline:", json.dumps(suite_roof))

    # ----------------------------------------------------------- CPU leg --
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(vs, counts, P.count_names(), args.cpu_seconds)
        cpu["output_oracle"] = output_oracle_timing(ctx, P)
        log("cpu oracle:", cpu)

    detail = {"model": model_info, "tiny_suite": c1, "work_group_sizes": wgs,
              "sweep_ranking": c4, "qpoly": qpoly,
              "autotune": tune, "serving": serving, "suite_roofline": suite_roof,
              "counter_schedule": {
                  "chosen": sched, "default": default_sched, "model": sched_model,
                  "tried_ms": [[c["inblock_items"], c["tail_wgs_per_cu"], round(t, 4)]
                               for c, t in sched_table]},
              "batch_stats": stats, "kernel_ms": phase_ms, "roofline": roof,
              "cpu_baseline": cpu}
    os.makedirs(os.path.join(ROOT, "gpurun_out"), exist_ok=True)
    with open(os.path.join(ROOT, "gpurun_out", "bench_detail.json"), "w") as fh:
        json.dump(detail, fh, indent=1, default=float)
    gm = None
    if model_info:
        gm = {p: model_info[p]["geomean"] for p in ("ext", "bank", "full", "p12")}
        gm["ext_paper_test_kernels"] = model_info["ext"]["geomean_paper_test_kernels"]
        gm["tiny_p3"] = c1["geomean"] if c1 else None
        gm["sweep_top8"] = c4["geomean_rel_err"] if c4 else None
    srv = None
    if serving:
        srv = {k: {x: serving[k][x] for x in ("p50_ms", "p99_ms", "mean_batch",
                                               "variants_per_s") if x in serving[k]}
               for k in ("batched", "plain", "batched_20k", "plain_20k",
                         "saturated_batched", "saturated_plain")}
    line = {
        "metric": "geomean rel. prediction error; variants counted+predicted/sec, batched vs plain",
        "value": round(value, 1), "unit": "variants/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int64", "data": "synthetic",
        "config": {"workload": "batched autotune sweep: 4096 matmul/stencil/transpose "
                               "variants, main domains 2^16..2^30 points, counted + "
                               "predicted in one pass", "variants": nv,
                   "model": "ext (the paper's property list and its named extensions)"},
        "geomean_rel_err": gm,
        "batched_over_plain": round(value / plain, 2),
        "plain_variants_per_s": round(plain, 1), "plain_us_per_call": round(t_call * 1e6, 2),
        "points_per_s": float("%.4g" % (points * value / nv)),
        "host_memory_batched_variants_per_s": round(host_batched, 1),
        "launch_floor_us": round(floor * 1e6, 2),
        "kernel_ms": {k: round(x, 4) for k, x in phase_ms.items()},
        "counter_schedule": {"model_choice": sched, "model_choice_ms": sched_model["chosen_ms"],
                             "fastest_timed_ms": sched_model["exhaustive_best_ms"]},
        "sweep_ranking": {k: c4[k] for k in ("mean_spearman", "geomean_rel_err",
                                             "spread_mean_spearman", "spread_geomean_rel_err")}
        if c4 else None,
        "qpoly": {k: qpoly[k] for k in ("variants", "us_per_eval", "equal_to_counter")},
        "work_group_sizes": {
            "runtime_spread_median": wgs["runtime_spread"]["median"],
            "ext_geomean_by_wg": wgs["ext"]["geomean_by_wg"],
            "ext_test_fit_wg256_vs_all": [wgs["ext"]["test_geomean_fit_wg256"],
                                          wgs["ext"]["test_geomean_fit_all_wg"]]}
        if wgs and "ext" in wgs else None,
        "autotune": {k: round(tune[k], 4) for k in ("choice_is_best", "geomean_slowdown",
                                                    "mean_spearman", "top2_geomean_slowdown",
                                                    "top3_geomean_slowdown")} if tune else None,
        "serving": srv,
        "hbm": {k: suite_roof[k]["frac_8TBs"] for k in
                ("best_load", "best_copy", "best_load_4B", "best_copy_4B")} if suite_roof else None,
        "fma_frac_peak": {r["dtype"]: r["frac_published_peak"] for r in suite_roof["fma"]}
        if suite_roof else None,
        "roofline": roof, "cpu_baseline": cpu,
        "detail": "gpurun_out/bench_detail.json",
    }
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
