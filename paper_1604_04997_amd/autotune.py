"""Model-ranked configuration selection (the paper's Sec. 6.2 use: pick the
fastest of several equivalent kernel configurations from predictions), and
the schedule tuner of the batched counter itself.

A *problem* is one computation at one size (family, op-independent sizes,
dtype); its *configurations* are the kernel variants that compute it
(tile size, tiled vs naive, coalescing side).  All configurations of all
problems are counted and predicted in one batched pass on the GPU; per
problem the predicted-fastest configurations are measured and compared
with the measured-fastest.
"""
from __future__ import annotations

import math

import numpy as np

from . import device_buffers, variant_array

TILES = (8, 16, 32)


def configurations(v: dict):
    """All kernel variants that compute the same result as `v`."""
    f = v["family"]
    if f == "matmul":
        return [dict(v, op=op, T=T) for op in ("tiled", "naive") for T in TILES]
    if f == "transpose":
        return [dict(v, op=op, T=T) for op in ("tiled", "naive_wc", "naive_rc")
                for T in TILES]
    if f == "stencil":
        return [dict(v, T=T) for T in TILES]
    if f == "nbody":
        return [dict(v, wg=g) for g in (64, 128, 256, 512, 1024)]
    return [dict(v)]


def problem_key(v: dict):
    keep = {k: x for k, x in v.items() if k not in ("op", "T", "wg", "seed")}
    return tuple(sorted(keep.items()))


def rank_and_measure(ctx, model, problems, top_k: int = 3, measure_all=False,
                     warmup: int = 4, reps: int = 26):
    """For each problem: predict every configuration (one batched count +
    predict), measure the top_k predicted (or all), and report the choice.

    Returns a list of dicts with the problem, predicted and measured times
    of the measured configurations, the chosen configuration (predicted
    best), the measured best among those measured, and the slowdown of the
    choice against that best."""
    import torch
    cfgs, owner = [], []
    for pi, p in enumerate(problems):
        for c in configurations(p):
            cfgs.append(c)
            owner.append(pi)
    pred = ctx.predict(model, variant_array(cfgs))
    out = []
    for pi, p in enumerate(problems):
        idx = [i for i, o in enumerate(owner) if o == pi]
        order = sorted(idx, key=lambda i: pred[i])
        meas_idx = order if measure_all else order[:top_k]
        meas = {}
        for i in meas_idx:
            ts, _ = device_buffers(cfgs[i], cfgs[i].get("seed", i), fast=True)
            meas[i], _ = ctx.measure(cfgs[i], ts, warmup=warmup, reps=reps)
            del ts
        torch.cuda.empty_cache()
        best = min(meas, key=meas.get)
        chosen = order[0]
        rec = {"problem": p, "n_configs": len(idx),
               "configs": [cfgs[i] for i in meas_idx],
               "predicted": [float(pred[i]) for i in meas_idx],
               "measured": [float(meas[i]) for i in meas_idx],
               "chosen": cfgs[chosen], "measured_best": cfgs[best],
               "slowdown": float(meas[chosen] / meas[best])}
        if len(meas_idx) >= 3:
            rp = np.argsort(np.argsort([pred[i] for i in meas_idx]))
            rm = np.argsort(np.argsort([meas[i] for i in meas_idx]))
            rec["spearman"] = float(np.corrcoef(rp, rm)[0, 1])
        out.append(rec)
    return out


def topk_slowdown(rec, k: int):
    """Slowdown, against the fastest configuration measured, of keeping the
    fastest of the k configurations with the lowest predicted time (the
    selection protocol of measuring only the model's best few).  Needs the
    record's k best-predicted configurations measured."""
    order = sorted(range(len(rec["predicted"])), key=lambda i: rec["predicted"][i])
    if k > len(order):
        k = len(order)
    return min(rec["measured"][i] for i in order[:k]) / min(rec["measured"])


def summary(results, ks=(2, 3)):
    """Geomean slowdown of the predicted choice, fraction of problems where
    it is the measured best, mean rank correlation, and the geomean slowdown
    of measuring the model's top k and keeping the fastest (for each k in
    `ks`; meaningful when every configuration was measured)."""
    sl = [r["slowdown"] for r in results]
    sp = [r["spearman"] for r in results if "spearman" in r and not math.isnan(r["spearman"])]
    out = {"problems": len(results),
           "choice_is_best": float(np.mean([s <= 1.0 + 1e-12 for s in sl])),
           "geomean_slowdown": float(math.exp(np.mean(np.log(sl)))),
           "max_slowdown": float(max(sl)),
           "mean_spearman": float(np.mean(sp)) if sp else None}
    for k in ks:
        tk = [topk_slowdown(r, k) for r in results]
        out["top%d_geomean_slowdown" % k] = float(math.exp(np.mean(np.log(tk))))
        out["top%d_max_slowdown" % k] = float(max(tk))
    return out


# Schedules of the batched counter tried by tune_counter: the in-block item
# limit decides which variants the expanding work-group counts itself and
# which go to the chip-wide kernels; the chip-wide kernels' work-groups per
# CU trade parallelism against launch cost.
COUNTER_SCHEDULES = [dict(inblock_items=i, tail_wgs_per_cu=w)
                     for i in (0, 1024, 4096, 16384, 65536) for w in (1, 2, 4, 8)]


def tune_counter(ctx, step, candidates=None, warmup: int = 2, reps: int = 10):
    """Time one batched counter pass `step()` (launched on torch's current
    stream) under each candidate schedule: HIP events around each pass,
    minimum over `reps` passes after `warmup`.  Sets the fastest on `ctx`
    and returns (chosen, [(schedule, ms), ...])."""
    import torch
    cands = candidates or COUNTER_SCHEDULES
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(reps)]
    table = []
    for sc in cands:
        cur = ctx.set_schedule(**sc)
        for _ in range(warmup):
            step()
        for e0, e1 in ev:
            e0.record()
            step()
            e1.record()
        torch.cuda.synchronize()
        table.append((cur, min(e0.elapsed_time(e1) for e0, e1 in ev)))
    chosen = min(table, key=lambda r: r[1])[0]
    ctx.set_schedule(**chosen)
    return chosen, table


def schedule_features(ctx, step, sched, n_cu: int = 256):
    """Properties of one counter pass under `sched` (the counter's own
    count vector, read from one untimed pass): 1, variants handed on to the
    chip-wide kernel, its work chunks, fill segments and bitmap words, and
    the chip-wide kernel's one-wavefront work-groups."""
    import torch
    ctx.set_schedule(**sched)
    step()
    torch.cuda.synchronize()
    st = ctx.batch_stats()
    wgs = 4 * n_cu * ctx.schedule()["tail_wgs_per_cu"]
    return np.array([1.0, st["handed_on"], st["chunks"], st["fill_segments"],
                     st["bitmap_words"], wgs], dtype=np.float64)


def _time_pass(step, warmup, reps):
    import torch
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(reps)]
    for _ in range(warmup):
        step()
    for e0, e1 in ev:
        e0.record()
        step()
        e1.record()
    torch.cuda.synchronize()
    return min(e0.elapsed_time(e1) for e0, e1 in ev)


def tune_counter_model(ctx, step, candidates=None, n_timed: int = 8, warmup: int = 2,
                       reps: int = 10, n_cu: int = 256):
    """The counter's schedule ranked by a linear model of its own pass time
    (the method of Sec. 4.3 applied to the counter): every candidate's
    properties come from one untimed pass; `n_timed` candidates spread over
    the list are timed; T = sum_i a_i f_i is fitted to them by relative-error
    least squares in FP64; every candidate is predicted and the predicted
    fastest is set on `ctx` and timed.  Returns (chosen, report)."""
    cands = candidates or COUNTER_SCHEDULES
    F = np.array([schedule_features(ctx, step, sc, n_cu) for sc in cands])
    idx = sorted(set(np.linspace(0, len(cands) - 1, min(n_timed, len(cands))).round().astype(int)))
    T = {}
    for i in idx:
        ctx.set_schedule(**cands[i])
        T[i] = _time_pass(step, warmup, reps)
    A = F[idx] / np.array([T[i] for i in idx])[:, None]
    keep = np.abs(A).sum(axis=0) > 0
    alpha = np.zeros(F.shape[1])
    alpha[keep] = np.linalg.lstsq(A[:, keep], np.ones(len(idx)), rcond=None)[0]
    pred = F @ alpha
    best = int(np.argmin(pred))
    chosen = ctx.set_schedule(**cands[best])
    t_best = T.get(best)
    if t_best is None:
        t_best = _time_pass(step, warmup, reps)
    timed_fast = min(T, key=T.get)
    rp = np.argsort(np.argsort([pred[i] for i in idx]))
    rm = np.argsort(np.argsort([T[i] for i in idx]))
    report = {"timed": [[cands[i]["inblock_items"], cands[i]["tail_wgs_per_cu"],
                         round(T[i], 4), round(float(pred[i]), 4)] for i in idx],
              "chosen_ms": round(t_best, 4), "fastest_timed_ms": round(T[timed_fast], 4),
              "spearman_timed": float(np.corrcoef(rp, rm)[0, 1]) if len(idx) > 2 else None,
              "passes": len(cands) + len(idx) * (warmup + reps) +
                        (0 if best in T else warmup + reps)}
    return chosen, report
