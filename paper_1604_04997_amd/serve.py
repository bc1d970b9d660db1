"""Serving loop: predict and measure requests with continuous batching.

Requests arrive over time (a Poisson trace, synth.serving_trace).  The loop,
every step:

  1. moves arrived requests into the wait queue;
  2. retires finished work: a predict batch is done when its event on the
     count stream has fired (its predictions and statuses were copied to
     pinned host memory behind it on the same stream); a measure request is
     done when its last event on the measure stream has fired;
  3. admits waiting predict requests into free slots of a device-resident
     slot ring (variants, count vectors, predictions and statuses stay in
     HBM) and launches them as ONE batched count + predict (libpm
     pm_count_device) on the count stream -- requests that arrived while
     earlier batches were on the GPU join the next batch;
  4. admits waiting measure requests while their kernel buffers fit the
     HBM budget next to those in flight -- at most `measure_admit` per
     step, so that the loop comes back to retire and launch predict
     batches between them -- and launches their warm-up and timed runs
     (pm_launch bracketed by events) on the measure stream, so they
     overlap with the count batches.

Latency of a request = time its result is on the host - its arrival time
(with realtime=False every request arrives at the start).
`run_plain` processes the same trace one request at a time, synchronously.
"""
from __future__ import annotations

import collections
import ctypes
import time

import numpy as np

from . import (PM_NCOUNT, Context, Model, Variant, buffers, counts_numpy,
               device_buffers, variant_array, variant_struct)

VSIZE = ctypes.sizeof(Variant)


class Server:
    def __init__(self, ctx: Context, model: Model, slots: int = 8192,
                 max_batch: int = 2048, hbm_budget: int = 32 << 30,
                 bitmap_bytes: int = 1 << 30, warmup: int = 2, reps: int = 5,
                 measure_admit: int = 1):
        import torch
        self.torch = torch
        self.ctx, self.model = ctx, model
        self.slots, self.max_batch = slots, min(max_batch, slots)
        self.budget = hbm_budget
        self.warmup, self.reps = warmup, reps
        self.measure_admit = measure_admit
        self.d_var = torch.zeros(slots * VSIZE, dtype=torch.uint8, device="cuda")
        self.d_counts = torch.zeros((slots, PM_NCOUNT), dtype=torch.int64, device="cuda")
        self.d_pred = torch.zeros(slots, dtype=torch.float64, device="cuda")
        self.d_status = torch.zeros(slots, dtype=torch.int32, device="cuda")
        self.h_var = torch.zeros(slots * VSIZE, dtype=torch.uint8).pin_memory()
        self.h_pred = torch.zeros(slots, dtype=torch.float64).pin_memory()
        self.h_status = torch.zeros(slots, dtype=torch.int32).pin_memory()
        self.h_counts = torch.zeros((slots, PM_NCOUNT), dtype=torch.int64).pin_memory()
        self.cs = torch.cuda.Stream()   # count / predict batches
        self.ms = torch.cuda.Stream()   # measure requests
        ctx.reserve(self.max_batch, bitmap_bytes)
        self.keep_counts = False

    # ------------------------------------------------------------ predict --
    def _launch_batch(self, reqs, head):
        """reqs: [(rid, variant)] placed in slots [head, head+n)."""
        n = len(reqs)
        va = variant_array([v for _, v in reqs])
        ctypes.memmove(self.h_var.data_ptr() + head * VSIZE, ctypes.addressof(va), n * VSIZE)
        with self.torch.cuda.stream(self.cs):
            dv = self.d_var[head * VSIZE:(head + n) * VSIZE]
            dv.copy_(self.h_var[head * VSIZE:(head + n) * VSIZE], non_blocking=True)
            self.ctx.count_device(dv.data_ptr(), n, self.d_counts[head:head + n].data_ptr(),
                                  self.model, self.d_pred[head:head + n].data_ptr(),
                                  self.d_status[head:head + n].data_ptr(),
                                  self.cs.cuda_stream)
            self.h_pred[head:head + n].copy_(self.d_pred[head:head + n], non_blocking=True)
            self.h_status[head:head + n].copy_(self.d_status[head:head + n], non_blocking=True)
            if self.keep_counts:
                self.h_counts[head:head + n].copy_(self.d_counts[head:head + n], non_blocking=True)
            ev = self.torch.cuda.Event()
            ev.record(self.cs)
        return ev

    # ------------------------------------------------------------ measure --
    def _launch_measure(self, rid, v):
        torch = self.torch
        with torch.cuda.stream(self.ms):
            ts, _ = device_buffers(v, v.get("seed", rid), fast=True)
            for _ in range(self.warmup):
                self.ctx.launch(v, ts, self.ms.cuda_stream)
            evs = []
            for _ in range(self.reps):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(self.ms)
                self.ctx.launch(v, ts, self.ms.cuda_stream)
                b.record(self.ms)
                evs.append((a, b))
        return ts, evs

    # --------------------------------------------------------------- loop --
    def run(self, trace, realtime: bool = True, keep_counts: bool = False,
            keep_outputs: bool = False):
        """Serve `trace` [(arrival_s, kind, variant)].  Returns per-request
        records {id, kind, arrival, done, pred | t_min, status, counts?,
        outputs?} and run statistics.  keep_counts keeps each predict
        request's count vector, keep_outputs each measured kernel's buffers."""
        torch = self.torch
        self.keep_counts = keep_counts
        arrivals = collections.deque(enumerate(trace))
        wait_p, wait_m = collections.deque(), collections.deque()
        batches = collections.deque()    # (event, head, [(rid, v)])
        measures = []                    # (rid, v, bytes, buffers, events)
        head, used_slots, mem = 0, 0, 0
        rec = {}
        n_batches, batch_sizes = 0, []
        t0 = time.perf_counter()
        total = len(trace)
        while len(rec) < total:
            now = time.perf_counter() - t0
            # 1. arrivals
            while arrivals and (not realtime or arrivals[0][1][0] <= now):
                rid, (ta, kind, v) = arrivals.popleft()
                if not realtime:  # every request is queued at the start
                    ta = 0.0
                (wait_p if kind == "predict" else wait_m).append((rid, v, ta))
            # 2. retire finished batches (in stream order) and measures
            while batches and batches[0][0].query():
                ev, h, reqs = batches.popleft()
                t = time.perf_counter() - t0
                n = len(reqs)
                hp = self.h_pred[h:h + n].numpy()
                hs = self.h_status[h:h + n].numpy()
                hc = self.h_counts[h:h + n].numpy() if keep_counts else None
                for k, (rid, v, ta) in enumerate(reqs):
                    r = {"id": rid, "kind": "predict", "arrival": ta, "done": t,
                         "pred": float(hp[k]), "status": int(hs[k])}
                    if keep_counts:
                        r["counts"] = hc[k].copy()
                    rec[rid] = r
                used_slots -= len(reqs)
            still = []
            for m in measures:
                rid, v, nbytes, ts, evs, ta = m
                if evs[-1][1].query():
                    t = time.perf_counter() - t0
                    times = [a.elapsed_time(b) * 1e-3 for a, b in evs]
                    rec[rid] = {"id": rid, "kind": "measure", "arrival": ta, "done": t,
                                "t_min": min(times), "status": 0}
                    if keep_outputs:
                        rec[rid]["outputs"] = ts
                    del ts
                    mem -= nbytes
                else:
                    still.append(m)
            measures = still
            # 3. admit and launch one predict batch
            free = self.slots - used_slots
            n = min(len(wait_p), free, self.max_batch)
            if n > 0:
                if head + n > self.slots:  # wrap: slots are a ring
                    if used_slots == 0:
                        head = 0
                    else:
                        n = min(n, self.slots - head)
                if n > 0:
                    reqs = [wait_p.popleft() for _ in range(n)]
                    ev = self._launch_batch([(rid, v) for rid, v, _ in reqs], head)
                    batches.append((ev, head, reqs))
                    head = (head + n) % self.slots
                    used_slots += n
                    n_batches += 1
                    batch_sizes.append(n)
            # 4. admit measures within the memory budget, a few per step
            admitted = 0
            while wait_m and admitted < self.measure_admit:
                rid, v, ta = wait_m[0]
                nbytes = sum(b for b, _ in buffers(v))
                if mem + nbytes > self.budget and measures:
                    break
                wait_m.popleft()
                ts, evs = self._launch_measure(rid, v)
                measures.append((rid, v, nbytes, ts, evs, ta))
                mem += nbytes
                admitted += 1
            if not realtime and not arrivals and not wait_p and not wait_m:
                torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        out = [rec[i] for i in range(total)]
        stats = {"requests": total, "wall_s": wall, "batches": n_batches,
                 "mean_batch": float(np.mean(batch_sizes)) if batch_sizes else 0.0,
                 "max_batch": int(max(batch_sizes)) if batch_sizes else 0}
        stats.update(latency_stats(out, wall))
        return out, stats


def run_plain(ctx: Context, model: Model, trace, realtime: bool = True,
              warmup: int = 2, reps: int = 5):
    """The same trace, one request at a time: pm_predict for one variant,
    or a synchronous pm_measure."""
    import torch
    t0 = time.perf_counter()
    rec = []
    for rid, (ta, kind, v) in enumerate(trace):
        if realtime:
            while time.perf_counter() - t0 < ta:
                pass
        else:  # every request is queued at the start
            ta = 0.0
        if kind == "predict":
            p = float(ctx.predict(model, [v])[0])
            rec.append({"id": rid, "kind": kind, "arrival": ta,
                        "done": time.perf_counter() - t0, "pred": p})
        else:
            ts, _ = device_buffers(v, v.get("seed", rid), fast=True)
            tmin, _ = ctx.measure(v, ts, warmup=warmup, reps=reps)
            del ts
            rec.append({"id": rid, "kind": kind, "arrival": ta,
                        "done": time.perf_counter() - t0, "t_min": tmin})
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stats = {"requests": len(rec), "wall_s": wall}
    stats.update(latency_stats(rec, wall))
    return rec, stats


def latency_stats(rec, wall):
    """p50 / p99 latency (ms) over all requests and per kind; predicted
    variants per second of wall time."""
    out = {}
    for name, sel in (("", None), ("predict_", "predict"), ("measure_", "measure")):
        lat = np.array([r["done"] - r["arrival"] for r in rec if sel is None or r["kind"] == sel])
        if len(lat):
            out[name + "p50_ms"] = float(np.percentile(lat, 50) * 1e3)
            out[name + "p99_ms"] = float(np.percentile(lat, 99) * 1e3)
    npred = sum(1 for r in rec if r["kind"] == "predict")
    out["predict"] = npred
    out["measure"] = len(rec) - npred
    out["variants_per_s"] = npred / wall
    return out
