"""GPU tests of the serving loop and the model-ranked autotuner.

Serving invariance: every predict request's count vector and prediction in
the continuously batched mix are bit-identical to the same variant counted
alone, and every measured kernel's output equals a solo launch of that
kernel on the same inputs."""
import numpy as np
import pytest

import paper_1604_04997_amd as P
from paper_1604_04997_amd import autotune, serve
from synth import serving_trace

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "no GPU visible"
    c = P.Context(0)
    yield c
    c.close()


def _model():
    # seconds per: [1, wg, barrier, f32 flop, f64 flop, special, LDS byte,
    # coalesced ld byte, coalesced st byte, other ld byte, other st byte, min]
    return P.model_struct("p12", [5e-6, 2e-9, 1e-10, 2e-14, 4e-14, 1e-13,
                                  1e-13, 2e-13, 2e-13, 1e-12, 1e-12, -5e-14])


def test_serving_results_equal_alone(ctx):
    import torch
    trace = serving_trace(rate=2000.0, duration=0.6, measure_frac=0.1, seed=77,
                          lo_log2=12, hi_log2=24)
    print("serving %d requests" % len(trace), flush=True)
    m = _model()
    srv = serve.Server(ctx, m, slots=1024, max_batch=256, bitmap_bytes=256 << 20)
    recs, stats = srv.run(trace, realtime=True, keep_counts=True, keep_outputs=True)
    print(stats, flush=True)
    assert stats["requests"] == len(trace) and stats["batches"] >= 1
    preds = [(i, t[2]) for i, t in enumerate(trace) if t[1] == "predict"]
    for i, v in preds:  # each variant counted and predicted alone
        r = recs[i]
        assert r["status"] == 0
        np.testing.assert_array_equal(r["counts"], P.counts_numpy(ctx.count_raw([v]))[0])
        assert r["pred"] == float(ctx.predict(m, [v])[0])
    for i, (ta, kind, v) in enumerate(trace):
        if kind != "measure":
            continue
        r = recs[i]
        assert r["t_min"] > 0
        ts, _ = P.device_buffers(v, v.get("seed", i), fast=True)
        ctx.launch(v, ts)
        torch.cuda.synchronize()
        for a, b in zip(r["outputs"], ts):
            assert torch.equal(a, b) or (torch.isnan(a).all() and torch.isnan(b).all()), v
    lat = [r["done"] - r["arrival"] for r in recs]
    assert min(lat) >= 0 and stats["p99_ms"] >= stats["p50_ms"] > 0
    # every request queued at once: batches form, results unchanged
    recs2, stats2 = srv.run(trace, realtime=False, keep_counts=True)
    assert stats2["max_batch"] > 1
    for i, v in preds:
        np.testing.assert_array_equal(recs2[i]["counts"], recs[i]["counts"])
        assert recs2[i]["pred"] == recs[i]["pred"]


def test_plain_replay(ctx):
    trace = serving_trace(rate=500.0, duration=0.2, measure_frac=0.1, seed=5,
                          lo_log2=12, hi_log2=20)
    recs, stats = serve.run_plain(ctx, _model(), trace, realtime=True)
    assert stats["requests"] == len(trace) and stats["p50_ms"] > 0


def test_autotune_ranks_and_measures(ctx):
    probs = [dict(family="matmul", n=200, m=300, l=150),
             dict(family="transpose", n=1500),
             dict(family="stencil", dtype="f32", n=1000),
             dict(family="nbody", n=3000)]
    res = autotune.rank_and_measure(ctx, _model(), probs, top_k=3, reps=5)
    assert len(res) == 4
    for r in res:
        assert len(r["measured"]) == min(3, r["n_configs"])
        assert r["slowdown"] >= 1.0
        assert r["chosen"] in r["configs"]
        # predictions come sorted: the chosen configuration is the first
        assert r["predicted"] == sorted(r["predicted"])
    s = autotune.summary(res)
    assert s["problems"] == 4 and s["geomean_slowdown"] >= 1.0
