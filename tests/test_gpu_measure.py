"""GPU tests of the measurement calls and of batch ordering, through the C
ABI: the launch floor of Sec. 4.2 (the empty kernel, run first), the
measurement deadline (PM_ETIMEDOUT while every enqueued kernel still runs
to completion), and batches of one context enqueued on different streams
and between host calls (they share the context's device arena)."""
import numpy as np
import pytest

import paper_1604_04997_amd as P
from oracle import count as C
from oracle import outputs as O

from test_lib_host import FAMILY_CASES

pytestmark = pytest.mark.gpu

PM_ETIMEDOUT = -6

# about 5 ms per launch: 2^22 work-items x 16384 FMAs (16 chains)
LONG_FMA = dict(family="fma", dtype="f32", n=1 << 22, wg=256, F=16384, K=16)


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "no GPU visible"
    c = P.Context(0)
    yield c
    c.close()


def test_launch_floor_and_below_floor_flag(ctx):
    import torch
    print("launch floor", flush=True)
    floor = ctx.launch_floor()
    assert 0 < floor < 1e-3
    empty = dict(family="empty", n=64, wx=64, wy=1)
    r = ctx.measure_until(empty, [], warmup=4, reps=26)
    assert r["status"] == 0 and len(r["t_reps"]) == 26
    assert r["below_floor"]
    ts, _ = P.device_buffers(LONG_FMA, 5, fast=True)
    r = ctx.measure_until(LONG_FMA, ts, warmup=1, reps=3)
    torch.cuda.synchronize()
    assert r["status"] == 0 and not r["below_floor"]
    assert r["t_min"] > 10 * floor


def test_deadline_times_out_and_kernels_complete(ctx):
    import torch
    print("deadline on %s" % LONG_FMA, flush=True)
    ts, host = P.device_buffers(LONG_FMA, 9)
    r = ctx.measure_until(LONG_FMA, ts, warmup=4, reps=26, deadline_s=0.002)
    assert r["status"] == PM_ETIMEDOUT
    assert len(r["t_reps"]) < 26
    torch.cuda.synchronize()
    # every enqueued launch ran to completion: the chains' outputs are exact
    # (sampled work-items; each launch recomputes the same outputs)
    idx = np.random.default_rng(3).choice(LONG_FMA["n"], 64, replace=False)
    got = ts[1].cpu().numpy()[idx]
    np.testing.assert_array_equal(got, O.fma_chain(LONG_FMA, host[0][idx]))
    # a zero deadline enqueues nothing
    r0 = ctx.measure_until(LONG_FMA, ts, warmup=4, reps=26, deadline_s=0.0)
    assert r0["status"] == PM_ETIMEDOUT and r0["t_reps"] == [] and r0["t_min"] == 0.0
    # the context measures normally afterwards
    small = dict(family="fma", dtype="f32", n=1 << 16, wg=256, F=64, K=4)
    ts2, _ = P.device_buffers(small, 2, fast=True)
    t, reps = ctx.measure(small, ts2, warmup=2, reps=5)
    assert t > 0 and len(reps) == 5
    r = ctx.measure_until(small, ts2, warmup=2, reps=5, deadline_s=30.0)
    assert r["status"] == 0 and len(r["t_reps"]) == 5


def _dev_variants(vs):
    import torch
    va = P.variant_array(vs)
    return torch.frombuffer(bytearray(bytes(memoryview(va).cast("B"))),
                            dtype=torch.uint8).cuda()


def test_batches_on_different_streams_are_ordered(ctx):
    """Two device batches on two side streams and a host call on the
    context's own stream, all enqueued before any wait: each gets the counts
    it gets alone (the arena is handed from batch to batch by events)."""
    import torch
    bm = [dict(v, bitmap=True) for v in FAMILY_CASES
          if v["family"] in ("transpose", "stream", "nbody")]
    a = (bm * 8)[:48]                                   # handed on: bitmaps
    b = [v for v in FAMILY_CASES if v["family"] in ("matmul", "stencil")][:40]
    c = [v for v in FAMILY_CASES if v["family"] in ("transpose", "conv")][:20]
    want = {k: [C.count(v) for v in vs] for k, vs in (("a", a), ("b", b), ("c", c))}
    ctx.reserve(64, sum(P.bitmap_bytes(v) for v in a))
    names = P.count_names()
    print("streams: %d + %d device variants, %d host" % (len(a), len(b), len(c)), flush=True)
    outs = {}
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    for key, vs, s in (("a", a, s1), ("b", b, s2)):
        d_v = _dev_variants(vs)
        d_c = torch.full((len(vs), P.PM_NCOUNT), 7, dtype=torch.int64, device="cuda")
        d_s = torch.full((len(vs),), 99, dtype=torch.int32, device="cuda")
        s.wait_stream(torch.cuda.current_stream())
        ctx.count_device(d_v.data_ptr(), len(vs), d_c.data_ptr(), None, 0,
                         d_s.data_ptr(), s.cuda_stream)
        outs[key] = (d_v, d_c, d_s)
    host = ctx.count(c)                                  # the context's stream
    torch.cuda.synchronize()
    for key, vs in (("a", a), ("b", b)):
        _, d_c, d_s = outs[key]
        assert (d_s.cpu().numpy() == 0).all(), key
        cnt = d_c.cpu().numpy()
        for k, v in enumerate(vs):
            got = {names[i]: int(x) for i, x in enumerate(cnt[k]) if x}
            assert got == want[key][k], (key, v)
    assert host == want["c"]


def test_null_stream_batch_then_side_stream_batch(ctx):
    """A device batch on the null stream (whose arena event the context
    records only when a batch on another stream needs it), then, before any
    wait, one on a side stream and another on the null stream: each gets the
    counts it gets alone."""
    import torch
    bm = [dict(v, bitmap=True) for v in FAMILY_CASES
          if v["family"] in ("transpose", "stream", "nbody")]
    a = (bm * 8)[:48]                                   # handed on: bitmaps
    b = [v for v in FAMILY_CASES if v["family"] in ("matmul", "stencil")][:40]
    c = [v for v in FAMILY_CASES if v["family"] in ("conv", "stream")][:30]
    want = {k: [C.count(v) for v in vs] for k, vs in (("a", a), ("b", b), ("c", c))}
    ctx.reserve(64, sum(P.bitmap_bytes(v) for v in a + c))
    names = P.count_names()
    print("null stream, side stream, null stream: %d, %d, %d variants" % (len(a), len(b), len(c)),
          flush=True)
    torch.cuda.synchronize()
    s1 = torch.cuda.Stream()
    outs = {}
    for key, vs, s in (("a", a, None), ("b", b, s1), ("c", c, None)):
        d_v = _dev_variants(vs)
        d_c = torch.full((len(vs), P.PM_NCOUNT), 7, dtype=torch.int64, device="cuda")
        d_s = torch.full((len(vs),), 99, dtype=torch.int32, device="cuda")
        if s is not None:
            s.wait_stream(torch.cuda.current_stream())
        ctx.count_device(d_v.data_ptr(), len(vs), d_c.data_ptr(), None, 0,
                         d_s.data_ptr(), s.cuda_stream if s is not None else 0)
        outs[key] = (d_v, d_c, d_s)
    torch.cuda.synchronize()
    for key, vs in (("a", a), ("b", b), ("c", c)):
        _, d_c, d_s = outs[key]
        assert (d_s.cpu().numpy() == 0).all(), key
        cnt = d_c.cpu().numpy()
        for k, v in enumerate(vs):
            got = {names[i]: int(x) for i, x in enumerate(cnt[k]) if x}
            assert got == want[key][k], (key, v)
