"""GPU edge cases of the batched counter, through the C ABI: per-variant
statuses in a batch that mixes valid, invalid and overflowing descriptors
(on both expansion kernels: batches of up to 32 variants and larger ones),
the empty batch, batch sizes around the switch between the two kernels,
the largest batch one call accepts, and the counter's schedule (counts do
not depend on it)."""
import numpy as np
import pytest

import paper_1604_04997_amd as P
from oracle import count as C

from closed_forms import counts as closed_counts
from test_lib_host import FAMILY_CASES

pytestmark = pytest.mark.gpu

PM_EINVAL, PM_EOVERFLOW = -1, -5

BAD = dict(family="matmul", op="tiled", n=16, m=16, l=16, T=12)          # tile not 8/16/32
HUGE = dict(family="stream", op="load", dtype="f32", n=1 << 40, wg=256,  # count > int64
            s=1 << 20, gs=1 << 20, vec=1, U=1)


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "no GPU visible"
    c = P.Context(0)
    yield c
    c.close()


def _strip(d):
    return {k: v for k, v in d.items() if not k.startswith("foot.")}


def _device_count(ctx, vs, model=None):
    import torch
    va = P.variant_array(vs)
    raw = bytes(memoryview(va).cast("B"))
    nv = len(vs)
    d_v = torch.frombuffer(bytearray(raw), dtype=torch.uint8).cuda()
    d_c = torch.full((nv, P.PM_NCOUNT), 7, dtype=torch.int64, device="cuda")
    d_t = torch.full((nv,), 7.0, dtype=torch.float64, device="cuda")
    d_s = torch.full((nv,), 99, dtype=torch.int32, device="cuda")
    ctx.reserve(nv, sum(P.bitmap_bytes(v) for v in vs if v is not BAD and v is not HUGE))
    ctx.count_device(d_v.data_ptr(), nv, d_c.data_ptr(), model, d_t.data_ptr(),
                     d_s.data_ptr(), torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return d_c.cpu().numpy(), d_t.cpu().numpy(), d_s.cpu().numpy()


@pytest.mark.parametrize("nv", [5, 40])
def test_per_variant_status_in_mixed_batch(ctx, nv):
    good = [v for v in FAMILY_CASES if v["family"] in ("stencil", "transpose", "matmul")]
    vs = []
    for k in range(nv):
        vs.append(BAD if k % 5 == 1 else HUGE if k % 5 == 3 else good[k % len(good)])
    m = P.model_struct("p12", np.linspace(1e-12, 1e-11, 12))
    print("mixed batch of %d variants" % nv, flush=True)
    cnt, t, st = _device_count(ctx, vs, m)
    names = P.count_names()
    for k, v in enumerate(vs):
        if v is BAD:
            assert st[k] == PM_EINVAL
        elif v is HUGE:
            assert st[k] == PM_EOVERFLOW
        else:
            assert st[k] == 0
            got = {names[i]: int(x) for i, x in enumerate(cnt[k]) if x}
            assert got == _strip(C.count(v)), v
            c = P.Counts()
            c.c[:] = [int(x) for x in cnt[k]]
            want = float(P.features(c, "p12") @ np.array(m.alpha[:m.nfeat]))
            assert t[k] == pytest.approx(want, rel=1e-12)
            continue
        assert (cnt[k] == 0).all() and t[k] == 0.0


def test_empty_batch(ctx):
    import torch
    assert ctx.count([]) == []
    small = torch.zeros(64, dtype=torch.int64, device="cuda")
    ctx.count_device(small.data_ptr(), 0, small.data_ptr(), None, small.data_ptr(),
                     small.data_ptr(), torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert (small.cpu() == 0).all()


@pytest.mark.parametrize("nv", [1, 32, 33, 65])
def test_batch_sizes_around_the_kernel_switch(ctx, nv):
    vs = [FAMILY_CASES[(7 * k) % len(FAMILY_CASES)] for k in range(nv)]
    print("batch of %d variants" % nv, flush=True)
    got = ctx.count(vs)
    for v, g in zip(vs, got):
        assert g == _strip(C.count(v)), v


def test_largest_batch(ctx):
    """PM_BATCH_MAX variants in one device call (closed forms check every
    one); one more is refused before anything runs."""
    kinds = [dict(family="transpose", op=op, n=n, T=16) for op in ("tiled", "naive_wc")
             for n in (17, 100, 333)]
    kinds += [dict(family="stencil", dtype="f32", n=n, T=16) for n in (31, 64, 250)]
    vs = [kinds[k % len(kinds)] for k in range(P.PM_BATCH_MAX)]
    print("batch of %d variants" % len(vs), flush=True)
    cnt, _, st = _device_count(ctx, vs)
    assert (st == 0).all()
    names = P.count_names()
    want = {}
    for k, v in enumerate(kinds):
        row = np.zeros(P.PM_NCOUNT, dtype=np.int64)
        for name, x in closed_counts(v).items():
            row[names.index(name)] = x
        want[k] = row
    for k in range(len(vs)):
        np.testing.assert_array_equal(cnt[k], want[k % len(kinds)], err_msg=str(vs[k]))
    import torch
    small = torch.zeros(64, dtype=torch.int64, device="cuda")  # never read: refused first
    with pytest.raises(P.PMError):
        ctx.count_device(small.data_ptr(), P.PM_BATCH_MAX + 1, small.data_ptr(), None,
                         small.data_ptr(), small.data_ptr(),
                         torch.cuda.current_stream().cuda_stream)


@pytest.mark.parametrize("nv", [12, 150])
def test_counts_do_not_depend_on_the_schedule(ctx, nv):
    """Every schedule the tuner tries, on a batch that mixes bitmap
    footprints, count jobs of every size and closed forms, gives the same
    counts (both expansion kernels: up to 32 variants and more)."""
    from paper_1604_04997_amd import autotune as AT
    from synth import suite_batched
    base = suite_batched(count=64, lo_log2=8, hi_log2=16, seed=21) + FAMILY_CASES[::9]
    vs = [dict(v, bitmap=True) if k % 4 == 1 else v for k, v in enumerate(base)][:nv]
    want = [_strip(C.count(v)) for v in vs]
    default = ctx.schedule()
    try:
        for sc in AT.COUNTER_SCHEDULES[::3] + [dict(inblock_items=0, fused_items=0,
                                                     tail_wgs_per_cu=32)]:
            ctx.set_schedule(**sc)
            print("schedule %s, %d variants" % (sc, nv), flush=True)
            got = ctx.count(vs)
            for v, g, w in zip(vs, got, want):
                assert g == w, (sc, v)
    finally:
        ctx.set_schedule(**default)
    assert ctx.schedule() == default


def test_schedule_range_checks(ctx):
    cur = ctx.schedule()
    for bad in (dict(inblock_items=-1), dict(inblock_items=(1 << 20) + 1),
                dict(fused_items=1 << 25), dict(tail_wgs_per_cu=0),
                dict(tail_wgs_per_cu=33)):
        with pytest.raises(P.PMError):
            ctx.set_schedule(**bad)
        assert ctx.schedule() == cur


def test_profile_and_batch_stats(ctx):
    """Phase timing windows (every phase, then the expansion kernel only)
    and the last batch's statistics: a batch with bitmap footprints hands
    variants on, one without hands none on."""
    import torch
    vs = [dict(v, bitmap=True) for v in FAMILY_CASES if v["family"] == "transpose"][:40]
    marked = sum(P.bitmap_bytes(v) > 0 for v in vs)  # these are handed on
    assert marked > 0
    va = P.variant_array(vs)
    nv = len(vs)
    d_v = torch.frombuffer(bytearray(bytes(memoryview(va).cast("B"))), dtype=torch.uint8).cuda()
    d_c = torch.zeros((nv, P.PM_NCOUNT), dtype=torch.int64, device="cuda")
    d_t = torch.zeros(nv, dtype=torch.float64, device="cuda")
    d_s = torch.zeros(nv, dtype=torch.int32, device="cuda")
    ctx.reserve(nv, sum(P.bitmap_bytes(v) for v in vs))
    stream = torch.cuda.current_stream().cuda_stream
    for mode, nph in ((1, len(P.Context.PHASES)), (2, 1)):
        ctx.profile(mode)
        for _ in range(3):
            ctx.count_device(d_v.data_ptr(), nv, d_c.data_ptr(), None, d_t.data_ptr(),
                             d_s.data_ptr(), stream)
        torch.cuda.synchronize()
        ms, nb = ctx.profile_read()
        ctx.profile(False)
        assert nb == 3
        assert ms["build"] > 0
        assert all(x >= 0 for x in ms.values())
        assert sum(x > 0 for x in ms.values()) <= nph
    st = ctx.batch_stats()
    assert st["handed_on"] == marked and st["chunks"] > 0 and st["fill_segments"] > 0
    assert st["bitmap_words"] > 0 and st["bitmap_words_requested"] >= st["bitmap_words"]
    got = d_c.cpu().numpy()
    names = P.count_names()
    for k, v in enumerate(vs):
        assert {names[i]: int(x) for i, x in enumerate(got[k]) if x} == _strip(C.count(v)), v
    plain = [v for v in FAMILY_CASES if v["family"] == "matmul"][:40]
    ctx.count(plain)
    assert ctx.batch_stats()["handed_on"] == 0


def test_model_ranked_counter_schedule(ctx):
    """The counter's schedule ranked by the model fitted to its own timed
    passes: the pick is one of the candidates, and the counts under it equal
    the oracle's (batches that hand variants on and ones that do not)."""
    import torch
    from paper_1604_04997_amd import autotune as AT
    vs = [dict(v, bitmap=True) if k % 2 else v
          for k, v in enumerate(FAMILY_CASES) if v["family"] in ("transpose", "stencil")][:48]
    va = P.variant_array(vs)
    nv = len(vs)
    d_v = torch.frombuffer(bytearray(bytes(memoryview(va).cast("B"))), dtype=torch.uint8).cuda()
    d_c = torch.zeros((nv, P.PM_NCOUNT), dtype=torch.int64, device="cuda")
    d_s = torch.zeros(nv, dtype=torch.int32, device="cuda")
    ctx.reserve(nv, sum(P.bitmap_bytes(v) for v in vs))
    stream = torch.cuda.current_stream().cuda_stream

    def step():
        ctx.count_device(d_v.data_ptr(), nv, d_c.data_ptr(), None, 0, d_s.data_ptr(), stream)

    default = ctx.schedule()
    try:
        chosen, rep = AT.tune_counter_model(ctx, step, n_timed=6, reps=3)
        assert {k: chosen[k] for k in ("inblock_items", "tail_wgs_per_cu")} in AT.COUNTER_SCHEDULES
        assert rep["chosen_ms"] > 0 and len(rep["timed"]) == 6
        d_c.zero_()
        step()
        torch.cuda.synchronize()
        assert (d_s.cpu() == 0).all()
        names = P.count_names()
        got = d_c.cpu().numpy()
        for k, v in enumerate(vs):
            assert {names[i]: int(x) for i, x in enumerate(got[k]) if x} == _strip(C.count(v)), v
    finally:
        ctx.set_schedule(**default)


def test_work_group_size_enters_predictions_through_the_group_count(ctx):
    """Sec. 5: kernel configurations that differ only in work-group size get
    the same prediction but for the per-group launch overhead.  For the
    study's measurement kernels (stream, FMA, rsqrt, LDS writes, barriers)
    at 128, 256 and 512 work-items per group, the counted features differ
    in the group count alone, and the device predictions differ by its
    weight times the change in groups."""
    from synth import suite_wg
    vs = [v for v in suite_wg() if v["family"] in ("stream", "fma", "rsqrt", "barrier")
          or (v["family"] == "lds" and v["op"] == "write")]
    print("wg study variants", len(vs), flush=True)
    counts = ctx.count_raw(vs)
    feats = np.array([P.features(counts[i], "ext") for i in range(len(vs))])
    alpha = np.random.default_rng(11).uniform(1e-12, 1e-9, P.NFEAT["ext"])
    pred = ctx.predict(P.model_struct("ext", alpha), vs)
    wg_col = set()
    for b in sorted({v["base"] for v in vs}):
        idx = [i for i, v in enumerate(vs) if v["base"] == b]
        for i in idx[1:]:
            j = idx[0]
            d = feats[i] - feats[j]
            nz = np.flatnonzero(d)
            assert len(nz) == 1, (vs[i], nz)
            k = int(nz[0])
            wg_col.add(k)
            groups = lambda v: v.get("groups", v.get("n", 0) // v["wg"])
            assert d[k] == groups(vs[i]) - groups(vs[j])
            want = alpha[k] * d[k]
            assert abs((pred[i] - pred[j]) - want) <= 1e-12 * max(abs(pred[i]), abs(pred[j]))
    assert len(wg_col) == 1
