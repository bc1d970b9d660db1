"""GPU parity: the HIP path (libpm through its C ABI) against the oracle.

Counts: bit-exact against the simulated-execution oracle at sizes it
finishes in seconds, against closed forms at the full workload sizes, and
bit-exact between batched and one-at-a-time counting.  Kernel outputs:
bit-exact where the kernel's arithmetic is fixed (data movement, fixed-order
sums, single-rounding FMA chains, the stencil), within stated error bounds
otherwise (matmul, n-body, rsqrt)."""
import ctypes
import math
import os

import numpy as np
import pytest

import paper_1604_04997_amd as P
from oracle import count as C
from oracle import outputs as O
from synth import suite_batched, suite_instructive, suite_test, suite_tiny, uniform

from closed_forms import counts as closed_counts
from golden.make_sweep_counts import variants_digest as sweep_digest
from test_lib_host import FAMILY_CASES, FILLED_SC

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
U64 = 2.0 ** -53


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "no GPU visible"
    c = P.Context(0)
    yield c
    c.close()


def _strip(d):
    return {k: v for k, v in d.items() if not k.startswith("foot.")}


# ---------------------------------------------------------------- counts --
def test_counts_match_oracle_in_one_batch(ctx):
    vs = FAMILY_CASES + suite_batched(count=64, lo_log2=8, hi_log2=13)
    # both footprint methods; count jobs where components are enumerated
    vs = vs + [dict(v, bitmap=True) for v in vs] + [dict(v, enumerate=True) for v in vs]
    print("counting %d variants in one batch" % len(vs), flush=True)
    got = ctx.count(vs)
    for v, g in zip(vs, got):
        assert g == _strip(C.count(v)), v


def test_counts_full_size_closed_forms(ctx):
    vs = suite_batched(4096) + suite_instructive() + suite_test() + suite_tiny()
    vs = vs + [dict(v, bitmap=True) for v in suite_batched(512, seed=3)]
    vs = vs + [dict(v, enumerate=True) for v in suite_batched(512, seed=5)]
    print("counting %d full-size variants" % len(vs), flush=True)
    got = ctx.count(vs)
    for v, g in zip(vs, got):
        assert g == closed_counts(v), v


def test_bench_workload_on_the_device_path(ctx):
    """The timed configuration itself: the 4096-variant sweep through
    pm_count_device in one launch sequence with the extension model, under
    the default schedule and the one the tuner picks on it; every count
    vector against the closed forms, every prediction against the host's
    features of those counts."""
    import torch
    from paper_1604_04997_amd import autotune as AT
    vs = suite_batched(4096)
    nv = len(vs)
    d_v = torch.frombuffer(bytearray(bytes(memoryview(P.variant_array(vs)).cast("B"))),
                           dtype=torch.uint8).cuda()
    d_c = torch.zeros((nv, P.PM_NCOUNT), dtype=torch.int64, device="cuda")
    d_t = torch.zeros(nv, dtype=torch.float64, device="cuda")
    d_s = torch.full((nv,), 99, dtype=torch.int32, device="cuda")
    alpha = np.linspace(1e-13, 1e-11, P.NFEAT["ext"])
    m = P.model_struct("ext", alpha)
    ctx.reserve(nv, sum(P.bitmap_bytes(v) for v in vs))
    stream = torch.cuda.current_stream().cuda_stream

    def step():
        ctx.count_device(d_v.data_ptr(), nv, d_c.data_ptr(), m, d_t.data_ptr(),
                         d_s.data_ptr(), stream)

    names = P.count_names()
    want = np.zeros((nv, P.PM_NCOUNT), dtype=np.int64)
    for k, v in enumerate(vs):
        for name, x in closed_counts(v).items():
            want[k, names.index(name)] = x
    # the oracle's enumeration of the same 4096 variants, stored by
    # tests/golden/make_sweep_counts.py (CPU only)
    gold = np.load(os.path.join(os.path.dirname(__file__), "golden", "sweep4096_counts.npz"))
    assert str(gold["digest"]) == sweep_digest(vs) and gold["done"].all()
    gcols = [names.index(str(name)) for name in gold["names"]]
    oracle = gold["counts"]
    pred = None
    default = ctx.schedule()
    try:
        for tune in (False, True):
            if tune:
                AT.tune_counter(ctx, step, candidates=AT.COUNTER_SCHEDULES[4:], reps=2)
            print("sweep on the device path, schedule %s" % ctx.schedule(), flush=True)
            d_c.zero_()
            step()
            torch.cuda.synchronize()
            assert (d_s.cpu() == 0).all()
            got = d_c.cpu().numpy()
            np.testing.assert_array_equal(got, want)
            np.testing.assert_array_equal(got[:, gcols], oracle)  # row by row, bit for bit
            if pred is None:
                arr = ctx.count_raw(vs)
                pred = np.array([P.features(arr[i], "ext") @ alpha for i in range(nv)])
            np.testing.assert_allclose(d_t.cpu().numpy(), pred, rtol=1e-12)
    finally:
        ctx.set_schedule(**default)


def test_batched_equals_one_at_a_time_and_any_order(ctx):
    vs = suite_batched(192, seed=11) + FAMILY_CASES[::7]
    whole = P.counts_numpy(ctx.count_raw(vs))
    rev = P.counts_numpy(ctx.count_raw(vs[::-1]))[::-1]
    np.testing.assert_array_equal(whole, rev)
    for i, v in enumerate(vs):
        one = P.counts_numpy(ctx.count_raw([v]))[0]
        np.testing.assert_array_equal(one, whole[i], err_msg=str(v))


@pytest.mark.parametrize("proj", ["p3", "p12", "full", "ext", "bank"])
def test_device_resident_path_and_prediction(ctx, proj):
    import torch
    vs = suite_batched(512, seed=5) + suite_test()
    va = P.variant_array(vs)
    raw = bytes(memoryview(va).cast("B"))
    d_v = torch.frombuffer(bytearray(raw), dtype=torch.uint8).cuda()
    nv = len(vs)
    d_c = torch.zeros((nv, P.PM_NCOUNT), dtype=torch.int64, device="cuda")
    d_t = torch.zeros(nv, dtype=torch.float64, device="cuda")
    d_s = torch.full((nv,), 99, dtype=torch.int32, device="cuda")
    alpha = np.linspace(1e-13, 1e-11, P.NFEAT[proj])
    m = P.model_struct(proj, alpha)
    ctx.reserve(nv, sum(P.bitmap_bytes(v) for v in vs))
    s = torch.cuda.current_stream()
    ctx.count_device(d_v.data_ptr(), nv, d_c.data_ptr(), m, d_t.data_ptr(),
                     d_s.data_ptr(), s.cuda_stream)
    torch.cuda.synchronize()
    assert (d_s.cpu() == 0).all()
    want = P.counts_numpy(ctx.count_raw(vs))
    np.testing.assert_array_equal(d_c.cpu().numpy(), want)
    arr = ctx.count_raw(vs)
    F = np.array([P.features(arr[i], proj) for i in range(nv)])
    pred = F @ alpha
    np.testing.assert_allclose(d_t.cpu().numpy(), pred, rtol=1e-12)
    np.testing.assert_allclose(ctx.predict(m, vs), pred, rtol=1e-12)
    # and bit for bit in the summation order the library fixes: 64 partial
    # sums over features i = l, l + 64, ... in increasing order, combined
    # pairwise at distances 32, 16, ..., 1
    want_bits = np.array([_butterfly(F[i], alpha) for i in range(nv)])
    np.testing.assert_array_equal(d_t.cpu().numpy(), want_bits)
    np.testing.assert_array_equal(ctx.predict(m, vs), want_bits)


def _butterfly(f, alpha):
    part = np.zeros(64)
    for lane in range(64):
        x = 0.0
        for i in range(lane, len(f), 64):
            x = x + float(alpha[i]) * float(f[i])
        part[lane] = x
    lanes = np.arange(64)
    for off in (32, 16, 8, 4, 2, 1):
        part = part + part[lanes ^ off]
    return part[0]


def test_small_budget_reports_enomem():
    # bitmap footprints: (30000^2 + 30000) bits, more than the 64 MiB budget
    big = dict(family="transpose", op="naive_wc", n=30000, T=16, bitmap=True)
    c = P.Context(0, hbm_budget=64 << 20)
    try:
        with pytest.raises(P.PMError) as e:
            c.count([big])
        assert e.value.code == -2
        # a variant that fits still counts in the same context
        assert c.count([dict(big, n=100)])[0] == closed_counts(dict(big, n=100))
    finally:
        c.close()


# --------------------------------------------------------------- outputs --
def _run(ctx, v, seed):
    import torch
    ts, host = P.device_buffers(v, seed)
    ctx.launch(v, ts)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in ts], host


def _np(dt):
    return np.float32 if dt == "f32" else np.float64


OUT_CASES = (
    [dict(family="stream", op=op, dtype=dt, n=4096, wg=256, s=s, gs=gs, vec=vec, U=U)
     for op in ("load", "store", "copy", "add4") for dt in ("f32", "f64")
     for (s, gs, vec, U) in ((1, 1, 1, 1), (3, 2, 2, 2), (8, 1, 1, 3))]
    + [dict(family="stream", op="filled", dtype=dt, n=4096, wg=128, s=k, gs=1, vec=1, U=2)
       for dt in ("f32", "f64") for k in (2, 3)]
    + [dict(family="stream", op="filled", dtype=dt, n=2048, wg=64, s=s, c=c, gs=1, vec=1, U=3)
       for dt in ("f32", "f64") for (s, c) in FILLED_SC]
    + [dict(family="lds", op=op, groups=8, wg=wg, b=b, R=R, W=W)
       for op in ("read", "write") for (wg, b, R, W) in ((256, 1, 256, 4096), (64, 5, 33, 1024),
                                                        (1024, 32, 17, 16384))]
    + [dict(family="fma", dtype=dt, n=8192, wg=256, F=F, K=K)
       for dt in ("f32", "f64") for (F, K) in ((16, 1), (64, 8), (256, 16))]
    + [dict(family="rsqrt", n=8192, wg=256, F=F, K=K) for (F, K) in ((8, 1), (64, 4), (256, 8))]
    + [dict(family="barrier", groups=8, wg=wg, B=3) for wg in (64, 1024)]
    + [dict(family="empty", n=1000, wx=16, wy=16)]
    + [dict(family="matmul", op=op, n=n, m=m, l=l, T=T)
       for op in ("tiled", "naive") for (n, m, l) in ((37, 29, 41), (64, 64, 64), (1, 70, 3), (130, 257, 65))
       for T in (8, 16, 32)]
    + [dict(family="transpose", op=op, n=n, T=T)
       for op in ("tiled", "naive_wc", "naive_rc") for n in (1, 37, 100, 257) for T in (8, 16, 32)]
    + [dict(family="stencil", dtype=dt, n=n, T=T)
       for dt in ("f32", "f64") for n in (1, 2, 37, 100, 129) for T in (8, 16, 32)]
    + [dict(family="nbody", n=n, wg=wg) for n in (1, 2, 63, 300, 1000, 4099) for wg in (64, 256)]
    + [dict(family="stream", op="axpby", dtype=dt, n=4096, wg=256, s=s, gs=gs, vec=vec, U=U)
       for dt in ("f32", "f64") for (s, gs, vec, U) in ((1, 1, 1, 1), (3, 2, 2, 2))]
    + [dict(family="arith", op=op, dtype=dt, n=8192, wg=256, F=F, K=K)
       for op in ("div", "exp") for dt in ("f32", "f64") for (F, K) in ((8, 1), (64, 8))]
    + [dict(family="conv", n=n, T=T) for n in (1, 5, 37, 100) for T in (8, 16)]
    # the streaming (non-temporal) hint changes no output
    + [dict(family="stream", op=op, dtype=dt, n=4096, wg=256, s=s, gs=gs, vec=vec, U=U,
            streaming=True)
       for op in ("load", "store", "copy", "add4", "axpby") for dt in ("f32", "f64")
       for (s, gs, vec, U) in ((1, 1, 1, 1), (3, 2, 2, 2), (1, 1, 4 if dt == "f32" else 2, 3))]
)


def check_output(v, outs, host):
    fam = v["family"]
    dt = v.get("dtype", "f32")
    if fam == "stream":
        op = v["op"]
        if op == "load":  # the sentinel store never fires
            assert np.isnan(outs[1]).all()
        elif op == "store":
            np.testing.assert_array_equal(outs[0], O.stream_store(v, host[0]))
        elif op == "copy":
            np.testing.assert_array_equal(outs[1], O.stream_copy(v, host[0], host[1]))
        elif op == "add4":
            np.testing.assert_array_equal(outs[4], O.stream_add4(v, *host[:5]))
        elif op == "axpby":
            np.testing.assert_array_equal(outs[2], O.stream_axpby(v, *host[:3]))
        else:
            np.testing.assert_array_equal(outs[1], O.stream_filled(v, host[0]))
    elif fam == "lds":
        np.testing.assert_array_equal(outs[0], O.lds_out(v))
    elif fam == "fma":
        np.testing.assert_array_equal(outs[1], O.fma_chain(v, host[0]))
    elif fam == "rsqrt":
        ref = O.rsqrt_chain(v, host[0])
        # each step contracts errors (|d y'/d y| <= 0.385); a few ulp each
        np.testing.assert_allclose(outs[1], ref, rtol=16 * U32 * v["K"], atol=0)
    elif fam == "arith":
        if v["op"] == "div":
            np.testing.assert_array_equal(outs[1], O.div_chain(v, host[0]))
        else:
            ref = O.exp_chain(v, host[0])
            u = U32 if dt == "f32" else U64
            # exp within a few ulp per step; |d exp(-y^2)/dy| <= 0.86 damps them
            np.testing.assert_allclose(outs[1], ref, rtol=64 * u * v["K"], atol=0)
    elif fam == "conv":
        n = v["n"]
        ref, scale = O.conv(host[0], host[1], n)
        err = np.abs(outs[2].reshape(3, 3, n, n).astype(np.float64) - ref)
        assert (err <= 1e-5 * scale).all(), float((err / np.maximum(scale, 1e-300)).max())
    elif fam == "barrier":
        np.testing.assert_array_equal(outs[0], O.barrier_out(v))
    elif fam == "matmul":
        n, m, l = v["n"], v["m"], v["l"]
        A, B = host[0].reshape(n, m), host[1].reshape(m, l)
        ref, scale = O.matmul(A, B), O.matmul_abs(A, B)
        err = np.abs(outs[2].reshape(n, l).astype(np.float64) - ref)
        assert (err <= 1e-5 * scale).all(), float((err / np.maximum(scale, 1e-300)).max())
    elif fam == "transpose":
        n = v["n"]
        np.testing.assert_array_equal(outs[1].reshape(n, n), O.transpose(host[0].reshape(n, n)))
    elif fam == "stencil":
        n = v["n"]
        np.testing.assert_array_equal(outs[1].reshape(n, n), O.stencil(host[0], n, dt))
    elif fam == "nbody":
        ref, scale = O.nbody(host[0])
        # the bar of the test kernel: 1e-5 of sum_j |1/r_ij| per body
        err = np.abs(outs[1].astype(np.float64) - ref)
        assert (err <= 1e-5 * scale).all(), float((err / np.maximum(scale, 1e-300)).max())


@pytest.mark.parametrize("v", OUT_CASES, ids=lambda v: "-".join(str(x) for x in v.values()))
def test_outputs_match_oracle(ctx, v):
    outs, host = _run(ctx, v, seed=1234)
    check_output(v, outs, host)


def test_outputs_full_size_sampled(ctx):
    """Every test-suite variant at its full size: every transpose and
    stencil element compared; sampled matmul entries (square and skinny),
    convolution outputs and n-body rows computed by the oracle one by one."""
    import torch
    rng = np.random.default_rng(0)
    for v in suite_test():
        fam, n = v["family"], v["n"]
        print("full-size output check", v, flush=True)
        ts, host = P.device_buffers(v, v["seed"])
        ctx.launch(v, ts)
        torch.cuda.synchronize()
        if fam == "matmul":
            m, l = v["m"], v["l"]
            out = ts[2].cpu().numpy().reshape(n, l)
            A, B = host[0].reshape(n, m), host[1].reshape(m, l)
            rows = np.concatenate([[0, n - 1], rng.integers(0, n, 14)])
            cols = np.concatenate([[0, l - 1], rng.integers(0, l, 62)])
            ref = A[rows].astype(np.float64) @ B[:, cols].astype(np.float64)
            scale = np.abs(A[rows]).astype(np.float64) @ np.abs(B[:, cols]).astype(np.float64)
            err = np.abs(out[np.ix_(rows, cols)] - ref)
            assert (err <= 1e-5 * scale).all(), v
        elif fam == "conv":
            out = ts[2].cpu().numpy().reshape(3, 3, n, n)
            idx = np.stack([rng.integers(0, 3, 256), rng.integers(0, 3, 256),
                            rng.integers(0, n, 256), rng.integers(0, n, 256)], axis=1)
            idx[:4, 2:] = [[0, 0], [n - 1, n - 1], [0, n - 1], [n - 1, 0]]
            ref, scale = O.conv_at(host[0], host[1], n, idx)
            got = out[idx[:, 0], idx[:, 1], idx[:, 2], idx[:, 3]].astype(np.float64)
            assert (np.abs(got - ref) <= 1e-5 * scale).all(), v
        elif fam == "transpose":
            np.testing.assert_array_equal(ts[1].cpu().numpy().reshape(n, n),
                                          host[0].reshape(n, n).T)
        elif fam == "stencil":
            np.testing.assert_array_equal(ts[1].cpu().numpy().reshape(n, n),
                                          O.stencil(host[0], n, v["dtype"]))
        elif fam == "nbody":
            rows = np.concatenate([[0, n - 1], rng.integers(0, n, 30)])
            ref, scale = O.nbody(host[0], rows)
            got = ts[1].cpu().numpy()[rows].astype(np.float64)
            assert (np.abs(got - ref) <= 1e-5 * scale).all(), v
        del ts
        torch.cuda.empty_cache()


def test_every_stride_class_counted_on_the_gpu(ctx):
    """The family cases counted on the GPU in one batch reach all 15 stride
    classes of Sec. 2.1, each count equal to the oracle's."""
    got = ctx.count(FAMILY_CASES)
    seen = set()
    for v, g in zip(FAMILY_CASES, got):
        assert g == _strip(C.count(v)), v
        seen |= {k.split(".", 2)[2] for k in g if k.startswith(("gld.", "gst."))}
    assert len(seen) == 15, sorted(seen)


# --------------------------------------------------------------- measure --
def test_measure_times_are_positive_and_ordered(ctx):
    import torch
    v = dict(family="stream", op="copy", dtype="f32", n=1 << 24, wg=256, s=1, gs=1, vec=1, U=1)
    ts, _ = P.device_buffers(v, 1)
    tmin, reps = ctx.measure(v, ts, warmup=4, reps=26)
    assert tmin > 0 and tmin == min(reps) and len(reps) == 26
    # copying 2^24 floats moves 128 MiB: it cannot beat 8 TB/s by far
    assert 2 * 4 * (1 << 24) / tmin < 12e12
    small = dict(v, n=1 << 20)
    ts2, _ = P.device_buffers(small, 1)
    t2, _ = ctx.measure(small, ts2, warmup=4, reps=26)
    assert t2 < tmin
    torch.cuda.synchronize()
