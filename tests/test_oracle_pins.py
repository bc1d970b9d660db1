"""Pins of the oracle against facts that do not come from the oracle itself:
hand-enumerated tiny domains, closed-form counts derived from the kernel
descriptions, the paper's textbook stride classes (Sec. 2.1), its Table 1
worked example (Sec. 5), exact least-squares recovery (Sec. 4.3) and exact
or error-bounded reference outputs."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import count as C
from oracle import model as M
from oracle import outputs as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def cdiv(a, b):
    return -(-a // b)


# --------------------------------------------------------------- counts ---
def test_tiny_hand_enumerated_counts():
    cases = json.load(open(os.path.join(GOLD, "tiny_counts.json")))["cases"]
    for c in cases:
        assert C.count(c["variant"]) == c["counts"], c["why"]


def _cls(s):
    return {0: "0", 1: "1", 2: "1/2", 3: "1/3", 4: "1/4"}.get(s, "1/>4")


@pytest.mark.parametrize("dt", ["f32", "f64"])
@pytest.mark.parametrize("s", [1, 2, 3, 4, 5, 8, 32])
@pytest.mark.parametrize("vec,U,gs", [(1, 1, 1), (2, 2, 1), (1, 3, 4)])
def test_stream_closed_forms(dt, s, vec, U, gs):
    if dt == "f64" and vec == 4:
        return
    e = 4 if dt == "f32" else 8
    n, wg = 512, 64
    base = dict(family="stream", dtype=dt, n=n, wg=wg, s=s, gs=gs, vec=vec, U=U)
    cl = _cls(s)
    sz = e * vec
    got = C.count(dict(base, op="load"))
    assert got == {"gld.%d.%s" % (sz, cl): n * U, "add.%s" % dt: n * U * vec,
                   "wg": n // wg, "wi": n}
    got = C.count(dict(base, op="store"))
    assert got == {"gst.%d.%s" % (sz, cl): n * U, "wg": n // wg, "wi": n}
    got = C.count(dict(base, op="copy"))
    assert got == {"gld.%d.%s" % (sz, cl): n * U, "gst.%d.%s" % (sz, cl): n * U,
                   "wg": n // wg, "wi": n}
    got = C.count(dict(base, op="add4"))
    assert got == {"gld.%d.%s" % (sz, cl): 4 * n * U,
                   "gst.%d.%s" % (sz, cl): n * U,
                   "add.%s" % dt: 3 * n * U * vec, "wg": n // wg, "wi": n}


@pytest.mark.parametrize("k,cls", [(2, "2/2"), (3, "3/3")])
def test_filled_closed_forms(k, cls):
    n, U = 1024, 2
    got = C.count(dict(family="stream", op="filled", dtype="f32", n=n, wg=256,
                       s=k, gs=1, vec=1, U=U))
    assert got == {"gld.4.%s" % cls: k * n * U, "gst.4.1": n,
                   "add.f32": k * n * U, "wg": 4, "wi": n}


# c of every s cells read: the utilization c/s (just under it: the last run
# reaches s - 1 cells past the array's used part) picks the class k/q of
# Sec. 2.1 with q = min(s, 4) quarters for s > 4 -- listed by hand here.
@pytest.mark.parametrize("s,c,cls", [
    (2, 1, "1/2"), (3, 1, "1/3"), (3, 2, "2/3"), (4, 1, "1/4"), (4, 2, "2/4"),
    (4, 3, "3/4"), (4, 4, "4/4"), (8, 1, "1/>4"), (8, 4, "2/>4"), (5, 2, "2/>4"),
    (8, 5, "3/>4"), (5, 3, "3/>4"), (5, 4, "4/>4"), (5, 5, "4/>4")])
def test_filled_c_of_s_classes(s, c, cls):
    n, U = 512, 3
    got = C.count(dict(family="stream", op="filled", dtype="f64", n=n, wg=128,
                       s=s, c=c, gs=1, vec=1, U=U), with_footprints=True)
    J = n * U
    assert got == {"gld.8.%s" % cls: c * J, "gst.8.1": n, "add.f64": c * J,
                   "wg": 4, "wi": n,
                   # |F|: c cells per group; Fill: up to the last read
                   # cell's run end, s*(J-1) + (c-1) + s
                   "foot.F.0": c * J, "foot.fill.0": s * J + c - 1,
                   "foot.F.1": n, "foot.fill.1": n}


@pytest.mark.parametrize("op", ["read", "write"])
def test_lds_closed_forms(op):
    G, wg, R, W = 3, 128, 17, 512
    got = C.count(dict(family="lds", op=op, groups=G, wg=wg, b=4, R=R, W=W))
    want = {"gst.4.1": G * wg, "bar.wi": G * wg, "bar.wg": G, "wg": G,
            "wi": G * wg}
    # bank stride 4 words: bin b4; the read kernel's initialisation moves one
    # word per lane
    if op == "read":
        want.update({"lst.4": G * W, "lld.4": G * wg * R, "add.f32": G * wg * R,
                     "lst.4.b1": G * W, "lld.4.b4": G * wg * R})
    else:
        want.update({"lst.4": G * wg * R, "lld.4": G * wg,
                     "lst.4.b4": G * wg * R, "lld.4.b4": G * wg})
    assert got == want


@pytest.mark.parametrize("b,bin_", [(1, "b1"), (3, "b1"), (2, "b2"), (6, "b2"), (4, "b4"),
                                    (12, "b4"), (8, "b8"), (16, "b16"), (48, "b16"),
                                    (32, "b32"), (64, "b32"), (96, "b32")])
def test_lds_bank_stride_bins(b, bin_):
    """Sec. 6.2 binning of the LDS stride: an access whose address moves b
    words per lane falls in the bin of the power of two in b (lanes of one
    wavefront that share a bank on power-of-two banks), 32 and beyond
    together; the stride, not its size, decides (3 and 1, 6 and 2 agree)."""
    G, wg, R, W = 2, 64, 5, 8192
    got = C.count(dict(family="lds", op="read", groups=G, wg=wg, b=b, R=R, W=W))
    assert got["lld.4." + bin_] == G * wg * R
    assert sum(x for k, x in got.items() if k.startswith("lld.4.")) == got["lld.4"]


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_fma_rsqrt_barrier_empty_closed_forms(dt):
    n, F, K = 2048, 64, 8
    got = C.count(dict(family="fma", dtype=dt, n=n, wg=256, F=F, K=K))
    s = dt
    assert got == {"gld.%d.1" % (4 if dt == "f32" else 8): n,
                   "gst.%d.1" % (4 if dt == "f32" else 8): n,
                   "fma." + s: n * F, "add." + s: n * (K - 1),
                   "wg": n // 256, "wi": n}
    got = C.count(dict(family="rsqrt", n=n, wg=256, F=F, K=4))
    assert got == {"gld.4.1": n, "gst.4.1": n, "mul.f32": n * F,
                   "add.f32": n * F + n * 3, "spec.f32": n * F,
                   "wg": n // 256, "wi": n}
    got = C.count(dict(family="barrier", groups=5, wg=128, B=7))
    assert got == {"bar.wi": 5 * 128 * 7, "bar.wg": 5 * 7, "gst.4.1": 5 * 128,
                   "wg": 5, "wi": 5 * 128}
    got = C.count(dict(family="empty", n=1000, wx=64, wy=4))
    assert got == {"wg": 16 * 250, "wi": 16 * 250 * 256}


@pytest.mark.parametrize("n,m,l,T", [(64, 64, 64, 16), (32, 48, 16, 8),
                                     (37, 29, 41, 16), (5, 70, 9, 32)])
def test_matmul_closed_forms(n, m, l, T):
    GX, GY, KT = cdiv(l, T), cdiv(n, T), cdiv(m, T)
    wi = GX * GY * T * T
    got = C.count(dict(family="matmul", op="tiled", n=n, m=m, l=l, T=T))
    # every A element is fetched once per column tile, every B element once
    # per row tile; inner products run over padded k-tiles
    # LDS by bank-stride bin (Sec. 6.2): the tiles are stored at lane stride
    # 1; in the inner product As[ly][k] is one word for all lanes of a row
    # (b0) and Bs[k][lx] moves one word per lane (b1)
    assert got == {"gld.4.1": n * m * GX + m * l * GY, "gst.4.1": n * l,
                   "lst.4": 2 * wi * KT, "lld.4": 2 * wi * KT * T,
                   "lst.4.b1": 2 * wi * KT, "lld.4.b0": wi * KT * T,
                   "lld.4.b1": wi * KT * T,
                   "fma.f32": wi * KT * T, "bar.wi": 2 * wi * KT,
                   "bar.wg": 2 * GX * GY * KT, "wg": GX * GY, "wi": wi}
    if T == 16 and n == m == l:  # the textbook n^3 forms
        assert got["fma.f32"] == n ** 3 and got["lld.4"] == 2 * n ** 3
        assert got["gld.4.1"] == 2 * n ** 3 // T and got["bar.wi"] == 2 * n ** 3 // T
    got = C.count(dict(family="matmul", op="naive", n=n, m=m, l=l, T=T))
    assert got == {"gld.4.0": n * m * l, "gld.4.1": n * m * l, "gst.4.1": n * l,
                   "fma.f32": n * m * l, "wg": GX * GY, "wi": wi}


@pytest.mark.parametrize("n,T", [(64, 16), (37, 16), (100, 32), (9, 8)])
def test_transpose_closed_forms(n, T):
    G = cdiv(n, T)
    got = C.count(dict(family="transpose", op="tiled", n=n, T=T))
    # the tile is stored by rows (lane stride 1) and read by columns of the
    # padded T + 1 rows: an odd word stride, bank-conflict free (b1)
    assert got == {"gld.4.1": n * n, "gst.4.1": n * n, "lst.4": n * n,
                   "lld.4": n * n, "lst.4.b1": n * n, "lld.4.b1": n * n,
                   "bar.wi": G * G * T * T, "bar.wg": G * G,
                   "wg": G * G, "wi": G * G * T * T}
    # the strided side moves n cells per lane; every cell is used: 4/>4
    got = C.count(dict(family="transpose", op="naive_wc", n=n, T=T))
    assert got == {"gld.4.4/>4": n * n, "gst.4.1": n * n, "wg": G * G,
                   "wi": G * G * T * T}
    got = C.count(dict(family="transpose", op="naive_rc", n=n, T=T))
    assert got == {"gld.4.1": n * n, "gst.4.4/>4": n * n, "wg": G * G,
                   "wi": G * G * T * T}


@pytest.mark.parametrize("dt", ["f32", "f64"])
@pytest.mark.parametrize("n,T", [(64, 16), (37, 16), (33, 8), (16, 32)])
def test_stencil_closed_forms(dt, n, T):
    G = cdiv(n, T)
    e = 4 if dt == "f32" else 8
    got = C.count(dict(family="stencil", dtype=dt, n=n, T=T))
    halo = 4 * n * G  # four tile edges per tile row / column
    # LDS stores: the halo columns go to a fixed column (one word for all
    # lanes: the left column in all G tile columns, the right one in the
    # n // T full ones); every other store and all five loads move one
    # element per lane -- one word in fp32 (b1), two in fp64 (b2)
    col0 = G * n + (n // T) * n
    s1 = "b1" if e == 4 else "b2"
    assert got == {"gld.%d.1" % e: n * n + halo, "lst.%d" % e: n * n + halo,
                   "lst.%d.b0" % e: col0, "lst.%d.%s" % (e, s1): n * n + halo - col0,
                   "lld.%d" % e: 5 * n * n, "lld.%d.%s" % (e, s1): 5 * n * n,
                   "add." + dt: 4 * n * n,
                   "mul." + dt: 3 * n * n, "gst.%d.1" % e: n * n,
                   "bar.wi": G * G * T * T, "bar.wg": G * G, "wg": G * G,
                   "wi": G * G * T * T}
    if n % T == 0:
        assert got["gld.%d.1" % e] * T == n * n * (T + 4)  # n^2 (1 + 4/T)


@pytest.mark.parametrize("N,G", [(1024, 256), (1000, 256), (300, 64)])
def test_nbody_closed_forms(N, G):
    B = cdiv(N, G)
    wi = B * G
    got = C.count(dict(family="nbody", n=N, wg=G))
    # per pair 3 differences, 2 adds in r^2 and 1 add into the block's
    # partial; per (work-item, block) 1 add of the partial into the total
    # a block's positions are stored at lane stride 1 and every pair reads
    # one word for all lanes (b0)
    assert got == {"gld.4.3/3": 3 * N + 3 * N * B, "gst.4.1": N,
                   "lst.4": 3 * N * B, "lld.4": 3 * wi * N,
                   "lst.4.b1": 3 * N * B, "lld.4.b0": 3 * wi * N,
                   "add.f32": 6 * wi * N + wi * B, "mul.f32": 3 * wi * N,
                   "spec.f32": wi * N, "bar.wi": 2 * wi * B,
                   "bar.wg": 2 * B * B, "wg": B, "wi": wi}


@pytest.mark.parametrize("n,T", [(16, 8), (20, 8), (37, 16), (7, 16)])
def test_conv_closed_forms(n, T):
    """Three 7x7 filters, three images: 147 FMAs and 294 LDS loads per
    output; the filter fetched once per work-group; every image row and
    column of the (T+6)-wide tiles that lies inside the padded image."""
    P, G, TT = n + 6, cdiv(n, T), T + 6
    rows = sum(min(TT, P - gy * T) for gy in range(G))
    got = C.count(dict(family="conv", n=n, T=T))
    assert got["fma.f32"] == 9 * 147 * n * n and got["lld.4"] == 9 * 294 * n * n
    assert got["gld.4.1"] == 9 * G * G * 147
    assert got["gld.4.3/3"] == 27 * rows * rows
    assert got["gst.4.1"] == 9 * n * n and got["bar.wi"] == 9 * G * G * T * T


@pytest.mark.parametrize("op", ["div", "exp"])
def test_arith_and_axpby_closed_forms(op):
    n, F, K = 2048, 32, 4
    got = C.count(dict(family="arith", op=op, dtype="f32", n=n, wg=256, F=F, K=K))
    assert got["mul.f32"] == n * F and got.get(op + ".f32") == n * F
    assert got["add.f32"] == (n * F if op == "div" else 0) + n * (K - 1)
    got = C.count(dict(family="stream", op="axpby", dtype="f64", n=n, wg=256, s=3,
                       gs=1, vec=1, U=1))
    assert got == {"gld.8.1/3": 2 * n, "gst.8.1/3": n, "mul.f64": 2 * n,
                   "add.f64": n, "wg": n // 256, "wi": n}


def test_div_chain_reference_exact_steps():
    """One division-chain step is (k+1) / (a*a + 1), each operation
    rounded once in float32: compare with rationals."""
    x = np.random.default_rng(8).uniform(-1, 1, 32).astype(np.float32)
    out = O.div_chain({"F": 1, "K": 1}, x)
    for i in range(32):
        sq = _round_f32(Fraction(float(x[i])) ** 2)
        den = _round_f32(Fraction(float(sq)) + 1)
        assert out[i] == _round_f32(Fraction(1) / Fraction(float(den)))


def test_conv_reference_single_tap():
    """With one non-zero filter tap (u, v, c) the convolution is a shifted
    copy of one image channel."""
    n = 5
    img = np.random.default_rng(9).uniform(-1, 1, 9 * (n + 6) ** 2).astype(np.float32)
    filt = np.zeros(3 * 147, dtype=np.float32)
    filt[1 * 147 + (2 * 7 + 4) * 3 + 1] = 2.0  # filter j=1, u=2, v=4, c=1
    r, _ = O.conv(img, filt, n)
    I = img.reshape(3, n + 6, n + 6, 3).astype(np.float64)
    np.testing.assert_array_equal(r[:, 1], 2.0 * I[:, 4:4 + n, 2:2 + n, 1])
    assert not r[:, 0].any() and not r[:, 2].any()


def test_conv_sampled_reference_single_tap():
    """The sampled convolution reference on one non-zero filter tap (filter
    j = 2, u = 5, v = 1, channel 0, weight -0.5): each output is that tap
    times img[i][x+1][y+5][0], and the other filters give 0."""
    n = 9
    img = np.random.default_rng(10).uniform(-1, 1, 9 * (n + 6) ** 2).astype(np.float32)
    filt = np.zeros(3 * 147, dtype=np.float32)
    filt[2 * 147 + (5 * 7 + 1) * 3 + 0] = -0.5
    I = img.reshape(3, n + 6, n + 6, 3).astype(np.float64)
    idx = [(i, j, x, y) for i in range(3) for j in (0, 2) for (x, y) in ((0, 0), (8, 3), (4, 8))]
    r, a = O.conv_at(img, filt, n, idx)
    for t, (i, j, x, y) in enumerate(idx):
        want = -0.5 * I[i, x + 1, y + 5, 0] if j == 2 else 0.0
        assert r[t] == want and a[t] == abs(want)


def test_counts_additive_over_a_domain_split():
    """Counts add when the launch is split: two half-size stream launches of
    a unit-stride kernel give the counts of the whole (Alg. 1 is a sum over
    domain points)."""
    whole = C.count(dict(family="stream", op="copy", dtype="f32", n=4096,
                         wg=256, s=1, gs=1, vec=1, U=1))
    half = C.count(dict(family="stream", op="copy", dtype="f32", n=2048,
                        wg=256, s=1, gs=1, vec=1, U=1))
    assert whole == {k: 2 * v for k, v in half.items()}


def test_wg_size_only_changes_overhead_counts():
    """Sec. 5: apart from halos and work-group counts, properties do not
    depend on the work-group size."""
    a = C.count(dict(family="fma", dtype="f32", n=4096, wg=64, F=16, K=4))
    b = C.count(dict(family="fma", dtype="f32", n=4096, wg=512, F=16, K=4))
    assert {k: v for k, v in a.items() if k != "wg"} == \
        {k: v for k, v in b.items() if k != "wg"}
    assert a["wg"] == 64 and b["wg"] == 8


# ------------------------------------------------------- stride classes ---
@pytest.mark.parametrize("sites,vec,want", [
    ([(0, 0)], 1, ["0"]),                                   # uniform
    ([(1, 0)], 1, ["1"]),
    ([(2, 0)], 1, ["1/2"]),                                 # <= 50% used
    ([(2, 0), (2, 1)], 1, ["2/2", "2/2"]),                  # all used
    ([(3, 0)], 1, ["1/3"]),
    ([(3, 0), (3, 1)], 1, ["2/3", "2/3"]),
    ([(3, 0), (3, 1), (3, 2)], 1, ["3/3"] * 3),
    ([(4, 0), (4, 2)], 1, ["2/4", "2/4"]),
    ([(8, 0)], 1, ["1/>4"]),
    ([(8, 0), (8, 4)], 1, ["1/>4", "1/>4"]),
    ([(8, c) for c in range(4)], 1, ["2/>4"] * 4),
    ([(8, c) for c in range(8)], 1, ["4/>4"] * 8),
    ([(8, 0)], 4, ["1/2"]),        # float4 accesses two accesses apart
    ([(4, 0)], 4, ["1"]),          # float4 accesses back to back
])
def test_textbook_stride_classes(sites, vec, want):
    n = 64
    cells = max(abs(c) * (n - 1) + o for c, o in sites) + vec
    assert C.classify_1d(cells, n, sites, elem=4, vec=vec) == want


def test_strided_transpose_read_is_uncoalesced_full():
    assert C.count(dict(family="transpose", op="naive_wc", n=50, T=16)) \
        ["gld.4.4/>4"] == 2500


# --------------------------------------------------- Table 1 and metric ---
def test_table1_worked_example():
    t = json.load(open(os.path.join(GOLD, "table1.json")))
    for kname, k in t["kernels"].items():
        P = np.array(k["pairs"])
        for g in range(4):
            if kname == "finite_difference" and g == 2:
                continue  # 0.70 vs 0.70: a zero error after rounding
            e = M.rel_errors(P[:, g, 1], P[:, g, 0])
            assert abs(M.geomean(e) - k["geomean"][g]) <= 0.02, (kname, g)
        if kname != "finite_difference":
            e = M.rel_errors(P[:, :, 1].ravel(), P[:, :, 0].ravel())
            assert abs(M.geomean(e) - k["cross_gpu"]) <= 0.01
    # the reversed column order does not reproduce the table
    P = np.array(t["kernels"]["nbody"]["pairs"])
    assert M.geomean(M.rel_errors(P[:, 3, 0], P[:, 3, 1])) > 2.0
    for g in (0, 1, 3):
        e = np.concatenate([M.rel_errors(np.array(k["pairs"])[:, g, 1],
                                         np.array(k["pairs"])[:, g, 0])
                            for k in t["kernels"].values()])
        assert abs(M.geomean(e) - t["cross_kernel"][g]) <= 0.01


def test_geomean_closed_form():
    assert M.geomean([0.5, 0.02]) == pytest.approx(0.1)
    assert M.geomean([0.3]) == pytest.approx(0.3)


# ------------------------------------------------------------------ fit ---
def test_fit_recovers_exact_weights():
    rng = np.random.default_rng(0)
    P = rng.uniform(1, 100, size=(40, 6))
    a = rng.uniform(1e-12, 1e-9, size=6)
    T = P @ a
    alpha, rank = M.fit(P, T)
    assert rank == 6
    np.testing.assert_allclose(alpha, a, rtol=1e-9)
    np.testing.assert_allclose(M.predict(P, alpha), T, rtol=1e-12)


def test_fit_minimises_relative_error():
    """The fitted weights make the relative residual orthogonal to every
    column of P/T (normal equations of Sec. 4.3), so no weight change can
    lower sum (1 - pred/T)^2; a plain absolute fit does not."""
    rng = np.random.default_rng(1)
    P = rng.uniform(1, 100, size=(30, 3))
    T = (P @ np.array([1.0, 2.0, 3.0])) * rng.uniform(0.7, 1.3, size=30)
    alpha, _ = M.fit(P, T)
    r = 1 - (P @ alpha) / T
    np.testing.assert_allclose((P / T[:, None]).T @ r, 0, atol=1e-9)
    a_abs = np.linalg.lstsq(P, T, rcond=None)[0]
    assert np.sum(r ** 2) < np.sum((1 - (P @ a_abs) / T) ** 2)


def test_fit_scaling_invariance_and_zero_columns():
    rng = np.random.default_rng(2)
    P = rng.uniform(1, 10, size=(20, 4))
    P[:, 2] = 0
    T = rng.uniform(1, 2, size=20)
    a1, r1 = M.fit(P, T)
    S = np.diag([1e3, 1e-4, 1.0, 7.0])
    a2, r2 = M.fit(P @ S, T)
    assert r1 == r2 == 3 and a1[2] == 0 and a2[2] == 0
    np.testing.assert_allclose(M.predict(P, a1), M.predict(P @ S, a2),
                               rtol=1e-9)


def test_features_of_a_known_count_dict():
    c = {"gld.4.1": 10, "gst.4.1": 4, "gld.8.1/2": 3, "gst.4.4/>4": 2,
         "gld.4.3/3": 5, "fma.f32": 7, "add.f32": 1, "mul.f64": 2,
         "spec.f32": 3, "lld.4": 6, "lst.8": 1, "bar.wi": 9, "wg": 11}
    assert M.features_p3(c) == [4 * 10 + 4 * 4 + 8 * 3 + 4 * 2 + 4 * 5, 7, 11]
    assert M.features_p12(c) == [1, 11, 9, 1 + 14, 2, 3, 24 + 8,
                                 40 + 20, 16, 24, 8, 16]
    f = dict(zip(M.full_names(), M.features_full(c)))
    assert f["add.f32"] == 8 and f["mul.f32"] == 7 and f["min.4.1"] == 4
    assert f["const"] == 1 and f["gst.4.4/>4"] == 2


@pytest.mark.parametrize("wi,div", [(1000, 1000), (1 << 20, 256 * 2048)])
def test_features_ext_of_a_known_count_dict(wi, div):
    """The three extension features on a hand-written count dict, once with
    a grid smaller than the GPU holds at once (256 CUs x 2048 work-items)
    and once larger: arithmetic instructions (an FMA once) and global bytes
    per resident work-item, and min(arithmetic instructions, global bytes)."""
    c = {"fma.f32": 100, "add.f32": 20, "mul.f64": 5, "spec.f32": 3,
         "div.f64": 2, "exp.f32": 1, "gld.4.1": 10, "gst.8.1/2": 3,
         "lld.4": 50, "bar.wi": 7, "wg": 4, "wi": wi}
    ops, gb = 131, 4 * 10 + 8 * 3
    f = M.features_ext(c)
    assert len(f) == 157 and f[:154] == M.features_full(c)
    assert f[154] == ops / div and f[155] == gb / div and f[156] == min(ops, gb)
    # arithmetic dominates the byte count the other way round
    c2 = dict(c, **{"gld.4.1": 1000})
    assert M.features_ext(c2)[156] == ops


def test_features_bank_of_a_known_count_dict():
    """The bank projection: the 90 global counts, then the 42 LDS counts by
    (direction, size, bank-stride bin) in that order -- loads before stores,
    4/8/16-byte, bins b0 b1 b2 b4 b8 b16 b32 -- in place of the 6 plain LDS
    counts, then the rest of the extended list."""
    c = {"gld.4.1": 10, "lld.4": 9, "lld.4.b0": 4, "lld.4.b1": 3, "lld.4.b32": 2,
         "lst.8": 5, "lst.8.b2": 5, "fma.f32": 7, "wg": 3, "wi": 300}
    f = M.features_bank(c)
    e = M.features_ext(c)
    assert len(f) == 193
    assert f[:90] == e[:90] and f[132:] == e[96:]
    lds = f[90:132]
    assert lds[0] == 4 and lds[1] == 3 and lds[6] == 2     # lld.4: b0, b1, b32
    assert lds[21 + 7 + 2] == 5                             # lst.8.b2
    assert sum(lds) == 9 + 5 and e[90] == 9 and e[94] == 5  # plain: lld.4, lst.8


# -------------------------------------------------------------- outputs ---
def _round_f32(q: Fraction) -> np.float32:
    """Correctly rounded (to nearest, ties to even) float32 of a rational."""
    r = np.float32(float(q))
    cands = [np.nextafter(r, np.float32(-np.inf)), r,
             np.nextafter(r, np.float32(np.inf))]
    best = min(abs(Fraction(float(c)) - q) for c in cands)
    ties = [c for c in cands if abs(Fraction(float(c)) - q) == best]
    ties.sort(key=lambda c: int(np.array(c).view(np.uint32)) & 1)
    return ties[0]


def test_fma_chain_rounds_once_per_step():
    """Each chain step is the exact a*c + b rounded once to float32."""
    x = np.random.default_rng(3).uniform(-1, 1, 64).astype(np.float32)
    v = {"F": 8, "K": 2}
    out = O.fma_chain(v, x)
    for i in range(64):
        a = Fraction(float(x[i]))
        c = [np.float32(x[i])] * 2
        for _ in range(4):
            for k in range(2):
                c[k] = _round_f32(Fraction(float(c[k])) * a + Fraction(k + 1, 64))
        assert out[i] == np.float32(c[0] + c[1])


def test_stencil_exact_on_small_integers():
    """n = 7: h^2 = 1/64 exactly; small-integer inputs make every step
    exact, so the reference equals the rational formula."""
    n = 7
    u = np.random.default_rng(4).integers(-3, 4, size=(n + 2) ** 2).astype(np.float32)
    out = O.stencil(u, n, "f32")
    U = u.reshape(n + 2, n + 2)
    for i in range(n):
        for j in range(n):
            q = Fraction(1, 4) * (int(U[i, j + 1]) + int(U[i + 2, j + 1])
                                  + int(U[i + 1, j]) + int(U[i + 1, j + 2])
                                  + Fraction(int(U[i + 1, j + 1]) ** 2, 64))
            assert Fraction(float(out[i, j])) == q


def test_nbody_known_geometry():
    pos = np.array([0, 0, 0, 3, 4, 0, 0, 0, 12], dtype=np.float32)
    out, _ = O.nbody(pos)
    np.testing.assert_allclose(out, [1 / 5 + 1 / 12, 1 / 5 + 1 / math.sqrt(9 + 16 + 144),
                                     1 / 12 + 1 / math.sqrt(9 + 16 + 144)])


def test_rsqrt_chain_from_zero():
    """a = 0: chain k runs y <- 1/sqrt(y^2 + (k+1)) from 0, so chain 0 gives
    1, 1/sqrt 2, sqrt(2/3) and chain 1 gives 1/sqrt 2, sqrt(2/5); the chains
    are summed."""
    x = np.zeros(4)
    np.testing.assert_allclose(O.rsqrt_chain({"F": 1, "K": 1}, x), 1.0, rtol=1e-15)
    np.testing.assert_allclose(O.rsqrt_chain({"F": 2, "K": 1}, x), 1 / math.sqrt(2), rtol=1e-15)
    np.testing.assert_allclose(O.rsqrt_chain({"F": 3, "K": 1}, x), math.sqrt(2 / 3), rtol=1e-15)
    np.testing.assert_allclose(O.rsqrt_chain({"F": 4, "K": 2}, x),
                               1 / math.sqrt(2) + math.sqrt(2 / 5), rtol=1e-15)
    # from a = 1 one step gives 1/sqrt(1 + 1)
    np.testing.assert_allclose(O.rsqrt_chain({"F": 1, "K": 1}, np.ones(2)),
                               1 / math.sqrt(2), rtol=1e-15)


def test_exp_chain_from_zero():
    """a = 0: y <- exp(-y^2) gives 1, exp(-1), exp(-exp(-2)); with two
    chains (no dependence on k) the sum is twice one chain."""
    x = np.zeros(3)
    np.testing.assert_allclose(O.exp_chain({"F": 1, "K": 1}, x), 1.0, rtol=1e-15)
    np.testing.assert_allclose(O.exp_chain({"F": 2, "K": 1}, x), math.exp(-1), rtol=1e-15)
    np.testing.assert_allclose(O.exp_chain({"F": 3, "K": 1}, x), math.exp(-math.exp(-2)),
                               rtol=1e-15)
    np.testing.assert_allclose(O.exp_chain({"F": 6, "K": 2}, x), 2 * math.exp(-math.exp(-2)),
                               rtol=1e-15)


def test_filled_reference_small():
    """s = 4, c = 3, U = 2, 2 work-items: work-item i adds x[4j]+x[4j+1]+x[4j+2]
    for j = i and j = i + 2 (integers: exact)."""
    x = np.arange(16, dtype=np.float32)
    out = O.stream_filled(dict(n=2, U=2, s=4, c=3), x)
    np.testing.assert_array_equal(out, [(0 + 1 + 2) + (8 + 9 + 10), (4 + 5 + 6) + (12 + 13 + 14)])


def test_matmul_reference_exact_small():
    rng = np.random.default_rng(5)
    A = rng.integers(-5, 6, size=(3, 4)).astype(np.float32)
    B = rng.integers(-5, 6, size=(4, 2)).astype(np.float32)
    Cm = O.matmul(A, B)
    for i in range(3):
        for j in range(2):
            assert Cm[i, j] == sum(int(A[i, k]) * int(B[k, j]) for k in range(4))


def test_lds_read_closed_form():
    v = dict(family="lds", op="read", groups=2, wg=64, b=1, R=32, W=4096)
    out = O.lds_out(v)
    l = np.arange(64)
    np.testing.assert_array_equal(out[:64], 32 * l + 32 * 31 // 2)
    v = dict(v, op="write", b=3)
    np.testing.assert_array_equal(O.lds_out(v)[64:], 3 * l)


def test_stream_touched_elements():
    v = dict(n=8, wg=4, s=2, gs=2, vec=1, U=1)
    # groups start gs*wg*s = 16 elements apart; lanes s = 2 apart
    assert list(O.stream_elements(v)) == [0, 2, 4, 6, 16, 18, 20, 22]
    v = dict(n=4, wg=2, s=1, gs=1, vec=2, U=2)
    assert list(O.stream_elements(v)) == [0, 1, 2, 3, 4, 5, 6, 7,
                                          8, 9, 10, 11, 12, 13, 14, 15]


def test_sweep_golden_file_matches_generator_and_closed_forms():
    """The stored oracle enumeration of the 4096-variant sweep (written by
    tests/golden/make_sweep_counts.py from oracle/ alone) belongs to the
    current variant generator, is complete, and agrees with the closed
    forms on every variant at its full size (2^16..2^30 domain points): the
    simulated execution and the hand-derived counts agree where no small
    case reaches."""
    import os
    from golden.make_sweep_counts import variants_digest
    from synth import suite_batched
    from closed_forms import counts as closed
    vs = suite_batched(4096)
    g = np.load(os.path.join(os.path.dirname(__file__), "golden", "sweep4096_counts.npz"))
    assert str(g["digest"]) == variants_digest(vs)
    assert g["done"].all()
    names = [str(x) for x in g["names"]]
    assert names == [x for x in C.names() if not x.startswith("foot.")]
    counts = g["counts"]  # an npz member is read again on every access
    for k, v in enumerate(vs):
        got = {nm: int(x) for nm, x in zip(names, counts[k]) if x}
        assert got == closed(v), (k, v)


WG_SMALL = [
    lambda wg: dict(family="stream", op="load", dtype="f32", n=1 << 13, wg=wg, s=2, gs=1, vec=1, U=1),
    lambda wg: dict(family="stream", op="copy", dtype="f32", n=1 << 13, wg=wg, s=4, gs=1, vec=1, U=1),
    lambda wg: dict(family="stream", op="store", dtype="f32", n=1 << 13, wg=wg, s=1, gs=1, vec=1, U=1),
    lambda wg: dict(family="fma", dtype="f64", n=1 << 12, wg=wg, F=16, K=8),
    lambda wg: dict(family="rsqrt", n=1 << 12, wg=wg, F=8, K=4),
    lambda wg: dict(family="lds", op="read", groups=(1 << 12) // wg, wg=wg, b=4, R=8, W=4096),
    lambda wg: dict(family="lds", op="write", groups=(1 << 12) // wg, wg=wg, b=32, R=8, W=4096),
    lambda wg: dict(family="barrier", groups=(1 << 12) // wg, wg=wg, B=4),
]


@pytest.mark.parametrize("mk", WG_SMALL, ids=lambda mk: "%s-%s" % (mk(128)["family"],
                                                                    mk(128).get("op", "")))
def test_work_group_size_changes_only_group_counts(mk):
    """Sec. 5: kernel configurations that differ only in work-group size have
    the same properties apart from the launch's group count (and barriers
    summed per group), so the model predicts them alike but for the
    per-group overhead -- except where a group does fixed work of its own,
    as the LDS read kernel's filling of its W words."""
    vs = {wg: mk(wg) for wg in (128, 256, 512)}
    cs = {wg: C.count(v) for wg, v in vs.items()}
    init = ("lst.4", "lst.4.b1") if vs[128]["family"] == "lds" and vs[128]["op"] == "read" else ()
    rest = [{k: x for k, x in c.items() if k not in ("wg", "bar.wg") + init}
            for c in cs.values()]
    assert rest[0] == rest[1] == rest[2]
    for wg, c in cs.items():
        assert c["wg"] * wg == c["wi"]
        if "bar.wi" in c:
            assert c["bar.wg"] * wg == c["bar.wi"]
        if init:  # every group first fills its W words of LDS
            assert c["lst.4"] == c["lst.4.b1"] == vs[wg]["groups"] * vs[wg]["W"]


def test_nbody_work_group_size_enters_staging():
    """The n-body kernel stages every body through LDS once per work-group
    (Sec. 5's exception: the group size changes the kernel's memory
    transactions): from 128 to 512 work-items per group the staged global
    loads, LDS stores and barriers per work-item fall as N/G, while the
    LDS loads and the pair arithmetic stay."""
    N = 4096
    c = {G: C.count(dict(family="nbody", n=N, wg=G)) for G in (128, 256, 512)}
    for G in (128, 256, 512):
        B = N // G
        assert c[G]["gld.4.3/3"] == 3 * N + 3 * N * B
        assert c[G]["lst.4"] == 3 * N * B
        assert c[G]["bar.wi"] == 2 * N * B
        assert c[G]["lld.4"] == 3 * N * N
        assert c[G]["mul.f32"] == 3 * N * N
