"""CPU tests of libpm: exported symbols, the descriptor / counting code run
on the host (pm_count_host) against the oracle, error paths, features and
the FP64 fit against the NumPy oracle.  No GPU calls."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import paper_1604_04997_amd as P
from oracle import count as C
from oracle import model as M
from synth import suite_batched, suite_instructive, suite_test, suite_tiny

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    syms = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            syms |= set(re.findall(r"^\s*(?:pm_status|void|const char \*)\s*(pm_\w+)\s*\(",
                                   txt, re.M))
    return syms


def test_library_exports_every_declared_symbol():
    syms = _declared_symbols()
    assert {"pm_create", "pm_count", "pm_predict", "pm_fit", "pm_measure",
            "pm_count_device", "pm_count_host"} <= syms
    out = subprocess.run(["nm", "-D", "--defined-only", P.LIB_PATH],
                         capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r" T (pm_\w+)", out))
    assert syms <= exported, syms - exported
    L = P.lib()
    for s in syms:
        assert hasattr(L, s)


def test_count_names_match_the_oracle_vocabulary():
    names = P.count_names()
    assert len(names) == P.PM_NCOUNT == 154 and len(set(names)) == 154
    orc = [n for n in C.names() if not n.startswith("foot.")]
    assert sorted(names) == sorted(orc)


def _strip(d):
    return {k: v for k, v in d.items() if not k.startswith("foot.")}


def _same(v):
    lib = P.count_host(v, with_footprints=True)
    orc = C.count(v, with_footprints=True)
    assert _strip(lib) == _strip(orc), v
    for k, x in lib.items():  # footprints the library computes agree too
        if k.startswith("foot."):
            assert orc[k] == x, (v, k)


# (s, c) pairs of the generalised filled access that between them reach the
# stride classes 1/2, 1/3, 2/3, 1/4..4/4 and 1/>4..4/>4
FILLED_SC = ((2, 1), (3, 1), (3, 2), (4, 1), (4, 2), (4, 3), (4, 4), (5, 2), (5, 3),
             (5, 4), (8, 1), (8, 4), (8, 5), (16, 5))

FAMILY_CASES = [
    dict(family="stream", op=op, dtype=dt, n=512, wg=64, s=s, gs=gs, vec=vec, U=U)
    for op in ("load", "store", "copy", "add4")
    for dt in ("f32", "f64") for s in (1, 2, 3, 5, 8)
    for (gs, vec, U) in ((1, 1, 1), (3, 2, 2), (1, 4, 3))
    if not (dt == "f64" and vec == 4)
] + [
    dict(family="stream", op="filled", dtype=dt, n=1024, wg=128, s=k, gs=1, vec=1, U=U)
    for dt in ("f32", "f64") for k in (2, 3) for U in (1, 3)
] + [
    # c of every s cells read: the classes k/q below q
    dict(family="stream", op="filled", dtype=dt, n=512, wg=64, s=s, c=c, gs=1, vec=1, U=U)
    for dt in ("f32", "f64") for (s, c) in FILLED_SC for U in (1, 2)
] + [
    dict(family="lds", op=op, groups=3, wg=wg, b=b, R=R, W=1024)
    for op in ("read", "write") for wg in (64, 256) for b in (1, 3, 32) for R in (0, 5)
] + [
    dict(family="fma", dtype=dt, n=2048, wg=wg, F=F, K=K)
    for dt in ("f32", "f64") for wg in (64, 1024) for (F, K) in ((16, 1), (64, 8), (256, 16))
] + [
    dict(family="rsqrt", n=4096, wg=256, F=F, K=K) for (F, K) in ((8, 1), (64, 4), (256, 8))
] + [
    dict(family="barrier", groups=G, wg=wg, B=B) for G in (1, 7) for wg in (64, 1024) for B in (0, 3)
] + [
    dict(family="empty", n=n, wx=wx, wy=wy) for n in (1, 1000) for (wx, wy) in ((64, 1), (16, 16))
] + [
    dict(family="matmul", op=op, n=n, m=m, l=l, T=T)
    for op in ("tiled", "naive") for (n, m, l) in ((37, 29, 41), (64, 64, 64), (1, 70, 3))
    for T in (8, 16, 32)
] + [
    dict(family="transpose", op=op, n=n, T=T)
    for op in ("tiled", "naive_wc", "naive_rc") for n in (1, 2, 37, 64, 100) for T in (8, 16, 32)
] + [
    dict(family="stencil", dtype=dt, n=n, T=T)
    for dt in ("f32", "f64") for n in (1, 2, 7, 16, 37) for T in (8, 16, 32)
] + [
    dict(family="nbody", n=n, wg=wg) for n in (1, 63, 300, 1000) for wg in (64, 256)
] + [
    dict(family="stream", op="axpby", dtype=dt, n=512, wg=64, s=s, gs=gs, vec=vec, U=U)
    for dt in ("f32", "f64") for s in (1, 2, 3) for (gs, vec, U) in ((1, 1, 1), (2, 2, 3))
] + [
    dict(family="arith", op=op, dtype=dt, n=1024, wg=256, F=F, K=K)
    for op in ("div", "exp") for dt in ("f32", "f64") for (F, K) in ((8, 1), (64, 8))
] + [
    dict(family="conv", n=n, T=T) for n in (1, 5, 16, 37) for T in (8, 16)
]


@pytest.mark.parametrize("v", FAMILY_CASES, ids=lambda v: "-".join(str(x) for x in v.values()))
def test_host_counts_match_oracle(v):
    _same(v)
    _same(dict(v, bitmap=True))  # bitmap footprints instead of intervals
    _same(dict(v, enumerate=True))  # count jobs instead of inline enumeration
    if v["family"] == "stream":  # the streaming cache hint changes no count
        _same(dict(v, streaming=True))


@pytest.mark.parametrize("v", FAMILY_CASES, ids=lambda v: "-".join(str(x) for x in v.values()))
def test_per_statement_expansion_matches_one_pass(v):
    """Statements expanded one by one in two job slots each (the GPU's
    layout, with its fall-back when a statement needs more jobs) give the
    same counts and footprints as the one-pass expansion."""
    for d in (v, dict(v, bitmap=True), dict(v, enumerate=True)):
        assert P.count_host(d, True) == P.count_host(d, True, sequential=True)


def test_per_statement_expansion_on_batched_workload():
    for v in suite_batched(count=256):
        assert P.count_host(v, True) == P.count_host(v, True, sequential=True)


def _classes(counts):
    return {k.split(".", 2)[2] for k in counts if k.startswith(("gld.", "gst."))}


def test_family_cases_reach_every_stride_class():
    """Between them the family cases give every one of the 15 classes of
    Sec. 2.1 (counted by the library on the host, checked against the
    oracle in test_host_counts_match_oracle)."""
    seen = set()
    for v in FAMILY_CASES:
        seen |= _classes(P.count_host(v))
    assert seen == set(M.CLASSES), set(M.CLASSES) - seen


def test_host_counts_on_batched_workload_sample():
    """Small-domain draws of the batched sweep (same generator, smaller
    domains so the oracle finishes quickly): uneven extents that are not
    multiples of the tile."""
    for v in suite_batched(count=48, lo_log2=8, hi_log2=13):
        _same(v)


def test_suites_are_valid_descriptors():
    for v in suite_tiny() + suite_instructive() + suite_test() + suite_batched(256):
        P.count_host(v) if v["family"] in ("empty",) else P.buffers(v)


@pytest.mark.parametrize("bad", [
    dict(family="stream", op="load", dtype="f32", n=1000, wg=256, s=1, gs=1, vec=1, U=1),
    dict(family="stream", op="load", dtype="f64", n=1024, wg=256, s=1, gs=1, vec=4, U=1),
    dict(family="stream", op="load", dtype="f32", n=1024, wg=256, s=0, gs=1, vec=1, U=1),
    dict(family="stream", op="filled", dtype="f32", n=1024, wg=256, s=8, gs=1, vec=1, U=1),
    dict(family="stream", op="filled", dtype="f32", n=1024, wg=256, s=4, c=5, gs=1, vec=1, U=1),
    dict(family="stream", op="filled", dtype="f32", n=1024, wg=256, s=1, c=1, gs=1, vec=1, U=1),
    dict(family="lds", op="read", groups=1, wg=256, b=1, R=1, W=1000),
    dict(family="fma", dtype="f32", n=1024, wg=256, F=10, K=4),
    dict(family="fma", dtype="f32", n=1024, wg=2048, F=16, K=4),
    dict(family="matmul", op="tiled", n=16, m=16, l=16, T=12),
    dict(family="transpose", op="tiled", n=0, T=16),
    dict(family="nbody", n=100, wg=100),
])
def test_invalid_descriptors_are_rejected(bad):
    with pytest.raises(P.PMError) as e:
        P.count_host(bad)
    assert e.value.code == -1
    with pytest.raises(P.PMError):
        P.buffers(bad)


def test_overflow_is_reported():
    v = dict(family="stream", op="load", dtype="f32", n=1 << 40, wg=256, s=1 << 20,
             gs=1 << 20, vec=1, U=1)
    with pytest.raises(P.PMError) as e:
        P.count_host(v)
    assert e.value.code == -5


def test_large_domains_count_in_closed_form():
    """Domains far beyond enumeration (2^40+ points) still count exactly:
    matmul n = m = l = 2^14 gives n^3 FMAs."""
    n = 1 << 14
    c = P.count_host(dict(family="matmul", op="tiled", n=n, m=n, l=n, T=16))
    assert c["fma.f32"] == n ** 3 and c["lld.4"] == 2 * n ** 3
    assert c["gld.4.1"] == 2 * n ** 3 // 16


def _lib_counts(variants):
    arr = (P.Counts * len(variants))()
    for i, v in enumerate(variants):
        vs = P.variant_struct(v)
        P._check(P.lib().pm_count_host(ctypes.byref(vs), ctypes.byref(arr[i]), None))
    return arr


def _small(v):
    """The same variant shape at a size the simulated-execution oracle
    finishes in milliseconds."""
    v = dict(v)
    if v["family"] in ("stream", "fma", "rsqrt", "arith"):
        v["n"] = min(v["n"], 1 << 12)
    if v["family"] == "conv":
        v["n"] = min(v["n"], 40) + 3
    if v["family"] in ("lds", "barrier"):
        v["groups"] = min(v["groups"], 8)
    if v["family"] in ("matmul", "transpose", "stencil"):
        v["n"] = min(v["n"], 40) + 3
        v["m"], v["l"] = v["n"] - 1, v["n"] + 2
    if v["family"] == "nbody":
        v["n"] = min(v["n"], 700)
    if v["family"] == "empty":
        v["n"] = min(v["n"], 1 << 10)
    return v


@pytest.fixture(scope="module")
def feature_cases():
    """Small variants of the tiny and test suites with their library and
    oracle counts (counted once for every projection)."""
    vs = [_small(v) for v in suite_tiny() + suite_test()[::3]]
    return vs, _lib_counts(vs), [C.count(v) for v in vs]


@pytest.fixture(scope="module")
def fit_cases():
    """Small variants of the instructive and test suites with their library
    and oracle counts (counted once for every projection)."""
    vs = [_small(v) for v in suite_instructive(roofline_points=False, extended=True)
          + suite_test()]
    return vs, _lib_counts(vs), [C.count(v) for v in vs]


@pytest.mark.parametrize("proj", ["p3", "p12", "full", "ext", "bank"])
def test_features_match_oracle(proj, feature_cases):
    vs, arr, oc = feature_cases
    for i, v in enumerate(vs):
        lib = P.features(arr[i], proj)
        orc = M.FEATURES[proj](oc[i])
        np.testing.assert_array_equal(lib, np.array(orc, dtype=np.float64))


@pytest.mark.parametrize("proj", ["p3", "p12", "full", "ext", "bank"])
def test_fit_matches_numpy_oracle(proj, fit_cases):
    vs, arr, oc = fit_cases
    F = np.array([P.features(arr[i], proj) for i in range(len(vs))])
    rng = np.random.default_rng(7)
    a_true = np.abs(rng.normal(size=F.shape[1])) * 1e-12 + 1e-15
    T = F @ a_true * rng.uniform(0.8, 1.25, size=len(vs)) + 2e-6
    m, cond, resid, rank = P.fit(arr, T, proj)
    alpha = P.model_alpha(m)
    Fo = M.feature_matrix(oc, proj)
    ao, rank_o = M.fit(Fo, T)
    pred, pred_o = F @ alpha, Fo @ ao
    np.testing.assert_allclose(pred, pred_o, rtol=1e-9)
    np.testing.assert_allclose(resid, 1 - pred / T, rtol=1e-9, atol=1e-12)
    assert rank == rank_o
    full_rank = rank == int(np.count_nonzero(np.any(F != 0, axis=0)))
    if full_rank and cond < 1e8:  # weights are unique only at full rank
        np.testing.assert_allclose(alpha, ao, rtol=1e-7, atol=1e-30)


def test_extension_features_at_full_size():
    """Full-size test kernels (grids above and below what the GPU holds at
    once): the library's extension features against the oracle's, on
    closed-form counts."""
    from closed_forms import counts as closed_counts
    for v in suite_test():
        lib = P.features(_lib_counts([v])[0], "ext")
        orc = M.features_ext(closed_counts(v))
        np.testing.assert_array_equal(lib, np.array(orc, dtype=np.float64), err_msg=str(v))


def test_fit_exact_recovery_and_errors():
    vs = suite_tiny()
    arr = _lib_counts(vs)
    F = np.array([P.features(arr[i], "p3") for i in range(len(vs))])
    a = np.array([1.0 / 5e12, 1.0 / 4e13, 2e-9])
    m, cond, resid, rank = P.fit(arr, F @ a, "p3")
    np.testing.assert_allclose(P.model_alpha(m), a, rtol=1e-9)
    assert rank == 3 and np.max(np.abs(resid)) < 1e-12
    with pytest.raises(P.PMError) as e:
        P.fit(arr, -np.ones(len(vs)), "p3")
    assert e.value.code == -1
    empty = (P.Counts * 2)()
    with pytest.raises(P.PMError) as e:
        P.fit(empty, [1.0, 2.0], "p3")
    assert e.value.code == -4


def test_buffers_layout():
    b = P.buffers(dict(family="matmul", op="tiled", n=3, m=5, l=7, T=8))
    assert b == [(60, 0), (140, 0), (84, 1)]
    b = P.buffers(dict(family="stream", op="load", dtype="f64", n=512, wg=256, s=2,
                       gs=2, vec=2, U=2))
    assert b == [(8 * 2 * 2 * 256 * 2 * 2 * 2, 0), (8 * 512, 3)]


def test_host_counts_full_size_closed_forms():
    """The full workloads (batched sweep, instructive and test suites) at
    their real sizes against closed forms derived from the kernels."""
    from closed_forms import counts as closed
    for v in suite_batched(4096) + suite_instructive() + suite_test() + suite_tiny():
        assert P.count_host(v) == closed(v), v


def test_partial_tile_guards_every_size():
    """Every size from 1 to 199 and every tile: the guards of the partial
    tiles (halo rows and columns of the last tile, matrix edges), counted
    in closed form where the coupled guards share one mixed-radix index and
    enumerated where they do not, against the closed forms derived from the
    kernels."""
    from closed_forms import counts as closed
    for n in range(1, 200):
        for T in (8, 16, 32):
            for v in (dict(family="stencil", dtype="f32", n=n, T=T),
                      dict(family="transpose", op="tiled", n=n, T=T),
                      dict(family="transpose", op="naive_rc", n=n, T=T),
                      dict(family="matmul", op="tiled", n=n, m=n + 5, l=max(n - 3, 1), T=T)):
                assert P.count_host(v) == closed(v), v


def test_qpoly_eval_binomial_basis():
    """pm_qpoly_eval on a hand-made form: on residue r of (x - x0) mod 2,
    count = c0 + c1 q + c2 C(q,2) + c3 C(q,3), q = (x - x0) div 2; below x0
    refused; a count past int64 reported."""
    import math
    qp = P.QPoly()
    qp.period, qp.x0, qp.scale, qp.fields = 2, 5, 1, 1
    co = {0: [3, 2, 4, 6], 1: [-7, 0, 0, 1]}
    for r, cs in co.items():
        for j, x in enumerate(cs):
            qp.coef[r][j][0] = x
            qp.coef[r][j][111] = 1 if j == 1 else 0   # wi = q on both residues
    for x in list(range(5, 40)) + [10 ** 6 + 3]:
        r, q = (x - 5) % 2, (x - 5) // 2
        want = sum(c * math.comb(q, j) for j, c in enumerate(co[r]))
        got = P.qpoly_eval(qp, x)
        assert got.c[0] == want and got.c[111] == q and got.c[5] == 0, x
    with pytest.raises(P.PMError):
        P.qpoly_eval(qp, 4)
    qp.coef[0][3][7] = 1 << 62
    with pytest.raises(P.PMError) as e:
        P.qpoly_eval(qp, 5 + 2 * 100)
    assert e.value.code == -5


def test_autotune_summary_top_k_selection():
    """The selection summaries on hand-made records: the model's pick, and
    keeping the fastest of its top k measured (host logic only)."""
    from paper_1604_04997_amd import autotune
    # predicted order c, a, b; measured fastest b
    r1 = {"predicted": [2.0, 3.0, 1.0], "measured": [1.5, 1.0, 2.0], "slowdown": 2.0,
          "spearman": -0.5}
    # the model's pick is the measured best
    r2 = {"predicted": [1.0, 2.0], "measured": [1.0, 4.0], "slowdown": 1.0}
    assert autotune.topk_slowdown(r1, 1) == 2.0
    assert autotune.topk_slowdown(r1, 2) == 1.5
    assert autotune.topk_slowdown(r1, 3) == 1.0
    assert autotune.topk_slowdown(r2, 5) == 1.0  # k past the configurations
    s = autotune.summary([r1, r2], ks=(2, 3))
    assert s["problems"] == 2 and s["choice_is_best"] == 0.5
    assert s["geomean_slowdown"] == pytest.approx(2.0 ** 0.5)
    assert s["top2_geomean_slowdown"] == pytest.approx(1.5 ** 0.5)
    assert s["top2_max_slowdown"] == 1.5
    assert s["top3_geomean_slowdown"] == 1.0
    assert s["mean_spearman"] == -0.5
