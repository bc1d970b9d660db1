"""Seeded input generators and workload parameter lists.

A *variant* is a plain dict naming a kernel family and its parameters.  The
families and their parameters (all sizes are element counts):

  stream    op in {load, store, copy, add4, filled}; dtype; n (work-items),
            wg, s (lane stride, or k for 'filled'), gs (group stride),
            vec (elements per access), U (accesses per work-item)
  lds       op in {read, write}; groups, wg, b (bank stride), R, W (words)
  fma       dtype; n (work-items), wg, F (FMAs per work-item), K (chains)
  rsqrt     n, wg, F (rsqrt per work-item), K (chains); fp32
  barrier   groups, wg, B (barriers per work-item)
  empty     n (side of the virtual n x n matrix), wx, wy
  matmul    op in {tiled, naive}; n, m, l (C[n,l] = A[n,m] B[m,l]), T
  transpose op in {tiled, naive_wc, naive_rc}; n, T
  stencil   dtype; n (interior side), T
  nbody     n (bodies), wg

Float inputs are uniform on [-1, 1], drawn in float64 from PCG64 and cast to
the kernel dtype; the same bytes feed the GPU and the oracle.
"""
from __future__ import annotations

import math

import numpy as np

SEED_BASE = 1604_04997


def seed_for(config: int, index: int) -> int:
    """Seed of variant `index` of workload `config` (1-based configs)."""
    return SEED_BASE + 1000 * config + index


def uniform(seed: int, count: int, dtype: str = "f32") -> np.ndarray:
    """`count` values uniform on [-1, 1] from PCG64(seed), cast to dtype."""
    g = np.random.Generator(np.random.PCG64(seed))
    x = g.uniform(-1.0, 1.0, size=int(count))
    return x.astype(np.float32 if dtype == "f32" else np.float64)


def _v(family, **kw):
    d = {"family": family}
    d.update(kw)
    return d


# ---------------------------------------------------------------------------
# workload 1: tiny plain-method suite
# ---------------------------------------------------------------------------
def suite_tiny():
    """4 fp32 global-load stream kernels (2^20 elements, lane stride 1/2/4/8,
    work-group 256) and 2 fp32 FMA loops (64 and 256 FMAs per thread,
    2^16 threads)."""
    out = []
    for s in (1, 2, 4, 8):
        out.append(_v("stream", op="load", dtype="f32", n=1 << 20, wg=256,
                      s=s, gs=1, vec=1, U=1))
    for F in (64, 256):
        out.append(_v("fma", dtype="f32", n=1 << 16, wg=256, F=F, K=4))
    for i, v in enumerate(out):
        v["seed"] = seed_for(1, i)
    return out


# ---------------------------------------------------------------------------
# workload 2: full performance-instructive measurement suite
# ---------------------------------------------------------------------------
def suite_instructive(roofline_points: bool = True, extended: bool = False):
    """Performance-instructive kernels: global stream access by dtype,
    direction, lane and group stride and size; stride-2/3 filled access;
    LDS by bank stride; FMA and rsqrt chains; barriers; empty kernels;
    tiled and naive matrix multiplication in four shapes; three transpose
    configurations.  `extended` appends grids smaller than the GPU holds at
    once (tagged "extension": True), the data for the extension features."""
    out = []
    ns = (1 << 20, 1 << 23, 1 << 26)
    for dt in ("f32", "f64"):
        for op in ("load", "store"):
            for s in (1, 2, 4, 8, 16, 32):
                for n in ns:
                    out.append(_v("stream", op=op, dtype=dt, n=n, wg=256, s=s,
                                  gs=1, vec=1, U=1))
        for s in (1, 2, 4):
            for n in ns:
                out.append(_v("stream", op="copy", dtype=dt, n=n, wg=256, s=s,
                              gs=1, vec=1, U=1))
    for gs in (2, 4, 8):
        for n in ns:
            out.append(_v("stream", op="load", dtype="f32", n=n, wg=256, s=1,
                          gs=gs, vec=1, U=1))
    for n in ns:
        for k in (2, 3):
            out.append(_v("stream", op="filled", dtype="f32", n=n, wg=256, s=k,
                          gs=1, vec=1, U=1))
        out.append(_v("stream", op="add4", dtype="f32", n=n, wg=256, s=1,
                      gs=1, vec=1, U=1))
    # vector scale and add at strides 1, 2, 3
    for dt in ("f32", "f64"):
        for s in (1, 2, 3):
            for n in (1 << 20, 1 << 24):
                out.append(_v("stream", op="axpby", dtype=dt, n=n, wg=256, s=s,
                              gs=1, vec=1, U=1))
    # division and exponential chains
    for dt in ("f32", "f64"):
        for op in ("div", "exp"):
            for F in (32, 128):
                out.append(_v("arith", op=op, dtype=dt, n=1 << 20, wg=256, F=F, K=4))
    # matrix multiplication, tiled: shapes n=m=l, l=n/2, m=n/2, n=m/2
    for n in (384, 768, 1536):
        for (a, b, c) in ((n, n, n), (n, n, n // 2), (n, n // 2, n), (n // 2, n, n)):
            for T in (16, 32):
                out.append(_v("matmul", op="tiled", n=a, m=b, l=c, T=T))
        for T in (16, 32):
            out.append(_v("matmul", op="naive", n=n, m=n, l=n, T=T))
    # transpose: LDS-tiled, naive with coalesced writes, naive with coalesced reads
    for n in (1536, 3072, 6144):
        for op in ("tiled", "naive_wc", "naive_rc"):
            out.append(_v("transpose", op=op, n=n, T=16))
    if roofline_points:
        for dt in ("f32", "f64"):
            for op in ("load", "copy"):
                out.append(_v("stream", op=op, dtype=dt, n=1 << 28, wg=256,
                              s=1, gs=1, vec=1, U=1))
    for op in ("read", "write"):
        for b in (1, 2, 4, 8, 16, 32):
            for R in (256, 1024):
                out.append(_v("lds", op=op, groups=4096, wg=256, b=b, R=R,
                              W=4096))
    for dt in ("f32", "f64"):
        for F in (16, 64, 256, 1024):
            for n in (1 << 20, 1 << 24):
                out.append(_v("fma", dtype=dt, n=n, wg=256, F=F, K=8))
    for F in (64, 256):
        for n in (1 << 20, 1 << 22):
            out.append(_v("rsqrt", n=n, wg=256, F=F, K=4))
    for B in (1, 4, 16, 64):
        for wg in (64, 256, 1024):
            out.append(_v("barrier", groups=4096, wg=wg, B=B))
    for (wx, wy) in ((64, 1), (128, 1), (256, 1), (512, 1), (1024, 1)):
        for n in (1 << 10, 1 << 12, 1 << 14):
            out.append(_v("empty", n=n, wx=wx, wy=wy))
    if extended:
        # grids smaller than the GPU holds at once: long per-work-item chains
        # of arithmetic and of global loads
        ext = []
        for F in (256, 1024, 4096):
            for n in (1 << 12, 1 << 14, 1 << 16):
                ext.append(_v("fma", dtype="f32", n=n, wg=256, F=F, K=8))
        for F in (256, 1024):
            for n in (1 << 12, 1 << 14):
                ext.append(_v("rsqrt", n=n, wg=256, F=F, K=4))
        for U in (16, 64):
            for n in (1 << 14, 1 << 16):
                ext.append(_v("stream", op="load", dtype="f32", n=n, wg=256, s=1, gs=1,
                              vec=1, U=U))
        for v in ext:
            v["extension"] = True
        out += ext
    for i, v in enumerate(out):
        v["seed"] = seed_for(2, i)
    return out


# ---------------------------------------------------------------------------
# workload 3: test-kernel suite whose run times the model predicts
# ---------------------------------------------------------------------------
def suite_test():
    """Test kernels: the paper's four (finite differences = stencil, skinny
    matmul n = l = m/8, n-body, convolution) and square matmul and
    transpose.  `kernel` names the test kernel."""
    out = []
    for n in (512, 1024, 2048, 4096):
        for T in (8, 16, 32):
            for op in ("tiled", "naive"):
                out.append(_v("matmul", op=op, n=n, m=n, l=n, T=T, kernel="matmul"))
    for m in (1024, 2048, 4096, 8192):
        out.append(_v("matmul", op="tiled", n=m // 8, m=m, l=m // 8, T=16,
                      kernel="skinny_mm"))
    for n in (256, 512, 1024, 2048):
        out.append(_v("conv", n=n, T=16, kernel="convolution"))
    for n in (1024, 2048, 4096, 8192):
        out.append(_v("transpose", op="naive_wc", n=n, T=16, kernel="transpose"))
        out.append(_v("transpose", op="tiled", n=n, T=32, kernel="transpose"))
    for dt in ("f32", "f64"):
        for n in (1024, 2048, 4096, 8192):
            out.append(_v("stencil", dtype=dt, n=n, T=16, kernel="finite_difference"))
    for n in (4096, 8192, 16384, 32768, 65536):
        out.append(_v("nbody", n=n, wg=256, kernel="nbody"))
    for i, v in enumerate(out):
        v["seed"] = seed_for(3, i)
    return out


# ---------------------------------------------------------------------------
# work-group size sensitivity (Sec. 5): the same kernels at several group sizes
# ---------------------------------------------------------------------------
WG_SIZES = (128, 256, 512)


def suite_wg(sizes=WG_SIZES):
    """Measurement kernels (global stream by direction and lane stride, FMA
    chains, rsqrt, LDS by bank stride, barriers) and the n-body test kernel,
    each at every work-group size in `sizes` with the total number of
    work-items fixed.  `base` numbers the kernel a variant belongs to: the
    variants of one base differ only in work-group size."""
    bases = []
    for op in ("load", "store", "copy"):
        for s in (1, 2, 4):
            for n in (1 << 23, 1 << 26):
                bases.append(lambda wg, op=op, s=s, n=n: _v(
                    "stream", op=op, dtype="f32", n=n, wg=wg, s=s, gs=1, vec=1, U=1))
    for dt in ("f32", "f64"):
        for F in (64, 256):
            bases.append(lambda wg, dt=dt, F=F: _v("fma", dtype=dt, n=1 << 24, wg=wg, F=F, K=8))
    bases.append(lambda wg: _v("rsqrt", n=1 << 22, wg=wg, F=64, K=4))
    for op in ("read", "write"):
        for b in (1, 4, 32):
            bases.append(lambda wg, op=op, b=b: _v("lds", op=op, groups=(1 << 20) // wg,
                                                   wg=wg, b=b, R=1024, W=4096))
    for B in (4, 16):
        bases.append(lambda wg, B=B: _v("barrier", groups=(1 << 20) // wg, wg=wg, B=B))
    for n in (16384, 65536):
        bases.append(lambda wg, n=n: _v("nbody", n=n, wg=wg, kernel="nbody"))
    out = []
    for bi, mk in enumerate(bases):
        for wg in sizes:
            v = mk(wg)
            v["base"] = bi
            out.append(v)
    for i, v in enumerate(out):
        v["seed"] = seed_for(6, i)
    return out


# ---------------------------------------------------------------------------
# workload 4: batched autotune sweep over uneven iteration domains
# ---------------------------------------------------------------------------
def _not_multiple(x: int, T: int) -> int:
    x = max(int(x), 1)
    return x + 1 if x % T == 0 else x


def suite_batched(count: int = 4096, seed: int | None = None,
                  lo_log2: float = 16.0, hi_log2: float = 30.0):
    """`count` matmul / stencil / transpose variants whose main iteration
    domain holds 2^U(lo, hi) points; extents avoid multiples of the tile."""
    g = np.random.Generator(np.random.PCG64(seed_for(4, 0) if seed is None
                                            else seed))
    out = []
    fams = ("matmul", "stencil", "transpose")
    for i in range(count):
        fam = fams[int(g.integers(0, 3))]
        P = 2.0 ** g.uniform(lo_log2, hi_log2)
        T = (8, 16, 32)[int(g.integers(0, 3))]
        if fam == "matmul":
            base = P ** (1.0 / 3.0)
            d = [_not_multiple(round(base * math.exp(g.normal(0, 0.3))), T)
                 for _ in range(3)]
            v = _v("matmul", op=("tiled", "naive")[int(g.integers(0, 2))],
                   n=d[0], m=d[1], l=d[2], T=T)
        elif fam == "stencil":
            n = _not_multiple(round(math.sqrt(P)), T)
            v = _v("stencil", dtype=("f32", "f64")[int(g.integers(0, 2))],
                   n=n, T=T)
        else:
            n = _not_multiple(round(math.sqrt(P)), T)
            v = _v("transpose",
                   op=("tiled", "naive_wc", "naive_rc")[int(g.integers(0, 3))],
                   n=n, T=T)
        v["seed"] = seed_for(4, i)
        out.append(v)
    return out


# ---------------------------------------------------------------------------
# workload 5: serving trace
# ---------------------------------------------------------------------------
def serving_trace(rate: float = 2000.0, duration: float = 10.0,
                  measure_frac: float = 0.1, seed: int | None = None,
                  lo_log2: float = 16.0, hi_log2: float = 28.0):
    """Poisson arrivals of predict / measure requests.  Returns a list of
    (arrival_seconds, kind, variant) with kind in {'predict', 'measure'}."""
    g = np.random.Generator(np.random.PCG64(seed_for(5, 0) if seed is None
                                            else seed))
    t = 0.0
    out = []
    fams = ("stream", "matmul", "transpose", "stencil", "nbody")
    i = 0
    while True:
        t += g.exponential(1.0 / rate)
        if t >= duration:
            break
        P = 2.0 ** g.uniform(lo_log2, hi_log2)
        fam = fams[int(g.integers(0, 5))]
        T = (8, 16, 32)[int(g.integers(0, 3))]
        if fam == "stream":
            n = max(256, int(P) // 256 * 256)
            v = _v("stream", op=("load", "store", "copy")[int(g.integers(0, 3))],
                   dtype="f32", n=n, wg=256, s=(1, 2, 4, 8)[int(g.integers(0, 4))],
                   gs=1, vec=1, U=1)
        elif fam == "matmul":
            base = P ** (1.0 / 3.0)
            d = [_not_multiple(round(base * math.exp(g.normal(0, 0.3))), T)
                 for _ in range(3)]
            v = _v("matmul", op=("tiled", "naive")[int(g.integers(0, 2))],
                   n=d[0], m=d[1], l=d[2], T=T)
        elif fam == "transpose":
            v = _v("transpose",
                   op=("tiled", "naive_wc", "naive_rc")[int(g.integers(0, 3))],
                   n=_not_multiple(round(math.sqrt(P)), T), T=T)
        elif fam == "stencil":
            v = _v("stencil", dtype="f32",
                   n=_not_multiple(round(math.sqrt(P)), T), T=T)
        else:
            v = _v("nbody", n=max(64, int(math.sqrt(P))), wg=256)
        v["seed"] = seed_for(5, i)
        kind = "measure" if g.uniform() < measure_frac else "predict"
        out.append((t, kind, v))
        i += 1
    return out
