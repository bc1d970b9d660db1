"""Randomised cross-checks on the host (CPU): seeded random small variants
of every family, counted by the library's own descriptor code and by the
simulated-execution oracle (brute force over every work-item), in all four
combinations of the footprint method and the job placement.  The draws
cover ragged extents, every tile size, odd strides and group strides,
vector widths and work-group shapes the descriptors accept."""
import numpy as np
import pytest

import paper_1604_04997_amd as P
from oracle import count as C

N_DRAWS = 1200


def _draw(rng):
    fam = str(rng.choice(["stream", "lds", "fma", "rsqrt", "arith", "barrier", "empty", "matmul",
                          "transpose", "stencil", "nbody", "conv"]))
    r = lambda lo, hi: int(rng.integers(lo, hi + 1))  # noqa: E731
    if fam == "stream":
        op = str(rng.choice(["load", "store", "copy", "add4", "axpby", "filled"]))
        dt = str(rng.choice(["f32", "f64"]))
        wg = int(rng.choice([64, 128, 256]))
        n = wg * r(1, 6)
        if op == "filled":
            s = r(2, 12)
            return dict(family=fam, op=op, dtype=dt, n=n, wg=wg, s=s, c=r(1, min(s, 5)), gs=1,
                        vec=1, U=r(1, 3))
        vec = int(rng.choice([1, 2] if dt == "f64" else [1, 2, 4]))
        return dict(family=fam, op=op, dtype=dt, n=n, wg=wg, s=r(1, 9), gs=r(1, 4), vec=vec,
                    U=r(1, 3))
    if fam == "lds":
        wg = int(rng.choice([64, 128, 256]))
        return dict(family=fam, op=str(rng.choice(["read", "write"])), groups=r(1, 4), wg=wg,
                    b=r(1, 40), R=r(0, 6), W=int(rng.choice([1024, 2048])))
    if fam in ("fma", "rsqrt", "arith"):
        K = int(rng.choice([1, 2, 4, 8]))
        v = dict(family=fam, n=256 * r(1, 4), wg=int(rng.choice([64, 256])), F=K * r(1, 8), K=K)
        if fam != "rsqrt":
            v["dtype"] = str(rng.choice(["f32", "f64"]))
        if fam == "arith":
            v["op"] = str(rng.choice(["div", "exp"]))
        return v
    if fam == "barrier":
        return dict(family=fam, groups=r(1, 5), wg=int(rng.choice([64, 256, 1024])), B=r(0, 4))
    if fam == "empty":
        wx, wy = [(64, 1), (128, 1), (16, 16), (32, 8)][r(0, 3)]
        return dict(family=fam, n=r(1, 300), wx=wx, wy=wy)
    T = int(rng.choice([8, 16, 32]))
    if fam == "matmul":
        return dict(family=fam, op=str(rng.choice(["tiled", "naive"])), n=r(1, 70), m=r(1, 70),
                    l=r(1, 70), T=T)
    if fam == "transpose":
        return dict(family=fam, op=str(rng.choice(["tiled", "naive_wc", "naive_rc"])),
                    n=r(1, 90), T=T)
    if fam == "stencil":
        return dict(family=fam, dtype=str(rng.choice(["f32", "f64"])), n=r(1, 70), T=T)
    if fam == "nbody":
        return dict(family=fam, n=r(1, 700), wg=int(rng.choice([64, 128, 256])))
    return dict(family=fam, n=r(1, 40), T=int(rng.choice([8, 16])))


def _strip(d):
    return {k: v for k, v in d.items() if not k.startswith("foot.")}


@pytest.mark.parametrize("seed", range(4))
def test_random_variants_match_oracle(seed):
    rng = np.random.default_rng(1604_04997 + 77 * seed)
    for _ in range(N_DRAWS // 4):
        v = _draw(rng)
        orc = C.count(v, with_footprints=True)
        for flags in ({}, {"bitmap": True}, {"enumerate": True}):
            d = dict(v, **flags)
            lib = P.count_host(d, with_footprints=True)
            assert _strip(lib) == _strip(orc), d
            for k, x in lib.items():  # footprints the library computes agree too
                if k.startswith("foot."):
                    assert orc[k] == x, (d, k)
            assert P.count_host(d, True, sequential=True) == lib, d
