"""GPU tests of the counts as quasi-polynomials of one size (pm_qpoly_derive
/ pm_qpoly_eval): derived once from the batched counter, evaluated on the
host at sizes far from the derivation points, and checked bit for bit
against the counter at those sizes; a period the counts do not have is
refused."""
import numpy as np
import pytest

import paper_1604_04997_amd as P

pytestmark = pytest.mark.gpu

# (variant, fields, scale, period, x0, largest x tried)
CASES = [
    (dict(family="stencil", dtype="f32", n=0, T=16), 1, 1, 16, 64, 40000),
    (dict(family="stencil", dtype="f64", n=0, T=8), 1, 1, 8, 32, 40000),
    (dict(family="transpose", op="tiled", n=0, T=32), 1, 1, 32, 64, 40000),
    (dict(family="transpose", op="naive_wc", n=0, T=16), 1, 1, 16, 64, 40000),
    (dict(family="transpose", op="naive_rc", n=0, T=8), 1, 1, 8, 32, 40000),
    (dict(family="matmul", op="tiled", n=0, m=0, l=0, T=16), 7, 1, 16, 32, 20000),
    (dict(family="matmul", op="naive", n=0, m=0, l=0, T=8), 7, 1, 8, 16, 20000),
    (dict(family="matmul", op="tiled", n=0, m=300, l=0, T=32), 5, 1, 32, 64, 20000),
    (dict(family="conv", n=0, T=8), 1, 1, 8, 16, 8000),
    (dict(family="nbody", n=0, wg=64), 1, 1, 64, 128, 60000),
    (dict(family="stream", op="load", dtype="f32", n=0, wg=256, s=2, gs=1, vec=1, U=1),
     1, 256, 1, 1, 200000),
]


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "no GPU visible"
    c = P.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("case", CASES, ids=lambda c: "%s-%s" % (c[0]["family"],
                                                                 c[0].get("op", c[0].get("dtype"))))
def test_qpoly_matches_counter(ctx, case):
    d, fields, scale, period, x0, xmax = case
    print("qpoly", d, flush=True)
    qp = ctx.qpoly_derive(d, fields=fields, scale=scale, period=period, x0=x0)
    rng = np.random.default_rng(7)
    xs = sorted(set([x0, x0 + 1, x0 + period * 6 + 1, xmax] +
                    [int(x) for x in rng.integers(x0, xmax, 40)]))
    vs = [P.qpoly_sizes(d, fields, scale, x) for x in xs]
    got = P.counts_numpy(ctx.count_raw(vs))
    for i, x in enumerate(xs):
        ev = np.ctypeslib.as_array(P.qpoly_eval(qp, x).c)
        np.testing.assert_array_equal(ev, got[i], err_msg="x=%d" % x)


def test_qpoly_refuses_a_wrong_period(ctx):
    d = dict(family="stencil", dtype="f32", n=0, T=16)
    with pytest.raises(P.PMError) as e:
        ctx.qpoly_derive(d, fields=1, period=3, x0=64)
    assert e.value.code == -1 and "no polynomial" in str(e.value)
