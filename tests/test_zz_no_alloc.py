"""GPU test of the allocation-free batched count (pm_count_device_noalloc)
through the C ABI: its count vectors, FP64 predictions and statuses equal
those of pm_count_device on the same variants, on two calls in a row (the
second with fewer variants), and a batch over its size limit is refused."""
import numpy as np
import pytest

import paper_1604_04997_amd as P
from synth import suite_batched

from test_lib_host import FAMILY_CASES

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "no GPU visible"
    c = P.Context(0)
    yield c
    c.close()


def _run(ctx, vs, model, noalloc):
    import torch
    va = P.variant_array(vs)
    nv = len(vs)
    d_v = torch.frombuffer(bytearray(bytes(memoryview(va).cast("B"))),
                           dtype=torch.uint8).cuda()
    d_c = torch.full((nv, P.PM_NCOUNT), 7, dtype=torch.int64, device="cuda")
    d_t = torch.full((nv,), 7.0, dtype=torch.float64, device="cuda")
    d_s = torch.full((nv,), 99, dtype=torch.int32, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    if noalloc:
        ctx.count_device_noalloc(d_v.data_ptr(), nv, d_c.data_ptr(), model,
                                 d_t.data_ptr(), d_s.data_ptr(), s)
    else:
        ctx.reserve(nv, sum(P.bitmap_bytes(v) for v in vs))
        ctx.count_device(d_v.data_ptr(), nv, d_c.data_ptr(), model, d_t.data_ptr(),
                         d_s.data_ptr(), s)
    torch.cuda.synchronize()
    return d_c.cpu().numpy(), d_t.cpu().numpy(), d_s.cpu().numpy()


def test_noalloc_matches_device_path_twice(ctx):
    # first call: 600 variants (the 64-wide expansion kernel) mixing count
    # jobs, closed forms, bitmaps (handed on to the chip-wide kernels) and
    # the sweep; second call: 20 variants (the fused kernel)
    mixed = [dict(v, bitmap=True) if k % 3 == 0 else v for k, v in enumerate(FAMILY_CASES)]
    first = (mixed * 4)[:300] + suite_batched(300, seed=5)
    second = mixed[5:25]
    m = P.model_struct("p12", np.linspace(1e-12, 1e-11, 12))
    for k, vs in enumerate((first, second)):
        print("noalloc call %d: %d variants" % (k, len(vs)), flush=True)
        want = _run(ctx, vs, m, noalloc=False)
        got = _run(ctx, vs, m, noalloc=True)
        np.testing.assert_array_equal(got[2], want[2])
        assert (got[2] == 0).all()
        np.testing.assert_array_equal(got[0], want[0])
        np.testing.assert_array_equal(got[1], want[1])


def test_noalloc_rejects_too_many_variants(ctx):
    import torch
    nv = P.PM_NOALLOC_MAX_VARIANTS + 1
    d = torch.zeros(nv * 88, dtype=torch.uint8, device="cuda")
    with pytest.raises(P.PMError) as e:
        ctx.count_device_noalloc(d.data_ptr(), nv, 0, None, 0, d.data_ptr(),
                                 torch.cuda.current_stream().cuda_stream)
    assert e.value.code == -1
