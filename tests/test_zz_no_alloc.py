"""The reduction entry point that allocates nothing (bl_reduce_async_noalloc): its
partial results live in the library's fixed device array.  Called through the C ABI,
it must give bl_reduce_async's result bit for bit, on two calls in a row (the second
on a smaller MultiFab, so stale partials of the first call lie beyond its chunks),
and refuse a MultiFab with more chunks than the array holds."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1604_03570_amd import inputs as I
from tests.gpu_helpers import lib, say

pytestmark = pytest.mark.gpu

OPS = ("sum", "max", "min", "norm0", "norm1", "norm2")


@pytest.fixture(scope="module")
def bt():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return lib()


def _mf(bt, shape, ncomp, dtype, seed):
    dom = I.domain_box(shape)
    boxes = I.random_chop(dom, 8, 32, 8, seed=seed)
    ba = bt.BoxArray.from_boxes(boxes, dom)
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((ncomp,) + tuple(shape[::-1]))
    if dtype == bt.F32:
        g = I.round_f32(g)
    m = bt.MultiFab(ba, ncomp, 1, dtype)
    m.set_val(1e30, with_ghosts=True)  # ghosts must not enter any result
    m.from_global(g)
    return boxes, dom, g, m


def _check(bt, m, ncomp, boxes, dom, g):
    ref = torch.empty(1, dtype=torch.float64, device="cuda")
    got = torch.empty(1, dtype=torch.float64, device="cuda")
    om = O.OracleMultiFab(boxes, dom, (1, 1, 1), ncomp, 1)
    om.load_global(g)
    for comp in range(ncomp):
        for op in OPS:
            got.fill_(float("nan"))
            m.reduce_async(comp, op, ref)
            m.reduce_async_noalloc(comp, op, got)
            torch.cuda.synchronize()
            r, x = float(ref.item()), float(got.item())
            assert x == r, (comp, op, x, r)
            o = O.reduce(om, comp, op)
            assert abs(x - o) <= 1e-13 * abs(o), (comp, op, x, o)


def test_noalloc_reduction_equals_the_allocating_one_twice(bt):
    shape1 = (96, 64, 80)
    boxes, dom, g, m = _mf(bt, shape1, 3, bt.F64, seed=1)
    say(f"noalloc reduce: first call, {len(boxes)} boxes {shape1} f64")
    _check(bt, m, 3, boxes, dom, g)
    shape2 = (32, 24, 16)
    boxes2, dom2, g2, m2 = _mf(bt, shape2, 2, bt.F32, seed=2)
    say(f"noalloc reduce: second call, {len(boxes2)} boxes {shape2} f32")
    _check(bt, m2, 2, boxes2, dom2, g2)


def test_noalloc_reduction_refuses_too_many_chunks(bt):
    """66560 boxes of 4^3: at least one reduction chunk per box, more than the 65536
    partial results the fixed array holds."""
    dom = (0, 0, 0, 127, 127, 259)
    ba = bt.BoxArray.from_boxes(I.regular_chop(dom, 4), dom)
    m = bt.MultiFab(ba, 1, 1, bt.F32)
    m.set_val(1.0)
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    with pytest.raises(bt.BoxtileError, match="no-allocation form holds at most 65536"):
        m.reduce_async_noalloc(0, "sum", out)
    m.reduce_async(0, "sum", out)  # the allocating form still takes it
    torch.cuda.synchronize()
    assert out.item() == 128 * 128 * 260
