"""Parity of the 8th-order heat step (9-cell span, HIP kernel through the C-ABI) with
the oracle.  FP64 bit for bit (same operand order, coefficients rounded once, no FMA
contraction); FP32 storage within 2e-5 of the FP64 oracle; the fill form, the fused form
(neighbour boxes read directly) and the fused form with the 4-layer edge mirrors agree bit
for bit.  Layouts: uneven boxes, holes
next to a non-periodic side, odd extents (scalar lanes), boxes whose last x tile is one
vector wide (its halo reaches past the row end into the x ghost slab), 5 ghost layers."""
import math

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1604_03570_amd import inputs as I
from tests.gpu_helpers import gpu_global, lib, make_pair, rel_err, say

pytestmark = pytest.mark.gpu

C8 = 0.09


@pytest.fixture(scope="module")
def bt():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return lib()


def _layout(name, rng):
    if name == "uneven_periodic":
        dom, periodic = I.domain_box(64), (1, 1, 1)
        boxes = I.random_chop(dom, 8, 32, 8, seed=4)
    elif name == "holes_mixed":
        dom, periodic = I.domain_box((48, 32, 40)), (1, 0, 1)
        boxes = I.random_chop(dom, 8, 24, 8, seed=9)
        boxes = boxes[np.sort(rng.permutation(len(boxes))[: len(boxes) * 3 // 4])]
    elif name == "odd_extents":
        dom, periodic = I.domain_box((37, 23, 18)), (1, 1, 1)
        boxes = I.random_chop(dom, 5, 14, 1, seed=2)
    else:  # x extent 34: 16 + 1 vectors of 2 cells, so the last x tile is one vector wide
        dom, periodic = I.domain_box((68, 40, 36)), (1, 1, 1)
        boxes = I.regular_chop(dom, (34, 20, 36))
    return dom, periodic, boxes


@pytest.mark.parametrize("form", ["fill", "fused", "fused_mirror"])
@pytest.mark.parametrize("ng", [4, 5])
@pytest.mark.parametrize("dtype_name", ["f64", "f32"])
@pytest.mark.parametrize("layout", ["uneven_periodic", "holes_mixed", "odd_extents", "narrow_last_tile"])
def test_heat8_equals_the_oracle(bt, layout, dtype_name, ng, form):
    rng = np.random.default_rng(5)
    dom, periodic, boxes = _layout(layout, rng)
    dtype = bt.F64 if dtype_name == "f64" else bt.F32
    N = tuple(int(dom[3 + d] + 1) for d in range(3))
    g = rng.random((2,) + N[::-1]) + 1.0
    if dtype == bt.F32:
        g = I.round_f32(g)
    steps = 7
    say(f"heat8 layout={layout} dtype={dtype_name} ng={ng} form={form} nbox={len(boxes)}")
    _, a, b, o = make_pair(boxes, dom, periodic, 2, ng, dtype, g, ghost_value=0.5)
    assert bt.heat8_fused_ok(a)
    if form == "fused_mirror" and layout == "odd_extents":  # boxes 5 cells wide: no 4-layer mirror form
        with pytest.raises(bt.BoxtileError) as e:
            bt.heat8_advance(a, b, steps, C8, form=form)
        assert e.value.code == bt.BL_EINVAL and "8 cells" in str(e.value)
        return
    res = bt.heat8_advance(a, b, steps, C8, form=form)
    ref = O.heat8_advance(o, steps, C8).to_global()
    got = gpu_global(res)
    if dtype == bt.F64:
        assert np.array_equal(got, ref, equal_nan=True)
    else:
        err = rel_err(got, ref)
        say(f"  fp32 rel err {err:.2e}")
        assert err <= 2e-5
    if form != "fill":  # the forms agree bit for bit, FP32 included
        _, a2, b2, _ = make_pair(boxes, dom, periodic, 2, ng, dtype, g, ghost_value=0.5)
        assert np.array_equal(gpu_global(bt.heat8_advance(a2, b2, steps, C8, form="fill")), got, equal_nan=True)


def test_heat8_fused_form_refused_where_a_neighbour_is_thin(bt):
    dom = I.domain_box(32)
    boxes = np.array([[0, 0, 0, 1, 31, 31], [2, 0, 0, 31, 31, 31]])  # a neighbour 2 cells thick across x
    g = np.random.default_rng(3).random((1, 32, 32, 32)) + 1.0
    _, a, b, o = make_pair(boxes, dom, (1, 1, 1), 1, 4, bt.F64, g)
    assert not bt.heat8_fused_ok(a)
    with pytest.raises(bt.BoxtileError):
        bt.heat8_advance(a, b, 1, C8, form="fused")
    res = bt.heat8_advance(a, b, 3, C8)  # auto: the fill form
    assert np.array_equal(gpu_global(res), O.heat8_advance(o, 3, C8).to_global())


def test_heat8_degenerate_calls(bt):
    dom = I.domain_box(16)
    boxes = I.regular_chop(dom, 8)
    g = np.random.default_rng(2).random((1, 16, 16, 16))
    _, a, b, _ = make_pair(boxes, dom, (1, 1, 1), 1, 4, bt.F64, g)
    before = gpu_global(a)
    assert bt.heat8_advance(a, b, 0, C8) is a
    assert np.array_equal(gpu_global(a), before)
    _, a1, b1, _ = make_pair(boxes, dom, (1, 1, 1), 1, 3, bt.F64, g)
    with pytest.raises(bt.BoxtileError):  # three ghost layers are too few
        bt.heat8_advance(a1, b1, 1, C8)
    with pytest.raises(bt.BoxtileError):
        bt.heat8_advance(a, b, -1, C8)
    # an unknown form: refused before any launch, the state untouched
    import ctypes
    arr = (ctypes.c_void_p * 2)(a.handle.value, b.handle.value)
    for form in (-1, 4):
        assert bt._L.bl_heat8_advance_form(arr, 1, ctypes.c_double(C8), form, None) == bt.BL_EINVAL
    assert np.array_equal(gpu_global(a), before)
    # the mirror form needs boxes at least 8 cells wide in x: 16 boxes of 4 x 16 x 16
    boxes4 = I.regular_chop(dom, (4, 16, 16))
    _, a4, b4, _ = make_pair(boxes4, dom, (1, 1, 1), 1, 4, bt.F64, g)
    with pytest.raises(bt.BoxtileError) as e:
        bt.heat8_advance(a4, b4, 1, C8, form="fused_mirror")
    assert e.value.code == bt.BL_EINVAL and "8 cells" in str(e.value)
