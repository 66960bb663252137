"""The one-pass red-black sweep (FillBoundary of 2 ghost layers, then one launch per
sweep into a second state buffer), used on periodic levels whose boxes cover the domain
when phi has 2 or more ghost layers.  Every cell update is the two-pass expression on the
same operands, so FP64 fields equal the oracle's bit for bit and FP32 fields equal the
two-pass GPU form's bit for bit; norms are held to 1e-13 (summation order)."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1604_03570_amd import inputs as I
from tests.gpu_helpers import gpu_global, lib, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bt():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return lib()


LAYOUTS = {
    "uneven64": lambda: (I.domain_box(64), I.random_chop(I.domain_box(64), 8, 32, 8, seed=4)),
    "boxes8_aniso": lambda: (I.domain_box((32, 24, 16)), I.regular_chop(I.domain_box((32, 24, 16)), 8)),
    "tiny_odd": lambda: (I.domain_box((18, 12, 10)), I.random_chop(I.domain_box((18, 12, 10)), 1, 6, 1, seed=3)),
    "wide_rows": lambda: (I.domain_box((96, 40, 12)), I.regular_chop(I.domain_box((96, 40, 12)), (96, 20, 12))),
}


def _run(bt, dom, boxes, dtype, ng, f, h2, sweeps):
    ba = bt.BoxArray.from_boxes(boxes, dom)
    phi, fm = bt.MultiFab(ba, 1, ng, dtype), bt.MultiFab(ba, 1, ng, dtype)
    phi.set_val(0.0, with_ghosts=True)
    fm.set_val(0.0, with_ghosts=True)
    fm.from_global(f)
    norms = bt.gsrb_sweeps(phi, fm, h2, sweeps)
    return gpu_global(phi), norms


@pytest.mark.parametrize("sweeps", [2, 3, 4])
@pytest.mark.parametrize("layout", sorted(LAYOUTS))
def test_one_pass_f64_equals_the_oracle(bt, layout, sweeps):
    dom, boxes = LAYOUTS[layout]()
    N = tuple(int(dom[3 + d] + 1) for d in range(3))
    f = I.zero_mean_normal_f32(N, seed=6)
    h2 = (1.0 / max(N)) ** 2
    say(f"gsrb one pass layout={layout} sweeps={sweeps} nbox={len(boxes)}")
    got, norms = _run(bt, dom, boxes, bt.F64, 2, f, h2, sweeps)
    ophi, ofm = O.OracleMultiFab(boxes, dom, (1, 1, 1), 1, 1), O.OracleMultiFab(boxes, dom, (1, 1, 1), 1, 1)
    ofm.load_global(f)
    on = O.gsrb_sweeps(ophi, ofm, h2, sweeps)
    assert np.array_equal(got, ophi.to_global())
    for a, b in zip(norms, on):
        assert abs(a - b) <= 1e-13 * b


@pytest.mark.parametrize("layout", sorted(LAYOUTS))
def test_one_pass_f32_equals_the_two_pass_form(bt, layout):
    dom, boxes = LAYOUTS[layout]()
    N = tuple(int(dom[3 + d] + 1) for d in range(3))
    f = I.zero_mean_normal_f32(N, seed=7)
    h2 = (1.0 / max(N)) ** 2
    one, n1 = _run(bt, dom, boxes, bt.F32, 2, f, h2, 6)   # one pass per sweep
    two, n2 = _run(bt, dom, boxes, bt.F32, 1, f, h2, 6)   # two colour passes per sweep
    assert np.array_equal(one, two)
    for a, b in zip(n1, n2):
        assert abs(a - b) <= 1e-13 * b


def test_one_pass_is_not_taken_where_ghosts_are_uncovered(bt):
    """Boxes leaving holes: the two-pass form runs (ghosts no box covers keep their value),
    bits as the oracle."""
    dom = I.domain_box(32)
    boxes = I.random_chop(dom, 8, 16, 8, seed=5)
    boxes = boxes[np.sort(np.random.default_rng(2).permutation(len(boxes))[: len(boxes) * 3 // 4])]
    f = I.zero_mean_normal_f32(32, seed=8)
    h2 = (1.0 / 32) ** 2
    ba = bt.BoxArray.from_boxes(boxes, dom)
    phi, fm = bt.MultiFab(ba, 1, 2, bt.F64), bt.MultiFab(ba, 1, 2, bt.F64)
    phi.set_val(0.25, with_ghosts=True)
    phi.from_global(np.zeros_like(f))
    fm.set_val(0.0, with_ghosts=True)
    fm.from_global(f)
    bt.gsrb_sweeps(phi, fm, h2, 4, with_norms=False)
    ophi, ofm = O.OracleMultiFab(boxes, dom, (1, 1, 1), 1, 2), O.OracleMultiFab(boxes, dom, (1, 1, 1), 1, 2)
    ophi.data[...] = 0.25
    ophi.load_global(np.zeros_like(f, dtype=np.float64))
    ofm.load_global(f)
    O.gsrb_sweeps(ophi, ofm, h2, 4, with_norms=False)
    assert np.array_equal(gpu_global(phi), ophi.to_global(), equal_nan=True)
