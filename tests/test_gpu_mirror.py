"""The edge mirror (each box's first and last valid x column, kept contiguous along y)
and the library's record of whether it is current.  Calls that find it current read
x faces from it: FillBoundary, the first step of an advance, the first GSRB pass,
the variable-coefficient step.  Every such use must give the oracle's bits, in call
sequences that leave the mirror current, stale, or declared modified."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1604_03570_amd import inputs as I
from tests.gpu_helpers import gpu_global, lib, make_pair, say

pytestmark = pytest.mark.gpu

LAYOUTS = {
    "uneven": (I.domain_box((64, 48, 40)), (1, 1, 1), dict(min_edge=8, max_edge=32, align=8, seed=6), 1.0),
    "odd_noncovering": (I.domain_box((35, 22, 27)), (0, 1, 1), dict(min_edge=3, max_edge=13, align=1, seed=8), 0.8),
}


@pytest.fixture(scope="module")
def bt():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return lib()


def _boxes(layout):
    dom, periodic, kw, keep = LAYOUTS[layout]
    boxes = I.random_chop(dom, kw["min_edge"], kw["max_edge"], kw["align"], seed=kw["seed"])
    if keep < 1.0:
        rng = np.random.default_rng(8)
        boxes = boxes[np.sort(rng.permutation(len(boxes))[: int(len(boxes) * keep)])]
    return dom, periodic, boxes


def _ghosts_equal(bt, mf, om, boxes):
    """Every ghost and valid cell of every FAB (grown boxes) equals the oracle's FAB."""
    for b in range(len(boxes)):
        got = mf.fab(b).double().cpu().numpy()
        ref = om.fab(b)
        m = np.isfinite(ref)
        assert np.array_equal(got[m], ref[m]), b


@pytest.mark.parametrize("layout", sorted(LAYOUTS))
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_fill_boundary_from_the_mirror_after_an_advance(bt, layout, dtype):
    """After a fused advance the mirror is current and FillBoundary reads the one-column
    x-face sources from it: every ghost equals the oracle's fill of the same state."""
    dom, periodic, boxes = _boxes(layout)
    N = tuple(dom[3 + d] + 1 for d in range(3))
    dt = bt.F64 if dtype == "f64" else bt.F32
    g = np.random.default_rng(1).random((2,) + N[::-1]) + 1.0
    if dt == bt.F32:
        g = I.round_f32(g)
    _, a, b, o = make_pair(boxes, dom, periodic, 2, 1, dt, g, ghost_value=np.nan)
    res = bt.heat_advance(a, b, 3, 0.15)
    res.fill_boundary()
    om = O.heat_advance(o, 3, 0.15)
    if dt == bt.F32:  # the oracle's fill of the GPU's own FP32 state
        om = O.OracleMultiFab(boxes, dom, periodic, 2, 1)
        om.data[...] = np.nan
        om.load_global(gpu_global(res))
    om.fill_boundary()
    _ghosts_equal(bt, res, om, boxes)


def _valid_indices(mf, boxes):
    """Element indices (into mf.elements()) of every valid cell, component 0."""
    out = []
    for b, bx in enumerate(boxes):
        grown, off, st = mf.layout(b)
        i = np.arange(bx[0], bx[3] + 1) - bx[0]
        j = np.arange(bx[1], bx[4] + 1) - grown[1]
        k = np.arange(bx[2], bx[5] + 1) - grown[2]
        out.append((off + i[None, None, :] * st[0] + j[None, :, None] * st[1] + k[:, None, None] * st[2]).ravel())
    return np.concatenate(out)


def test_fill_boundary_after_an_outside_write_declared_modified(bt):
    """Valid cells doubled around the library (through the raw element view; the edge
    mirrors keep the old values) and declared with modified(): FillBoundary reads the
    rows again and fills the new values."""
    dom, periodic, boxes = _boxes("uneven")
    N = tuple(dom[3 + d] + 1 for d in range(3))
    rng = np.random.default_rng(2)
    g = rng.random((1,) + N[::-1])
    _, a, b, o = make_pair(boxes, dom, periodic, 1, 1, bt.F64, g)
    res = bt.heat_advance(a, b, 2, 0.15)  # res's mirror is now current
    el = res.elements()
    idx = torch.as_tensor(_valid_indices(res, boxes), device=el.device)
    el[idx] *= 2.0  # the valid cells change, their mirror copies do not...
    res.modified()  # ...and the write is declared
    x = gpu_global(res)
    res.fill_boundary()
    om = O.OracleMultiFab(boxes, dom, periodic, 1, 1)
    om.load_global(x)
    om.fill_boundary()
    got = [res.fab(k).double().cpu().numpy() for k in range(len(boxes))]
    for k in range(len(boxes)):
        m = np.isfinite(om.fab(k))
        assert np.array_equal(got[k][m], om.fab(k)[m]), k


@pytest.mark.parametrize("layout", sorted(LAYOUTS))
def test_advances_in_sequence_continue_from_the_mirror(bt, layout):
    """Advances of 1, 1, 2, 3 and 1 steps alternating the pair's roles, an unfused step
    and a per-box step in between: each continues from the state (and, where current,
    the edge mirror) the last call left, and every state equals the oracle's."""
    dom, periodic, boxes = _boxes(layout)
    N = tuple(dom[3 + d] + 1 for d in range(3))
    g = np.random.default_rng(3).random((2,) + N[::-1]) + 1.0
    _, a, b, o = make_pair(boxes, dom, periodic, 2, 1, bt.F64, g, ghost_value=0.25)
    c = 0.15
    ox, oy = o, o.copy()
    x, y = a, b
    total = 0
    for kind, n in (("adv", 1), ("adv", 1), ("adv", 2), ("unfused", 1), ("adv", 3), ("perbox", 1), ("adv", 1),
                    ("unfused", 1), ("unfused", 1), ("adv", 2)):
        if kind == "adv":
            r = bt.heat_advance(x, y, n, c)
        elif kind == "unfused":
            bt.heat_step_unfused(x, y, c)
            r = y
        else:
            bt.heat_step(x, y, c)
            r = y
        if r is not x:
            x, y = y, x
        for _ in range(n):
            O.heat_step(ox, oy, c)
            ox, oy = oy, ox
        total += n
        ref = ox.to_global()
        m = np.isfinite(ref)
        assert np.array_equal(gpu_global(x)[m], ref[m]), (kind, n, total)
    say(f"mirror continuation {layout}: {total} steps bit-exact")


@pytest.mark.parametrize("one_pass", [0, 1])
def test_gsrb_calls_in_sequence_skip_the_extraction(bt, one_pass):
    """Two GSRB calls in a row (the second finds phi's mirror current and extracts
    nothing) give the oracle's field and norms of one run of all the sweeps, in the
    two-pass form and in the one-pass form."""
    bt.set_gsrb_config(one_pass, 0, 0)
    try:
        _gsrb_in_sequence(bt)
    finally:
        bt.set_gsrb_config(1, 0, 0)


def _gsrb_in_sequence(bt):
    dom, periodic, boxes = _boxes("uneven")
    N = tuple(dom[3 + d] + 1 for d in range(3))
    rng = np.random.default_rng(4)
    f = rng.standard_normal((1,) + N[::-1])
    g0 = 0.1 * rng.random((1,) + N[::-1])
    h2 = 1.0 / 1024.0
    _, phi, fm, ophi = make_pair(boxes, dom, periodic, 1, 1, bt.F64, g0, ghost_value=0.25)
    fm.set_val(0.0, with_ghosts=True)
    fm.from_global(f)
    n1 = bt.gsrb_sweeps(phi, fm, h2, 2)
    n2 = bt.gsrb_sweeps(phi, fm, h2, 3)
    r = bt.residual_norm(phi, fm, h2)
    ofm = O.OracleMultiFab(boxes, dom, periodic, 1, 1)
    ofm.load_global(f)
    on = O.gsrb_sweeps(ophi, ofm, h2, 5)
    ref = ophi.to_global()
    m = np.isfinite(ref)
    assert np.array_equal(gpu_global(phi)[m], ref[m])
    for x, y in zip(n1 + n2, on):
        assert abs(x - y) <= 1e-13 * y
    assert abs(r - on[-1]) <= 1e-13 * on[-1]


def test_varcoef_calls_in_sequence_skip_the_extraction(bt):
    """Variable-coefficient advances of 2 and 3 steps in a row equal the oracle's 5."""
    dom, periodic, boxes = _boxes("uneven")
    N = tuple(dom[3 + d] + 1 for d in range(3))
    rng = np.random.default_rng(5)
    g = rng.random((1,) + N[::-1]) + 1.0
    beta = 0.5 + rng.random((1,) + N[::-1])
    dx = 1.0 / 64
    dt = 0.9 * dx * dx / 9.0
    ba, a, b, o = make_pair(boxes, dom, periodic, 1, 1, bt.F64, g)
    bm = bt.MultiFab(ba, 1, 1, bt.F64)
    bm.set_val(0.0, with_ghosts=True)
    bm.from_global(beta)
    ob = O.OracleMultiFab(boxes, dom, periodic, 1, 1)
    ob.load_global(beta)
    r = bt.heat_varcoef_advance(a, b, bm, 2, dt, dx)
    other = a if r is b else b
    r = bt.heat_varcoef_advance(r, other, bm, 3, dt, dx)
    ref = O.heat_varcoef_advance(o, ob, 5, dt, dx).to_global()
    assert np.array_equal(gpu_global(r), ref)


C8 = 0.09


def _check_4_layer_mirror(bt, mf, boxes, ncomp, rng, nsample=200):
    """The 4-layer mirror of mf holds its first and last 4 valid x columns: every
    corner of every box's mirror and a random sample of its other elements."""
    el = mf.elements()
    ba, ng, dt = mf.ba, mf.nghost, mf.dtype
    pts = []
    for b, bx in enumerate(boxes):
        for side in (0, 1):
            for layer in range(4):
                for j in (bx[1], bx[4]):
                    for k in (bx[2], bx[5]):
                        pts.append((b, side, layer, int(j), int(k), ncomp - 1))
    for _ in range(nsample):
        b = int(rng.integers(len(boxes)))
        bx = boxes[b]
        pts.append((b, int(rng.integers(2)), int(rng.integers(4)), int(rng.integers(bx[1], bx[4] + 1)),
                    int(rng.integers(bx[2], bx[5] + 1)), int(rng.integers(ncomp))))
    mi, ci = [], []
    for b, side, layer, j, k, comp in pts:
        bx = boxes[b]
        i = bx[0] + layer if side == 0 else bx[3] - layer
        mi.append(ba.layout_mirror_index(ncomp, ng, dt, b, side, layer, j, k, comp))
        ci.append(ba.layout_index(ncomp, ng, dt, b, (int(i), j, k), comp))
    mi = torch.as_tensor(mi, device=el.device)
    ci = torch.as_tensor(ci, device=el.device)
    assert torch.equal(el[mi], el[ci])


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_heat8_calls_in_sequence_continue_from_the_4_layer_mirror(bt, dtype):
    """8th-order advances in the mirror form of 1, 2, 3, 1, 2, 1 and 2 steps alternating
    the pair's roles, with a 7-point advance (which writes the first mirror layer only), a
    fill-form call (which writes none) and an outside write declared modified between
    them: every call reads a neighbour's 4-layer mirror only where the last write left all
    4 layers current.
    FP64 states equal the oracle's bit for bit; FP32 states equal those of the same
    calls in the fill form throughout (the forms agree bit for bit).  After each
    8th-order call the result's mirror holds its edge columns; FillBoundary then reads
    the first mirror layer, and every ghost equals the oracle's fill."""
    dom, periodic, boxes = _boxes("uneven")
    N = tuple(dom[3 + d] + 1 for d in range(3))
    dt = bt.F64 if dtype == "f64" else bt.F32
    rng = np.random.default_rng(12)
    g = rng.random((2,) + N[::-1]) + 1.0
    if dt == bt.F32:
        g = I.round_f32(g)
    ba, a, b, o = make_pair(boxes, dom, periodic, 2, 4, dt, g, ghost_value=0.25)
    _, a2, b2, _ = make_pair(boxes, dom, periodic, 2, 4, dt, g, ghost_value=0.25)
    assert bt.heat8_fused_ok(a)
    ba.heat8_fused_layout(2, 4, dt, from_mirror=True)  # the mirror form applies
    ox, oy = o, o.copy()
    pairs = [[a, b], [a2, b2]]  # the default form, the fill form
    idx = torch.as_tensor(_valid_indices(a, boxes), device=a.elements().device)
    seq = (("h8", 1), ("h8", 2), ("h8", 3), ("heat", 1), ("h8", 1), ("fill", 2), ("h8", 2), ("modified", 0),
           ("h8", 1), ("h8", 2))
    for kind, n in seq:
        say(f"heat8 mirror sequence {dtype}: {kind} {n}")
        for p, pair in enumerate(pairs):
            x, y = pair
            if kind == "h8":
                r = bt.heat8_advance(x, y, n, C8, form="fused_mirror" if p == 0 else "fill")
            elif kind == "fill":
                r = bt.heat8_advance(x, y, n, C8, form="fill")
            elif kind == "heat":
                r = bt.heat_advance(x, y, n, 0.15)
            else:  # valid cells scaled around the library, the write declared
                el = x.elements()  # (every MultiFab of one shape has one layout)
                el[idx] *= 0.5
                x.modified()
                r = x
            if r is not x:
                pair.reverse()
        if dt == bt.F64:
            for _ in range(n):
                if kind == "heat":
                    O.heat_step(ox, oy, 0.15)
                elif kind == "modified":
                    break
                else:
                    O.heat8_step(ox, oy, C8)
                ox, oy = oy, ox
            if kind == "modified":
                ox.load_global(gpu_global(pairs[0][0]))
            ref = ox.to_global()
            m = np.isfinite(ref)
            assert np.array_equal(gpu_global(pairs[0][0])[m], ref[m]), (kind, n)
        assert np.array_equal(gpu_global(pairs[0][0]), gpu_global(pairs[1][0]), equal_nan=True), (kind, n)
        if kind == "h8":
            _check_4_layer_mirror(bt, pairs[0][0], boxes, 2, rng)
    res = pairs[0][0]
    res.fill_boundary()
    om = O.OracleMultiFab(boxes, dom, periodic, 2, 4)
    om.data[...] = np.nan
    om.load_global(gpu_global(res))
    om.fill_boundary()
    _ghosts_equal(bt, res, om, boxes)
