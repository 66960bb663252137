"""Host logic of the fused 8th-order form (CPU only, no kernels run): its tiles cover
every valid cell of every component exactly once, and every cell of every tile strip
outside its box is read from the element FillBoundary would copy into that ghost cell
(the periodic image's box), or from the box's own ghost cell where no box covers it."""
import numpy as np
import pytest

from paper_1604_03570_amd import boxtile as bt
from paper_1604_03570_amd import inputs as I


def _layouts():
    dom = I.domain_box(32)
    return {
        "uneven": (I.random_chop(dom, 8, 16, 8, seed=4), dom, (1, 1, 1)),
        "regular": (I.regular_chop(dom, 16), dom, (1, 1, 1)),
        "one_box": (np.array([[0, 0, 0, 31, 31, 31]]), dom, (1, 1, 1)),
        "nonperiodic_x": (I.regular_chop(dom, 16), dom, (0, 1, 1)),
        "slab_hole": (np.array([[0, 0, 0, 31, 15, 31]]), dom, (1, 0, 1)),  # y faces of a half-domain slab: uncovered
        "odd_extents": (I.random_chop(I.domain_box((23, 13, 11)), 5, 10, 1, seed=2), I.domain_box((23, 13, 11)),
                        (1, 1, 1)),
        "holes_mixed": (_holes(), I.domain_box((24, 16, 20)), (1, 0, 1)),
    }


def _holes():
    boxes = I.random_chop(I.domain_box((24, 16, 20)), 4, 8, 4, seed=9)
    keep = np.sort(np.random.default_rng(5).permutation(len(boxes))[: len(boxes) * 3 // 4])
    return boxes[keep]


def _source(boxes, dom, periodic, b, g):
    """Box and cell FillBoundary copies ghost cell g of box b from; (b, g) if none."""
    gp = list(g)
    for d in range(3):
        n = dom[3 + d] - dom[d] + 1
        if periodic[d]:
            gp[d] = dom[d] + (g[d] - dom[d]) % n
        elif g[d] < dom[d] or g[d] > dom[3 + d]:
            return b, tuple(g)
    for b2, bx in enumerate(boxes):
        if all(bx[d] <= gp[d] <= bx[3 + d] for d in range(3)):
            return b2, tuple(gp)
    return b, tuple(g)


def _strip_region(t, s, e):
    x0, W, y0, rows, z0, z1 = int(t[2]), int(t[3]), int(t[4]), int(t[5]), int(t[6]), int(t[7])
    lo, hi = [x0, y0, z0], [x0 + W - 1, y0 + rows - 1, z1 - 1]
    a, side = s // 2, s % 2
    if side == 0:
        lo[a] -= 4
        hi[a] = min(lo[a] + 3, -1)
    else:
        top = hi[a]
        lo[a], hi[a] = max(top + 1, e[a]), top + 4
    return lo, hi


@pytest.mark.parametrize("name", list(_layouts()))
@pytest.mark.parametrize("dtype", [bt.F64, bt.F32])
@pytest.mark.parametrize("ng", [4, 5])
def test_fused_heat8_strips_read_the_fillboundary_source(name, dtype, ng):
    boxes, dom, periodic = _layouts()[name]
    ncomp = 2
    ba = bt.BoxArray.from_boxes(boxes, dom, periodic)
    tiles, strips, total = ba.heat8_fused_layout(ncomp, ng, dtype)
    idx = lambda b, cell, comp: ba.layout_index(ncomp, ng, dtype, b, cell, comp)
    # coverage: every valid cell of every component exactly once
    count = {}
    for t in tiles:
        b, comp = int(t[0]), int(t[1])
        count[(b, comp)] = count.get((b, comp), 0) + int(t[3]) * int(t[5]) * (int(t[7]) - int(t[6]))
        assert t[2] % t[8] == 0 and t[3] % t[8] == 0
    for b, bx in enumerate(boxes):
        vol = int(np.prod(np.asarray(bx[3:]) - np.asarray(bx[:3]) + 1))
        for comp in range(ncomp):
            assert count.get((b, comp), 0) == vol, (b, comp)
    cover = {}
    for t in tiles:
        key = (int(t[0]), int(t[1]))
        m = cover.setdefault(key, np.zeros(tuple(np.asarray(boxes[key[0]][3:]) - boxes[key[0]][:3] + 1)[::-1], bool))
        sl = (slice(t[6], t[7]), slice(t[4], t[4] + t[5]), slice(t[2], t[2] + t[3]))
        assert not m[sl].any()
        m[sl] = True
    assert all(m.all() for m in cover.values())
    # strips: every cell outside the box reads FillBoundary's source element
    checked = 0
    for t, S in zip(tiles, strips):
        b, comp = int(t[0]), int(t[1])
        bx = boxes[b]
        e = [int(bx[3 + d] - bx[d] + 1) for d in range(3)]
        for s in range(6):
            lo, hi = _strip_region(t, s, e)
            if lo[s // 2] > hi[s // 2]:
                continue
            o, sx, sy, sz = (int(v) for v in S[s])
            for z in range(lo[2], hi[2] + 1):
                for y in range(lo[1], hi[1] + 1):
                    for x in range(lo[0], hi[0] + 1):
                        g = (bx[0] + x, bx[1] + y, bx[2] + z)
                        b2, gs = _source(boxes, dom, periodic, b, g)
                        want = idx(b2, gs, comp)
                        got = o + x * sx + y * sy + z * sz
                        assert got == want, (name, b, s, (x, y, z), got, want)
                        assert 0 <= got < total
                        checked += 1
    assert checked > 0


def test_fused_heat8_reports_layouts_it_cannot_take():
    dom = I.domain_box(32)
    # a neighbour 2 cells thick across x: a 4-deep strip would have two sources
    boxes = np.array([[0, 0, 0, 1, 31, 31], [2, 0, 0, 31, 31, 31]])
    ba = bt.BoxArray.from_boxes(boxes, dom)
    with pytest.raises(bt.BoxtileError) as e:
        ba.heat8_fused_layout(1, 4, bt.F64)
    assert e.value.code == bt.BL_EINVAL and "thinner" in str(e.value)
    # fewer than 4 ghost layers
    with pytest.raises(bt.BoxtileError) as e:
        bt.BoxArray.from_boxes(I.regular_chop(dom, 16), dom).heat8_fused_layout(1, 3, bt.F64)
    assert e.value.code == bt.BL_EINVAL
    # a box 6 cells wide: FP32 vectors of one cell, and every strip still resolves
    boxes = np.array([[0, 0, 0, 31, 15, 31], [0, 16, 0, 5, 31, 31], [6, 16, 0, 31, 31, 31]])
    tiles, _, _ = bt.BoxArray.from_boxes(boxes, dom).heat8_fused_layout(1, 4, bt.F32)
    assert (tiles[:, 8] == 1).all()
