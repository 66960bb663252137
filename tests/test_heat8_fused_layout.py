"""Host logic of the fused 8th-order form (CPU only, no kernels run): the segments of
every box face tile the face's 4 cell layers exactly, and every cell found through them
the way the kernel finds it (the first segment of the face that covers its tangential
coordinates, else the last) is the element FillBoundary copies into that ghost cell: the
periodic image's box, or the box's own ghost cell where no box covers it."""
import numpy as np
import pytest

from paper_1604_03570_amd import boxtile as bt
from paper_1604_03570_amd import inputs as I


def _holes():
    boxes = I.random_chop(I.domain_box((24, 16, 20)), 4, 8, 4, seed=9)
    keep = np.sort(np.random.default_rng(5).permutation(len(boxes))[: len(boxes) * 3 // 4])
    return boxes[keep]


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


TANGENT = {0: (1, 2), 1: (0, 2), 2: (0, 1)}


@pytest.mark.parametrize("name", list(_layouts()))
@pytest.mark.parametrize("dtype", [bt.F64, bt.F32])
@pytest.mark.parametrize("ng", [4, 5])
def test_fused_heat8_segments_read_the_fillboundary_source(name, dtype, ng):
    boxes, dom, periodic = _layouts()[name]
    ncomp = 2
    ba = bt.BoxArray.from_boxes(boxes, dom, periodic)
    segs, total = ba.heat8_fused_layout(ncomp, ng, dtype)
    vec = int(segs[0, 11])
    idx = lambda b, cell, comp: ba.layout_index(ncomp, ng, dtype, b, cell, comp)
    checked = 0
    for b, bx in enumerate(boxes):
        e = [int(bx[3 + d] - bx[d] + 1) for d in range(3)]
        for f in range(6):
            a, side = f // 2, f % 2
            u1, u2 = TANGENT[a]
            face = segs[(segs[:, 0] == b) & (segs[:, 1] == f)]
            assert len(face) >= 1
            # the segments tile the face exactly
            cover = np.zeros((e[u1], e[u2]), dtype=np.int32)
            for g in face:
                cover[g[2]:g[3] + 1, g[4]:g[5] + 1] += 1
                if a > 0 and vec > 1:  # whole vectors of x cells in one segment
                    assert g[2] % vec == 0 and (g[3] + 1) % vec == 0
            assert (cover == 1).all(), (name, b, f)
            layers = range(e[a], e[a] + 4) if side else range(-4, 0)
            for t1 in range(e[u1]):
                for t2 in range(e[u2]):
                    hit = [g for g in face[:-1] if g[2] <= t1 <= g[3] and g[4] <= t2 <= g[5]]
                    g = hit[0] if hit else face[-1]
                    o, sc, sx, sy, sz = (int(v) for v in g[6:11])
                    for depth in layers:
                        q = [0, 0, 0]
                        q[a], q[u1], q[u2] = depth, t1, t2
                        glob = (bx[0] + q[0], bx[1] + q[1], bx[2] + q[2])
                        b2, gs = _source(boxes, dom, periodic, b, glob)
                        for comp in (0, ncomp - 1):
                            got = o + comp * sc + q[0] * sx + q[1] * sy + q[2] * sz
                            assert got == idx(b2, gs, comp), (name, b, f, q, comp)
                            assert 0 <= got < total
                            checked += 1
    assert checked > 0


def test_fused_heat8_reports_layouts_it_cannot_take():
    dom = I.domain_box(32)
    # a neighbour 2 cells thick across x: its face cells would need two sources in depth
    boxes = np.array([[0, 0, 0, 1, 31, 31], [2, 0, 0, 31, 31, 31]])
    with pytest.raises(bt.BoxtileError) as e:
        bt.BoxArray.from_boxes(boxes, dom).heat8_fused_layout(1, 4, bt.F64)
    assert e.value.code == bt.BL_EINVAL and "thinner" in str(e.value)
    # fewer than 4 ghost layers
    with pytest.raises(bt.BoxtileError) as e:
        bt.BoxArray.from_boxes(I.regular_chop(dom, 16), dom).heat8_fused_layout(1, 3, bt.F64)
    assert e.value.code == bt.BL_EINVAL
    # a box 6 cells wide: FP32 vectors of one cell, and the form still applies
    boxes = np.array([[0, 0, 0, 31, 15, 31], [0, 16, 0, 5, 31, 31], [6, 16, 0, 31, 31, 31]])
    segs, _ = bt.BoxArray.from_boxes(boxes, dom).heat8_fused_layout(1, 4, bt.F32)
    assert (segs[:, 11] == 1).all()


def test_layout_index_bounds_and_errors():
    dom = I.domain_box(16)
    boxes = I.regular_chop(dom, 8)
    ba = bt.BoxArray.from_boxes(boxes, dom)
    # cells of one box's grown box map to distinct elements inside the MultiFab
    _, total = ba.heat8_fused_layout(2, 4, bt.F64)
    seen = set()
    for k in range(-4, 12):
        for j in (-4, 0, 7, 11):
            for i in range(-4, 12):
                for comp in (0, 1):
                    at = ba.layout_index(2, 4, bt.F64, 0, (i, j, k), comp)
                    assert 0 <= at < total
                    seen.add(at)
    assert len(seen) == 16 * 4 * 16 * 2
    for bad in (((12, 0, 0), 0, 0), ((0, 0, 0), 0, 2), ((0, -5, 0), 0, 0)):
        cell, box, comp = bad
        with pytest.raises(bt.BoxtileError) as e:
            ba.layout_index(2, 4, bt.F64, box, cell, comp)
        assert e.value.code == bt.BL_EINVAL
    with pytest.raises(bt.BoxtileError):
        ba.layout_index(2, 4, bt.F64, len(boxes), (0, 0, 0), 0)


def _mirror_element(ba, ncomp, ng, dtype, boxes, b2, gs, comp):
    """Element of box b2's 4-layer edge mirror that holds its valid cell gs."""
    bx = boxes[b2]
    ex = int(bx[3] - bx[0] + 1)
    cx = int(gs[0] - bx[0])
    side, layer = (0, cx) if cx < 4 else (1, ex - 1 - cx)
    assert 0 <= layer < 4, (b2, gs)
    return ba.layout_mirror_index(ncomp, ng, dtype, b2, side, layer, gs[1], gs[2], comp)


@pytest.mark.parametrize("name", ["uneven", "regular", "one_box", "nonperiodic_x", "slab_hole"])
@pytest.mark.parametrize("dtype", [bt.F64, bt.F32])
def test_fused_heat8_mirror_segments_read_the_neighbours_mirror(name, dtype):
    """The segments of a step whose input's 4-layer mirror is current: y and z faces
    and uncovered x faces as in the rows form; an x-face cell a box covers is the
    element of that box's mirror holding FillBoundary's source cell (a sample of 300
    cells per layout, found the way the kernel searches, plus every segment corner)."""
    boxes, dom, periodic = _layouts()[name]
    ncomp, ng = 2, 4
    ba = bt.BoxArray.from_boxes(boxes, dom, periodic)
    rows, total = ba.heat8_fused_layout(ncomp, ng, dtype)
    mir, total2 = ba.heat8_fused_layout(ncomp, ng, dtype, from_mirror=True)
    assert total2 == total and mir.shape == rows.shape
    assert np.array_equal(mir[:, :6], rows[:, :6])  # the same segments, in the same order
    xf = mir[:, 1] < 2
    assert np.array_equal(mir[~xf], rows[~xf])      # y and z faces: unchanged
    idx = lambda b, cell, comp: ba.layout_index(ncomp, ng, dtype, b, cell, comp)
    rng = np.random.default_rng(8)
    cases = []
    for g in mir[xf]:
        b, f = int(g[0]), int(g[1])
        for t1 in (g[2], g[3]):
            for t2 in (g[4], g[5]):
                cases.append((b, f, int(t1), int(t2), None))
    for _ in range(300):
        b = int(rng.integers(len(boxes)))
        bx = boxes[b]
        cases.append((b, int(rng.integers(2)), int(rng.integers(bx[4] - bx[1] + 1)),
                      int(rng.integers(bx[5] - bx[2] + 1)), None))
    moved = 0
    for b, f, t1, t2, _ in cases:
        bx = boxes[b]
        e0 = int(bx[3] - bx[0] + 1)
        face = mir[(mir[:, 0] == b) & (mir[:, 1] == f)]
        hit = [g for g in face[:-1] if g[2] <= t1 <= g[3] and g[4] <= t2 <= g[5]]
        g = hit[0] if hit else face[-1]
        o, sc, sx, sy, sz = (int(v) for v in g[6:11])
        for depth in (range(e0, e0 + 4) if f else range(-4, 0)):
            glob = (bx[0] + depth, bx[1] + t1, bx[2] + t2)
            b2, gs = _source(boxes, dom, periodic, b, glob)
            covered = all(boxes[b2][d] <= gs[d] <= boxes[b2][3 + d] for d in range(3))
            for comp in (0, ncomp - 1):
                got = o + comp * sc + depth * sx + t1 * sy + t2 * sz
                if covered:
                    assert got == _mirror_element(ba, ncomp, ng, dtype, boxes, b2, gs, comp), (name, b, f, depth)
                    moved += 1
                else:
                    assert got == idx(b2, gs, comp)
                assert 0 <= got < total
    if name != "slab_hole" or periodic[0]:
        assert moved > 0


def test_fused_heat8_mirror_form_needs_boxes_8_wide():
    for name in ("odd_extents", "holes_mixed"):  # boxes 5 and 4 cells wide in x
        boxes, dom, periodic = _layouts()[name]
        ba = bt.BoxArray.from_boxes(boxes, dom, periodic)
        ba.heat8_fused_layout(1, 4, bt.F64)  # the rows form applies
        with pytest.raises(bt.BoxtileError) as e:
            ba.heat8_fused_layout(1, 4, bt.F64, from_mirror=True)
        assert e.value.code == bt.BL_EINVAL and "8 cells" in str(e.value)


def test_mirror_layout_holds_4_layers_apart_from_the_cells():
    """With 4 ghost layers every box's mirror has 2 sides x 4 layers of ey*ez
    elements per component, all distinct, inside the MultiFab and apart from every
    cell of the grown boxes; with 1 ghost layer one layer per side (BL_EINVAL for
    layer 1)."""
    dom = I.domain_box(16)
    boxes = I.regular_chop(dom, (8, 16, 8))
    ba = bt.BoxArray.from_boxes(boxes, dom)
    ncomp = 2
    _, total = ba.heat8_fused_layout(ncomp, 4, bt.F64)
    cells = set()
    for b, bx in enumerate(boxes):
        for k in range(bx[2] - 4, bx[5] + 5):
            for j in range(bx[1] - 4, bx[4] + 5):
                for i in range(bx[0] - 4, bx[3] + 5):
                    for comp in range(ncomp):
                        cells.add(ba.layout_index(ncomp, 4, bt.F64, b, (i, j, k), comp))
    mir = set()
    for b, bx in enumerate(boxes):
        for side in (0, 1):
            for layer in range(4):
                for k in range(bx[2], bx[5] + 1):
                    for j in range(bx[1], bx[4] + 1):
                        for comp in range(ncomp):
                            mir.add(ba.layout_mirror_index(ncomp, 4, bt.F64, b, side, layer, j, k, comp))
    n = sum(2 * 4 * (bx[4] - bx[1] + 1) * (bx[5] - bx[2] + 1) * ncomp for bx in boxes)
    assert len(mir) == n and not (mir & cells)
    assert min(mir) >= 0 and max(mir) < total
    bx = boxes[0]
    ba.layout_mirror_index(1, 1, bt.F64, 0, 1, 0, bx[1], bx[2], 0)
    for bad in ((0, 1), (2, 0), (0, 4)):
        with pytest.raises(bt.BoxtileError) as e:
            ba.layout_mirror_index(1, 1 if bad == (0, 1) else 4, bt.F64, 0, bad[0], bad[1], bx[1], bx[2], 0)
        assert e.value.code == bt.BL_EINVAL
