"""Logical tiles of a BoxArray (tile boxes, face tiles, grown tiles; Sec. 3.2): host
metadata from the library, checked on the CPU by counting cells and faces, and by
computing the paper's flux form face tile by face tile."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1604_03570_amd import inputs as I

bt = pytest.importorskip("paper_1604_03570_amd.boxtile")

CASES = [
    ((16, 12, 8), (4, 4, 4), 2, 7, 1),
    ((24, 16, 20), (1024, 8, 8), 4, 12, 2),   # no tiling along x
    ((9, 7, 5), (2, 3, 1), 1, 5, 3),          # odd edges, tiles of any size
    ((32, 32, 32), (1, 1, 1), 8, 16, 4),      # one cell per tile
    ((20, 20, 20), (64, 64, 64), 4, 10, 5),   # tiles larger than the boxes
]


def _ba(shape, min_edge, max_edge, seed):
    dom = I.domain_box(shape)
    boxes = I.random_chop(dom, min_edge, max_edge, 1, seed=seed)
    return dom, boxes, bt.BoxArray.from_boxes(boxes, dom)


@pytest.mark.parametrize("shape,ts,mn,mx,seed", CASES)
def test_cell_tiles_partition_every_box(shape, ts, mn, mx, seed):
    dom, boxes, ba = _ba(shape, mn, mx, seed)
    t = ba.tile_boxes(ts, "cell")
    count = np.zeros(shape[::-1], dtype=np.int32)
    expected = 0
    for b, bx in enumerate(boxes):
        expected += int(np.prod([-(-(bx[3 + d] - bx[d] + 1) // ts[d]) for d in range(3)]))
    assert len(t) == expected
    for b, *r in t:
        lo, hi = np.array(r[:3]), np.array(r[3:])
        assert np.all(lo >= boxes[b][:3]) and np.all(hi <= boxes[b][3:]) and np.all(hi - lo + 1 <= ts)
        count[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1] += 1
    assert np.all(count == 1)  # boxes cover this domain, tiles partition the boxes
    # box by box, then z, y, x with x fastest
    assert np.all(np.diff(t[:, 0]) >= 0)
    for b in range(len(boxes)):
        rows = t[t[:, 0] == b]
        keys = [(r[3], r[2], r[1]) for r in rows]
        assert keys == sorted(keys)


@pytest.mark.parametrize("shape,ts,mn,mx,seed", CASES)
@pytest.mark.parametrize("d", [0, 1, 2])
def test_face_tiles_partition_every_box_faces(shape, ts, mn, mx, seed, d):
    dom, boxes, ba = _ba(shape, mn, mx, seed)
    t = ba.tile_boxes(ts, "nodal", d)
    cells = ba.tile_boxes(ts, "cell")
    assert len(t) == len(cells)
    for b, bx in enumerate(boxes):
        fshape = [bx[3 + e] - bx[e] + 1 + (1 if e == d else 0) for e in range(3)]
        count = np.zeros(fshape[::-1], dtype=np.int32)
        for _, *r in t[t[:, 0] == b]:
            lo, hi = np.array(r[:3]) - bx[:3], np.array(r[3:]) - bx[:3]
            count[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1] += 1
        assert np.all(count == 1), b
    # only the face tiles that end at the box's high side grow, and by one face
    grown = (t[:, 4 + d] - cells[:, 4 + d])
    ends = cells[:, 4 + d] == np.array([boxes[b][3 + d] for b in cells[:, 0]])
    assert np.array_equal(grown, ends.astype(np.int32))
    assert np.array_equal(np.delete(t, 4 + d, axis=1), np.delete(cells, 4 + d, axis=1))


@pytest.mark.parametrize("ng", [0, 1, 2])
def test_grown_tiles_cover_each_grown_box_once(ng):
    dom, boxes, ba = _ba((16, 12, 10), 3, 8, 6)
    t = ba.tile_boxes((4, 5, 3), "grown", ng)
    for b, bx in enumerate(boxes):
        gshape = [bx[3 + e] - bx[e] + 1 + 2 * ng for e in range(3)]
        count = np.zeros(gshape[::-1], dtype=np.int32)
        for _, *r in t[t[:, 0] == b]:
            lo, hi = np.array(r[:3]) - bx[:3] + ng, np.array(r[3:]) - bx[:3] + ng
            count[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1] += 1
        assert np.all(count == 1), b


def test_bad_arguments_are_refused():
    _, _, ba = _ba((8, 8, 8), 2, 4, 0)
    for ts, kind, arg in [((0, 4, 4), "cell", 0), ((4, 4, 4), "nodal", 3), ((4, 4, 4), "nodal", -1),
                          ((4, 4, 4), "grown", -1)]:
        with pytest.raises(bt.BoxtileError):
            ba.tile_boxes(ts, kind, arg)


def test_flux_form_face_tile_by_face_tile_equals_the_oracle():
    """The flux form computed as the paper structures it: per face tile of each direction
    the face fluxes, then per cell tile the divergence and the update.  Every face is
    written once and the result equals the oracle's flux-form step bit for bit."""
    n = 20
    dom, boxes, ba = _ba((n, n, n), 3, 9, 4)
    rng = np.random.default_rng(3)
    g = rng.random((1, n, n, n))
    dx = 1.0 / n
    inv_dx = 1.0 / dx
    dt = 0.9 * dx * dx / 6.0
    u = O.OracleMultiFab(boxes, dom, (1, 1, 1), 1, 1)
    u.load_global(g)
    u.fill_boundary()
    ref = O.OracleMultiFab(boxes, dom, (1, 1, 1), 1, 1)
    O.heat_flux_step(u.copy(), ref, dt, dx)
    ts = (4, 3, 5)
    cell_tiles = ba.tile_boxes(ts, "cell")
    face_tiles = [ba.tile_boxes(ts, "nodal", d) for d in range(3)]
    for b, bx in enumerate(boxes):
        fab = u.fab(b)[0]  # (z, y, x) with one ghost layer
        ext = bx[3:] - bx[:3] + 1
        flux = [np.full(tuple((ext + (np.arange(3) == d))[::-1]), np.nan) for d in range(3)]
        for d in range(3):
            for _, *r in face_tiles[d][face_tiles[d][:, 0] == b]:
                lo, hi = np.array(r[:3]) - bx[:3], np.array(r[3:]) - bx[:3]
                sl = tuple(slice(lo[e], hi[e] + 1) for e in (2, 1, 0))
                hi_c = tuple(slice(lo[e] + 1, hi[e] + 2) for e in (2, 1, 0))   # cell i (ghost offset 1)
                lo_c = tuple(slice(lo[e] + 1 - (e == d), hi[e] + 2 - (e == d)) for e in (2, 1, 0))  # cell i-1
                assert np.all(np.isnan(flux[d][sl]))  # each face once
                flux[d][sl] = (fab[hi_c] - fab[lo_c]) * inv_dx
        assert all(not np.isnan(f).any() for f in flux)
        new = np.full(tuple(ext[::-1]), np.nan)
        for _, *r in cell_tiles[cell_tiles[:, 0] == b]:
            lo, hi = np.array(r[:3]) - bx[:3], np.array(r[3:]) - bx[:3]
            sl = tuple(slice(lo[e], hi[e] + 1) for e in (2, 1, 0))
            up = [tuple(slice(lo[e] + (e == d), hi[e] + 1 + (e == d)) for e in (2, 1, 0)) for d in range(3)]
            dfx, dfy, dfz = ((flux[d][up[d]] - flux[d][sl]) * inv_dx for d in range(3))
            uc = fab[tuple(slice(lo[e] + 1, hi[e] + 2) for e in (2, 1, 0))]
            new[sl] = uc + dt * ((dfx + dfy) + dfz)
        assert np.array_equal(new, ref.valid(b)[0]), b
