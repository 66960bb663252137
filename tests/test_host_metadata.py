"""Host-side logic of the library (CPU only, no kernels run): exported symbols,
BoxArray validation, box chops against the shared input generators, the
FillBoundary copy plan against the oracle's fill, the face-source records,
tile-list coverage and the static tile partition of the paper's worked example."""
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_1604_03570_amd import inputs as I

bt = pytest.importorskip("paper_1604_03570_amd.boxtile", reason="libboxtile.so not built")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_library_exports_every_declared_function():
    names = bt.header_functions()
    assert len(names) >= 30
    missing = [n for n in names if not hasattr(bt.lib(), n)]
    assert not missing, missing


def test_boxarray_validation_errors():
    dom = (0, 0, 0, 7, 7, 7)
    with pytest.raises(bt.BoxtileError) as e:
        bt.BoxArray.from_boxes([(0, 0, 0, 3, 3, 3), (3, 3, 3, 5, 5, 5)], dom)
    assert e.value.code == bt.BL_EOVERLAP
    with pytest.raises(bt.BoxtileError) as e:
        bt.BoxArray.from_boxes([(0, 0, 0, 3, 3, 8)], dom)
    assert e.value.code == bt.BL_EDOMAIN
    with pytest.raises(bt.BoxtileError) as e:
        bt.BoxArray.from_boxes([(2, 0, 0, 1, 3, 3)], dom)
    assert e.value.code == bt.BL_EINVAL
    with pytest.raises(bt.BoxtileError) as e:
        bt.BoxArray.chop_random(dom, min_edge=4, max_edge=6)
    assert e.value.code == bt.BL_EINVAL
    with pytest.raises(bt.BoxtileError) as e:
        bt.DistributionMapping(bt.BoxArray.chop(dom, 4), ndevices=2)
    assert e.value.code == bt.BL_EINVAL
    ba = bt.BoxArray.from_boxes([(0, 0, 0, 3, 3, 3), (4, 4, 4, 7, 7, 7)], dom)  # non-covering is fine
    assert len(ba) == 2


@pytest.mark.parametrize("n,edge", [(64, 32), (96, 64), ((40, 24, 16), (16, 8, 16)), (256, 64)])
def test_regular_chop_matches_generator(n, edge):
    dom = I.domain_box(n)
    assert np.array_equal(bt.BoxArray.chop(dom, edge).boxes(), I.regular_chop(dom, edge))


@pytest.mark.parametrize("seed", [0, 1, 2, 3, 17])
def test_random_chop_matches_generator(seed):
    dom = I.domain_box(512)
    lib_boxes = bt.BoxArray.chop_random(dom, 16, 128, 8, seed).boxes()
    assert np.array_equal(lib_boxes, I.random_chop(dom, 16, 128, 8, seed))
    e = lib_boxes[:, 3:] - lib_boxes[:, :3] + 1
    assert e.min() >= 16 and e.max() <= 128 and np.all(e % 8 == 0)
    assert int(np.prod(e, axis=1).sum()) == 512 ** 3


def _fabs_from_plan(boxes, shape, periodic, ng, plan):
    """Per-box grown arrays with unique valid values, ghosts set by applying the plan records."""
    nx, ny, nz = shape
    g = np.arange(nx * ny * nz, dtype=np.float64).reshape(nz, ny, nx) + 0.5
    fabs = []
    for bx in boxes:
        a = np.full((bx[5] - bx[2] + 1 + 2 * ng, bx[4] - bx[1] + 1 + 2 * ng, bx[3] - bx[0] + 1 + 2 * ng), -1e300)
        a[ng:-ng, ng:-ng, ng:-ng] = g[bx[2]:bx[5] + 1, bx[1]:bx[4] + 1, bx[0]:bx[3] + 1]
        fabs.append(a)
    hits = [np.zeros(f.shape, dtype=np.int32) for f in fabs]
    for r in plan:
        dst, src, lo, hi, sh = r[0], r[1], r[2:5], r[5:8], r[8:11]
        db, sb = boxes[dst], boxes[src]
        dsl = tuple(slice(lo[d] - db[d] + ng, hi[d] - db[d] + ng + 1) for d in (2, 1, 0))
        ssl = tuple(slice(lo[d] + sh[d] - sb[d] + ng, hi[d] + sh[d] - sb[d] + ng + 1) for d in (2, 1, 0))
        fabs[dst][dsl] = fabs[src][ssl]
        hits[dst][dsl] += 1
    return g, fabs, hits


@pytest.mark.parametrize("case", range(16))
def test_fill_plan_matches_oracle_fill(case):
    rng = np.random.default_rng(500 + case)
    shape = [(8, 6, 4), (5, 5, 5), (12, 8, 10), (7, 4, 6)][case % 4]
    ng = 1 + case % 2
    periodic = tuple(int(v) for v in rng.integers(0, 2, 3))
    boxes = I.random_chop(I.domain_box(shape), min_edge=1 + case % 2, max_edge=4 + case % 3, align=1, seed=case)
    if case % 3 == 2 and len(boxes) > 2:  # non-covering
        boxes = boxes[np.sort(rng.permutation(len(boxes))[: max(1, len(boxes) * 2 // 3)])]
    if any(periodic[d] and ng > shape[d] for d in range(3)):
        pytest.skip("ghost width above a periodic extent")
    ba = bt.BoxArray.from_boxes(boxes, I.domain_box(shape), periodic)
    g, fabs, hits = _fabs_from_plan(boxes, shape, periodic, ng, ba.fill_plan(ng))
    m = O.OracleMultiFab(boxes, I.domain_box(shape), periodic, 1, ng)
    m.data[...] = -1e300
    m.load_global(g[None])
    m.fill_boundary()
    for b in range(len(boxes)):
        assert np.array_equal(fabs[b], m.fab(b)[0]), b
        assert hits[b].max() <= 1  # no ghost cell written twice
        inner = hits[b][ng:-ng, ng:-ng, ng:-ng]
        assert inner.max() == 0  # valid cells never written


@pytest.mark.parametrize("case", range(10))
def test_face_plan_partitions_every_face_and_matches_wrap(case):
    rng = np.random.default_rng(900 + case)
    shape = [(8, 6, 4), (12, 8, 10), (9, 7, 5)][case % 3]
    periodic = tuple(int(v) for v in rng.integers(0, 2, 3))
    boxes = I.random_chop(I.domain_box(shape), min_edge=1, max_edge=4, align=1, seed=40 + case)
    if case % 2 and len(boxes) > 2:
        boxes = boxes[np.sort(rng.permutation(len(boxes))[: len(boxes) // 2])]
    ba = bt.BoxArray.from_boxes(boxes, I.domain_box(shape), periodic)
    recs = ba.face_plan()
    N = shape
    owner = {}
    for b, bx in enumerate(boxes):
        for k in range(bx[2], bx[5] + 1):
            for j in range(bx[1], bx[4] + 1):
                for i in range(bx[0], bx[3] + 1):
                    owner[(i, j, k)] = b
    for b, bx in enumerate(boxes):
        for face in range(6):
            a, side = divmod(face, 2)
            layer = list(bx)
            layer[a] = layer[3 + a] = bx[3 + a] + 1 if side else bx[a] - 1
            count = {}
            for r in recs[(recs[:, 0] == b) & (recs[:, 1] == face)]:
                src, lo, hi, sh = r[2], r[3:6], r[6:9], r[9:12]
                for k in range(lo[2], hi[2] + 1):
                    for j in range(lo[1], hi[1] + 1):
                        for i in range(lo[0], hi[0] + 1):
                            p = (i, j, k)
                            count[p] = count.get(p, 0) + 1
                            q = [p[d] % N[d] if periodic[d] else p[d] for d in range(3)]
                            inside = all(0 <= q[d] < N[d] for d in range(3))
                            want = owner.get(tuple(q)) if inside else None
                            if want is None:
                                assert src == b and tuple(sh) == (0, 0, 0)
                            else:
                                assert src == want
                                assert tuple(p[d] + sh[d] for d in range(3)) == tuple(q)
            cells = {(i, j, k) for k in range(layer[2], layer[5] + 1) for j in range(layer[1], layer[4] + 1)
                     for i in range(layer[0], layer[3] + 1)}
            assert set(count) == cells and max(count.values()) == 1


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("boxes_kind", ["regular", "uneven", "odd"])
def test_tile_list_covers_every_cell_once(dtype, boxes_kind):
    if boxes_kind == "regular":
        dom, boxes = I.domain_box(64), I.regular_chop(I.domain_box(64), 32)
    elif boxes_kind == "uneven":
        dom = I.domain_box(128)
        boxes = I.random_chop(dom, 16, 64, 8, seed=3)
    else:
        dom = I.domain_box((21, 13, 9))
        boxes = I.random_chop(dom, 3, 8, 1, seed=5)
    ncomp = 2
    ba = bt.BoxArray.from_boxes(boxes, dom)
    tiles = ba.tile_list(ncomp, 1, dtype)
    for b, bx in enumerate(boxes):
        ex, ey, ez = bx[3] - bx[0] + 1, bx[4] - bx[1] + 1, bx[5] - bx[2] + 1
        cover = np.zeros((ncomp, ez, ey, ex), dtype=np.int32)
        for t in tiles[tiles[:, 0] == b]:
            comp, xv0, nvt, y0, rows, z0, z1, vec = t[1:]
            assert nvt * rows <= 256  # fits the default workgroup
            cover[comp, z0:z1, y0:y0 + rows, xv0 * vec:(xv0 + nvt) * vec] += 1
        assert cover.min() == 1 and cover.max() == 1


@pytest.mark.parametrize("dtype", [0, 1])
def test_small_levels_take_shorter_tiles(dtype):
    """Where the configured shape (4 planes, 4 waves, 2 z steps) gives fewer than 1024
    tiles, every tile takes one z step, and if that is still fewer than 1024, one z block
    per step: more and shorter workgroups for latency-bound launches.  A level with
    enough tiles keeps two z steps."""
    saved = bt.get_tile_config()
    bt.set_tile_config(4, 4, 0, 3, 2)
    try:
        def tiles(n, edge):
            dom = I.domain_box(n)
            return bt.BoxArray.from_boxes(I.regular_chop(dom, edge), dom).stencil_tiles(1, 1, dtype)
        large = tiles(256, 64)   # 64 boxes of 64^3: thousands of tiles
        mid = tiles(64, 32)      # 8 boxes of 32^3: under 1024 even with one z step
        tiny = tiles(32, 8)      # 64 boxes of 8^3: whole planes stacked in z blocks
    finally:
        bt.set_tile_config(*saved)
    planes = lambda t: t[:, 6] - t[:, 5]
    assert len(large) >= 1024 and (planes(large) == 2 * 4 * large[:, 4]).any()
    for t in (mid, tiny):
        assert len(t) < 1024
        assert (t[:, 4] == 1).all() and (planes(t) <= 4).all()
    assert len(tiny) == 64 * 2  # 8 planes per box in z blocks of 4: two tiles each


@pytest.mark.parametrize("dtype", [0, 1])
@pytest.mark.parametrize("boxes_kind", ["regular", "uneven", "odd", "cells"])
@pytest.mark.parametrize("shape", [(4, 4, 1), (2, 4, 2), (8, 2, 1), (4, 3, 4), (4, 4, 8)])
def test_stencil_tiles_cover_every_cell_once(dtype, boxes_kind, shape):
    """Linear tiles (runs of consecutive vectors of a plane, whole planes stacked in z
    blocks for small planes) cover every valid cell of every component exactly once,
    fit the workgroup, and do not straddle a z boundary of an x or y face record."""
    if boxes_kind == "regular":
        dom, boxes = I.domain_box(64), I.regular_chop(I.domain_box(64), 32)
    elif boxes_kind == "uneven":
        dom = I.domain_box(128)
        boxes = I.random_chop(dom, 16, 64, 8, seed=3)
    elif boxes_kind == "odd":
        dom = I.domain_box((21, 13, 9))
        boxes = I.random_chop(dom, 3, 8, 1, seed=5)
    else:  # boxes of one and two cells, as on the coarse levels of a V-cycle
        dom = I.domain_box((6, 4, 4))
        boxes = I.random_chop(dom, 1, 2, 1, seed=7)
    ncomp = 2
    saved = bt.get_tile_config()
    bt.set_tile_config(shape[0], shape[1], 0, 3, shape[2])
    try:
        ba = bt.BoxArray.from_boxes(boxes, dom)
        tiles = ba.stencil_tiles(ncomp, 1, dtype)
        faces = ba.face_plan()
    finally:
        bt.set_tile_config(*saved)
    assert len(tiles)
    for b, bx in enumerate(boxes):
        ex, ey, ez = bx[3] - bx[0] + 1, bx[4] - bx[1] + 1, bx[5] - bx[2] + 1
        cover = np.zeros((ncomp, ez, ey * ex), dtype=np.int32)
        cuts = set()
        for r in faces[(faces[:, 0] == b) & (faces[:, 1] < 4)]:
            cuts.add(int(r[5] - bx[2]))
            cuts.add(int(r[8] - bx[2] + 1))
        for t in tiles[tiles[:, 0] == b]:
            comp, q0, nq, nzs, z0, z1, zc, vec, lanes, zsteps = t[1:]
            assert vec in (1, 2, 4) and ex % vec == 0 and nzs * nq <= lanes == 64 * shape[1]
            assert zsteps == shape[2] and z1 - z0 <= nzs * zc * zsteps and nzs <= -(-(z1 - z0) // zc)
            assert not any(z0 < c < z1 for c in cuts)
            cover[comp, z0:z1, q0 * vec:(q0 + nq) * vec] += 1
        assert cover.min() == 1 and cover.max() == 1


def test_tiles_do_not_straddle_face_record_z_boundaries():
    dom = I.domain_box(128)
    boxes = I.random_chop(dom, 16, 64, 8, seed=2)
    ba = bt.BoxArray.from_boxes(boxes, dom)
    tiles = ba.tile_list(1, 1, bt.F64)
    faces = ba.face_plan()
    for b, bx in enumerate(boxes):
        cuts = set()
        for r in faces[(faces[:, 0] == b) & (faces[:, 1] < 4)]:
            cuts.add(int(r[5] - bx[2]))          # region lo z, box-local
            cuts.add(int(r[8] - bx[2] + 1))      # region hi z + 1
        for t in tiles[tiles[:, 0] == b]:
            z0, z1 = t[6], t[7]
            assert not any(z0 < c < z1 for c in cuts)


def test_static_partition_reproduces_the_papers_worked_example():
    path = os.path.join(GOLDEN, "static_schedule_sec3_3.txt")
    expect = {}
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        parts = line.split()
        expect[int(parts[0])] = [tuple(int(v) for v in p.split(",")) for p in parts[1:]]
    tiles_per_grid = [4, 2, 2, 4]
    flat = [(g, t) for g, n in enumerate(tiles_per_grid) for t in range(n)]  # collapsed (grid, tile) loop
    first = bt.static_partition(len(flat), 4)
    for w in range(4):
        assert flat[first[w]:first[w + 1]] == expect[w]


def test_static_partition_general():
    for n, w in [(0, 3), (5, 8), (100, 7), (12, 4)]:
        f = bt.static_partition(n, w)
        sizes = np.diff(f)
        assert f[0] == 0 and f[-1] == n and sizes.max() - sizes.min() <= 1
        assert list(sizes) == sorted(sizes, reverse=True)


def test_multifab_bytes_cover_the_grown_boxes():
    boxes = I.random_chop(I.domain_box(128), 16, 64, 8, seed=1)
    ba = bt.BoxArray.from_boxes(boxes, I.domain_box(128))
    e = boxes[:, 3:] - boxes[:, :3] + 3
    grown = int(np.prod(e, axis=1).sum())
    for dtype, es in ((bt.F64, 8), (bt.F32, 4)):
        nb = ba.multifab_bytes(3, 1, dtype)
        assert 3 * grown * es <= nb <= 3 * grown * es * 1.35


def test_device_copy_refuses_bad_arguments_before_any_launch():
    """Argument errors return BL_EINVAL without touching a device (this runs on the CPU)."""
    import ctypes
    from paper_1604_03570_amd import boxtile as bt
    L = bt.lib()
    vp = ctypes.c_void_p
    assert L.bl_device_copy(vp(0x1000), vp(0x9000), 0, None) == bt.BL_OK  # nothing to copy
    for dst, src, n in [(0, 0x9000, 64), (0x1000, 0, 64), (0x1008, 0x9000, 64), (0x1000, 0x9000, 24),
                        (0x1000, 0x1010, 64)]:
        assert L.bl_device_copy(vp(dst), vp(src), n, None) != bt.BL_OK, (dst, src, n)
