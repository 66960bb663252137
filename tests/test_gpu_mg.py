"""Parity of the multigrid path (restriction, prolongation, V-cycles; HIP kernels through
the C-ABI) with the oracle.

FP64 fields are bit-identical to the oracle's: the smoother is the GSRB pass already held
bit for bit, the restriction evaluates the oracle's residual expression and sums the
children in the oracle's order, the prolongation is one addition.  Residual norms are
held to 1e-13 (summation order).  FP32 storage: transfers within one FP32 rounding of the
oracle on the same inputs, V-cycles within 1e-5 of the FP64 run.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1604_03570_amd import inputs as I
from tests.gpu_helpers import gpu_global, lib, rel_err, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bt():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return lib()


def _layout(name):
    if name == "uneven64":
        dom, periodic = I.domain_box(64), (1, 1, 1)
        boxes = I.random_chop(dom, 8, 32, 8, seed=4)
    elif name == "cells32":  # down to 64 boxes of one cell
        dom, periodic = I.domain_box(32), (1, 1, 1)
        boxes = I.regular_chop(dom, 8)
    elif name == "holes_mixed":  # boxes leave holes; y is not periodic
        dom, periodic = I.domain_box((48, 32, 40)), (1, 0, 1)
        boxes = I.random_chop(dom, 8, 24, 8, seed=9)
        rng = np.random.default_rng(1)
        boxes = boxes[np.sort(rng.permutation(len(boxes))[: len(boxes) * 3 // 4])]
    else:  # tiny: boxes of 2 cells, coarse boxes of one
        dom, periodic = I.domain_box(8), (1, 1, 1)
        boxes = I.regular_chop(dom, 2)
    return dom, periodic, boxes


def _pair(bt, ba, boxes, dom, periodic, dtype, g, ghost=0.0):
    m = bt.MultiFab(ba, 1, 1, dtype)
    m.set_val(ghost, with_ghosts=True)
    m.from_global(g)
    o = O.OracleMultiFab(boxes, dom, periodic, 1, 1)
    o.data[...] = ghost
    o.load_global(np.asarray(g, dtype=np.float64))
    return m, o


@pytest.mark.parametrize("dtype_name", ["f64", "f32"])
@pytest.mark.parametrize("layout", ["uneven64", "cells32", "holes_mixed", "tiny"])
def test_transfers_equal_the_oracle(bt, layout, dtype_name):
    dtype = bt.F64 if dtype_name == "f64" else bt.F32
    dom, periodic, boxes = _layout(layout)
    say(f"mg transfers layout={layout} dtype={dtype_name}")
    N = tuple(int(dom[3 + d] + 1) for d in range(3))
    rng = np.random.default_rng(17)
    g_phi, g_f = rng.random((1,) + N[::-1]), rng.random((1,) + N[::-1]) - 0.5
    if dtype == bt.F32:
        g_phi, g_f = I.round_f32(g_phi), I.round_f32(g_f)
    h2 = (1.0 / max(N)) ** 2
    ba = bt.BoxArray.from_boxes(boxes, dom, periodic)
    cba = ba.coarsen(2)
    phi, ophi = _pair(bt, ba, boxes, dom, periodic, dtype, g_phi, ghost=0.25)
    f, of = _pair(bt, ba, boxes, dom, periodic, dtype, g_f)
    fc = bt.MultiFab(cba, 1, 1, dtype)
    cdom = O.coarsen_boxes(dom)[0]
    ofc = O.OracleMultiFab(O.coarsen_boxes(boxes), cdom, periodic, 1, 1)
    bt.restrict_residual(phi, f, h2, fc)
    O.restrict_residual(ophi, of, h2, ofc)
    got, ref = gpu_global(fc), ofc.to_global()
    if dtype == bt.F64:
        assert np.array_equal(got, ref, equal_nan=True)
    else:
        m = np.isfinite(ref)
        assert np.all(np.abs(got[m] - ref[m]) <= 6e-8 * np.abs(ref[m]) + 1e-30)
    # prolongation of a random coarse field
    CN = tuple(int(cdom[3 + d] + 1) for d in range(3))
    g_c = rng.random((1,) + CN[::-1])
    if dtype == bt.F32:
        g_c = I.round_f32(g_c)
    fc.from_global(g_c)
    ofc.load_global(g_c)
    bt.prolong_add(phi, fc)
    O.prolong_add(ophi, ofc)
    got, ref = gpu_global(phi), ophi.to_global()
    if dtype == bt.F64:
        assert np.array_equal(got, ref, equal_nan=True)
    else:
        m = np.isfinite(ref)
        assert np.all(np.abs(got[m] - ref[m]) <= 6e-8 * np.abs(ref[m]))


def _problem(bt, layout, dtype, seed=0):
    dom, periodic, boxes = _layout(layout)
    N = tuple(int(dom[3 + d] + 1) for d in range(3))
    f = I.zero_mean_normal_f32(N, seed=seed)
    h2 = (1.0 / max(N)) ** 2
    ba = bt.BoxArray.from_boxes(boxes, dom, periodic)
    phi, ophi = _pair(bt, ba, boxes, dom, periodic, dtype, np.zeros_like(f))
    fm, ofm = _pair(bt, ba, boxes, dom, periodic, dtype, f)
    return dict(ba=ba, phi=phi, ophi=ophi, f=fm, of=ofm, h2=h2)


@pytest.mark.parametrize("layout", ["uneven64", "cells32", "holes_mixed"])
def test_vcycles_bit_exact_f64(bt, layout):
    P = _problem(bt, layout, bt.F64)
    mg = bt.Multigrid(P["ba"], bt.F64)
    say(f"mg vcycles layout={layout} levels={mg.nlevels}")
    norms = mg.vcycles(P["phi"], P["f"], P["h2"], 2, 2, 2, 8)
    onorms = O.mg_vcycles(P["ophi"], P["of"], P["h2"], 2, 2, 2, 8)
    assert mg.nlevels == len(O.mg_level_boxes(P["ophi"].boxes, P["ophi"].domain, P["ophi"].periodic, 32))
    assert np.array_equal(gpu_global(P["phi"]), P["ophi"].to_global(), equal_nan=True)
    for a, b in zip(norms, onorms):
        assert abs(a - b) <= 1e-13 * b
    assert norms[1] < 0.3 * norms[0]


@pytest.mark.parametrize("shape", [(4, 4, 0, 3), (2, 2, 0, 3), (4, 4, 0, 2), (4, 4, 0, 0), (4, 4, 0, 3, 4)],
                         ids=["z4_w4_b3", "z2_w2_b3", "z4_w4_b2", "march", "z4_w4_b3_s4"])
def test_vcycles_every_tile_shape(bt, shape):
    """The fused smoother (form 3) and the fill-then-pass smoother give the same bits."""
    bt.set_tile_config(*shape)
    try:
        P = _problem(bt, "uneven64", bt.F64, seed=3)
        mg = bt.Multigrid(P["ba"], bt.F64, max_levels=3)
        mg.vcycles(P["phi"], P["f"], P["h2"], 1, 2, 1, 6, with_norms=False)
        O.mg_vcycles(P["ophi"], P["of"], P["h2"], 1, 2, 1, 6, max_levels=3)
        assert np.array_equal(gpu_global(P["phi"]), P["ophi"].to_global())
    finally:
        bt.set_tile_config(4, 4, 0, 3)


def test_vcycles_f32_follow_the_oracle(bt):
    """FP32 storage: 5 V-cycles against the oracle's 5 (FP64) on the same f: the field
    within 1e-5; every norm within 1e-5 of the oracle's plus the FP32 floor (a norm from
    FP32 state differs from the exact one by at most the norm of the residual of the
    FP32 rounding error, which the cycles converge to; the last FP32 norm bounds it);
    the FP32 residual still falls 3x per cycle at first."""
    P32 = _problem(bt, "uneven64", bt.F32)
    n32 = bt.Multigrid(P32["ba"], bt.F32).vcycles(P32["phi"], P32["f"], P32["h2"], 5)
    on = O.mg_vcycles(P32["ophi"], P32["of"], P32["h2"], 5)
    err = rel_err(gpu_global(P32["phi"]), P32["ophi"].to_global())
    say(f"mg f32 vs oracle: field rel err {err:.2e}, norms {n32} vs {on}")
    assert err <= 1e-5
    assert all(abs(a - b) <= 1e-5 * b + n32[-1] for a, b in zip(n32, on)), (n32, on)
    assert abs(n32[0] - on[0]) <= 1e-5 * on[0]
    assert all(b < 0.3 * a for a, b in zip(n32[:3], n32[1:4]))


def test_single_level_is_the_smoother(bt):
    """max_levels = 1: a V-cycle is nu_bottom GSRB sweeps."""
    P = _problem(bt, "uneven64", bt.F64, seed=2)
    Q = _problem(bt, "uneven64", bt.F64, seed=2)
    mg = bt.Multigrid(P["ba"], bt.F64, max_levels=1)
    assert mg.nlevels == 1
    mg.vcycles(P["phi"], P["f"], P["h2"], 1, 2, 2, 5, with_norms=False)
    bt.gsrb_sweeps(Q["phi"], Q["f"], Q["h2"], 5, with_norms=False)
    assert np.array_equal(gpu_global(P["phi"]), gpu_global(Q["phi"]))


def test_mg_degenerate_calls(bt):
    P = _problem(bt, "cells32", bt.F64)
    mg = bt.Multigrid(P["ba"], bt.F64)
    assert mg.vcycles(P["phi"], P["f"], P["h2"], 0) == []
    other = bt.BoxArray.chop(I.domain_box(32), 16)
    with pytest.raises(bt.BoxtileError):  # phi on another BoxArray
        mg.vcycles(bt.MultiFab(other, 1, 1, bt.F64), bt.MultiFab(other, 1, 1, bt.F64), P["h2"], 1)
    with pytest.raises(bt.BoxtileError):  # dtype differs from the hierarchy's
        mg.vcycles(bt.MultiFab(P["ba"], 1, 1, bt.F32), bt.MultiFab(P["ba"], 1, 1, bt.F32), P["h2"], 1)
    with pytest.raises(bt.BoxtileError):  # two ghost layers
        mg.vcycles(bt.MultiFab(P["ba"], 1, 2, bt.F64), bt.MultiFab(P["ba"], 1, 2, bt.F64), P["h2"], 1)
    with pytest.raises(bt.BoxtileError):  # negative counts
        mg.vcycles(P["phi"], P["f"], P["h2"], 1, -1, 2, 2)
    with pytest.raises(bt.BoxtileError):  # fc not on the coarsened boxes
        bt.restrict_residual(P["phi"], P["f"], P["h2"], bt.MultiFab(P["ba"], 1, 1, bt.F64))
    with pytest.raises(bt.BoxtileError):  # fine boxes of odd extent
        dom = I.domain_box(6)
        odd = bt.BoxArray.from_boxes(I.regular_chop(dom, 3), dom)
        bt.prolong_add(bt.MultiFab(odd, 1, 1, bt.F64), bt.MultiFab(bt.BoxArray.chop(I.domain_box(3), 3), 1, 1, bt.F64))


@pytest.mark.parametrize("periodic", [(1, 1, 1), (1, 1, 0)], ids=["periodic", "z_walls"])
def test_vcycles_with_one_pass_smoothing(bt, periodic):
    """A finest level of 4M cells (128 x 128 x 256, 32 boxes of 64^3), which the V-cycle
    smooths with the one-pass sweep where the sweep count is even: two V(2,2) cycles, a
    V(1,3) cycle (odd counts: the two colour passes there) and a V(2,2) cycle again give
    the oracle's FP64 bits and norms; so does the two-pass form.  Between one-pass calls
    the cycle skips the FillBoundary of the face ghosts the last sweep pushed; with z not
    periodic the ghost planes beyond the z walls, which no box covers, keep their value
    throughout."""
    dom = I.domain_box((128, 128, 256))
    boxes = I.regular_chop(dom, 64)
    N = (128, 128, 256)
    f = I.zero_mean_normal_f32(N, seed=3)
    h2 = (1.0 / 256) ** 2
    for one_pass in (1, 0):
        say(f"mg one-pass smoothing on 4M cells, periodic={periodic}, one_pass={one_pass}")
        ba = bt.BoxArray.from_boxes(boxes, dom, periodic)
        phi, ophi = _pair(bt, ba, boxes, dom, periodic, bt.F64, np.zeros_like(f))
        fm, ofm = _pair(bt, ba, boxes, dom, periodic, bt.F64, f)
        assert bt.gsrb_one_pass_applies(phi)
        mg = bt.Multigrid(ba, bt.F64)
        bt.set_gsrb_config(one_pass, 0, 0)
        try:
            for cycles, nu1, nu2 in ((2, 2, 2), (1, 1, 3), (1, 2, 2)):
                norms = mg.vcycles(phi, fm, h2, cycles, nu1, nu2, 8)
                onorms = O.mg_vcycles(ophi, ofm, h2, cycles, nu1, nu2, 8)
                assert np.array_equal(gpu_global(phi), ophi.to_global()), (one_pass, cycles, nu1, nu2)
                for a, b in zip(norms, onorms):
                    assert abs(a - b) <= 1e-13 * b
            if not periodic[2]:  # the ghost plane below the lowest boxes: no box covers it
                for k in np.nonzero(boxes[:, 2] == 0)[0][:2]:
                    fab = phi.fab(int(k)).double().cpu().numpy()  # (comp, z, y, x) of the grown box
                    assert np.all(fab[0, 0, 1:-1, 1:-1] == 0.0)
        finally:
            bt.set_gsrb_config(1, 0, 0)
        del mg, phi, fm


def test_repeated_vcycle_calls_on_one_hierarchy(bt):
    """Several calls on one hierarchy, with other sweep counts and another h2, continue
    from the state left by the last one and give the oracle's bits."""
    P = _problem(bt, "uneven64", bt.F64, seed=9)
    mg = bt.Multigrid(P["ba"], bt.F64)
    h2 = P["h2"]
    plan = [(1, 2, 2, 8, h2), (2, 2, 2, 8, h2), (1, 1, 3, 5, h2), (1, 2, 2, 8, 2.0 * h2)]
    for cycles, nu1, nu2, nub, hh in plan:
        mg.vcycles(P["phi"], P["f"], hh, cycles, nu1, nu2, nub, with_norms=(cycles == 2))
        O.mg_vcycles(P["ophi"], P["of"], hh, cycles, nu1, nu2, nub)
        assert np.array_equal(gpu_global(P["phi"]), P["ophi"].to_global()), (cycles, nu1, nu2, nub)


@pytest.mark.parametrize("dtype_name", ["f64", "f32"])
@pytest.mark.parametrize("layout,expect", [("uneven64", "coarse"), ("cells32", "coarse"), ("tiny", 0),
                                           ("holes_mixed", -1)])
def test_fused_bottom_equals_the_oracle(bt, layout, dtype_name, expect):
    """Where every level from some level down covers a fully periodic domain and fits one
    workgroup's LDS, that bottom of the cycle runs as one launch (dense periodic arrays in
    LDS); from level 0 itself on the tiny grid.  FP64: the oracle's bits and norms to
    1e-13 over 3 cycles with other sweep counts too; FP32: within 1e-5.  Layouts with holes
    or a non-periodic axis keep the level-by-level passes."""
    dtype = bt.F64 if dtype_name == "f64" else bt.F32
    P = _problem(bt, layout, dtype, seed=5)
    mg = bt.Multigrid(P["ba"], dtype)
    say(f"fused bottom layout={layout} {dtype_name}: levels {mg.nlevels}, bottom {mg.bottom_level}")
    if expect == "coarse":
        assert 0 < mg.bottom_level < mg.nlevels
    else:
        assert mg.bottom_level == expect
    for ncyc, nu1, nu2, nub in ((2, 2, 2, 8), (1, 1, 3, 5)):
        n = mg.vcycles(P["phi"], P["f"], P["h2"], ncyc, nu1, nu2, nub)
        on = O.mg_vcycles(P["ophi"], P["of"], P["h2"], ncyc, nu1, nu2, nub)
        got, ref = gpu_global(P["phi"]), P["ophi"].to_global()
        if dtype == bt.F64:
            assert np.array_equal(got, ref, equal_nan=True)
            assert all(abs(a - b) <= 1e-13 * b for a, b in zip(n, on))
        else:
            assert rel_err(got, ref) <= 1e-5
