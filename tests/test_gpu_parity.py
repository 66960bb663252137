"""Parity of the HIP path (through the C-ABI) with the CPU oracle on seeded inputs.

FP64 results must be bit-identical to the oracle: both sides evaluate every cell
update in the same operand order without FMA contraction.  FP32-storage results
are compared with the FP64 oracle at 2e-5 relative (after 100 steps); FP64
reductions that sum (sum, norm1, norm2, the residual norm) at 1e-13 relative,
since the GPU's summation order differs from exactly rounded fsum.
"""
import math

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1604_03570_amd import inputs as I
from tests.gpu_helpers import gpu_global, lib, make_pair, rel_err, say

pytestmark = pytest.mark.gpu

F64_SUM_TOL = 1e-13
F32_TOL = 2e-5


@pytest.fixture(scope="module")
def bt():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return lib()


def _gauss64():
    n = 64
    return I.domain_box(n), I.regular_chop(I.domain_box(n), 32), I.gaussian(n), I.heat_c(n)


# ----------------------------------------------------------------------------- FillBoundary
@pytest.mark.parametrize("case", range(10))
def test_fill_boundary_bit_exact(bt, case):
    rng = np.random.default_rng(300 + case)
    shape = [(8, 6, 4), (12, 10, 8), (16, 8, 12), (9, 7, 5), (24, 16, 8)][case % 5]
    ng = 1 + case % 2
    ncomp = 1 + case % 3
    dtype = bt.F64 if case % 4 else bt.F32
    periodic = tuple(int(v) for v in rng.integers(0, 2, 3))
    dom = I.domain_box(shape)
    boxes = I.random_chop(dom, min_edge=2, max_edge=6, align=1, seed=case)
    if case % 3 == 2 and len(boxes) > 2:
        boxes = boxes[np.sort(rng.permutation(len(boxes))[: len(boxes) * 2 // 3])]
    say(f"fill case={case} shape={shape} ng={ng} ncomp={ncomp} dtype={dtype} periodic={periodic} nbox={len(boxes)}")
    g = rng.random((ncomp,) + shape[::-1])
    if dtype == bt.F32:
        g = I.round_f32(g)
    ba, a, _, o = make_pair(boxes, dom, periodic, ncomp, ng, dtype, g, ghost_value=-7.0)
    a.fill_boundary()
    o.fill_boundary()
    torch.cuda.synchronize()
    for b in range(len(boxes)):
        got = a.fab(b).double().cpu().numpy()
        assert np.array_equal(got, o.fab(b)), f"box {b}"


def test_fill_boundary_partial_components(bt):
    dom = I.domain_box(16)
    boxes = I.regular_chop(dom, 8)
    g = np.random.default_rng(1).random((3, 16, 16, 16))
    ba, a, _, o = make_pair(boxes, dom, (1, 1, 1), 3, 1, bt.F64, g, ghost_value=-7.0)
    a.fill_boundary(scomp=1, ncomp=1)
    o.fill_boundary(scomp=1, ncomp=1)
    torch.cuda.synchronize()
    for b in range(len(boxes)):
        assert np.array_equal(a.fab(b).cpu().numpy(), o.fab(b))


# ----------------------------------------------------------------------------- heat step
@pytest.mark.parametrize("form", ["per_box", "unfused", "fused"])
def test_heat_64cube_8boxes_bit_exact(bt, form):
    dom, boxes, u0, c = _gauss64()
    steps = 20
    say(f"heat 64^3, 8 boxes, form={form}")
    ba, a, b, o = make_pair(boxes, dom, (1, 1, 1), 1, 1, bt.F64, u0)
    if form == "fused":
        res = bt.heat_advance(a, b, steps, c)
    else:
        x, y = a, b
        for _ in range(steps):
            if form == "per_box":
                bt.heat_step(x, y, c)
            else:
                bt.heat_step_unfused(x, y, c)
            x, y = y, x
        res = x
    ref = O.heat_advance(o, steps, c).to_global()
    assert np.array_equal(gpu_global(res), ref)


@pytest.mark.parametrize("dtype_name", ["f64", "f32"])
@pytest.mark.parametrize("layout", ["uneven_periodic", "noncovering_mixed", "odd_extents"])
def test_heat_fused_equals_oracle_and_per_box(bt, dtype_name, layout):
    rng = np.random.default_rng(7)
    if layout == "uneven_periodic":
        dom, periodic = I.domain_box(64), (1, 1, 1)
        boxes = I.random_chop(dom, 8, 32, 8, seed=4)
    elif layout == "noncovering_mixed":
        dom, periodic = I.domain_box((48, 32, 40)), (1, 0, 1)
        boxes = I.random_chop(dom, 8, 24, 8, seed=9)
        boxes = boxes[np.sort(rng.permutation(len(boxes))[: len(boxes) * 3 // 4])]
    else:
        dom, periodic = I.domain_box((37, 23, 18)), (1, 1, 1)
        boxes = I.random_chop(dom, 3, 14, 1, seed=2)
    dtype = bt.F64 if dtype_name == "f64" else bt.F32
    ncomp, steps, c = 3, 12, 0.15
    N = tuple(dom[3 + d] + 1 for d in range(3))
    g = rng.random((ncomp,) + N[::-1]) + 1.0
    if dtype == bt.F32:
        g = I.round_f32(g)
    say(f"heat fused layout={layout} dtype={dtype_name} nbox={len(boxes)}")
    ba, a, b, o = make_pair(boxes, dom, periodic, ncomp, 1, dtype, g, ghost_value=0.5)
    fused = gpu_global(bt.heat_advance(a, b, steps, c))
    # per-box form from the same start
    _, a2, b2, _ = make_pair(boxes, dom, periodic, ncomp, 1, dtype, g, ghost_value=0.5)
    x, y = a2, b2
    for _ in range(steps):
        bt.heat_step(x, y, c)
        x, y = y, x
    per_box = gpu_global(x)
    m = np.isfinite(fused)
    assert np.array_equal(fused[m], per_box[m])
    ref = O.heat_advance(o, steps, c).to_global()
    if dtype == bt.F64:
        assert np.array_equal(fused[m], ref[m])
    else:
        assert rel_err(fused, ref) <= F32_TOL


def test_heat_fp32_storage_error_after_100_steps(bt):
    n = 64
    dom = I.domain_box(n)
    boxes = I.random_chop(dom, 8, 32, 8, seed=1)
    u0 = I.round_f32(I.uniform(n, 2, seed=3))
    c = I.heat_c(n)
    ba, a, b, o = make_pair(boxes, dom, (1, 1, 1), 2, 1, bt.F32, u0)
    got = gpu_global(bt.heat_advance(a, b, 100, c))
    ref = O.heat_advance(o, 100, c).to_global()
    err = rel_err(got, ref)
    say(f"fp32 storage rel err after 100 steps: {err:.3e}")
    assert err <= F32_TOL


def test_heat_single_box_equals_many_boxes_gpu(bt):
    n = 64
    dom = I.domain_box(n)
    u0, _ = I.sine_modes(n, seed=1)
    c = I.heat_c(n)
    outs = []
    for boxes in (I.regular_chop(dom, 64), I.regular_chop(dom, 32), I.random_chop(dom, 8, 32, 8, seed=5)):
        ba = bt.BoxArray.from_boxes(boxes, dom)
        a, b = bt.MultiFab(ba), bt.MultiFab(ba)
        a.from_global(u0)
        outs.append(gpu_global(bt.heat_advance(a, b, 15, c)))
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])


def test_heat_sine_decay_and_conservation_gpu(bt):
    n, steps = 64, 40
    dom = I.domain_box(n)
    u0, modes = I.sine_modes(n, seed=2)
    u0 = u0 + 2.0
    c = I.heat_c(n)
    ba = bt.BoxArray.chop(dom, 32)
    a, b = bt.MultiFab(ba), bt.MultiFab(ba)
    a.from_global(u0)
    s0 = a.sum()
    res = bt.heat_advance(a, b, steps, c)
    got = gpu_global(res)
    exact = np.full_like(u0, 2.0)
    for md in modes:
        gm = 1.0 - 4.0 * c * sum(math.sin(math.pi * kd / n) ** 2 for kd in md.k)
        exact[0] += md.amp * gm ** steps * I.sine_product(n, md.k)
    assert np.abs(got - exact).max() / np.abs(exact - 2.0).max() <= 1e-12
    assert abs(res.sum() - s0) <= 1e-13 * abs(s0)


def test_heat_advance_graph_replay(bt):
    dom, boxes, u0, c = _gauss64()
    ba, a, b, o = make_pair(boxes, dom, (1, 1, 1), 1, 1, bt.F64, u0)
    for _ in range(5):  # the captured 2-step graph is replayed five times
        r = bt.heat_advance(a, b, 2, c)
        assert r is a
    r = bt.heat_advance(a, b, 3, c)  # a second graph, odd length
    ref = O.heat_advance(o, 13, c).to_global()
    assert np.array_equal(gpu_global(r), ref)


# ----------------------------------------------------------------------------- reductions
@pytest.mark.parametrize("dtype_name", ["f64", "f32"])
def test_reductions_match_oracle(bt, dtype_name):
    dom = I.domain_box((40, 24, 32))
    boxes = I.random_chop(dom, 8, 16, 8, seed=3)
    g = np.random.default_rng(4).standard_normal((2, 32, 24, 40)) * 3.0
    dtype = bt.F64 if dtype_name == "f64" else bt.F32
    if dtype == bt.F32:
        g = I.round_f32(g)
    ba, a, _, o = make_pair(boxes, dom, (1, 1, 1), 2, 1, dtype, g)
    for comp in range(2):
        for op in ("sum", "max", "min", "norm0", "norm1", "norm2"):
            got, ref = a.reduce(comp, op), O.reduce(o, comp, op)
            if op in ("max", "min", "norm0"):
                assert got == ref, (comp, op)
            elif op == "sum":  # cancellation: bound by the sum of magnitudes
                assert abs(got - ref) <= F64_SUM_TOL * O.reduce(o, comp, "norm1"), (comp, op)
            else:
                assert abs(got - ref) <= F64_SUM_TOL * abs(ref), (comp, op)
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    a.reduce_async(1, "max", out)
    torch.cuda.synchronize()
    assert out.item() == O.reduce(o, 1, "max")


# ----------------------------------------------------------------------------- Gauss-Seidel
def _gsrb_problem(n, boxes_edge, dtype, seed=5):
    dom = I.domain_box(n)
    boxes = I.regular_chop(dom, boxes_edge)
    f = I.zero_mean_normal_f32(n, seed=seed)
    bt = lib()
    ba = bt.BoxArray.from_boxes(boxes, dom)
    phi, fm = bt.MultiFab(ba, 1, 1, dtype), bt.MultiFab(ba, 1, 1, dtype)
    phi.set_val(0.0, with_ghosts=True)
    fm.set_val(0.0, with_ghosts=True)
    fm.from_global(f)
    ophi, ofm = O.OracleMultiFab(boxes, dom, (1, 1, 1), 1, 1), O.OracleMultiFab(boxes, dom, (1, 1, 1), 1, 1)
    ofm.load_global(f)
    return phi, fm, ophi, ofm


@pytest.mark.parametrize("one_pass", [0, 1])
def test_gsrb_fp64_bit_exact_with_norms(bt, one_pass):
    n, sweeps = 32, 6
    h2 = (1.0 / n) ** 2
    phi, fm, ophi, ofm = _gsrb_problem(n, 16, bt.F64)
    bt.set_gsrb_config(one_pass, 0, 0)
    try:
        assert bt.gsrb_one_pass_applies(phi) == bool(one_pass)
        norms = bt.gsrb_sweeps(phi, fm, h2, sweeps)
    finally:
        bt.set_gsrb_config(1, 0, 0)
    onorms = O.gsrb_sweeps(ophi, ofm, h2, sweeps)
    assert np.array_equal(gpu_global(phi), ophi.to_global())
    for g, r in zip(norms, onorms):
        assert abs(g - r) <= F64_SUM_TOL * r
    assert abs(bt.residual_norm(phi, fm, h2) - onorms[-1]) <= F64_SUM_TOL * onorms[-1]


@pytest.mark.parametrize("one_pass", [0, 1])
def test_gsrb_fp32_state_against_fp64_oracle(bt, one_pass):
    n, sweeps = 64, 20
    h2 = (1.0 / n) ** 2
    phi, fm, ophi, ofm = _gsrb_problem(n, 32, bt.F32)
    bt.set_gsrb_config(one_pass, 0, 0)
    try:
        norms = bt.gsrb_sweeps(phi, fm, h2, sweeps)
    finally:
        bt.set_gsrb_config(1, 0, 0)
    onorms = O.gsrb_sweeps(ophi, ofm, h2, sweeps)
    err = rel_err(gpu_global(phi), ophi.to_global())
    nerr = max(abs(g - r) / r for g, r in zip(norms, onorms))
    say(f"gsrb fp32: phi rel err {err:.3e}, norm rel err {nerr:.3e}")
    assert err <= 1e-5 and nerr <= 1e-5
    assert all(b2 < a2 for a2, b2 in zip(norms, norms[1:]))


def test_gsrb_rejects_odd_periodic_extent(bt):
    dom = I.domain_box((10, 9, 8))
    ba = bt.BoxArray.chop(dom, 8)
    phi, f = bt.MultiFab(ba), bt.MultiFab(ba)
    with pytest.raises(bt.BoxtileError) as e:
        bt.gsrb_sweeps(phi, f, 1.0, 1)
    assert e.value.code == bt.BL_EINVAL


# ----------------------------------------------------------------------------- argument errors
def test_shape_and_dtype_errors(bt):
    dom = I.domain_box(16)
    ba1, ba2 = bt.BoxArray.chop(dom, 8), bt.BoxArray.chop(dom, 16)
    a = bt.MultiFab(ba1)
    with pytest.raises(bt.BoxtileError) as e:
        bt.heat_step(a, bt.MultiFab(ba2), 0.1)
    assert e.value.code == bt.BL_ESHAPE
    with pytest.raises(bt.BoxtileError) as e:
        bt.heat_step(a, bt.MultiFab(ba1, dtype=bt.F32), 0.1)
    assert e.value.code == bt.BL_EDTYPE
    with pytest.raises(bt.BoxtileError) as e:
        bt.heat_step(bt.MultiFab(ba1, nghost=0), bt.MultiFab(ba1, nghost=0), 0.1)
    assert e.value.code == bt.BL_EINVAL
    small = torch.empty(1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(bt.BoxtileError) as e:
        bt.MultiFab(ba1, buffer=small)
    assert e.value.code == bt.BL_ENOMEM
    with pytest.raises(bt.BoxtileError) as e:
        bt.MultiFab(bt.BoxArray.chop(I.domain_box(2), 2), nghost=3)
    assert e.value.code == bt.BL_EINVAL


# ----------------------------------------------------------------------------- batching
def test_batch_alone_equals_in_the_mix(bt):
    rng = np.random.default_rng(11)
    specs = [(32, 16, bt.F64, 9), (48, 32, bt.F32, 14), (64, 32, bt.F64, 5), (32, 32, bt.F32, 11),
             (40, 16, bt.F64, 7)]
    join_at = [0, 0, 2, 3, 3]
    alone, probs = [], []
    for (n, be, dt, steps), j in zip(specs, join_at):
        dom = I.domain_box(n)
        ba = bt.BoxArray.chop(dom, be)
        center = tuple(rng.uniform(0.25, 0.75, 3))
        g = I.gaussian(n, center)
        if dt == bt.F32:
            g = I.round_f32(g)
        c = I.heat_c(n)
        a, b = bt.MultiFab(ba, 1, 1, dt), bt.MultiFab(ba, 1, 1, dt)
        a.from_global(g)
        alone.append(gpu_global(bt.heat_advance(a, b, steps, c)))
        a2, b2 = bt.MultiFab(ba, 1, 1, dt), bt.MultiFab(ba, 1, 1, dt)
        a2.from_global(g)
        probs.append(dict(a=a2, b=b2, c=c, steps=steps, join=j, id=None, done=False))
    batch = bt.Batch()
    tick = 0
    results = [None] * len(probs)
    while not all(p["done"] for p in probs):
        for p in probs:
            if p["id"] is None and p["join"] <= tick:
                p["id"] = batch.add(p["a"], p["b"], p["c"])
        batch.step()
        tick += 1
        for i, p in enumerate(probs):
            if p["id"] is not None and not p["done"] and batch.steps_done(p["id"]) == p["steps"]:
                results[i] = gpu_global(batch.current(p["id"]))
                batch.remove(p["id"])
                p["done"] = True
    for i in range(len(probs)):
        assert np.array_equal(results[i], alone[i]), i


# ----------------------------------------------------------------------------- tile configurations
TILE_CONFIGS = [(1, 4, 0, 0), (2, 2, 0, 0), (3, 4, 0, 0), (8, 1, 0, 0), (1024, 4, 0, 0), (5, 3, 0, 0), (4, 4, 2, 0),
                (1024, 2, 3, 0), (8, 4, 1, 0), (16, 1, 0, 0), (2, 4, 0, 1), (4, 4, 0, 1), (8, 2, 0, 1), (8, 4, 2, 1),
                (2, 4, 0, 2), (4, 4, 0, 2), (8, 3, 0, 2), (4, 4, 2, 2), (4, 1, 0, 2),
                (2, 4, 0, 3), (4, 4, 0, 3), (8, 3, 0, 3), (4, 4, 2, 3), (4, 1, 0, 3), (8, 2, 0, 3),
                # z steps of form 3: a workgroup carries two planes from one step into the next
                (4, 4, 0, 3, 1), (2, 4, 0, 3, 1), (4, 4, 0, 3, 4), (2, 4, 0, 3, 8), (8, 3, 0, 3, 2), (4, 4, 2, 3, 4),
                (4, 1, 0, 3, 3)]


@pytest.mark.parametrize("cfg", TILE_CONFIGS)
@pytest.mark.parametrize("layout", ["uneven", "odd_noncovering"])
def test_every_tile_configuration_bit_exact(bt, cfg, layout):
    """Every stencil kernel variant (z march, block forms of 2/4/8 planes with
    registers, LDS neighbours or LDS halos, z steps with carried planes, persistent
    grid) gives the oracle's FP64 result, fused and per box, on ragged tiles."""
    rng = np.random.default_rng(31)
    if layout == "uneven":
        dom, periodic = I.domain_box((64, 48, 40)), (1, 1, 1)
        boxes = I.random_chop(dom, 8, 32, 8, seed=6)
    else:
        dom, periodic = I.domain_box((35, 22, 27)), (0, 1, 1)
        boxes = I.random_chop(dom, 3, 13, 1, seed=8)
        boxes = boxes[np.sort(rng.permutation(len(boxes))[: len(boxes) * 4 // 5])]
    N = tuple(dom[3 + d] + 1 for d in range(3))
    ncomp, steps, c = 2, 5, 0.15
    g = rng.random((ncomp,) + N[::-1]) + 1.0
    saved = bt.get_tile_config()
    bt.set_tile_config(*cfg)
    try:
        say(f"tile cfg {cfg} layout={layout}")
        _, a, b, o = make_pair(boxes, dom, periodic, ncomp, 1, bt.F64, g, ghost_value=0.25)
        fused = gpu_global(bt.heat_advance(a, b, steps, c))
        _, a2, b2, _ = make_pair(boxes, dom, periodic, ncomp, 1, bt.F64, g, ghost_value=0.25)
        x, y = a2, b2
        for s in range(steps):
            if s % 2:
                bt.heat_step(x, y, c)
            else:
                bt.heat_step_unfused(x, y, c)
            x, y = y, x
        other = gpu_global(x)
    finally:
        bt.set_tile_config(*saved)
    ref = O.heat_advance(o, steps, c).to_global()
    m = np.isfinite(ref)
    assert np.array_equal(fused[m], ref[m])
    assert np.array_equal(other[m], ref[m])


# ----------------------------------------------------------------------------- autotuner
def test_autotune_picks_the_fastest_and_stays_bit_exact(bt):
    """The autotuner times every candidate shape, keeps the fastest, and the tuned
    MultiFabs (and ones created afterwards) still give the oracle's FP64 result."""
    dom = I.domain_box((64, 48, 40))
    boxes = I.random_chop(dom, 8, 32, 8, seed=21)
    g = np.random.default_rng(5).random((2, 40, 48, 64)) + 1.0
    c = 0.15
    saved = bt.get_tile_config()
    try:
        ba = bt.BoxArray.from_boxes(boxes, dom)
        s0, s1 = bt.MultiFab(ba, 2, 1, bt.F64), bt.MultiFab(ba, 2, 1, bt.F64)
        s0.set_val(1.0)
        s1.set_val(1.0)
        best, table = bt.autotune(ba, s0, s1, c, trial_steps=2)
        say(f"autotune best {best}, {len(table)} candidates")
        assert len(table) == 45  # form 3: 3 zchunk x 3 waves x 4 zsteps; form 2: 3 x 3
        assert best == min(table, key=lambda t: t[1])[0]
        assert all(ms > 0 for _, ms in table)
        # the scratch pair, and a fresh pair of the same shape, now run the tuned shape
        for a, b in ((s0, s1), (bt.MultiFab(ba, 2, 1, bt.F64), bt.MultiFab(ba, 2, 1, bt.F64))):
            _, _, _, o = make_pair(boxes, dom, (1, 1, 1), 2, 1, bt.F64, g)
            a.from_global(g)
            got = gpu_global(bt.heat_advance(a, b, 5, c))
            ref = O.heat_advance(o, 5, c).to_global()
            assert np.array_equal(got, ref)
    finally:
        bt.set_tile_config(*saved)


# ----------------------------------------------------------------------------- fused GSRB
GSRB_CONFIGS = [(4, 4, 0, 3), (2, 4, 0, 3), (8, 2, 0, 3), (4, 3, 0, 3), (4, 4, 2, 3), (4, 4, 0, 2),
                (4, 4, 0, 3, 1), (4, 4, 0, 3, 4), (2, 4, 0, 3, 8), (8, 2, 0, 3, 2), (4, 4, 2, 3, 3)]


@pytest.mark.parametrize("cfg", GSRB_CONFIGS)
@pytest.mark.parametrize("layout", ["uneven", "odd_noncovering"])
def test_gsrb_every_form_bit_exact_on_uneven_layouts(bt, cfg, layout):
    """GSRB sweeps in the two-pass form (fused colour passes with face records, or
    fill + colour passes) give the oracle's FP64 field bit for bit and its norms to
    1e-13, on uneven and on non-covering, partly non-periodic layouts, under every
    tile configuration."""
    rng = np.random.default_rng(41)
    if layout == "uneven":
        dom, periodic = I.domain_box((48, 40, 32)), (1, 1, 1)
        boxes = I.random_chop(dom, 8, 24, 8, seed=3)
    else:
        dom, periodic = I.domain_box((30, 21, 26)), (0, 0, 1)
        boxes = I.random_chop(dom, 3, 12, 1, seed=9)
        boxes = boxes[np.sort(rng.permutation(len(boxes))[: len(boxes) * 4 // 5])]
    N = tuple(dom[3 + d] + 1 for d in range(3))
    f = rng.standard_normal((1,) + N[::-1])
    g0 = 0.1 * rng.random((1,) + N[::-1])
    h2, sweeps = 1.0 / 1024.0, 4
    saved = bt.get_tile_config()
    bt.set_tile_config(*cfg)
    bt.set_gsrb_config(0, 0, 0)
    try:
        say(f"gsrb cfg {cfg} layout={layout}")
        _, phi, fm, ophi = make_pair(boxes, dom, periodic, 1, 1, bt.F64, g0, ghost_value=0.25)
        fm.set_val(0.0, with_ghosts=True)
        fm.from_global(f)
        norms = bt.gsrb_sweeps(phi, fm, h2, sweeps)
        res = bt.residual_norm(phi, fm, h2)
        got = gpu_global(phi)
    finally:
        bt.set_tile_config(*saved)
        bt.set_gsrb_config(1, 0, 0)
    ofm = O.OracleMultiFab(boxes, dom, periodic, 1, 1)
    ofm.load_global(f)
    onorms = O.gsrb_sweeps(ophi, ofm, h2, sweeps)
    ref = ophi.to_global()
    m = np.isfinite(ref)
    assert np.array_equal(got[m], ref[m])
    for a, b in zip(norms, onorms):
        assert abs(a - b) <= F64_SUM_TOL * b
    assert abs(res - onorms[-1]) <= F64_SUM_TOL * onorms[-1]


# ----------------------------------------------------------------------------- degenerate calls
def test_degenerate_calls(bt):
    """Zero steps and sweeps are no-ops; empty batches step; bad ids, components and
    trial counts are rejected with EINVAL."""
    dom = I.domain_box(32)
    ba = bt.BoxArray.chop(dom, 16)
    a, b = bt.MultiFab(ba, 2, 1, bt.F64), bt.MultiFab(ba, 2, 1, bt.F64)
    g = np.random.default_rng(3).random((2, 32, 32, 32))
    a.from_global(g)
    assert bt.heat_advance(a, b, 0, 0.15) is a
    assert np.array_equal(gpu_global(a), g)
    phi, f = bt.MultiFab(ba, 1, 1, bt.F64), bt.MultiFab(ba, 1, 1, bt.F64)
    phi.from_global(g[:1])
    f.set_val(0.0, with_ghosts=True)
    assert bt.gsrb_sweeps(phi, f, 1e-3, 0) == []
    assert np.array_equal(gpu_global(phi), g[:1])
    batch = bt.Batch()
    batch.step()  # no members
    batch.steps(0)
    batch.steps(3)
    for call in (lambda: batch.remove(12345), lambda: a.reduce(2, "sum"), lambda: a.reduce(-1, "max"),
                 lambda: batch.steps(-1),
                 lambda: bt.autotune(ba, a, b, 0.15, trial_steps=0), lambda: bt.heat_advance(a, b, -1, 0.15)):
        with pytest.raises(bt.BoxtileError) as e:
            call()
        assert e.value.code == bt.BL_EINVAL
    torch.cuda.synchronize()


@pytest.mark.parametrize("nbytes", [16, 4096 + 16, 64 << 20])
def test_device_copy(bt, nbytes):
    src = torch.randint(0, 255, (nbytes,), dtype=torch.uint8, device="cuda")
    dst = torch.zeros_like(src)
    bt.device_copy(dst, src)
    torch.cuda.synchronize()
    assert torch.equal(dst, src)
