"""The workloads at their full sizes, in the launch configurations the benchmark uses.

The 7-point heat step (per box at 256^3, fused and batched on the 512^3 uneven
level), the GSRB sweeps at 384^3 and V-cycles at 256^3 are compared with whole
oracle runs, field by field.  The variable-coefficient and 8th-order steps at
512^3 are checked on sampled cells through the oracle's dependence-cone
windows, beside the closed form of discrete sine modes and conservation.
"""
import math

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1604_03570_amd import inputs as I
from tests.gpu_helpers import lib, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bt():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return lib()


def _cell(mf, boxes, comp, cell):
    """Value of global cell (i, j, k), component comp, read from the FAB that holds it."""
    i, j, k = cell
    for b, bx in enumerate(boxes):
        if bx[0] <= i <= bx[3] and bx[1] <= j <= bx[4] and bx[2] <= k <= bx[5]:
            g, _, _ = mf.layout(b)
            fab = mf.fab(b)
            return float(fab[comp, k - g[2], j - g[1], i - g[0]])
    raise AssertionError(f"no box holds {cell}")


def test_256cube_per_box_launches_follow_the_sine_closed_form(bt):
    """256^3 periodic, 64 boxes of 64^3, FP64, 3 seeded sine modes, 100 steps of the
    plain per-box form (FillBoundary, then one launch per box)."""
    n, steps = 256, 100
    dom = I.domain_box(n)
    ba = bt.BoxArray.chop(dom, 64)
    u0, modes = I.sine_modes(n, seed=1)
    c = I.heat_c(n)
    a, b = bt.MultiFab(ba, 1, 1, bt.F64), bt.MultiFab(ba, 1, 1, bt.F64)
    a.from_global(u0)
    x, y = a, b
    for _ in range(steps):
        bt.heat_step(x, y, c, fill_first=True)
        x, y = y, x
    got = x.to_global()[0].cpu().numpy()
    exact = np.zeros_like(got)
    for md in modes:
        g = 1.0 - 4.0 * c * sum(math.sin(math.pi * kd / n) ** 2 for kd in md.k)
        exact += md.amp * g ** steps * I.sine_product(n, md.k)
    err = np.abs(got - exact).max() / np.abs(exact).max()
    say(f"256^3 per box: closed-form rel err {err:.3e}")
    assert err <= 1e-12
    o = O.OracleMultiFab(ba.boxes(), dom, (1, 1, 1), 1, 1)
    o.load_global(u0)
    ref = O.heat_advance(o, steps, c).to_global()[0]
    assert np.array_equal(got, ref), "per-box field differs from the oracle's"
    say("256^3 per box: whole field equals the oracle's bit for bit")


CFG2_N, CFG2_NCOMP, CFG2_STEPS = 512, 5, 50


@pytest.fixture(scope="module")
def cfg2_oracle():
    """The 512^3 uneven level (seeded chop, 5 comps, U(0,1) data): the oracle's state
    after 50 steps, every component, in global (comp, z, y, x) order (FP64); and the
    same from the data rounded to FP32."""
    n, ncomp, steps = CFG2_N, CFG2_NCOMP, CFG2_STEPS
    dom = I.domain_box(n)
    boxes = I.random_chop(dom, 16, 128, 8, seed=0)
    c = I.heat_c(n)
    u0 = I.uniform(n, ncomp, seed=0)
    out = {"boxes": boxes, "dom": dom, "c": c, "u0": u0}
    o = O.OracleMultiFab(boxes, dom, (1, 1, 1), ncomp, 1)
    o.load_global(u0)
    say(f"512^3 uneven: oracle running {steps} steps on {O.num_threads()} threads")
    out["ref"] = O.heat_advance(o, steps, c).to_global()
    del o
    return out


@pytest.mark.parametrize("dtype_name", ["f64", "f32"])
def test_512cube_uneven_fused_step_whole_field(bt, cfg2_oracle, dtype_name):
    """512^3 periodic, seeded chop into ~1270 uneven boxes, 5 comps, 50 fused steps in
    one graph (the benchmark's form, its chunked workgroup order included): every cell
    of every component equals the oracle's whole run (FP64 bit for bit; FP32 storage
    within 2e-5 of the FP64 oracle) and every component's sum is conserved."""
    n, ncomp, steps = CFG2_N, CFG2_NCOMP, CFG2_STEPS
    dt = bt.F64 if dtype_name == "f64" else bt.F32
    boxes, dom, c, u0, ref = (cfg2_oracle[k] for k in ("boxes", "dom", "c", "u0", "ref"))
    ba = bt.BoxArray.from_boxes(boxes, dom)
    a, b = bt.MultiFab(ba, ncomp, 1, dt), bt.MultiFab(ba, ncomp, 1, dt)
    for comp in range(ncomp):
        g = u0[comp:comp + 1] if dt == bt.F64 else I.round_f32(u0[comp:comp + 1])
        a.from_global(g, scomp=comp)
    s0 = [a.sum(comp) for comp in range(ncomp)]
    res = bt.heat_advance(a, b, steps, c)
    torch.cuda.synchronize()
    worst = 0.0
    for comp in range(ncomp):
        drift = abs(res.sum(comp) - s0[comp]) / abs(s0[comp])
        assert drift <= (1e-13 if dt == bt.F64 else 1e-6), (comp, drift)
        got = res.to_global(scomp=comp, ncomp=1)[0].double().cpu().numpy()
        if dt == bt.F64:
            assert np.array_equal(got, ref[comp]), f"component {comp} differs from the oracle's"
        else:
            worst = max(worst, float(np.abs(got - ref[comp]).max() / np.abs(ref[comp]).max()))
        del got
    say(f"512^3 uneven {dtype_name}: whole field vs oracle ok, worst rel err {worst:.2e}")
    assert worst <= 2e-5


def test_512cube_uneven_varcoef_at_full_size(bt):
    """512^3 periodic, the seeded uneven chop, 5 comps, FP64, beta = 0.5 + U(0,1): 10
    flux-form steps in the benchmark's launch configuration; sampled cells equal the
    oracle's dependence-cone window bit for bit and every component's sum is conserved."""
    n, ncomp, steps = 512, 5, 10
    dom = I.domain_box(n)
    boxes = I.random_chop(dom, 16, 128, 8, seed=0)
    ba = bt.BoxArray.from_boxes(boxes, dom)
    u0 = I.uniform(n, ncomp, seed=0)
    beta = I.uniform(n, ncomp, seed=1) + 0.5
    dx = 1.0 / n
    dt = 0.9 * dx * dx / (6.0 * 1.5)
    a, b, bm = (bt.MultiFab(ba, ncomp, 1, bt.F64) for _ in range(3))
    for comp in range(ncomp):
        a.from_global(u0[comp:comp + 1], scomp=comp)
        bm.from_global(beta[comp:comp + 1], scomp=comp)
    s0 = [a.sum(comp) for comp in range(ncomp)]
    res = bt.heat_varcoef_advance(a, b, bm, steps, dt, dx)
    torch.cuda.synchronize()
    for comp in range(ncomp):
        drift = abs(res.sum(comp) - s0[comp]) / abs(s0[comp])
        assert drift <= 1e-13, (comp, drift)
    rng = np.random.default_rng(9)
    for comp in (0, 2, 4):
        for _ in range(3):
            cell = tuple(int(v) for v in rng.integers(0, n, 3))
            ref = O.heat_varcoef_window(u0[comp], beta[comp], cell, steps, dt, dx)
            assert _cell(res, boxes, comp, cell) == ref, (comp, cell)
    say("512^3 uneven varcoef: sampled cells bit-exact, sums conserved")


@pytest.mark.parametrize("form", ["auto", "fused_mirror"])
def test_512cube_uneven_heat8_fused_at_full_size(bt, form):
    """512^3 periodic, the seeded uneven chop, 5 comps, 4 ghost layers, FP64: 10 steps of
    the 8th-order form in the benchmark's configuration (the default, fused form, which
    reads neighbour boxes directly, and the fused form with the 4-layer edge mirrors);
    sampled cells equal the oracle's dependence-cone window bit for bit and every
    component's sum is conserved."""
    n, ncomp, steps, c = 512, 5, 10, 0.09
    dom = I.domain_box(n)
    boxes = I.random_chop(dom, 16, 128, 8, seed=0)
    ba = bt.BoxArray.from_boxes(boxes, dom)
    u0 = I.uniform(n, ncomp, seed=0)
    a, b = bt.MultiFab(ba, ncomp, 4, bt.F64), bt.MultiFab(ba, ncomp, 4, bt.F64)
    for comp in range(ncomp):
        a.from_global(u0[comp:comp + 1], scomp=comp)
    assert bt.heat8_auto_form(a) == "fused"
    s0 = [a.sum(comp) for comp in range(ncomp)]
    res = bt.heat8_advance(a, b, steps, c, form=form)
    torch.cuda.synchronize()
    for comp in range(ncomp):
        drift = abs(res.sum(comp) - s0[comp]) / abs(s0[comp])
        assert drift <= 1e-13, (comp, drift)
    rng = np.random.default_rng(11)
    for comp in (0, 2, 4):
        for _ in range(3):
            cell = tuple(int(v) for v in rng.integers(0, n, 3))
            assert _cell(res, boxes, comp, cell) == O.heat8_window(u0[comp], cell, steps, c), (comp, cell)
    say(f"512^3 uneven heat8 ({form}): sampled cells bit-exact, sums conserved")


def test_512cube_uneven_heat8_fp32_forms_agree(bt):
    """512^3 periodic, the seeded uneven chop, 5 comps, 4 ghost layers, FP32 storage: 4
    steps of the 8th-order step in the fill form, the fused form and the fused form with
    the 4-layer edge mirrors give the same bits on every valid cell (the same operations
    on the same operands; the forms differ only in where a face cell is read from)."""
    n, ncomp, steps, c = 512, 5, 4, 0.09
    dom = I.domain_box(n)
    boxes = I.random_chop(dom, 16, 128, 8, seed=0)
    ba = bt.BoxArray.from_boxes(boxes, dom)
    u0 = I.round_f32(I.uniform(n, ncomp, seed=2))
    got = {}
    for form in ("fill", "fused", "fused_mirror"):
        a, b = bt.MultiFab(ba, ncomp, 4, bt.F32), bt.MultiFab(ba, ncomp, 4, bt.F32)
        a.set_val(0.0, with_ghosts=True)
        for comp in range(ncomp):
            a.from_global(u0[comp:comp + 1], scomp=comp)
        got[form] = bt.heat8_advance(a, b, steps, c, form=form).to_global()
        del a, b
        torch.cuda.synchronize()
    assert torch.equal(got["fused"], got["fill"]) and torch.equal(got["fused_mirror"], got["fill"])
    say("512^3 uneven heat8 FP32: fill, fused and mirror forms bit-identical")


def test_384cube_gsrb_at_full_size(bt):
    """384^3 periodic, 216 boxes of 64^3, zero-mean f, phi0 = 0, 20 sweeps with the FP64
    residual norm after each (the benchmark's GSRB workload) against the oracle's whole
    run: the FP64 state bit for bit and all 20 norms to 1e-13, in the one-pass and in the
    two-pass form; the FP32 state of both forms the same bits, within 1e-5 of the
    oracle's field, and all 20 FP32 norms within 1e-5; the norms fall every sweep."""
    n, sweeps = 384, 20
    dom = I.domain_box(n)
    boxes = I.regular_chop(dom, 64)
    ba = bt.BoxArray.from_boxes(boxes, dom)
    f = I.zero_mean_normal_f32(n, seed=0)
    h2 = (1.0 / n) ** 2

    ophi, ofm = O.OracleMultiFab(boxes, dom, (1, 1, 1), 1, 1), O.OracleMultiFab(boxes, dom, (1, 1, 1), 1, 1)
    ofm.load_global(f)
    on = O.gsrb_sweeps(ophi, ofm, h2, sweeps)
    ref = ophi.to_global()[0]
    del ophi, ofm

    def run(dt, one_pass):
        phi, fm = bt.MultiFab(ba, 1, 1, dt), bt.MultiFab(ba, 1, 1, dt)
        phi.set_val(0.0, with_ghosts=True)
        fm.set_val(0.0, with_ghosts=True)
        fm.from_global(f)
        bt.set_gsrb_config(one_pass, 0, 0)
        try:
            assert bt.gsrb_one_pass_applies(phi) == bool(one_pass)
            norms = bt.gsrb_sweeps(phi, fm, h2, sweeps)
        finally:
            bt.set_gsrb_config(1, 0, 0)
        return phi.to_global()[0].double().cpu().numpy(), norms

    for one_pass in (1, 0):  # the one-pass sweep (the default here) and the two colour passes
        g64, n64 = run(bt.F64, one_pass)
        assert np.array_equal(g64, ref), f"FP64 GSRB field differs from the oracle's (one_pass={one_pass})"
        assert all(abs(g - r) <= 1e-13 * r for g, r in zip(n64, on)), (one_pass, n64, on)
        del g64
    g32, n32 = run(bt.F32, 1)
    g32b, _ = run(bt.F32, 0)
    assert np.array_equal(g32, g32b), "FP32 one-pass and two-pass fields differ"
    del g32b
    ferr = float(np.abs(g32 - ref).max() / np.abs(ref).max())
    nerr = max(abs(x - y) / y for x, y in zip(n32, on))
    say(f"384^3 gsrb: fp64 bit-exact; fp32 field rel err {ferr:.2e}, norm rel err {nerr:.2e}, "
        f"norms {on[0]:.4e} -> {on[-1]:.4e}")
    assert ferr <= 1e-5 and nerr <= 1e-5
    assert all(y < x for x, y in zip(on, on[1:]))


def test_256cube_vcycles_at_full_size(bt):
    """256^3 periodic, 64 boxes of 64^3, FP64, zero-mean f: 7 levels down to 64 boxes of
    one cell; after one V(2,2) cycle the field equals the oracle's bit for bit; four
    more cycles cut the residual by 10^4."""
    n = 256
    dom = I.domain_box(n)
    boxes = I.regular_chop(dom, 64)
    ba = bt.BoxArray.from_boxes(boxes, dom)
    f = I.zero_mean_normal_f32(n, seed=0)
    h2 = (1.0 / n) ** 2
    phi, fm = bt.MultiFab(ba, 1, 1, bt.F64), bt.MultiFab(ba, 1, 1, bt.F64)
    phi.set_val(0.0, with_ghosts=True)
    fm.set_val(0.0, with_ghosts=True)
    fm.from_global(f)
    mg = bt.Multigrid(ba, bt.F64)
    assert mg.nlevels == 7
    n1 = mg.vcycles(phi, fm, h2, 1)
    ophi, ofm = O.OracleMultiFab(boxes, dom, (1, 1, 1), 1, 1), O.OracleMultiFab(boxes, dom, (1, 1, 1), 1, 1)
    ofm.load_global(f)
    on = O.mg_vcycles(ophi, ofm, h2, 1)
    assert np.array_equal(phi.to_global().cpu().numpy(), ophi.to_global())
    assert abs(n1[0] - on[0]) <= 1e-13 * on[0]
    more = mg.vcycles(phi, fm, h2, 4)
    on4 = O.mg_vcycles(ophi, ofm, h2, 4)
    ref = ophi.to_global()
    assert np.array_equal(phi.to_global().cpu().numpy(), ref)
    assert all(abs(g - r) <= 1e-13 * r for g, r in zip(more, on4))
    say(f"256^3 vcycles: norms {n1[0]:.4e} then {[f'{x:.3e}' for x in more]}")
    assert more[-1] <= 1e-4 * n1[0]
    # FP32 storage: 5 cycles against the oracle's 5 (FP64)
    p32, f32 = bt.MultiFab(ba, 1, 1, bt.F32), bt.MultiFab(ba, 1, 1, bt.F32)
    p32.set_val(0.0, with_ghosts=True)
    f32.set_val(0.0, with_ghosts=True)
    f32.from_global(f)
    n32 = bt.Multigrid(ba, bt.F32).vcycles(p32, f32, h2, 5)
    ferr = float(np.abs(p32.to_global().double().cpu().numpy() - ref).max() / np.abs(ref).max())
    on5 = [on[0]] + list(on4)
    say(f"256^3 vcycles fp32: field rel err {ferr:.2e} vs the oracle, norms {n32} vs {on5}")
    assert ferr <= 1e-5
    # a norm from FP32 state differs from the exact one by at most the norm of the
    # residual of the FP32 rounding error, a floor the cycles converge to (the last FP32
    # norm bounds it): each norm within 1e-5 of the oracle's plus that floor
    floor = n32[-1]
    assert all(abs(a - b) <= 1e-5 * b + floor for a, b in zip(n32, on5)), (n32, on5)
    assert abs(n32[0] - on5[0]) <= 1e-5 * on5[0]
    assert all(b < 0.3 * a for a, b in zip(n32[:3], n32[1:4]))


def test_256cube_heat8_at_full_size(bt):
    """256^3 periodic, 64 boxes of 64^3, 4 ghost layers, FP64, 3 seeded sine modes, 20
    steps of the 8th-order form: the closed form of the stencil's symbol to 1e-12 and
    sampled cells equal the oracle's dependence-cone window bit for bit."""
    n, steps, c = 256, 20, 0.09
    dom = I.domain_box(n)
    ba = bt.BoxArray.chop(dom, 64)
    u0, modes = I.sine_modes(n, seed=4)
    a, b = bt.MultiFab(ba, 1, 4, bt.F64), bt.MultiFab(ba, 1, 4, bt.F64)
    a.from_global(u0)
    got = bt.heat8_advance(a, b, steps, c).to_global()[0].cpu().numpy()
    coef = (-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0)
    exact = np.zeros_like(got)
    for md in modes:
        sym = sum(coef[0] + 2.0 * sum(coef[m] * math.cos(2 * math.pi * m * kd / n) for m in range(1, 5))
                  for kd in md.k)
        exact += md.amp * (1.0 + c * sym) ** steps * I.sine_product(n, md.k)
    err = np.abs(got - exact).max() / np.abs(exact).max()
    say(f"256^3 heat8: closed-form rel err {err:.3e}")
    assert err <= 1e-12
    rng = np.random.default_rng(3)
    for cell in [(0, 0, 0), (255, 64, 130)] + [tuple(int(v) for v in rng.integers(0, n, 3))]:
        i, j, k = cell
        assert got[k, j, i] == O.heat8_window(u0[0], cell, steps, c), cell
