"""Pins of the CPU oracle against facts fixed by the paper and by the mathematics,
not by the oracle itself (CPU only).

Each pin is chosen so that a plausible mistake in the oracle fails at least one
of them (``test_planted_mistakes_are_caught`` plants such mistakes in a copy of
the oracle and checks exactly that):
  * a periodic sine mode is a discrete eigenfunction of the 7-point Laplacian,
    so n heat steps multiply it by g^n, g = 1 - 4c sum_d sin^2(pi k_d / N_d);
  * the domain sum is conserved on periodic domains;
  * a single-box and a many-box decomposition give bit-identical results;
  * FillBoundary equals a brute-force search over boxes on tiny grids;
  * one periodic box equals a numpy.roll 7-point update;
  * the paper's flux form agrees with the 7-point form;
  * the variable-coefficient flux form is second order against the analytic
    div(beta grad u) of a smooth periodic problem, with the closed-form leading error
    term of the mean face coefficient; a unit impulse spreads exactly the face
    coefficients; it equals a numpy.roll implementation, reduces to the flux form at
    unit coefficient, conserves the sum and is self-adjoint;
  * red-black Gauss-Seidel equals dense Gauss-Seidel in red-then-black order;
  * residual invariants (zero on the colour just relaxed, sum r = sum f);
  * reductions against exactly known sums.
"""
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_1604_03570_amd import inputs as I


def _mf(boxes, n, ncomp=1, ng=1, periodic=(1, 1, 1)):
    return O.OracleMultiFab(boxes, I.domain_box(n), periodic, ncomp, ng)


def _uneven_boxes(n, seed):
    """A seeded uneven decomposition of an (nx, ny, nz) domain (small edges)."""
    nx, ny, nz = (n, n, n) if np.isscalar(n) else n
    return I.random_chop(I.domain_box((nx, ny, nz)), min_edge=2, max_edge=8, align=2, seed=seed)


# ---------------------------------------------------------------------------------------------
# heat step
# ---------------------------------------------------------------------------------------------
def _sine_decay_error(shape=(32, 24, 16), steps=20, boxes=None):
    nx, ny, nz = shape
    c = 0.1  # modes stay O(1e-2) after 20 steps, far above the rounding noise
    modes = [(0.7, (1, 2, 3)), (0.3, (5, 1, 2))]
    u0 = np.zeros((1, nz, ny, nx))
    exact = np.zeros_like(u0)
    for amp, k in modes:
        phi = I.sine_product(shape, k)
        g = 1.0 - 4.0 * c * sum(math.sin(math.pi * k[d] / shape[d]) ** 2 for d in range(3))
        u0[0] += amp * phi
        exact[0] += amp * g ** steps * phi
    if boxes is None:
        boxes = I.random_chop(I.domain_box(shape), min_edge=4, max_edge=16, align=4, seed=3)
    m = _mf(boxes, shape)
    m.load_global(u0)
    out = O.heat_advance(m, steps, c).to_global()
    return np.abs(out - exact).max() / np.abs(exact).max()


def test_sine_mode_decay_closed_form():
    # anisotropic domain and wavenumbers: axis mix-ups change the decay factor
    assert _sine_decay_error() <= 1e-12
    assert _sine_decay_error(boxes=I.regular_chop(I.domain_box((32, 24, 16)), 8)) <= 1e-12


def test_sine_mode_decay_with_the_256cube_modes():
    # the 256^3 workload's seeded modes (wavenumbers 1..8), on a 64^3 grid
    n, steps = 64, 10
    u0, modes = I.sine_modes(n, seed=1)
    c = I.heat_c(n)
    m = _mf(I.regular_chop(I.domain_box(n), 32), n)
    m.load_global(u0)
    out = O.heat_advance(m, steps, c).to_global()
    exact = np.zeros_like(u0)
    for md in modes:
        g = 1.0 - 4.0 * c * sum(math.sin(math.pi * kd / n) ** 2 for kd in md.k)
        exact[0] += md.amp * g ** steps * I.sine_product(n, md.k)
    assert np.abs(out - exact).max() / np.abs(exact).max() <= 1e-12


def test_domain_sum_conserved_periodic():
    shape = (12, 10, 8)
    u0 = I.uniform(shape, 2, seed=5)
    m = _mf(_uneven_boxes(shape, seed=1), shape, ncomp=2)
    m.load_global(u0)
    s0 = [O.reduce(m, comp, "sum") for comp in range(2)]
    out = O.heat_advance(m, 30, 0.15)
    for comp in range(2):
        assert abs(O.reduce(out, comp, "sum") - s0[comp]) <= 1e-13 * abs(s0[comp])


def test_single_box_equals_many_boxes_bit_identical():
    n = 32
    u0 = I.gaussian(n)
    c = I.heat_c(n)
    results = []
    for boxes in (I.regular_chop(I.domain_box(n), n), I.regular_chop(I.domain_box(n), 16),
                  I.regular_chop(I.domain_box(n), (8, 16, 32)),
                  I.random_chop(I.domain_box(n), min_edge=4, max_edge=16, align=4, seed=7)):
        m = _mf(boxes, n)
        m.load_global(u0)
        results.append(O.heat_advance(m, 10, c).to_global())
    for r in results[1:]:
        assert np.array_equal(r, results[0])


def _roll_step(u, c):
    """Textbook periodic 7-point update with numpy.roll, same operand order."""
    xm, xp = np.roll(u, 1, axis=2), np.roll(u, -1, axis=2)
    ym, yp = np.roll(u, 1, axis=1), np.roll(u, -1, axis=1)
    zm, zp = np.roll(u, 1, axis=0), np.roll(u, -1, axis=0)
    s = ((xm + xp) + (ym + yp)) + (zm + zp)
    return u + c * (s - 6.0 * u)


def test_single_periodic_box_equals_numpy_roll():
    shape = (10, 6, 8)
    u = I.uniform(shape, 1, seed=11)
    m = _mf(I.regular_chop(I.domain_box(shape), 64), shape)
    m.load_global(u)
    ref = u[0]
    for _ in range(7):
        ref = _roll_step(ref, 0.15)
    assert np.array_equal(O.heat_advance(m, 7, 0.15).to_global()[0], ref)


def test_many_boxes_equal_numpy_roll():
    shape = (10, 6, 8)
    u = I.uniform(shape, 1, seed=12)
    m = _mf(_uneven_boxes(shape, seed=4), shape)
    m.load_global(u)
    ref = u[0]
    for _ in range(5):
        ref = _roll_step(ref, 0.15)
    assert np.array_equal(O.heat_advance(m, 5, 0.15).to_global()[0], ref)


def _roll_varcoef_step(u, beta, dt, dx):
    """Textbook periodic variable-coefficient flux form with numpy.roll: face coefficient
    the mean of the two cells, same operand order as the oracle's C loop."""
    out = []
    inv_dx = 1.0 / dx
    for axis in (2, 1, 0):  # x, y, z
        um, up = np.roll(u, 1, axis=axis), np.roll(u, -1, axis=axis)
        bm, bp = np.roll(beta, 1, axis=axis), np.roll(beta, -1, axis=axis)
        fm = (0.5 * (bm + beta)) * ((u - um) * inv_dx)
        fp = (0.5 * (beta + bp)) * ((up - u) * inv_dx)
        out.append((fp - fm) * inv_dx)
    dfx, dfy, dfz = out
    return u + dt * ((dfx + dfy) + dfz)


def test_varcoef_single_periodic_box_equals_numpy_roll():
    shape = (10, 6, 8)
    rng = np.random.default_rng(5)
    u = rng.random((1,) + shape[::-1])
    beta = 0.5 + rng.random((1,) + shape[::-1])
    dx, dt = 0.1, 0.001
    m, bm = _mf(I.regular_chop(I.domain_box(shape), 64), shape), _mf(I.regular_chop(I.domain_box(shape), 64), shape)
    m.load_global(u)
    bm.load_global(beta)
    ref = u[0]
    for _ in range(4):
        ref = _roll_varcoef_step(ref, beta[0], dt, dx)
    assert np.array_equal(O.heat_varcoef_advance(m, bm, 4, dt, dx).to_global()[0], ref)


def test_varcoef_many_boxes_equal_one_box_and_conserve_the_sum():
    shape = (12, 10, 8)
    rng = np.random.default_rng(6)
    u = rng.random((2,) + shape[::-1])
    beta = 0.5 + rng.random((2,) + shape[::-1])
    dx, dt = 0.1, 0.0005
    out = []
    for boxes in (I.regular_chop(I.domain_box(shape), 64), _uneven_boxes(shape, seed=7)):
        m, bm = _mf(boxes, shape, ncomp=2), _mf(boxes, shape, ncomp=2)
        m.load_global(u)
        bm.load_global(beta)
        out.append(O.heat_varcoef_advance(m, bm, 6, dt, dx).to_global())
    assert np.array_equal(out[0], out[1])
    for comp in range(2):
        s0, s1 = math.fsum(u[comp].ravel()), math.fsum(out[0][comp].ravel())
        assert abs(s1 - s0) <= 1e-13 * abs(s0)


def test_varcoef_unit_coefficient_is_the_flux_form():
    shape = (9, 7, 6)
    u = I.uniform(shape, 1, seed=9)
    dx, dt = 1.0 / 9, 0.9 * (1.0 / 9) ** 2 / 6
    boxes = _uneven_boxes(shape, seed=8)
    a, b, bm = _mf(boxes, shape), _mf(boxes, shape), _mf(boxes, shape)
    a.load_global(u)
    bm.load_global(np.ones_like(u))
    O.heat_varcoef_step(a, b, bm, dt, dx)
    a2, b2 = _mf(boxes, shape), _mf(boxes, shape)
    a2.load_global(u)
    O.heat_flux_step(a2, b2, dt, dx)
    assert np.array_equal(b.to_global(), b2.to_global())


# A manufactured smooth periodic problem for the variable-coefficient operator: u and beta
# are products of one sinusoid per axis, different on every axis, so that any derivative
# is known in closed form.  Each factor is (k, phase, amplitude, offset):
# f(t) = amp * sin(k t + phase) + offset, whose m-th derivative is
# amp * k^m * sin(k t + phase + m pi / 2).
_VC_U = [(2 * math.pi, 1.0, 1.0, 0.0), (2 * math.pi, math.pi / 2, 1.0, 0.0), (2 * math.pi, 0.0, 0.5, 1.0)]
_VC_B = [(2 * math.pi, 0.0, 1.0, 0.0), (4 * math.pi, 0.3 + math.pi / 2, 1.0, 0.0), (2 * math.pi, math.pi / 2, 1.0, 0.0)]
_VC_B_OFFSET = 2.0  # beta = 2 + P(x) Q(y) R(z) lies in [1, 3]


def _vc_manufactured(n):
    """u, beta, the exact div(beta grad u) and the exact leading truncation term E at the
    cell centres of an n^3 periodic grid on [0,1)^3.

    For the flux form whose face coefficient is the mean of the two cells, Taylor
    expansion of the one-axis difference b(+)(u(+) - u) - b(-)(u - u(-)) about the cell
    centre gives, per axis d (h = dx),
        L_h u = (beta u_d)_d + h^2 [beta u_dddd / 12 + beta_d u_ddd / 6
                                    + beta_dd u_dd / 4 + beta_ddd u_d / 6] + O(h^4),
    so E is that bracket summed over the axes.  A one-sided face coefficient leaves an
    O(h) error; a harmonic or geometric mean is second order too but with another h^2
    term (it differs by multiples of beta_d^2 / beta)."""
    t = (np.arange(n) + 0.5) / n
    co = [t[None, None, :], t[None, :, None], t[:, None, None]]

    def deriv(factors, d, m):
        out = 1.0
        for a, (k, ph, amp, off) in enumerate(factors):
            mm = m if a == d else 0
            out = out * (amp * k ** mm * np.sin(k * co[a] + ph + mm * math.pi / 2) + (off if mm == 0 else 0.0))
        return out

    def du(d, m):
        return deriv(_VC_U, d, m)

    def db(d, m):
        return deriv(_VC_B, d, m) + (_VC_B_OFFSET if m == 0 else 0.0)

    u, beta = du(0, 0), db(0, 0)
    div = sum(beta * du(d, 2) + db(d, 1) * du(d, 1) for d in range(3))
    lead = sum(beta * du(d, 4) / 12 + db(d, 1) * du(d, 3) / 6 + db(d, 2) * du(d, 2) / 4 + db(d, 3) * du(d, 1) / 6
               for d in range(3))
    return u, beta, div, lead


def _vc_truncation(n):
    """(max |L_h u - div(beta grad u)|, max |(L_h u - div)/h^2 - E|, max |E|) for the
    oracle's operator on an uneven chop of an n^3 periodic grid; L_h u is one step with
    dt = 1 minus u."""
    u, beta, div, lead = _vc_manufactured(n)
    shape = (n, n, n)
    boxes = I.random_chop(I.domain_box(shape), 4, 16, 4, seed=n)
    m, bm, out = _mf(boxes, shape), _mf(boxes, shape), _mf(boxes, shape)
    m.load_global(u[None])
    bm.load_global(beta[None])
    O.heat_varcoef_step(m, out, bm, 1.0, 1.0 / n)
    lh = out.to_global()[0] - u
    return (float(np.abs(lh - div).max()), float(np.abs((lh - div) * (n * n) - lead).max()),
            float(np.abs(lead).max()))


def test_varcoef_is_second_order_with_the_mean_face_coefficient():
    """The variable-coefficient flux form (Sec. 4.1's flux-then-divergence kernel with a
    coefficient per cell) against the analytic operator div(beta grad u) of a smooth
    periodic problem: the error falls 4x per halving of dx (second order), and the error
    divided by dx^2 converges to the closed-form leading term of the mean-coefficient
    scheme.  Neither fact restates the oracle's formula."""
    e16, r16, _ = _vc_truncation(16)
    e32, r32, _ = _vc_truncation(32)
    e64, r64, lead = _vc_truncation(64)
    assert 3.5 <= e16 / e32 <= 4.5 and 3.7 <= e32 / e64 <= 4.3, (e16, e32, e64)
    # the remainder after the h^2 term is O(h^2) itself and small against that term
    assert r32 / r64 >= 3.5 and r64 <= 0.01 * lead, (r32, r64, lead)


def test_varcoef_face_coefficient_is_the_mean_of_the_two_cells():
    """A unit impulse at one cell spreads, in one step with dt = dx = 1, exactly its face
    coefficient b to the neighbour across each face and keeps 1 - sum(b): the flux between
    two cells is b times their difference, b the mean of their coefficients (the reading
    of the paper's flux form with a coefficient per cell)."""
    shape = (8, 6, 10)
    rng = np.random.default_rng(21)
    beta = 0.5 + rng.random((1,) + shape[::-1])
    boxes = _uneven_boxes(shape, seed=22)
    for cell in [(0, 0, 0), (7, 5, 9), (3, 2, 4)]:
        i, j, k = cell
        u = np.zeros((1,) + shape[::-1])
        u[0, k, j, i] = 1.0
        m, bm, out = _mf(boxes, shape), _mf(boxes, shape), _mf(boxes, shape)
        m.load_global(u)
        bm.load_global(beta)
        O.heat_varcoef_step(m, out, bm, 1.0, 1.0)
        got = out.to_global()[0]
        total = 0.0
        for axis, n in enumerate(shape):
            for s in (-1, 1):
                q = [i, j, k]
                q[axis] = (q[axis] + s) % n
                b = 0.5 * (beta[0, k, j, i] + beta[0, q[2], q[1], q[0]])
                assert abs(got[q[2], q[1], q[0]] - b) <= 1e-15, (cell, axis, s)
                total += b
        assert abs(got[k, j, i] - (1.0 - total)) <= 1e-14
        assert np.count_nonzero(got) == 7


def test_varcoef_operator_is_symmetric():
    """div(beta grad) is self-adjoint on periodic grids: <v, A u> = <u, A v>."""
    shape = (8, 8, 6)
    rng = np.random.default_rng(10)
    beta = 0.5 + rng.random((1,) + shape[::-1])
    boxes = _uneven_boxes(shape, seed=11)

    def apply(w):
        m, out, bm = _mf(boxes, shape), _mf(boxes, shape), _mf(boxes, shape)
        m.load_global(w)
        bm.load_global(beta)
        O.heat_varcoef_step(m, out, bm, 1.0, 1.0)
        return out.to_global() - w

    u, v = rng.random((1,) + shape[::-1]), rng.random((1,) + shape[::-1])
    lhs, rhs = float((v * apply(u)).sum()), float((u * apply(v)).sum())
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), abs(rhs))
    assert float((u * apply(u)).sum()) < 0  # and negative definite on non-constant fields


def test_flux_form_agrees_with_seven_point():
    n = 24
    dx = 1.0 / n
    dt = 0.9 * dx * dx / 6.0
    c = dt / (dx * dx)
    u0 = I.uniform(n, 2, seed=2) + 1.0
    a = _mf(_uneven_boxes(n, seed=2), n, ncomp=2)
    a.load_global(u0)
    b = a.copy()
    a2, b2 = a.copy(), b.copy()
    for _ in range(5):
        O.heat_step(a, a2, c)
        a, a2 = a2, a
        O.heat_flux_step(b, b2, dt, dx)
        b, b2 = b2, b
    ga, gb = a.to_global(), b.to_global()
    assert np.abs(ga - gb).max() / np.abs(ga).max() <= 1e-14
    assert not np.array_equal(ga, gb)  # genuinely a different formulation


def test_heat_window_equals_full_run():
    n, steps = 16, 6
    u0 = I.uniform(n, 1, seed=3)
    c = I.heat_c(n)
    m = _mf(I.regular_chop(I.domain_box(n), 8), n)
    m.load_global(u0)
    full = O.heat_advance(m, steps, c).to_global()[0]
    rng = np.random.default_rng(0)
    for _ in range(10):
        i, j, k = (int(v) for v in rng.integers(0, n, 3))
        assert O.heat_window(u0[0], (i, j, k), steps, c) == full[k, j, i]


def test_varcoef_window_equals_full_run():
    """The dependence-cone window (one box, fixed ghosts) gives the full periodic run's
    cell bit for bit, also for a window that wraps around the domain."""
    n, steps = 18, 7
    rng = np.random.default_rng(11)
    u0 = rng.random((1, n, n, n))
    beta = 0.5 + rng.random((1, n, n, n))
    dx = 1.0 / n
    dt = 0.9 * dx * dx / (6 * 1.5)
    boxes = I.random_chop(I.domain_box(n), 3, 9, 1, seed=2)
    m, bm = _mf(boxes, n), _mf(boxes, n)
    m.load_global(u0)
    bm.load_global(beta)
    full = O.heat_varcoef_advance(m, bm, steps, dt, dx).to_global()[0]
    for cell in [(0, 0, 0), (17, 9, 3)] + [tuple(int(v) for v in rng.integers(0, n, 3)) for _ in range(6)]:
        i, j, k = cell
        assert O.heat_varcoef_window(u0[0], beta[0], cell, steps, dt, dx) == full[k, j, i]


# ---------------------------------------------------------------------------------------------
# FillBoundary
# ---------------------------------------------------------------------------------------------
POISON = -1.0e300


def _brute_fill(boxes, shape, periodic, ng, ncomp, values):
    """For every ghost cell of every box, search all boxes for the wrapped index."""
    nx, ny, nz = shape
    N = (nx, ny, nz)
    expect = {}
    for b, bx in enumerate(boxes):
        for k in range(bx[2] - ng, bx[5] + ng + 1):
            for j in range(bx[1] - ng, bx[4] + ng + 1):
                for i in range(bx[0] - ng, bx[3] + ng + 1):
                    if bx[0] <= i <= bx[3] and bx[1] <= j <= bx[4] and bx[2] <= k <= bx[5]:
                        continue
                    p = [i, j, k]
                    ok = True
                    for d in range(3):
                        if periodic[d]:
                            p[d] %= N[d]
                        if not 0 <= p[d] < N[d]:
                            ok = False
                    owner = None
                    if ok:
                        for bb in boxes:
                            if bb[0] <= p[0] <= bb[3] and bb[1] <= p[1] <= bb[4] and bb[2] <= p[2] <= bb[5]:
                                owner = bb
                    for comp in range(ncomp):
                        v = values[comp, p[2], p[1], p[0]] if owner is not None else POISON
                        expect[(b, comp, k, j, i)] = v
    return expect


@pytest.mark.parametrize("case", range(12))
def test_fill_boundary_brute_force(case):
    rng = np.random.default_rng(100 + case)
    shape = [(8, 6, 4), (5, 5, 5), (7, 4, 6)][case % 3]
    ng = 1 + case % 2
    ncomp = 1 + case % 3
    periodic = tuple(int(v) for v in rng.integers(0, 2, 3))
    boxes = I.random_chop(I.domain_box(shape), min_edge=1, max_edge=4, align=1, seed=case)
    if case % 4 == 3 and len(boxes) > 2:  # non-covering box list: drop some boxes
        keep = rng.permutation(len(boxes))[: len(boxes) // 2]
        boxes = boxes[np.sort(keep)]
    nx, ny, nz = shape
    # unique value per (comp, cell): any mis-copied ghost is seen
    values = np.arange(ncomp * nx * ny * nz, dtype=np.float64).reshape(ncomp, nz, ny, nx) + 0.25
    m = O.OracleMultiFab(boxes, I.domain_box(shape), periodic, ncomp, ng)
    m.data[...] = POISON
    m.load_global(values)
    before = [m.valid(b).copy() for b in range(m.nbox)]
    m.fill_boundary()
    expect = _brute_fill(boxes, shape, periodic, ng, ncomp, values)
    for (b, comp, k, j, i), v in expect.items():
        bx = boxes[b]
        got = m.fab(b)[comp, k - bx[2] + ng, j - bx[1] + ng, i - bx[0] + ng]
        assert got == v, (b, comp, k, j, i)
    for b in range(m.nbox):
        assert np.array_equal(m.valid(b), before[b])


def test_fill_boundary_partial_components():
    shape = (6, 6, 6)
    boxes = I.regular_chop(I.domain_box(shape), 3)
    vals = I.uniform(shape, 3, seed=9)
    m = O.OracleMultiFab(boxes, I.domain_box(shape), (1, 1, 1), 3, 1)
    m.data[...] = POISON
    m.load_global(vals)
    m.fill_boundary(scomp=1, ncomp=1)
    for b in range(m.nbox):
        f = m.fab(b)
        assert np.sum(f[0] == POISON) == f[0].size - m.valid(b)[0].size  # comp 0 ghosts untouched
        assert np.sum(f[2] == POISON) == f[2].size - m.valid(b)[2].size  # comp 2 ghosts untouched
        assert not np.any(f[1] == POISON)                                   # comp 1 fully filled


# ---------------------------------------------------------------------------------------------
# red-black Gauss-Seidel
# ---------------------------------------------------------------------------------------------
def _dense_minus_laplacian(shape, h2):
    nx, ny, nz = shape
    n = nx * ny * nz
    A = np.zeros((n, n))
    idx = lambda i, j, k: (k % nz) * ny * nx + (j % ny) * nx + (i % nx)
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                r = idx(i, j, k)
                A[r, r] += 6.0 / h2
                for di, dj, dk in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
                    A[r, idx(i + di, j + dj, k + dk)] -= 1.0 / h2
    return A


@pytest.mark.parametrize("shape", [(4, 4, 4), (6, 4, 8)])
def test_gsrb_equals_dense_gauss_seidel_red_then_black(shape):
    nx, ny, nz = shape
    h2 = (1.0 / 8) ** 2
    f = I.uniform(shape, 1, seed=21)[0] - 0.5
    phi0 = I.uniform(shape, 1, seed=22)[0]
    A = _dense_minus_laplacian(shape, h2)
    kk, jj, ii = np.meshgrid(range(nz), range(ny), range(nx), indexing="ij")
    color = ((ii + jj + kk) % 2).ravel()
    order = np.concatenate([np.flatnonzero(color == 0), np.flatnonzero(color == 1)])
    Ap = A[np.ix_(order, order)]
    x = phi0.ravel()[order].copy()
    b = f.ravel()[order]
    DL = np.tril(Ap)
    for _ in range(2):  # two sweeps: x <- x + (D+L)^{-1} (b - A x)
        x = x + np.linalg.solve(DL, b - Ap @ x)
    expect = np.empty_like(x)
    expect[order] = x
    boxes = I.regular_chop(I.domain_box(shape), (nx // 2, ny // 2, nz))  # several boxes
    phi = _mf(boxes, shape)
    phi.load_global(phi0[None])
    fm = _mf(boxes, shape)
    fm.load_global(f[None])
    O.gsrb_sweeps(phi, fm, h2, 2, with_norms=False)
    got = phi.to_global()[0].ravel()
    assert np.abs(got - expect).max() / np.abs(expect).max() <= 1e-14


def test_gsrb_residual_invariants():
    shape = (8, 8, 6)
    h2 = (1.0 / 8) ** 2
    f = I.zero_mean_normal_f32(shape, seed=4)
    boxes = _uneven_boxes(shape, seed=5)
    phi = _mf(boxes, shape)
    fm = _mf(boxes, shape)
    fm.load_global(f)
    kk, jj, ii = np.meshgrid(range(shape[2]), range(shape[1]), range(shape[0]), indexing="ij")
    red = ((ii + jj + kk) % 2) == 0
    scale = np.abs(f).max()

    def r_global():
        r = O.residual(phi, fm, h2)
        g = np.empty(shape[::-1])
        n = 0
        for bx in boxes:
            e = (bx[3] - bx[0] + 1, bx[4] - bx[1] + 1, bx[5] - bx[2] + 1)
            sz = e[0] * e[1] * e[2]
            g[bx[2]:bx[5] + 1, bx[1]:bx[4] + 1, bx[0]:bx[3] + 1] = r[n:n + sz].reshape(e[::-1])
            n += sz
        return g

    for _ in range(3):
        O.gsrb_color(phi, fm, h2, 0)
        r = r_global()
        assert np.abs(r[red]).max() <= 1e-12 * scale
        O.gsrb_color(phi, fm, h2, 1)
        r = r_global()
        assert np.abs(r[~red]).max() <= 1e-12 * scale
        # periodic: sum of L_h phi vanishes, so sum r = sum f
        assert abs(math.fsum(r.ravel().tolist()) - math.fsum(f.ravel().tolist())) <= 1e-10 * scale * r.size


def test_gsrb_exact_discrete_solution_is_fixed_point():
    shape = (8, 8, 8)
    h2 = (1.0 / 8) ** 2
    k = (1, 2, 3)
    phi_exact = I.sine_product(shape, k)
    lam = 4.0 / h2 * sum(math.sin(math.pi * kd / 8) ** 2 for kd in k)  # -L_h phi = lam phi
    boxes = I.regular_chop(I.domain_box(shape), 4)
    phi = _mf(boxes, shape)
    phi.load_global(phi_exact[None])
    fm = _mf(boxes, shape)
    fm.load_global(lam * phi_exact[None])
    norms = O.gsrb_sweeps(phi, fm, h2, 3)
    assert np.abs(phi.to_global()[0] - phi_exact).max() <= 1e-13
    assert max(norms) <= 1e-10 * lam


def test_gsrb_decomposition_invariance_and_single_fill_breaks_it():
    n = 8
    h2 = (1.0 / n) ** 2
    f = I.zero_mean_normal_f32(n, seed=6)
    out = {}
    for name, boxes in (("one", I.regular_chop(I.domain_box(n), n)),
                        ("many", I.regular_chop(I.domain_box(n), 4))):
        for per_color in (True, False):
            phi = _mf(boxes, n)
            fm = _mf(boxes, n)
            fm.load_global(f)
            O.gsrb_sweeps(phi, fm, h2, 3, with_norms=False, fill_per_color=per_color)
            out[(name, per_color)] = phi.to_global()
    assert np.array_equal(out[("one", True)], out[("many", True)])
    # one fill per sweep: black cells at box faces read stale red ghosts
    assert not np.array_equal(out[("one", False)], out[("many", False)])


def test_gsrb_residual_decreases():
    n = 16
    h2 = (1.0 / n) ** 2
    f = I.zero_mean_normal_f32(n, seed=7)
    boxes = I.regular_chop(I.domain_box(n), 8)
    phi, fm = _mf(boxes, n), _mf(boxes, n)
    fm.load_global(f)
    r0 = math.sqrt(math.fsum((f.ravel() ** 2).tolist()))
    norms = O.gsrb_sweeps(phi, fm, h2, 10)
    assert norms[0] < r0 and all(b < a for a, b in zip(norms, norms[1:]))


# ---------------------------------------------------------------------------------------------
# reductions
# ---------------------------------------------------------------------------------------------
def test_reductions_exact_cases():
    shape = (4, 4, 2)
    boxes = I.regular_chop(I.domain_box(shape), 2)
    g = np.zeros((2,) + shape[::-1])
    flat = g[0].ravel()
    flat[:] = 1.0
    flat[3] = 1e16
    flat[17] = -1e16  # naive left-to-right summation loses the ones next to 1e16
    g[1] = -np.arange(32, dtype=np.float64).reshape(shape[::-1]) * 0.5
    m = _mf(boxes, shape, ncomp=2)
    m.load_global(g)
    assert O.reduce(m, 0, "sum") == 30.0
    assert O.reduce(m, 0, "max") == 1e16 and O.reduce(m, 0, "min") == -1e16
    assert O.reduce(m, 0, "norm0") == 1e16
    assert O.reduce(m, 0, "norm1") == 2e16 + 30.0
    assert O.reduce(m, 1, "sum") == -0.5 * 31 * 32 / 2
    assert O.reduce(m, 1, "norm1") == 0.5 * 31 * 32 / 2
    assert O.reduce(m, 1, "norm2") == math.sqrt(0.25 * sum(i * i for i in range(32)))
    assert O.reduce(m, 1, "max") == 0.0 and O.reduce(m, 1, "min") == -15.5


def _exact_sum(values) -> float:
    """The real sum of the values (rational arithmetic, no rounding), rounded once to the
    nearest double (Fraction -> float rounds correctly, ties to even)."""
    from fractions import Fraction
    return float(sum((Fraction(float(v)) for v in values), Fraction(0)))


def _fsum_cases():
    rng = np.random.default_rng(31)
    tiny = 2.0 ** -1074
    cases = [
        [],
        [3.5],
        [1.0, 1e100, 1.0, -1e100],                      # the ones survive the cancellation
        [1.0, 2.0 ** -53],                              # a tie: rounds to even (1.0)
        [1.0, 2.0 ** -53, 2.0 ** -106],                 # just above the tie: rounds up
        [1.0, -(2.0 ** -53), -(2.0 ** -106)],           # below 1 the spacing halves: no tie
        [1.0 + 2.0 ** -52, 2.0 ** -53],                 # a tie from an odd last bit: rounds up
        [1.0 + 2.0 ** -52, 2.0 ** -53, -(2.0 ** -110)],  # below that tie: stays
        [tiny, tiny, -tiny, 2.0 ** 1000, -(2.0 ** 1000)],
        list(rng.standard_normal(5000)),
        list(rng.standard_normal(3000) * 10.0 ** rng.integers(-30, 30, 3000)),
        list(np.concatenate([rng.random(2000) * 1e20, -rng.random(2000) * 1e20, rng.random(7) * 1e-20])),
    ]
    big = rng.standard_normal(400_000) ** 2  # long enough to be split over threads
    return cases, big


def test_fsum_is_the_exactly_rounded_sum():
    """The oracle's sum (Shewchuk's expansions in C, split over threads) equals the real
    sum rounded once, computed with rationals, on cancellation, ties, subnormals, wide
    exponent ranges and a long array; and it equals math.fsum."""
    cases, big = _fsum_cases()
    for vals in cases:
        assert O.fsum(np.array(vals, dtype=np.float64)) == _exact_sum(vals), vals[:4]
        assert O.fsum(np.array(vals, dtype=np.float64)) == math.fsum(vals)
    assert O.fsum(big) == math.fsum(big.tolist())
    for nt in (1, 3, 8):
        O.set_num_threads(nt)
        try:
            assert O.fsum(big) == math.fsum(big.tolist())
        finally:
            O.set_num_threads(os.cpu_count() or 1)


# ---------------------------------------------------------------------------------------------
# planted mistakes: each must make at least one pin fail
# ---------------------------------------------------------------------------------------------
# ---------------------------------------------------------------------------------------------
# Multigrid V-cycle (restriction, prolongation, levels)
# ---------------------------------------------------------------------------------------------
def _dense_transfer(shape):
    """R (coarse x fine): mean of the 8 children; P (fine x coarse): parent injection."""
    nx, ny, nz = shape
    cx, cy, cz = nx // 2, ny // 2, nz // 2
    R = np.zeros((cx * cy * cz, nx * ny * nz))
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                R[((k // 2) * cy + j // 2) * cx + i // 2, (k * ny + j) * nx + i] = 0.125
    return R, 8.0 * R.T


@pytest.mark.parametrize("shape", [(4, 4, 4), (8, 4, 6)])
def test_mg_transfers_equal_dense_matrices(shape):
    """Restriction = R (f - A phi) and prolongation = phi + P pc with the dense periodic
    operator A = -L_h and the textbook transfer matrices, on several boxes."""
    nx, ny, nz = shape
    h2 = (1.0 / 8) ** 2
    phi0 = I.uniform(shape, 1, seed=31)[0]
    f = I.uniform(shape, 1, seed=32)[0] - 0.5
    A = _dense_minus_laplacian(shape, h2)
    R, P = _dense_transfer(shape)
    boxes = I.regular_chop(I.domain_box(shape), (nx // 2, ny // 2, 2))
    phi, fm = _mf(boxes, shape), _mf(boxes, shape)
    phi.load_global(phi0[None])
    fm.load_global(f[None])
    cshape = (nx // 2, ny // 2, nz // 2)
    fc = O.OracleMultiFab(O.coarsen_boxes(boxes), I.domain_box(cshape), (1, 1, 1), 1, 1)
    O.restrict_residual(phi, fm, h2, fc)
    expect = R @ (f.ravel() - A @ phi0.ravel())
    got = fc.to_global()[0].ravel()
    assert np.abs(got - expect).max() <= 1e-12 * np.abs(A).max() * np.abs(phi0).max()
    pc = I.uniform(cshape, 1, seed=33)[0]
    fc.load_global(pc[None])
    O.prolong_add(phi, fc)
    assert np.array_equal(phi.to_global()[0].ravel(), phi0.ravel() + P @ pc.ravel())


def test_mg_levels_follow_the_coarsening_rule():
    dom = I.domain_box(256)
    lv = O.mg_level_boxes(I.regular_chop(dom, 64), dom, (1, 1, 1), 32)
    assert len(lv) == 7  # boxes 64 -> 1, domain 256 -> 4
    assert np.array_equal(lv[-1][1], [0, 0, 0, 3, 3, 3]) and len(lv[-1][0]) == 64
    assert np.all(lv[-1][0][:, 3:] == lv[-1][0][:, :3])  # single cells
    assert len(O.mg_level_boxes(I.regular_chop(dom, 64), dom, (1, 1, 1), 3)) == 3
    odd = I.domain_box((12, 8, 8))
    assert len(O.mg_level_boxes(I.regular_chop(odd, (3, 4, 4)), odd, (1, 1, 1), 32)) == 1  # odd box edges
    six = I.domain_box((12, 16, 16))  # 12 -> 6 -> 3: the periodic x axis stops at 6
    assert len(O.mg_level_boxes(I.regular_chop(six, (12, 16, 16)), six, (1, 1, 1), 32)) == 2
    assert len(O.mg_level_boxes(I.regular_chop(six, (12, 16, 16)), six, (0, 1, 1), 32)) == 3


def _sine_problem(n):
    """A zero-mean eigenvector of -L_h (cell-centred, periodic) and f = lambda * phi*."""
    h2 = (1.0 / n) ** 2
    k = (1, 2, 3)
    x = (np.arange(n) + 0.5) / n
    sx, sy, sz = (np.sin(2 * np.pi * kd * x) for kd in k)
    star = sz[:, None, None] * sy[None, :, None] * sx[None, None, :]
    lam = sum(4.0 * np.sin(np.pi * kd / n) ** 2 for kd in k) / h2
    return star, lam * star, h2


@pytest.mark.parametrize("chop", ["one_box", "boxes_of_8", "uneven"])
def test_mg_converges_to_the_discrete_sine_solution(chop):
    """V(2,2) cycles reach the exact discrete solution of -L_h phi = lambda phi* (up to the
    constant null mode), the residual falling by at least 5x per cycle."""
    n = 32
    dom = I.domain_box(n)
    boxes = {"one_box": I.regular_chop(dom, n), "boxes_of_8": I.regular_chop(dom, 8),
             "uneven": I.random_chop(dom, 8, 16, 8, seed=3)}[chop]
    star, f, h2 = _sine_problem(n)
    phi, fm = _mf(boxes, n), _mf(boxes, n)
    fm.load_global(f[None])
    r0 = O.residual_norm(phi, fm, h2)
    norms = O.mg_vcycles(phi, fm, h2, 10, 2, 2, 16)
    rates = [b / a for a, b in zip([r0] + norms, norms)]
    assert max(rates[:6]) <= 0.2, rates
    got = phi.to_global()[0]
    err = np.abs(got - got.mean() - star).max()
    assert err <= 1e-8, err


def test_mg_vcycle_is_decomposition_invariant():
    """The same level count on one box, regular boxes and an uneven chop gives the same
    bits after two cycles (every step is local per cell, or a fill)."""
    n = 32
    dom = I.domain_box(n)
    f = I.zero_mean_normal_f32(n, seed=5)
    h2 = (1.0 / n) ** 2
    outs = []
    for boxes in (I.regular_chop(dom, n), I.regular_chop(dom, 16), I.random_chop(dom, 8, 16, 8, seed=2)):
        phi, fm = _mf(boxes, n), _mf(boxes, n)
        fm.load_global(f)
        O.mg_vcycles(phi, fm, h2, 2, 2, 2, 8, max_levels=4)
        outs.append(phi.to_global())
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])


# ---------------------------------------------------------------------------------------------
# The 8th-order heat step (9-cell span, 4 ghost layers)
# ---------------------------------------------------------------------------------------------
H8 = (-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0)


def _h8_symbol(theta):
    """Eigenvalue (times h^2) of the 8th-order second difference on exp(i theta x)."""
    return H8[0] + 2.0 * sum(H8[m] * math.cos(m * theta) for m in range(1, 5))


def _h8_sine_error(shape=(32, 24, 16), steps=12, boxes=None):
    nx, ny, nz = shape
    c = 0.09
    modes = [(0.7, (1, 2, 3)), (0.3, (5, 1, 2))]
    u0 = np.zeros((1, nz, ny, nx))
    exact = np.zeros_like(u0)
    for amp, k in modes:
        phi = I.sine_product(shape, k)
        g = 1.0 + c * sum(_h8_symbol(2 * math.pi * k[d] / shape[d]) for d in range(3))
        u0[0] += amp * phi
        exact[0] += amp * g ** steps * phi
    if boxes is None:
        boxes = I.random_chop(I.domain_box(shape), min_edge=4, max_edge=16, align=4, seed=3)
    m = _mf(boxes, shape, ng=4)
    m.load_global(u0)
    out = O.heat8_advance(m, steps, c).to_global()
    return np.abs(out - exact).max() / np.abs(exact).max()


def test_heat8_sine_modes_decay_by_the_stencil_symbol():
    assert _h8_sine_error() <= 1e-12
    assert _h8_sine_error(boxes=I.regular_chop(I.domain_box((32, 24, 16)), 8)) <= 1e-12


def test_heat8_is_eighth_order():
    """One step of a smooth field recovers the exact Laplacian with an error that falls
    by 2^8 when the grid is refined: the coefficients are those of the 8th-order formula."""
    errs = []
    for n in (16, 32):
        x = (np.arange(n) + 0.5) / n
        u = np.sin(2 * np.pi * x)[None, None, None, :] * np.ones((1, 8, 8, 1))
        m = _mf(I.regular_chop(I.domain_box((n, 8, 8)), (n // 2, 8, 8)), (n, 8, 8), ng=4)
        m.load_global(u)
        c = 0.05
        out = O.heat8_advance(m, 1, c).to_global()
        lap = (out - u) / c * (n * n)  # (u_new - u) / (c h^2) = L_h u
        exact = -(2 * np.pi) ** 2 * u
        errs.append(np.abs(lap - exact).max())
    assert 200 <= errs[0] / errs[1] <= 300, errs


def _h8_roll(u, c):
    D = []
    for axis in (2, 1, 0):
        p = [None] + [np.roll(u, mm, axis=axis) + np.roll(u, -mm, axis=axis) for mm in range(1, 5)]
        D.append(((8.0 / 5.0 * p[1] + -1.0 / 5.0 * p[2]) + 8.0 / 315.0 * p[3]) + -1.0 / 560.0 * p[4])
    return u + c * (((D[0] + D[1]) + D[2]) + (-205.0 / 24.0) * u)


def test_heat8_single_periodic_box_equals_numpy_roll():
    shape = (12, 10, 9)
    u = I.uniform(shape, 1, seed=41)[0]
    m = _mf(I.regular_chop(I.domain_box(shape), shape), shape, ng=4)
    m.load_global(u[None])
    ref = u
    for _ in range(3):
        ref = _h8_roll(ref, 0.09)
    assert np.array_equal(O.heat8_advance(m, 3, 0.09).to_global()[0], ref)


def test_heat8_many_boxes_equal_one_box_and_conserve_the_sum():
    shape = (24, 20, 16)
    u = I.uniform(shape, 2, seed=42)
    outs = []
    for boxes in (I.regular_chop(I.domain_box(shape), shape), I.random_chop(I.domain_box(shape), 4, 12, 4, seed=8)):
        m = _mf(boxes, shape, ncomp=2, ng=4)
        m.load_global(u)
        outs.append(O.heat8_advance(m, 4, 0.09).to_global())
    assert np.array_equal(outs[0], outs[1])
    for comp in range(2):
        assert abs(outs[0][comp].sum() - u[comp].sum()) <= 1e-12 * u[comp].sum()


def test_heat8_window_equals_full_run():
    n, steps = 24, 3
    u0 = I.uniform(n, 1, seed=43)
    m = _mf(I.random_chop(I.domain_box(n), 4, 12, 4, seed=1), n, ng=4)
    m.load_global(u0)
    full = O.heat8_advance(m, steps, 0.09).to_global()[0]
    rng = np.random.default_rng(4)
    for cell in [(0, 0, 0), (23, 11, 5)] + [tuple(int(v) for v in rng.integers(0, n, 3)) for _ in range(4)]:
        i, j, k = cell
        assert O.heat8_window(u0[0], cell, steps, 0.09) == full[k, j, i]


MUTATIONS = {
    "heat_drops_z_pair": ("double s = (sx + sy) + sz;\n            v[", "double s = (sx + sy);\n            v["),
    "heat_wrong_sign": ("uc + c * (s - 6.0 * uc)", "uc - c * (s - 6.0 * uc)"),
    "heat_shifted_index": ("u[fab_index(&g, comp, i, j - 1, k)] + u[fab_index(&g, comp, i, j + 1, k)]",
                           "u[fab_index(&g, comp, i, j - 1, k)] + u[fab_index(&g, comp, i, j + 2, k)]"),
    "layout_transposed": ("return (((int64_t)comp * g->nz + lk) * g->ny + lj) * g->nx + li;",
                          "return (((int64_t)comp * g->nz + lk) * g->nx + li) * g->ny + lj;"),
    "fill_no_wrap": ("if (periodic[d]) p[d] = lo[d] + floor_mod(p[d] - lo[d], N[d]);", ""),
    "gsrb_black_first": ("if (floor_mod(i + j + k, 2) != color) continue;",
                         "if (floor_mod(i + j + k + 1, 2) != color) continue;"),
    "gsrb_drops_rhs": ("p[q] = (((sx + sy) + sz) + h2 * fb[q]) * inv6;", "p[q] = (((sx + sy) + sz)) * inv6;"),
    "varcoef_cell_coefficient": ("const double b = 0.5 * (bt[lo] + bt[hi]);", "const double b = bt[hi];"),
    "varcoef_flux_sign": ("return b * ((u[hi] - u[lo]) * inv_dx);", "return b * ((u[lo] - u[hi]) * inv_dx);"),
    "varcoef_harmonic_mean": ("const double b = 0.5 * (bt[lo] + bt[hi]);",
                              "const double b = 2.0 * bt[lo] * bt[hi] / (bt[lo] + bt[hi]);"),
    "heat8_swapped_coefficients": ("H8_A3 = 8.0 / 315.0, H8_A4 = -1.0 / 560.0;", "H8_A3 = -1.0 / 560.0, H8_A4 = 8.0 / 315.0;"),
    "heat8_drops_far_y": ("u[fab_index(&g, comp, i, j - m, k)] + u[fab_index(&g, comp, i, j + m, k)]",
                          "u[fab_index(&g, comp, i, j - m, k)] + u[fab_index(&g, comp, i, j + (m < 4 ? m : 0), k)]"),
    "heat8_centre": ("static const double H8_A0X3 = -205.0 / 24.0;", "static const double H8_A0X3 = -205.0 / 36.0;"),
    "mg_restrict_weight": ("out[fab_index(&gc, 0, I, J, K)] = acc * 0.125;", "out[fab_index(&gc, 0, I, J, K)] = acc * 0.25;"),
    "mg_restrict_drops_children": ("residual_at(p, fb, &gf, 2 * I + a, 2 * J + bb, 2 * K + c, h2)",
                                   "residual_at(p, fb, &gf, 2 * I + a, 2 * J, 2 * K + c, h2)"),
    "mg_residual_sign": ("return fb[q] + (((sx + sy) + sz) - 6.0 * p[q]) / h2;",
                         "return fb[q] - (((sx + sy) + sz) - 6.0 * p[q]) / h2;"),
    "mg_prolong_parent": ("floor_half(i), floor_half(j), floor_half(k))", "floor_half(i + 1), floor_half(j), floor_half(k))"),
    "fsum_drops_errors": ("if (lo != 0.0) p[m++] = lo;", "(void)lo;"),
    "fsum_no_tie_correction": ("if (y == x - hi) hi = x;", "(void)x;"),
}


def _pins_pass():
    checks = []
    try:
        checks.append(_sine_decay_error() <= 1e-12)
        test_single_periodic_box_equals_numpy_roll()
        test_many_boxes_equal_numpy_roll()
        test_fill_boundary_brute_force(1)
        test_gsrb_equals_dense_gauss_seidel_red_then_black((4, 4, 4))
        test_gsrb_exact_discrete_solution_is_fixed_point()
        test_varcoef_is_second_order_with_the_mean_face_coefficient()
        test_mg_transfers_equal_dense_matrices((4, 4, 4))
        checks.append(_h8_sine_error() <= 1e-12)
        test_heat8_is_eighth_order()
        test_mg_converges_to_the_discrete_sine_solution("boxes_of_8")
        test_fsum_is_the_exactly_rounded_sum()
    except (AssertionError, ValueError, IndexError):
        return False
    return all(checks)


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistakes_are_caught(name, tmp_path):
    old, new = MUTATIONS[name]
    src = O.source()
    assert src.count(old) >= 1, "mutation anchor not found"
    with O.variant(src.replace(old, new), str(tmp_path)):
        assert not _pins_pass(), f"pins did not catch planted mistake {name}"


def test_unmodified_oracle_passes_the_mutation_harness():
    assert _pins_pass()
