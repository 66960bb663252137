"""Plain FP64 CPU oracle for the single-level BoxLib hot path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the package smoke check and the
CPU-baseline leg of the benchmark import this module; the product library and
its Python binding never do.  It shares no code with the GPU path: the box
geometry, the FAB layout and every update below are written here again, from
the paper and the plain mathematical definitions.

The arithmetic lives in ``boxlib_oracle.c`` (plain C, compiled with
``-O2 -ffp-contract=off``); this module holds the oracle's own MultiFab (one
float64 numpy buffer, FABs contiguous, x fastest then y, z, component), calls
the C routines box by box, and computes reductions as exactly rounded sums
(Shewchuk's adaptive expansions, ``orc_fsum``: the same number as ``math.fsum``),
so that sums do not depend on order or decomposition.

Citations are to the paper "BoxLib with Tiling: An AMR Software Framework":
  Sec. 3.1  Box (six integers), FArrayBox (contiguous multi-component data on a
            box grown by ghost cells), MultiFab (the FABs of one level),
            ``mf.max(comp)`` and ``mf.FillBoundary()``.
  Sec. 3.3  ghost-cell filling by local copies.
  Sec. 4.1  the heat test: forward Euler, second-order centred differences,
            periodic boundaries; flux loops followed by a divergence loop.
The red-black Gauss-Seidel smoother is not written out in the paper (which only
names multigrid solvers, Sec. 1 and Sec. 3.3); it is the textbook method for
the 7-point discrete Poisson problem, as stated on each routine.
"""
from __future__ import annotations

import contextlib
import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "boxlib_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (plain, no FMA contraction, OpenMP over boxes)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _configure(L):
    L.orc_num_threads.restype = ctypes.c_int
    L.orc_set_num_threads.argtypes = [ctypes.c_int]
    L.orc_set_num_threads.restype = None
    L.orc_owner_map.argtypes = [ctypes.c_int, _ip, _ip, _i32p]
    L.orc_owner_map.restype = ctypes.c_int
    L.orc_fill_boundary.argtypes = [ctypes.c_int, _ip, _ip, _ip, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_int, _dp, _i64p, _dp, _i32p]
    L.orc_fill_boundary.restype = None
    L.orc_heat_step.argtypes = [ctypes.c_int, _ip, ctypes.c_int, ctypes.c_int, _dp, _dp, _i64p,
                                ctypes.c_double]
    L.orc_heat_step.restype = None
    L.orc_heat_flux_step.argtypes = [ctypes.c_int, _ip, ctypes.c_int, ctypes.c_int, _dp, _dp,
                                     _i64p, ctypes.c_double, ctypes.c_double]
    L.orc_heat_flux_step.restype = ctypes.c_int
    L.orc_heat_varcoef_step.argtypes = [ctypes.c_int, _ip, ctypes.c_int, ctypes.c_int, _dp, _dp, _dp, _i64p,
                                        ctypes.c_double, ctypes.c_double]
    L.orc_heat_varcoef_step.restype = None
    L.orc_gsrb_color.argtypes = [ctypes.c_int, _ip, ctypes.c_int, _dp, _dp, _i64p,
                                 ctypes.c_double, ctypes.c_double, ctypes.c_int]
    L.orc_gsrb_color.restype = None
    L.orc_residual.argtypes = [ctypes.c_int, _ip, ctypes.c_int, _dp, _dp, _i64p,
                               ctypes.c_double, _dp]
    L.orc_residual.restype = None
    L.orc_restrict_residual.argtypes = [ctypes.c_int, _ip, _ip, ctypes.c_int, _dp, _dp, _i64p, _dp, _i64p,
                                        ctypes.c_double]
    L.orc_restrict_residual.restype = None
    L.orc_prolong_add.argtypes = [ctypes.c_int, _ip, _ip, ctypes.c_int, _dp, _i64p, _dp, _i64p]
    L.orc_prolong_add.restype = None
    L.orc_heat8_step.argtypes = [ctypes.c_int, _ip, ctypes.c_int, ctypes.c_int, _dp, _dp, _i64p, ctypes.c_double]
    L.orc_heat8_step.restype = None
    L.orc_heat_window.argtypes = [_dp, _dp, ctypes.c_int, ctypes.c_double]
    L.orc_heat_window.restype = ctypes.c_double
    L.orc_fsum.argtypes = [_dp, ctypes.c_int64]
    L.orc_fsum.restype = ctypes.c_double
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = _configure(ctypes.CDLL(_LIB))
    return _lib


@contextlib.contextmanager
def variant(source: str, workdir: str):
    """Use an oracle compiled from ``source`` (a modified copy of boxlib_oracle.c)
    inside the block.  Exists so that tests can plant a mistake in the oracle and
    show that the pins catch it."""
    global _lib
    path_c = os.path.join(workdir, "oracle_variant.c")
    path_so = os.path.join(workdir, "liboracle_variant.so")
    with open(path_c, "w") as fh:
        fh.write(source)
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                           "-o", path_so, path_c])
    saved = lib()
    _lib = _configure(ctypes.CDLL(path_so))
    try:
        yield
    finally:
        _lib = saved


def source() -> str:
    with open(_SRC) as fh:
        return fh.read()


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the box loops from here on (results do not depend on it)."""
    lib().orc_set_num_threads(int(n))


def _ptr(a, t):
    return a.ctypes.data_as(t)


class OracleMultiFab:
    """The oracle's MultiFab: FABs of one level on a list of disjoint boxes (Sec. 3.1).

    boxes    : (nbox, 6) int array of inclusive {lo[3], hi[3]} cell indices
    domain   : 6 ints, the level's domain box
    periodic : 3 flags
    ncomp, ng: components and ghost cells per FAB
    FAB b holds its box grown by ng cells, all ncomp components, contiguous,
    x fastest, then y, z, component.
    """

    def __init__(self, boxes, domain, periodic, ncomp: int, ng: int):
        self.boxes = np.ascontiguousarray(np.asarray(boxes, dtype=np.int32).reshape(-1, 6))
        self.domain = np.ascontiguousarray(np.asarray(domain, dtype=np.int32).reshape(6))
        self.periodic = np.ascontiguousarray(np.asarray(periodic, dtype=np.int32).reshape(3))
        self.ncomp, self.ng = int(ncomp), int(ng)
        self.nbox = self.boxes.shape[0]
        ext = self.boxes[:, 3:] - self.boxes[:, :3] + 1 + 2 * self.ng
        self.shapes = [(self.ncomp, int(e[2]), int(e[1]), int(e[0])) for e in ext]
        sizes = np.array([int(np.prod(s)) for s in self.shapes], dtype=np.int64)
        self.fab_off = np.ascontiguousarray(np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64))
        self.data = np.zeros(int(sizes.sum()), dtype=np.float64)
        N = self.domain[3:] - self.domain[:3] + 1
        self.N = tuple(int(n) for n in N)
        self._owner = None
        self._G = None

    # -- views ---------------------------------------------------------------
    def fab(self, b: int) -> np.ndarray:
        """View of FAB b as (comp, z, y, x) over the grown box."""
        n = int(np.prod(self.shapes[b]))
        return self.data[self.fab_off[b]:self.fab_off[b] + n].reshape(self.shapes[b])

    def valid(self, b: int) -> np.ndarray:
        g = self.ng
        f = self.fab(b)
        return f[:, g:f.shape[1] - g, g:f.shape[2] - g, g:f.shape[3] - g]

    def _owner_map(self):
        if self._owner is None:
            owner = np.empty(int(np.prod(self.N)), dtype=np.int32)
            rc = lib().orc_owner_map(self.nbox, _ptr(self.boxes, _ip), _ptr(self.domain, _ip),
                                     _ptr(owner, _i32p))
            if rc != 0:
                raise ValueError("boxes overlap or leave the domain")
            self._owner = owner
        return self._owner

    # -- data in and out, in global (comp, z, y, x) order ---------------------
    def load_global(self, g: np.ndarray) -> None:
        """Set the valid cells from a global array of shape (ncomp, Nz, Ny, Nx)."""
        lo = self.domain[:3]
        for b in range(self.nbox):
            bx = self.boxes[b]
            self.valid(b)[...] = g[:, bx[2] - lo[2]:bx[5] - lo[2] + 1, bx[1] - lo[1]:bx[4] - lo[1] + 1,
                                   bx[0] - lo[0]:bx[3] - lo[0] + 1]

    def to_global(self, fill=np.nan) -> np.ndarray:
        """Valid cells as a global array; cells no box covers hold ``fill``."""
        lo = self.domain[:3]
        g = np.full((self.ncomp,) + self.N[::-1], fill, dtype=np.float64)
        for b in range(self.nbox):
            bx = self.boxes[b]
            g[:, bx[2] - lo[2]:bx[5] - lo[2] + 1, bx[1] - lo[1]:bx[4] - lo[1] + 1,
              bx[0] - lo[0]:bx[3] - lo[0] + 1] = self.valid(b)
        return g

    def copy(self) -> "OracleMultiFab":
        m = OracleMultiFab(self.boxes, self.domain, self.periodic, self.ncomp, self.ng)
        m.data[...] = self.data
        m._owner = self._owner
        return m

    # -- Sec. 3.1 / 3.3: FillBoundary with periodic wrap -------------------------
    def fill_boundary(self, scomp: int = 0, ncomp: int | None = None) -> None:
        ncomp = self.ncomp - scomp if ncomp is None else ncomp
        owner = self._owner_map()
        if self._G is None:
            self._G = np.empty(int(np.prod(self.N)), dtype=np.float64)
        lib().orc_fill_boundary(self.nbox, _ptr(self.boxes, _ip), _ptr(self.domain, _ip),
                                _ptr(self.periodic, _ip), self.ng, scomp, ncomp,
                                _ptr(self.data, _dp), _ptr(self.fab_off, _i64p), _ptr(self._G, _dp),
                                _ptr(owner, _i32p))


def _same_layout(a: OracleMultiFab, b: OracleMultiFab) -> None:
    if a.ncomp != b.ncomp or a.ng != b.ng or not np.array_equal(a.boxes, b.boxes):
        raise ValueError("MultiFabs differ in boxes, components or ghost width")


# -- Sec. 4.1: forward-Euler heat step ------------------------------------------
def heat_step(u_old: OracleMultiFab, u_new: OracleMultiFab, c: float, fill_first: bool = True) -> None:
    """One heat step, u_new = u + c*(sum of 6 neighbours - 6u), c = dt/dx^2, after FillBoundary(u_old)."""
    _same_layout(u_old, u_new)
    if fill_first:
        u_old.fill_boundary()
    lib().orc_heat_step(u_old.nbox, _ptr(u_old.boxes, _ip), u_old.ng, u_old.ncomp,
                        _ptr(u_old.data, _dp), _ptr(u_new.data, _dp), _ptr(u_old.fab_off, _i64p), c)


def heat_flux_step(u_old: OracleMultiFab, u_new: OracleMultiFab, dt: float, dx: float) -> None:
    """The paper's structure of the same step: face-flux loops, then a divergence loop (Sec. 4.1);
    differences are multiplied by 1/dx, formed once here."""
    _same_layout(u_old, u_new)
    u_old.fill_boundary()
    rc = lib().orc_heat_flux_step(u_old.nbox, _ptr(u_old.boxes, _ip), u_old.ng, u_old.ncomp,
                                  _ptr(u_old.data, _dp), _ptr(u_new.data, _dp),
                                  _ptr(u_old.fab_off, _i64p), dt, 1.0 / dx)
    if rc != 0:
        raise MemoryError("flux scratch")


def heat_varcoef_step(u_old: OracleMultiFab, u_new: OracleMultiFab, beta: OracleMultiFab, dt: float,
                      dx: float) -> None:
    """du/dt = div(beta grad u) in the flux form, face coefficients the mean of the two
    cells (Sec. 4.1's flux form with a variable coefficient), differences multiplied by
    1/dx formed once here; fills u_old's and beta's ghosts first."""
    _same_layout(u_old, u_new)
    _same_layout(u_old, beta)
    u_old.fill_boundary()
    beta.fill_boundary()
    lib().orc_heat_varcoef_step(u_old.nbox, _ptr(u_old.boxes, _ip), u_old.ng, u_old.ncomp, _ptr(u_old.data, _dp),
                                _ptr(beta.data, _dp), _ptr(u_new.data, _dp), _ptr(u_old.fab_off, _i64p), dt,
                                1.0 / dx)


def heat_varcoef_advance(u: OracleMultiFab, beta: OracleMultiFab, nsteps: int, dt: float,
                         dx: float) -> OracleMultiFab:
    a, b = u, u.copy()
    for _ in range(nsteps):
        heat_varcoef_step(a, b, beta, dt, dx)
        a, b = b, a
    return a


def heat_varcoef_window(u0_global: np.ndarray, beta_global: np.ndarray, center, nsteps: int, dt: float,
                        dx: float) -> float:
    """Value at global cell ``center`` = (i, j, k) after nsteps heat_varcoef_step steps of a
    fully periodic, fully covered single component (Nz, Ny, Nx) pair u0, beta.  The cube of
    half-width nsteps around the cell, cut out with periodic wrap, becomes the one box of a
    non-periodic domain whose ghost layer holds the wrapped neighbours and stays fixed; a
    fixed ghost first changes a result in step 2 and then moves in one cell per step, so
    after nsteps steps the cells within distance 1 of the centre are exact."""
    i, j, k = center
    n = int(nsteps)
    Nz, Ny, Nx = u0_global.shape
    h = n + 1
    ix = np.arange(i - h, i + h + 1) % Nx
    iy = np.arange(j - h, j + h + 1) % Ny
    iz = np.arange(k - h, k + h + 1) % Nz
    m = 2 * n + 1
    box = np.array([[0, 0, 0, m - 1, m - 1, m - 1]], dtype=np.int64)
    u = OracleMultiFab(box, box[0], (0, 0, 0), 1, 1)
    beta = OracleMultiFab(box, box[0], (0, 0, 0), 1, 1)
    u.fab(0)[0] = u0_global[np.ix_(iz, iy, ix)]
    beta.fab(0)[0] = beta_global[np.ix_(iz, iy, ix)]
    res = heat_varcoef_advance(u, beta, n, dt, dx)
    return float(res.fab(0)[0, h, h, h])


def heat_advance(u: OracleMultiFab, nsteps: int, c: float) -> OracleMultiFab:
    """nsteps heat steps with ping-pong buffers; returns the MultiFab holding the result."""
    a, b = u, u.copy()
    for _ in range(nsteps):
        heat_step(a, b, c)
        a, b = b, a
    return a


# -- the 8th-order heat step (9-cell span, ng >= 4) ------------------------------------
H8_COEF = (-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0)  # centre, then m = 1..4


def heat8_step(u_old: OracleMultiFab, u_new: OracleMultiFab, c: float) -> None:
    """FillBoundary(u_old), then the 8th-order step on every valid cell (needs ng >= 4)."""
    _same_layout(u_old, u_new)
    if u_old.ng < 4:
        raise ValueError("the 8th-order stencil needs 4 ghost layers")
    u_old.fill_boundary()
    lib().orc_heat8_step(u_old.nbox, _ptr(u_old.boxes, _ip), u_old.ng, u_old.ncomp, _ptr(u_old.data, _dp),
                         _ptr(u_new.data, _dp), _ptr(u_old.fab_off, _i64p), c)


def heat8_advance(u: OracleMultiFab, nsteps: int, c: float) -> OracleMultiFab:
    a, b = u, u.copy()
    for _ in range(nsteps):
        heat8_step(a, b, c)
        a, b = b, a
    return a


def heat8_window(u0_global: np.ndarray, center, nsteps: int, c: float) -> float:
    """Value at global cell ``center`` after nsteps 8th-order steps of a fully periodic,
    fully covered single component (Nz, Ny, Nx) array: the cube of half-width 4*nsteps
    around the cell (periodic wrap) as the one box of a non-periodic domain whose 4 ghost
    layers hold the wrapped neighbours and stay fixed.  A fixed ghost first changes a
    result in step 2 and moves in 4 cells per step, so the centre is exact."""
    i, j, k = center
    n = int(nsteps)
    Nz, Ny, Nx = u0_global.shape
    h = 4 * n + 4
    ix = np.arange(i - h, i + h + 1) % Nx
    iy = np.arange(j - h, j + h + 1) % Ny
    iz = np.arange(k - h, k + h + 1) % Nz
    m = 8 * n + 1
    box = np.array([[0, 0, 0, m - 1, m - 1, m - 1]], dtype=np.int64)
    u = OracleMultiFab(box, box[0], (0, 0, 0), 1, 4)
    u.fab(0)[0] = u0_global[np.ix_(iz, iy, ix)]
    res = heat8_advance(u, n, c)
    return float(res.fab(0)[0, h, h, h])


def heat_window(u0_global: np.ndarray, center, nsteps: int, c: float) -> float:
    """Value at global cell ``center`` = (i, j, k) after nsteps heat steps of a fully
    periodic, fully covered single component (Nz, Ny, Nx) array: the cube of
    half-width nsteps around the cell is cut out with periodic wrap and advanced
    on shrinking windows with the same per-cell expression as heat_step."""
    i, j, k = center
    n = int(nsteps)
    Nz, Ny, Nx = u0_global.shape
    ix = np.arange(i - n, i + n + 1) % Nx
    iy = np.arange(j - n, j + n + 1) % Ny
    iz = np.arange(k - n, k + n + 1) % Nz
    w = np.ascontiguousarray(u0_global[np.ix_(iz, iy, ix)], dtype=np.float64)
    if n == 0:
        return float(w[0, 0, 0])
    tmp = np.empty_like(w)
    return float(lib().orc_heat_window(_ptr(w, _dp), _ptr(tmp, _dp), n, c))


# -- red-black Gauss-Seidel for -L_h phi = f (textbook; multigrid smoother) ----------
def gsrb_color(phi: OracleMultiFab, f: OracleMultiFab, h2: float, color: int) -> None:
    """Fill phi's ghosts, then solve every cell of one colour exactly, in place."""
    _same_layout(phi, f)
    if phi.ncomp != 1:
        raise ValueError("GSRB acts on one component")
    phi.fill_boundary()
    lib().orc_gsrb_color(phi.nbox, _ptr(phi.boxes, _ip), phi.ng, _ptr(phi.data, _dp),
                         _ptr(f.data, _dp), _ptr(phi.fab_off, _i64p), h2, 1.0 / 6.0, int(color))


def residual(phi: OracleMultiFab, f: OracleMultiFab, h2: float, fill_first: bool = True) -> np.ndarray:
    """r = f + L_h phi on the valid cells (FP64), box after box, each in (k, j, i) order."""
    _same_layout(phi, f)
    if fill_first:
        phi.fill_boundary()
    n = int(sum(np.prod(phi.boxes[b, 3:] - phi.boxes[b, :3] + 1) for b in range(phi.nbox)))
    r = np.empty(n, dtype=np.float64)
    lib().orc_residual(phi.nbox, _ptr(phi.boxes, _ip), phi.ng, _ptr(phi.data, _dp),
                       _ptr(f.data, _dp), _ptr(phi.fab_off, _i64p), h2, _ptr(r, _dp))
    return r


def fsum(values) -> float:
    """The exactly rounded sum of finite values (the same number as ``math.fsum``:
    the real sum rounded once, ties to even), computed in C by Shewchuk's adaptive
    expansions so that sums over whole levels take seconds, not minutes."""
    a = np.ascontiguousarray(values, dtype=np.float64).ravel()
    s = float(lib().orc_fsum(_ptr(a, _dp), a.size))
    if math.isnan(s):
        raise ValueError("fsum of non-finite values")
    return s


def residual_norm(phi: OracleMultiFab, f: OracleMultiFab, h2: float) -> float:
    """||r||_2 = sqrt(sum r^2) with the sum exactly rounded."""
    r = residual(phi, f, h2)
    return math.sqrt(fsum(r * r))


# -- multigrid V-cycle for -L_h phi = f (textbook geometric multigrid; the paper names
#    multigrid solvers and their coarse levels of small grids, Sec. 1 and Sec. 3.3) ------
def coarsen_boxes(boxes) -> np.ndarray:
    """Boxes coarsened by 2: lo/2 .. (hi+1)/2 - 1 (every lo and extent must be even)."""
    b = np.asarray(boxes, dtype=np.int64).reshape(-1, 6)
    return np.concatenate([b[:, :3] // 2, (b[:, 3:] + 1) // 2 - 1], axis=1)


def mg_level_boxes(boxes, domain, periodic, max_levels: int):
    """The levels of the hierarchy: level 0 is (boxes, domain); level l+1 is level l
    coarsened by 2, made while every box and the domain have even lo and even extents
    and every periodic axis of the coarse domain keeps an even extent (red-black
    colouring across the wrap), up to max_levels levels."""
    levels = [(np.asarray(boxes, dtype=np.int64).reshape(-1, 6), np.asarray(domain, dtype=np.int64).reshape(6))]
    while len(levels) < max_levels:
        b, d = levels[-1]
        allb = np.concatenate([b, d[None]], axis=0)
        if np.any(allb[:, :3] % 2) or np.any((allb[:, 3:] - allb[:, :3] + 1) % 2):
            break
        cd = coarsen_boxes(d)[0]
        if any(periodic[a] and (cd[3 + a] - cd[a] + 1) % 2 for a in range(3)):
            break
        levels.append((coarsen_boxes(b), cd))
    return levels


def restrict_residual(phi: OracleMultiFab, f: OracleMultiFab, h2: float, fc: OracleMultiFab) -> None:
    """fc (on the coarsened boxes) = mean of the 8 fine residuals of each coarse cell; fills
    phi's ghosts first."""
    _same_layout(phi, f)
    if fc.nbox != phi.nbox or not np.array_equal(fc.boxes, coarsen_boxes(phi.boxes)) or fc.ng != phi.ng:
        raise ValueError("fc must live on the coarsened boxes with the same ghost width")
    phi.fill_boundary()
    lib().orc_restrict_residual(phi.nbox, _ptr(phi.boxes, _ip), _ptr(fc.boxes, _ip), phi.ng, _ptr(phi.data, _dp),
                                _ptr(f.data, _dp), _ptr(phi.fab_off, _i64p), _ptr(fc.data, _dp),
                                _ptr(fc.fab_off, _i64p), h2)


def prolong_add(phi: OracleMultiFab, pc: OracleMultiFab) -> None:
    """phi (valid cells) += the value of the coarse cell containing each cell."""
    if pc.nbox != phi.nbox or not np.array_equal(pc.boxes, coarsen_boxes(phi.boxes)) or pc.ng != phi.ng:
        raise ValueError("pc must live on the coarsened boxes with the same ghost width")
    lib().orc_prolong_add(phi.nbox, _ptr(phi.boxes, _ip), _ptr(pc.boxes, _ip), phi.ng, _ptr(phi.data, _dp),
                          _ptr(phi.fab_off, _i64p), _ptr(pc.data, _dp), _ptr(pc.fab_off, _i64p))


def _smooth(phi: OracleMultiFab, f: OracleMultiFab, h2: float, nsweeps: int) -> None:
    for _ in range(nsweeps):
        gsrb_color(phi, f, h2, 0)
        gsrb_color(phi, f, h2, 1)


def mg_vcycles(phi: OracleMultiFab, f: OracleMultiFab, h2: float, ncycles: int, nu1: int = 2, nu2: int = 2,
               nu_bottom: int = 8, max_levels: int = 32):
    """ncycles V-cycles on -L_h phi = f, phi updated in place; returns the residual norm
    after each cycle.  On level l (h^2 = 4^l h2): nu1 GSRB sweeps, the residual
    restricted to level l+1 as its f, phi there set to zero (ghosts too), the cycle on
    level l+1, the coarse phi added back by prolongation, nu2 sweeps.  The coarsest level
    takes nu_bottom sweeps.  Ghosts no box covers keep their value on level 0 and are 0
    on the coarse levels (the correction vanishes there)."""
    _same_layout(phi, f)
    if phi.ncomp != 1:
        raise ValueError("multigrid acts on one component")
    levels = mg_level_boxes(phi.boxes, phi.domain, phi.periodic, max_levels)
    P = [phi] + [OracleMultiFab(b, d, phi.periodic, 1, phi.ng) for b, d in levels[1:]]
    F = [f] + [OracleMultiFab(b, d, phi.periodic, 1, phi.ng) for b, d in levels[1:]]

    def cycle(l, h2l):
        if l == len(levels) - 1:
            _smooth(P[l], F[l], h2l, nu_bottom)
            return
        _smooth(P[l], F[l], h2l, nu1)
        restrict_residual(P[l], F[l], h2l, F[l + 1])
        P[l + 1].data[...] = 0.0
        cycle(l + 1, 4.0 * h2l)
        prolong_add(P[l], P[l + 1])
        _smooth(P[l], F[l], h2l, nu2)

    norms = []
    for _ in range(ncycles):
        cycle(0, h2)
        norms.append(residual_norm(phi, f, h2))
    return norms


def gsrb_sweeps(phi: OracleMultiFab, f: OracleMultiFab, h2: float, nsweeps: int,
                with_norms: bool = True, fill_per_color: bool = True):
    """nsweeps red-black sweeps (red = even i+j+k first), FillBoundary before each
    colour; after each sweep the residual norm is taken (with a fresh fill).
    ``fill_per_color=False`` fills only once per sweep (a deliberately wrong
    variant, kept to show that the second fill is needed)."""
    norms = []
    for _ in range(nsweeps):
        gsrb_color(phi, f, h2, 0)
        if fill_per_color:
            gsrb_color(phi, f, h2, 1)
        else:
            _same_layout(phi, f)
            lib().orc_gsrb_color(phi.nbox, _ptr(phi.boxes, _ip), phi.ng, _ptr(phi.data, _dp),
                                 _ptr(f.data, _dp), _ptr(phi.fab_off, _i64p), h2, 1.0 / 6.0, 1)
        if with_norms:
            norms.append(residual_norm(phi, f, h2))
    return norms


# -- Sec. 3.1: MultiFab reductions over valid cells ------------------------------
def reduce(mf: OracleMultiFab, comp: int, op: str) -> float:
    """sum / max / min / norm0 (max |u|) / norm1 (sum |u|) / norm2 (sqrt sum u^2) over valid cells."""
    vals = np.concatenate([mf.valid(b)[comp].ravel() for b in range(mf.nbox)])
    if op == "sum":
        return fsum(vals)
    if op == "max":
        return float(vals.max())
    if op == "min":
        return float(vals.min())
    if op == "norm0":
        return float(np.abs(vals).max())
    if op == "norm1":
        return fsum(np.abs(vals))
    if op == "norm2":
        return math.sqrt(fsum(vals * vals))
    raise ValueError(op)
