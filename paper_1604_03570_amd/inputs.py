"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds no arithmetic of the method itself (no fill, stencil, smoother
or reduction): only box decompositions, initial fields and request streams,
generated on the host in global order so that they do not depend on how a
domain is cut into boxes.  Both the CPU oracle and the GPU library receive what
it produces.

Random draws:
  * fields use numpy's PCG64 (``numpy.random.default_rng(seed)``) in global
    (comp, z, y, x) order;
  * the recursive box chop uses SplitMix64 as a counter-based generator
    (Steele, Lea and Flood, "Fast splittable pseudorandom number generators",
    OOPSLA 2014): draw n of seed s is mix(s + (n + 1) * 0x9E3779B97F4A7C15),
    so the library's C++ chop can produce the identical box list from the
    same seed.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

MASK64 = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15


def splitmix64(seed: int, n: int) -> int:
    """Draw n (n = 0, 1, ...) of the counter-based SplitMix64 stream of ``seed``."""
    z = (seed + (n + 1) * GOLDEN) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def unit_double(z: int) -> float:
    """Top 53 bits of a 64-bit draw as a double in [0, 1)."""
    return (z >> 11) * (1.0 / 9007199254740992.0)


# -- box decompositions -------------------------------------------------------------
def domain_box(n) -> tuple:
    """Domain [0, n-1] per axis; n is an int or three ints."""
    nx, ny, nz = (n, n, n) if np.isscalar(n) else tuple(n)
    return (0, 0, 0, nx - 1, ny - 1, nz - 1)


def regular_chop(domain, max_edge) -> np.ndarray:
    """Cut the domain into boxes of edge max_edge along each axis, from lo, with
    the remainder as the last box of an axis (e.g. 96 with 64 gives 64 + 32).
    Boxes are listed x fastest, then y, then z."""
    me = (max_edge,) * 3 if np.isscalar(max_edge) else tuple(max_edge)
    cuts = []
    for d in range(3):
        lo, hi = domain[d], domain[3 + d]
        e = max(1, min(me[d], hi - lo + 1))
        cuts.append([(a, min(a + e - 1, hi)) for a in range(lo, hi + 1, e)])
    out = []
    for (zl, zh) in cuts[2]:
        for (yl, yh) in cuts[1]:
            for (xl, xh) in cuts[0]:
                out.append((xl, yl, zl, xh, yh, zh))
    return np.array(out, dtype=np.int32)


def random_chop(domain, min_edge: int = 16, max_edge: int = 128, align: int = 8, seed: int = 0) -> np.ndarray:
    """Seeded recursive chop of the domain into uneven boxes.

    Depth first, low half first.  A box whose longest edge m satisfies m <= max_edge
    is kept if m < 2*min_edge, or else if a uniform draw is below 1/2.  Otherwise
    its longest axis (the lowest such axis on ties) is cut at an offset from the
    box's lower end chosen uniformly among {min_edge, min_edge+align, ...,
    m-min_edge} (draw mod the number of choices).  Every draw advances the
    SplitMix64 counter by one.
    """
    if min_edge < 1 or align < 1 or min_edge % align or max_edge < 2 * min_edge:
        raise ValueError("need min_edge % align == 0 and max_edge >= 2*min_edge")
    counter = [0]

    def draw() -> int:
        z = splitmix64(seed, counter[0])
        counter[0] += 1
        return z

    out = []
    stack = [tuple(int(v) for v in domain)]
    while stack:
        b = stack.pop()
        e = [b[3 + d] - b[d] + 1 for d in range(3)]
        m = max(e)
        if m <= max_edge and (m < 2 * min_edge or unit_double(draw()) < 0.5):
            out.append(b)
            continue
        axis = e.index(m)
        nchoice = (m - 2 * min_edge) // align + 1
        off = min_edge + align * (draw() % nchoice)
        lo_half = list(b)
        hi_half = list(b)
        lo_half[3 + axis] = b[axis] + off - 1
        hi_half[axis] = b[axis] + off
        stack.append(tuple(hi_half))  # popped after the low half: low half first
        stack.append(tuple(lo_half))
    return np.array(out, dtype=np.int32)


# -- initial fields (global arrays of shape (ncomp, Nz, Ny, Nx), float64) -------------------
def heat_c(n: int) -> float:
    """c = dt/dx^2 for dx = 1/n and dt = 0.9 dx^2/6 (0.9 of the 3-D explicit limit)."""
    dx = 1.0 / n
    dt = 0.9 * dx * dx / 6.0
    return dt / (dx * dx)


def cell_centers(n: int) -> np.ndarray:
    return (np.arange(n, dtype=np.float64) + 0.5) / n


def gaussian(n: int, center=(0.5, 0.5, 0.5), width2: float = 0.01) -> np.ndarray:
    """u0 = 1 + exp(-|x - c|^2 / width2) at cell centres of an n^3 unit cube (plain distance)."""
    x = cell_centers(n)
    dx2 = (x - center[0]) ** 2
    dy2 = (x - center[1]) ** 2
    dz2 = (x - center[2]) ** 2
    r2 = dz2[:, None, None] + dy2[None, :, None] + dx2[None, None, :]
    return (1.0 + np.exp(-r2 / width2))[None]


def gaussian_factors(n: int, center=(0.5, 0.5, 0.5), width2: float = 0.01):
    """The 1-D factors (gx, gy, gz) of exp(-|x - c|^2 / width2) = gx(x) gy(y) gz(z) at the
    cell centres of an n^3 unit cube: a separable Gaussian bump, cheap to expand on a device."""
    x = cell_centers(n)
    return tuple(np.exp(-((x - center[d]) ** 2) / width2) for d in range(3))


def gaussian_separable(n: int, center=(0.5, 0.5, 0.5), width2: float = 0.01) -> np.ndarray:
    """u0 = 1 + (gz (x) gy) (x) gx from gaussian_factors, products in that order (the serving
    loop expands the same factors in the same order on the GPU)."""
    gx, gy, gz = gaussian_factors(n, center, width2)
    return (1.0 + (gz[:, None, None] * gy[None, :, None]) * gx[None, None, :])[None]


@dataclass
class SineMode:
    amp: float
    k: tuple  # (kx, ky, kz)


def sine_modes(n: int, seed: int, nmodes: int = 3, kmax: int = 8):
    """Sum of nmodes products sin(2 pi kx x) sin(2 pi ky y) sin(2 pi kz z) at cell centres,
    integer wavenumbers uniform in 1..kmax and amplitudes uniform in (0, 1)."""
    rng = np.random.default_rng(seed)
    modes = []
    for _ in range(nmodes):
        k = tuple(int(v) for v in rng.integers(1, kmax + 1, size=3))
        modes.append(SineMode(float(rng.random()), k))
    u = np.zeros((1, n, n, n), dtype=np.float64)
    for m in modes:
        u[0] += m.amp * sine_product(n, m.k)
    return u, modes


def sine_product(n, k) -> np.ndarray:
    """sin(2 pi kx x) sin(2 pi ky y) sin(2 pi kz z) on an (nz, ny, nx) grid of cell centres."""
    nx, ny, nz = (n, n, n) if np.isscalar(n) else tuple(n)
    sx = np.sin(2 * np.pi * k[0] * cell_centers(nx))
    sy = np.sin(2 * np.pi * k[1] * cell_centers(ny))
    sz = np.sin(2 * np.pi * k[2] * cell_centers(nz))
    return sz[:, None, None] * sy[None, :, None] * sx[None, None, :]


def uniform(n, ncomp: int, seed: int) -> np.ndarray:
    """Independent U(0,1) per cell and component, PCG64, global (comp, z, y, x) order."""
    nx, ny, nz = (n, n, n) if np.isscalar(n) else tuple(n)
    return np.random.default_rng(seed).random((ncomp, nz, ny, nx))


def zero_mean_normal_f32(n, seed: int) -> np.ndarray:
    """N(0,1) per cell drawn in FP64 in global order, the exactly rounded mean
    subtracted, then rounded to FP32.  Returned as float64 holding FP32 values."""
    nx, ny, nz = (n, n, n) if np.isscalar(n) else tuple(n)
    f = np.random.default_rng(seed).standard_normal((1, nz, ny, nx))
    mean = math.fsum(f.ravel().tolist()) / f.size
    return (f - mean).astype(np.float32).astype(np.float64)


def round_f32(a: np.ndarray) -> np.ndarray:
    return a.astype(np.float32).astype(np.float64)


# -- serving request stream ----------------------------------------------------------------
@dataclass
class Request:
    rid: int
    arrival: float      # seconds after the stream starts
    n: int              # cubic domain edge
    box_edge: int       # boxes of this edge (remainder box last)
    steps: int
    dtype: str          # "f64" or "f32"
    center: tuple       # Gaussian bump centre


def request_stream(nreq: int = 2000, rate: float = 200.0, seed: int = 0,
                   edges=tuple(range(32, 257, 32)), box_edges=(32, 64),
                   steps_lo: int = 10, steps_hi: int = 200):
    """Independent periodic heat problems with Poisson arrivals (exponential gaps of
    mean 1/rate), cubic edge uniform over ``edges``, box edge uniform over
    ``box_edges``, steps uniform in [steps_lo, steps_hi], FP32 or FP64 with equal
    probability and a Gaussian bump centred uniformly in [1/4, 3/4]^3."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for r in range(nreq):
        t += float(rng.exponential(1.0 / rate))
        n = int(rng.choice(edges))
        be = int(rng.choice(box_edges))
        steps = int(rng.integers(steps_lo, steps_hi + 1))
        dtype = "f32" if rng.random() < 0.5 else "f64"
        center = tuple(float(v) for v in rng.uniform(0.25, 0.75, size=3))
        out.append(Request(r, t, n, be, steps, dtype, center))
    return out
