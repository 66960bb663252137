"""Python binding of libboxtile (ctypes): argument marshalling only.

Every computation runs in the library's HIP kernels; torch supplies device
memory (a uint8 tensor per MultiFab) and the stream (torch's current stream by
default).  The library must be built (``python -m paper_1604_03570_amd.build``);
importing this module without it raises ImportError.

Names follow the paper's objects: BoxArray, DistributionMapping, MultiFab,
fill_boundary (FillBoundary), heat_step, reductions (Sec. 3.1, Sec. 4.1).
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np
import torch  # loads the HIP runtime first, so the library shares torch's copy

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libboxtile.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "boxtile.h")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1604_03570_amd.build`")
_L = ctypes.CDLL(LIB_PATH)

BL_OK, BL_EINVAL, BL_EOVERLAP, BL_EDOMAIN, BL_ESHAPE, BL_EDTYPE, BL_ENOMEM, BL_EHIP = 0, -1, -2, -3, -4, -5, -6, -7
F64, F32 = 0, 1
REDUCE_OPS = {"sum": 0, "max": 1, "min": 2, "norm0": 3, "norm1": 4, "norm2": 5}
_ERR_NAMES = {-1: "EINVAL", -2: "EOVERLAP", -3: "EDOMAIN", -4: "ESHAPE", -5: "EDTYPE", -6: "ENOMEM", -7: "EHIP"}


class BoxtileError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_ERR_NAMES.get(code, code)}: {msg}")
        self.code = code


class bl_box(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_int32 * 3), ("hi", ctypes.c_int32 * 3)]


_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_dp = ctypes.POINTER(ctypes.c_double)
_boxp = ctypes.POINTER(bl_box)
_szp = ctypes.POINTER(ctypes.c_size_t)
_vpp = ctypes.POINTER(ctypes.c_void_p)

_SIGS = {
    "bl_boxarray_create": [_boxp, _i32, _boxp, _i32p, _vpp],
    "bl_boxarray_chop": [_boxp, _i32p, _i32p, _vpp],
    "bl_boxarray_chop_random": [_boxp, _i32p, _i32, _i32, _i32, ctypes.c_uint64, _vpp],
    "bl_boxarray_get": [_vp, _i32p, _boxp],
    "bl_boxarray_domain": [_vp, _boxp, _i32p],
    "bl_distmap_create": [_vp, _i32, _i32p, _vpp],
    "bl_multifab_bytes": [_vp, _i32, _i32, _i32, _szp],
    "bl_multifab_create": [_vp, _vp, _i32, _i32, _i32, _vp, ctypes.c_size_t, _vpp],
    "bl_multifab_layout": [_vp, _i32, _boxp, _szp, _i64p],
    "bl_multifab_xghost_layout": [_vp, _i32, _szp, _i64p],
    "bl_multifab_copy_fab": [_vp, _i32, _i32, _i32, _vp, _i32, _vp],
    "bl_multifab_modified": [_vp],
    "bl_multifab_info": [_vp, _i32p, _i32p, _i32p, _i32p],
    "bl_multifab_copy_global": [_vp, _i32, _i32, _vp, _i32, _vp],
    "bl_multifab_set_val": [_vp, ctypes.c_double, _i32, _i32, _i32, _vp],
    "bl_fill_boundary": [_vp, _i32, _i32, _vp],
    "bl_heat_step": [_vp, _vp, ctypes.c_double, _i32, _vp],
    "bl_heat_advance": [_vpp, _i32, ctypes.c_double, _vp],
    "bl_heat_varcoef_advance": [_vpp, _vp, _i32, ctypes.c_double, ctypes.c_double, _vp],
    "bl_heat8_advance": [_vpp, _i32, ctypes.c_double, _vp],
    "bl_heat8_advance_form": [_vpp, _i32, ctypes.c_double, _i32, _vp],
    "bl_heat8_fused_ok": [_vp, _i32p],
    "bl_heat8_fused_layout": [_vp, _i32, _i32, _i32, _i32, _i32p, _i64p, _i64p],
    "bl_layout_index": [_vp, _i32, _i32, _i32, _i32, _i32p, _i32, _i64p],
    "bl_layout_mirror_index": [_vp, _i32, _i32, _i32, _i32, _i32, _i32, _i32, _i32, _i32, _i64p],
    "bl_device_copy": [_vp, _vp, ctypes.c_size_t, _vp],
    "bl_heat_step_unfused": [_vp, _vp, ctypes.c_double, _vp],
    "bl_gsrb_sweeps": [_vp, _vp, ctypes.c_double, _i32, _dp, _vp],
    "bl_residual_norm": [_vp, _vp, ctypes.c_double, _dp, _vp],
    "bl_reduce": [_vp, _i32, _i32, _dp, _vp],
    "bl_reduce_async": [_vp, _i32, _i32, _vp, _vp],
    "bl_reduce_async_noalloc": [_vp, _i32, _i32, _vp, _vp],
    "bl_set_tile_config": [_i32, _i32, _i32, _i32, _i32],
    "bl_set_gsrb_config": [_i32, _i32, _i32],
    "bl_get_gsrb_config": [_i32p, _i32p, _i32p],
    "bl_gsrb_one_pass_applies": [_vp, _i32p],
    "bl_autotune": [_vp, _vp, _vp, ctypes.c_double, _i32, _i32, _i32p, _i32p, ctypes.POINTER(ctypes.c_float), _i32p,
                    _vp],
    "bl_get_tile_config": [_i32p, _i32p, _i32p, _i32p, _i32p],
    "bl_batch_create": [_vpp],
    "bl_batch_add": [_vp, _vp, _vp, ctypes.c_double, _i32p],
    "bl_batch_remove": [_vp, _i32],
    "bl_batch_parity": [_vp, _i32, _i32p],
    "bl_batch_step": [_vp, _vp],
    "bl_batch_steps": [_vp, _i32, _vp],
    "bl_fill_plan": [_vp, _i32, _i32p, _i32p],
    "bl_face_plan": [_vp, _i32p, _i32p],
    "bl_tile_list": [_vp, _i32, _i32, _i32, _i32p, _i32p],
    "bl_stencil_tiles": [_vp, _i32, _i32, _i32, _i32p, _i32p],
    "bl_tile_boxes": [_vp, _i32p, _i32, _i32, _i32p, _i32p],
    "bl_boxarray_coarsen": [_vp, _i32, _vpp],
    "bl_mg_restrict_residual": [_vp, _vp, ctypes.c_double, _vp, _vp],
    "bl_mg_prolong_add": [_vp, _vp, _vp],
    "bl_mg_workspace_bytes": [_vp, _i32, _i32, _szp, _i32p],
    "bl_mg_create": [_vp, _i32, _i32, _vp, ctypes.c_size_t, _vpp],
    "bl_mg_levels": [_vp, _i32p],
    "bl_mg_bottom_level": [_vp, _i32p],
    "bl_mg_vcycles": [_vp, _vp, _vp, ctypes.c_double, _i32, _i32, _i32, _i32, _dp, _vp],
    "bl_static_partition": [_i32, _i32, _i32p],
}
for _name, _args in _SIGS.items():
    _f = getattr(_L, _name)
    _f.argtypes = _args
    _f.restype = ctypes.c_int32
for _name in ("bl_boxarray_destroy", "bl_distmap_destroy", "bl_multifab_destroy", "bl_batch_destroy",
              "bl_mg_destroy"):
    getattr(_L, _name).argtypes = [_vp]
    getattr(_L, _name).restype = None
_L.bl_last_error.restype = ctypes.c_char_p
_L.bl_version.restype = ctypes.c_char_p


def _check(rc: int) -> None:
    if rc != BL_OK:
        raise BoxtileError(rc, _L.bl_last_error().decode())


def header_functions() -> list:
    """Names of the functions include/boxtile.h declares."""
    with open(HEADER_PATH) as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bl_[a-z0-9_]+)\s*\(", text)))


def version() -> str:
    return _L.bl_version().decode()


def lib() -> ctypes.CDLL:
    return _L


def _stream(stream) -> int:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


def _box(b) -> bl_box:
    r = bl_box()
    for d in range(3):
        r.lo[d] = int(b[d])
        r.hi[d] = int(b[3 + d])
    return r


def _per(periodic) -> ctypes.Array:
    return (ctypes.c_int32 * 3)(*[int(bool(v)) for v in periodic])


# --------------------------------------------------------------------------- BoxArray
class BoxArray:
    """The grids of one level (Sec. 3.1): disjoint boxes inside a domain, periodic flags."""

    def __init__(self, handle: int):
        self._h = ctypes.c_void_p(handle)

    @classmethod
    def from_boxes(cls, boxes, domain, periodic=(1, 1, 1)) -> "BoxArray":
        boxes = np.asarray(boxes, dtype=np.int64).reshape(-1, 6)
        arr = (bl_box * len(boxes))(*[_box(b) for b in boxes])
        h = ctypes.c_void_p()
        _check(_L.bl_boxarray_create(arr, len(boxes), ctypes.byref(_box(domain)), _per(periodic), ctypes.byref(h)))
        return cls(h.value)

    @classmethod
    def chop(cls, domain, max_edge, periodic=(1, 1, 1)) -> "BoxArray":
        me = (max_edge,) * 3 if np.isscalar(max_edge) else tuple(max_edge)
        h = ctypes.c_void_p()
        _check(_L.bl_boxarray_chop(ctypes.byref(_box(domain)), _per(periodic), (ctypes.c_int32 * 3)(*me),
                                   ctypes.byref(h)))
        return cls(h.value)

    def coarsen(self, ratio: int = 2) -> "BoxArray":
        """Every box and the domain coarsened by ratio (same box order and periodic flags)."""
        h = ctypes.c_void_p()
        _check(_L.bl_boxarray_coarsen(self._h, int(ratio), ctypes.byref(h)))
        return BoxArray(h.value)

    @classmethod
    def chop_random(cls, domain, min_edge=16, max_edge=128, align=8, seed=0, periodic=(1, 1, 1)) -> "BoxArray":
        h = ctypes.c_void_p()
        _check(_L.bl_boxarray_chop_random(ctypes.byref(_box(domain)), _per(periodic), min_edge, max_edge, align,
                                          ctypes.c_uint64(seed), ctypes.byref(h)))
        return cls(h.value)

    @property
    def handle(self):
        return self._h

    def boxes(self) -> np.ndarray:
        n = ctypes.c_int32()
        _check(_L.bl_boxarray_get(self._h, ctypes.byref(n), None))
        arr = (bl_box * n.value)()
        _check(_L.bl_boxarray_get(self._h, ctypes.byref(n), arr))
        return np.array([list(b.lo) + list(b.hi) for b in arr], dtype=np.int32).reshape(-1, 6)

    def __len__(self) -> int:
        n = ctypes.c_int32()
        _check(_L.bl_boxarray_get(self._h, ctypes.byref(n), None))
        return n.value

    def domain(self):
        d = bl_box()
        p = (ctypes.c_int32 * 3)()
        _check(_L.bl_boxarray_domain(self._h, ctypes.byref(d), p))
        return tuple(d.lo) + tuple(d.hi), tuple(p)

    def fill_plan(self, nghost: int) -> np.ndarray:
        n = ctypes.c_int32()
        _check(_L.bl_fill_plan(self._h, nghost, ctypes.byref(n), None))
        out = np.zeros((n.value, 11), dtype=np.int32)
        _check(_L.bl_fill_plan(self._h, nghost, ctypes.byref(n), out.ctypes.data_as(_i32p)))
        return out

    def face_plan(self) -> np.ndarray:
        n = ctypes.c_int32()
        _check(_L.bl_face_plan(self._h, ctypes.byref(n), None))
        out = np.zeros((n.value, 12), dtype=np.int32)
        _check(_L.bl_face_plan(self._h, ctypes.byref(n), out.ctypes.data_as(_i32p)))
        return out

    def tile_list(self, ncomp: int, nghost: int, dtype: int = F64) -> np.ndarray:
        n = ctypes.c_int32()
        _check(_L.bl_tile_list(self._h, ncomp, nghost, dtype, ctypes.byref(n), None))
        out = np.zeros((n.value, 9), dtype=np.int32)
        _check(_L.bl_tile_list(self._h, ncomp, nghost, dtype, ctypes.byref(n), out.ctypes.data_as(_i32p)))
        return out

    def stencil_tiles(self, ncomp: int, nghost: int, dtype: int = F64) -> np.ndarray:
        """Linear tiles of the stencil (block form 3): rows of
        {box, comp, q0, nq, nzs, z0, z1, zchunk, vec, lanes, zsteps}."""
        n = ctypes.c_int32()
        _check(_L.bl_stencil_tiles(self._h, ncomp, nghost, dtype, ctypes.byref(n), None))
        out = np.zeros((n.value, 11), dtype=np.int32)
        _check(_L.bl_stencil_tiles(self._h, ncomp, nghost, dtype, ctypes.byref(n), out.ctypes.data_as(_i32p)))
        return out

    TILE_KINDS = {"cell": 0, "nodal": 1, "grown": 2}

    def tile_boxes(self, tile_size, kind: str = "cell", arg: int = 0) -> np.ndarray:
        """Logical tiles of every box: rows of {box, lo[3], hi[3]}.  kind "cell" (tilebox),
        "nodal" with arg = the face direction (nodaltilebox), "grown" with arg = ghost width
        (growntilebox)."""
        ts = np.ascontiguousarray(np.broadcast_to(np.asarray(tile_size, dtype=np.int32), (3,)))
        k = self.TILE_KINDS[kind]
        n = ctypes.c_int32()
        _check(_L.bl_tile_boxes(self._h, ts.ctypes.data_as(_i32p), k, int(arg), ctypes.byref(n), None))
        out = np.zeros((n.value, 7), dtype=np.int32)
        _check(_L.bl_tile_boxes(self._h, ts.ctypes.data_as(_i32p), k, int(arg), ctypes.byref(n),
                                out.ctypes.data_as(_i32p)))
        return out

    def heat8_fused_layout(self, ncomp: int, nghost: int, dtype: int = F64, from_mirror: bool = False):
        """Host-only: the face segments of the fused 8th-order form for a MultiFab of this
        shape, as (segs, total_elems): segs rows {box, face, t1lo, t1hi, t2lo, t2hi, o, sc, sx,
        sy, sz, vec}.  from_mirror: the segments of a step whose input's 4-layer edge mirror is
        current (covered x faces read the neighbours' mirrors).  BoxtileError where the form
        does not apply."""
        n = ctypes.c_int32()
        total = ctypes.c_int64()
        fm = 1 if from_mirror else 0
        _check(_L.bl_heat8_fused_layout(self._h, ncomp, nghost, dtype, fm, ctypes.byref(n), None,
                                        ctypes.byref(total)))
        segs = np.zeros((n.value, 12), dtype=np.int64)
        _check(_L.bl_heat8_fused_layout(self._h, ncomp, nghost, dtype, fm, ctypes.byref(n),
                                        segs.ctypes.data_as(_i64p), ctypes.byref(total)))
        return segs, total.value

    def layout_mirror_index(self, ncomp: int, nghost: int, dtype: int, box: int, side: int, layer: int, j: int,
                            k: int, comp: int) -> int:
        """Host-only: element index of row j, plane k (global) of layer `layer` of side `side` of
        a box's edge mirror (the copy of valid column `layer`, or ex-1-layer on side 1)."""
        out = ctypes.c_int64()
        _check(_L.bl_layout_mirror_index(self._h, ncomp, nghost, dtype, int(box), int(side), int(layer), int(j),
                                         int(k), int(comp), ctypes.byref(out)))
        return out.value

    def layout_index(self, ncomp: int, nghost: int, dtype: int, box: int, cell, comp: int) -> int:
        """Host-only: element index of a cell (global indices, in the box's grown box)."""
        c = (ctypes.c_int32 * 3)(*[int(v) for v in cell])
        out = ctypes.c_int64()
        _check(_L.bl_layout_index(self._h, ncomp, nghost, dtype, int(box), c, int(comp), ctypes.byref(out)))
        return out.value

    def multifab_bytes(self, ncomp: int, nghost: int, dtype: int = F64) -> int:
        b = ctypes.c_size_t()
        _check(_L.bl_multifab_bytes(self._h, ncomp, nghost, dtype, ctypes.byref(b)))
        return b.value

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _L is not None:
            try:
                _L.bl_boxarray_destroy(h)
            except Exception:  # interpreter shutdown
                pass
            self._h = ctypes.c_void_p()


class DistributionMapping:
    """Owner of each box; one GPU here (Sec. 3.1)."""

    def __init__(self, ba: BoxArray, ndevices: int = 1, owner=None):
        h = ctypes.c_void_p()
        own = None
        if owner is not None:
            own = (ctypes.c_int32 * len(owner))(*owner)
        _check(_L.bl_distmap_create(ba.handle, ndevices, own, ctypes.byref(h)))
        self._h = h
        self.ba = ba

    @property
    def handle(self):
        return self._h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _L is not None:
            try:
                _L.bl_distmap_destroy(h)
            except Exception:  # interpreter shutdown
                pass
            self._h = ctypes.c_void_p()


def static_partition(ntiles: int, nworkers: int) -> list:
    first = (ctypes.c_int32 * (nworkers + 1))()
    _check(_L.bl_static_partition(ntiles, nworkers, first))
    return list(first)


def set_tile_config(zchunk: int = 4, waves: int = 4, persist: int = 0, block: int = 3, zsteps: int = 2) -> None:
    _check(_L.bl_set_tile_config(zchunk, waves, persist, block, zsteps))


def get_tile_config() -> tuple:
    """(zchunk, waves, persist, block, zsteps)"""
    v = [ctypes.c_int32() for _ in range(5)]
    _check(_L.bl_get_tile_config(*(ctypes.byref(x) for x in v)))
    return tuple(x.value for x in v)


def autotune(ba: "BoxArray", u0: "MultiFab", u1: "MultiFab", c: float, trial_steps: int = 4, stream=None):
    """Time every candidate tile shape of the fused heat step on u0/u1 (their contents are
    overwritten) and keep the fastest for this (BoxArray, ncomp, nghost, dtype).
    Returns (best (zchunk, waves, persist, block, zsteps),
    [((zchunk, waves, persist, block, zsteps), ms_per_step), ...])."""
    nmax = 64
    cfgs = (ctypes.c_int32 * (5 * nmax))()
    ms = (ctypes.c_float * nmax)()
    n = ctypes.c_int32()
    best = (ctypes.c_int32 * 5)()
    _check(_L.bl_autotune(ba.handle, u0.handle, u1.handle, float(c), int(trial_steps), nmax, ctypes.byref(n), cfgs, ms,
                          best, _stream(stream)))
    table = [(tuple(cfgs[5 * i:5 * i + 5]), float(ms[i])) for i in range(n.value)]
    return tuple(best), table


# --------------------------------------------------------------------------- MultiFab
_TORCH = {F64: torch.float64, F32: torch.float32}


class MultiFab:
    """FABs of one level on device memory held by a torch uint8 tensor (Sec. 3.1)."""

    def __init__(self, ba: BoxArray, ncomp: int = 1, nghost: int = 1, dtype: int = F64, dm=None,
                 device: str = "cuda", buffer: torch.Tensor | None = None):
        self.ba, self.ncomp, self.nghost, self.dtype = ba, ncomp, nghost, dtype
        nbytes = ba.multifab_bytes(ncomp, nghost, dtype)
        if buffer is None:
            buffer = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        ptr = buffer.data_ptr()
        pad = (-ptr) % 256
        self.buffer = buffer
        self.nbytes = nbytes
        self._ptr = ptr + pad
        h = ctypes.c_void_p()
        _check(_L.bl_multifab_create(ba.handle, dm.handle if dm is not None else None, ncomp, nghost, dtype,
                                     ctypes.c_void_p(self._ptr), buffer.numel() - pad, ctypes.byref(h)))
        self._h = h
        dom, self.periodic = ba.domain()
        self.domain = dom
        self.N = tuple(dom[3 + d] - dom[d] + 1 for d in range(3))

    @property
    def handle(self):
        return self._h

    @property
    def data_ptr(self) -> int:
        return self._ptr

    def elements(self) -> torch.Tensor:
        """The whole allocation viewed as elements of the MultiFab's dtype.  After writing
        through this view (or any other way around the library), call modified()."""
        esize = 8 if self.dtype == F64 else 4
        off = self._ptr - self.buffer.data_ptr()
        return self.buffer[off:off + self.nbytes].view(_TORCH[self.dtype])[: self.nbytes // esize]

    def modified(self) -> None:
        """Declare that the storage was written outside the library, so that no later
        call trusts the boxes' edge mirrors before it has rewritten them."""
        _check(_L.bl_multifab_modified(self._h))

    def layout(self, box: int):
        g = bl_box()
        off = ctypes.c_size_t()
        st = (ctypes.c_int64 * 4)()
        _check(_L.bl_multifab_layout(self._h, box, ctypes.byref(g), ctypes.byref(off), st))
        return tuple(g.lo) + tuple(g.hi), off.value, tuple(st)

    def fab(self, box: int, stream=None) -> torch.Tensor:
        """FAB `box` over its grown box, all components, as a dense (comp, z, y, x) device tensor (a copy)."""
        g, _, _ = self.layout(box)
        shape = (self.ncomp, g[5] - g[2] + 1, g[4] - g[1] + 1, g[3] - g[0] + 1)
        t = torch.empty(shape, dtype=_TORCH[self.dtype], device=self.buffer.device)
        _check(_L.bl_multifab_copy_fab(self._h, box, 0, self.ncomp, ctypes.c_void_p(t.data_ptr()), 1,
                                       _stream(stream)))
        return t

    def set_fab(self, box: int, values: torch.Tensor, stream=None) -> None:
        """Overwrite FAB `box` (grown box, all components) from a dense (comp, z, y, x) tensor."""
        t = values.to(device=self.buffer.device, dtype=_TORCH[self.dtype]).contiguous()
        _check(_L.bl_multifab_copy_fab(self._h, box, 0, self.ncomp, ctypes.c_void_p(t.data_ptr()), 0,
                                       _stream(stream)))
        self._keep = t

    def from_global(self, g, scomp: int = 0, stream=None) -> None:
        """Set valid cells from a dense (ncomp', Nz, Ny, Nx) array (numpy or torch)."""
        t = torch.as_tensor(np.ascontiguousarray(g) if isinstance(g, np.ndarray) else g)
        t = t.to(device=self.buffer.device, dtype=_TORCH[self.dtype]).contiguous()
        if t.dim() == 3:
            t = t[None]
        _check(_L.bl_multifab_copy_global(self._h, scomp, t.shape[0], ctypes.c_void_p(t.data_ptr()), 0,
                                          _stream(stream)))
        self._keep = t  # the copy is asynchronous: keep the source alive

    def to_global(self, scomp: int = 0, ncomp: int | None = None, fill=float("nan"), stream=None) -> torch.Tensor:
        ncomp = self.ncomp - scomp if ncomp is None else ncomp
        t = torch.full((ncomp,) + self.N[::-1], fill, dtype=_TORCH[self.dtype], device=self.buffer.device)
        _check(_L.bl_multifab_copy_global(self._h, scomp, ncomp, ctypes.c_void_p(t.data_ptr()), 1, _stream(stream)))
        return t

    def set_val(self, val: float, scomp: int = 0, ncomp: int | None = None, with_ghosts: bool = False,
                stream=None) -> None:
        ncomp = self.ncomp - scomp if ncomp is None else ncomp
        _check(_L.bl_multifab_set_val(self._h, float(val), scomp, ncomp, int(with_ghosts), _stream(stream)))

    def fill_boundary(self, scomp: int = 0, ncomp: int | None = None, stream=None) -> None:
        ncomp = self.ncomp - scomp if ncomp is None else ncomp
        _check(_L.bl_fill_boundary(self._h, scomp, ncomp, _stream(stream)))

    def reduce(self, comp: int, op: str, stream=None) -> float:
        out = ctypes.c_double()
        _check(_L.bl_reduce(self._h, comp, REDUCE_OPS[op], ctypes.byref(out), _stream(stream)))
        return out.value

    def reduce_async(self, comp: int, op: str, out: torch.Tensor, stream=None) -> None:
        assert out.dtype == torch.float64 and out.is_cuda
        _check(_L.bl_reduce_async(self._h, comp, REDUCE_OPS[op], ctypes.c_void_p(out.data_ptr()), _stream(stream)))

    def reduce_async_noalloc(self, comp: int, op: str, out: torch.Tensor, stream=None) -> None:
        """reduce_async whose partial results live in the library's fixed device array
        (no allocation; calls that overlap on one GPU race)."""
        assert out.dtype == torch.float64 and out.is_cuda
        _check(_L.bl_reduce_async_noalloc(self._h, comp, REDUCE_OPS[op], ctypes.c_void_p(out.data_ptr()),
                                          _stream(stream)))

    def sum(self, comp: int = 0) -> float:
        return self.reduce(comp, "sum")

    def max(self, comp: int = 0) -> float:
        return self.reduce(comp, "max")

    def min(self, comp: int = 0) -> float:
        return self.reduce(comp, "min")

    def norm0(self, comp: int = 0) -> float:
        return self.reduce(comp, "norm0")

    def norm1(self, comp: int = 0) -> float:
        return self.reduce(comp, "norm1")

    def norm2(self, comp: int = 0) -> float:
        return self.reduce(comp, "norm2")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _L is not None:
            try:
                _L.bl_multifab_destroy(h)
            except Exception:  # interpreter shutdown
                pass
            self._h = ctypes.c_void_p()


# --------------------------------------------------------------------------- stencils
def heat_step(u_old: MultiFab, u_new: MultiFab, c: float, fill_first: bool = True, stream=None) -> None:
    """One heat step, plain per-box form (FillBoundary, then one launch per box)."""
    _check(_L.bl_heat_step(u_old.handle, u_new.handle, float(c), int(fill_first), _stream(stream)))


def heat_step_unfused(u_old: MultiFab, u_new: MultiFab, c: float, stream=None) -> None:
    """One heat step: one FillBoundary kernel, then one stencil kernel over all tiles."""
    _check(_L.bl_heat_step_unfused(u_old.handle, u_new.handle, float(c), _stream(stream)))


def heat_advance(u0: MultiFab, u1: MultiFab, nsteps: int, c: float, stream=None) -> MultiFab:
    """nsteps fused steps (one launch per step, captured in a HIP graph); returns the result holder."""
    arr = (ctypes.c_void_p * 2)(u0.handle.value, u1.handle.value)
    _check(_L.bl_heat_advance(arr, int(nsteps), float(c), _stream(stream)))
    return u0 if nsteps % 2 == 0 else u1


def device_copy(dst: torch.Tensor, src: torch.Tensor, stream=None) -> None:
    """dst = src (contiguous device tensors of the same byte size, 16-byte multiples)."""
    if dst.nbytes != src.nbytes or not dst.is_contiguous() or not src.is_contiguous():
        raise ValueError("device_copy needs contiguous tensors of one byte size")
    _check(_L.bl_device_copy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()), dst.nbytes,
                             _stream(stream)))


H8_FORMS = {"auto": 0, "fill": 1, "fused": 2, "fused_mirror": 3}


def heat8_advance(u0: MultiFab, u1: MultiFab, nsteps: int, c: float, stream=None, form: str = "auto") -> MultiFab:
    """nsteps heat steps with the 8th-order second difference (nghost >= 4), one stencil
    launch per step: form "fill" (FillBoundary first), "fused" (neighbour boxes read
    directly; BoxtileError where the layout does not allow it), "fused_mirror" (the fused
    form writing and reading the 4-layer edge mirrors; boxes at least 8 cells wide in x)
    or "auto" (heat8_auto_form); returns the result holder."""
    arr = (ctypes.c_void_p * 2)(u0.handle.value, u1.handle.value)
    _check(_L.bl_heat8_advance_form(arr, int(nsteps), float(c), H8_FORMS[form], _stream(stream)))
    return u0 if nsteps % 2 == 0 else u1


def heat8_fused_ok(mf: MultiFab) -> bool:
    """True where the fused 8th-order form applies to mf's layout."""
    ok = ctypes.c_int32(0)
    _check(_L.bl_heat8_fused_ok(mf.handle, ctypes.byref(ok)))
    return ok.value > 0


def heat8_auto_form(mf: MultiFab) -> str:
    """The form heat8_advance(form="auto") takes on mf's layout: "fused" or "fill"."""
    return "fused" if heat8_fused_ok(mf) else "fill"


def heat_varcoef_advance(u0: MultiFab, u1: MultiFab, beta: MultiFab, nsteps: int, dt: float, dx: float,
                         stream=None) -> MultiFab:
    """nsteps steps of du/dt = div(beta grad u) in the flux form (face coefficient: the mean
    of the two cells'), one launch per step; 1/dx is formed here; returns the result holder."""
    arr = (ctypes.c_void_p * 2)(u0.handle.value, u1.handle.value)
    _check(_L.bl_heat_varcoef_advance(arr, beta.handle, int(nsteps), float(dt), 1.0 / float(dx), _stream(stream)))
    return u0 if nsteps % 2 == 0 else u1


def restrict_residual(phi: MultiFab, f: MultiFab, h2: float, fc: MultiFab, stream=None) -> None:
    """fc (on phi's BoxArray coarsened by 2) = mean of the 8 fine residuals f + L_h phi of each
    coarse cell; fills phi's ghosts first."""
    _check(_L.bl_mg_restrict_residual(phi.handle, f.handle, float(h2), fc.handle, _stream(stream)))


def prolong_add(phi: MultiFab, pc: MultiFab, stream=None) -> None:
    """phi (valid cells) += the value of the coarse cell containing each cell."""
    _check(_L.bl_mg_prolong_add(phi.handle, pc.handle, _stream(stream)))


class Multigrid:
    """V-cycle hierarchy for -L_h phi = f over ba; coarse levels in a device workspace held
    by a torch uint8 tensor."""

    def __init__(self, ba: BoxArray, dtype: int = F64, max_levels: int = 32, device: str = "cuda"):
        nb = ctypes.c_size_t()
        nl = ctypes.c_int32()
        _check(_L.bl_mg_workspace_bytes(ba.handle, dtype, int(max_levels), ctypes.byref(nb), ctypes.byref(nl)))
        self.ba, self.dtype = ba, dtype
        self.workspace = torch.empty(nb.value + 256, dtype=torch.uint8, device=device)
        ptr = self.workspace.data_ptr()
        pad = (-ptr) % 256
        h = ctypes.c_void_p()
        _check(_L.bl_mg_create(ba.handle, dtype, int(max_levels), ctypes.c_void_p(ptr + pad),
                               self.workspace.numel() - pad, ctypes.byref(h)))
        self._h = h
        self.nlevels = nl.value
        bl_ = ctypes.c_int32()
        _check(_L.bl_mg_bottom_level(h, ctypes.byref(bl_)))
        self.bottom_level = bl_.value  # first level solved in one workgroup, -1: none

    def vcycles(self, phi: MultiFab, f: MultiFab, h2: float, ncycles: int, nu1: int = 2, nu2: int = 2,
                nu_bottom: int = 8, with_norms: bool = True, stream=None):
        """ncycles V-cycles, phi updated in place; the level-0 residual norm after each (or None)."""
        norms = (ctypes.c_double * max(1, ncycles))() if with_norms else None
        _check(_L.bl_mg_vcycles(self._h, phi.handle, f.handle, float(h2), int(ncycles), int(nu1), int(nu2),
                                int(nu_bottom), norms, _stream(stream)))
        return list(norms)[:ncycles] if with_norms else None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _L is not None:
            try:
                _L.bl_mg_destroy(h)
            except Exception:
                pass
            self._h = ctypes.c_void_p()


def gsrb_sweeps(phi: MultiFab, f: MultiFab, h2: float, nsweeps: int, with_norms: bool = True, stream=None):
    """Red-black Gauss-Seidel sweeps; returns the FP64 residual norm after each sweep (or None)."""
    norms = (ctypes.c_double * max(1, nsweeps))() if with_norms else None
    _check(_L.bl_gsrb_sweeps(phi.handle, f.handle, float(h2), int(nsweeps), norms, _stream(stream)))
    return list(norms)[:nsweeps] if with_norms else None


def set_gsrb_config(one_pass: int = 1, zchunk: int = 0, vectors_per_lane: int = 0) -> None:
    """Form of gsrb_sweeps: the one-pass sweep where it applies (one_pass=1) or the
    two colour passes; planes per workgroup and vectors per lane of the one-pass sweep."""
    _check(_L.bl_set_gsrb_config(int(one_pass), int(zchunk), int(vectors_per_lane)))


def get_gsrb_config():
    a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(_L.bl_get_gsrb_config(ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return a.value, b.value, c.value


def gsrb_one_pass_applies(phi: MultiFab) -> bool:
    out = ctypes.c_int32()
    _check(_L.bl_gsrb_one_pass_applies(phi.handle, ctypes.byref(out)))
    return bool(out.value)


def residual_norm(phi: MultiFab, f: MultiFab, h2: float, stream=None) -> float:
    out = ctypes.c_double()
    _check(_L.bl_residual_norm(phi.handle, f.handle, float(h2), ctypes.byref(out), _stream(stream)))
    return out.value


class Batch:
    """Independent heat problems advanced together, one fused launch per dtype per step."""

    def __init__(self):
        h = ctypes.c_void_p()
        _check(_L.bl_batch_create(ctypes.byref(h)))
        self._h = h
        self._members = {}

    def add(self, u0: MultiFab, u1: MultiFab, c: float) -> int:
        mid = ctypes.c_int32()
        _check(_L.bl_batch_add(self._h, u0.handle, u1.handle, float(c), ctypes.byref(mid)))
        self._members[mid.value] = (u0, u1)
        return mid.value

    def remove(self, mid: int) -> None:
        _check(_L.bl_batch_remove(self._h, mid))
        self._members.pop(mid, None)

    def steps_done(self, mid: int) -> int:
        s = ctypes.c_int32()
        _check(_L.bl_batch_parity(self._h, mid, ctypes.byref(s)))
        return s.value

    def current(self, mid: int) -> MultiFab:
        u0, u1 = self._members[mid]
        return u0 if self.steps_done(mid) % 2 == 0 else u1

    def step(self, stream=None) -> None:
        _check(_L.bl_batch_step(self._h, _stream(stream)))

    def steps(self, nsteps: int, stream=None) -> None:
        """nsteps steps of every member in one call (no joins or leaves in between)."""
        _check(_L.bl_batch_steps(self._h, int(nsteps), _stream(stream)))

    def __len__(self) -> int:
        return len(self._members)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _L is not None:
            try:
                _L.bl_batch_destroy(h)
            except Exception:  # interpreter shutdown
                pass
            self._h = ctypes.c_void_p()
