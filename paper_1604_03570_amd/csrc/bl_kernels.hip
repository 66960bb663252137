// gfx950 kernels of libboxtile: FillBoundary copy, the 7-point heat step
// (per-box and fused forms), red-black Gauss-Seidel colour passes, the FP64
// residual, reductions and data movement between MultiFabs and dense arrays.
//
// Thread mapping shared by the stencil kernels: a workgroup takes one tile
// (box, component, whole rows of x vectors, a z range).  Each lane owns `V`
// consecutive x cells of one row (V*sizeof(T) = 16 bytes when all x extents
// allow it, so every row access is one aligned 16-byte load) and marches up
// the tile's z range keeping the planes z-1, z, z+1 in registers, with the
// next plane already in flight; x and y neighbours inside the tile come from
// the other lanes through LDS, those outside from the FAB (or, fused, from the
// neighbouring box).
//
// Every cell update is one fixed expression (heat_cell / gsrb_cell), compiled
// without FMA contraction, so the per-box, fused and batched forms produce
// bit-identical results.
#include <hip/hip_runtime.h>

#include <cmath>
#include <limits>
#include <mutex>

#include "bl_internal.h"
#include "bl_launch.h"

#pragma clang fp contract(off)

namespace bl {
namespace {

template <typename T, int V>
struct alignas(sizeof(T) * V) Vec {
  T v[V];
};

template <typename T, int V>
__device__ __forceinline__ Vec<T, V> ldv(const T* p) {
  return *reinterpret_cast<const Vec<T, V>*>(p);
}
template <typename T, int V>
__device__ __forceinline__ void stv(T* p, const Vec<T, V>& x) {
  *reinterpret_cast<Vec<T, V>*>(p) = x;
}

// Field pointers reach the stencil through descriptors in memory, so the
// compiler cannot tell they are global; generic (flat) accesses would count
// against the scalar-load counter too and serialise every scalar wait with the
// data loads in flight.  These views pin them to the global address space.
#if defined(__HIP_DEVICE_COMPILE__)
#define BL_GLOBAL __attribute__((address_space(1)))
template <typename T, int V>
__device__ __forceinline__ Vec<T, V> ldv(const BL_GLOBAL T* p) {
  return *reinterpret_cast<const BL_GLOBAL Vec<T, V>*>(p);
}
template <typename T, int V>
__device__ __forceinline__ void stv(BL_GLOBAL T* p, const Vec<T, V>& x) {
  *reinterpret_cast<BL_GLOBAL Vec<T, V>*>(p) = x;
}
#else
#define BL_GLOBAL
#endif
#if defined(__HIP_DEVICE_COMPILE__)
// Store that does not keep the line in the caches (the new state is read back
// only in the next step, long after).
template <typename T, int V>
__device__ __forceinline__ void stv_nt(BL_GLOBAL T* p, const Vec<T, V>& x) {
  using E = T __attribute__((ext_vector_type(V)));
  E e;
#pragma unroll
  for (int i = 0; i < V; ++i) e[i] = x.v[i];
  __builtin_nontemporal_store(e, reinterpret_cast<BL_GLOBAL E*>(p));
}
#else
template <typename T, int V>
__device__ __forceinline__ void stv_nt(T* p, const Vec<T, V>& x) {
  *reinterpret_cast<Vec<T, V>*>(p) = x;
}
#endif
template <typename T>
__device__ __forceinline__ const BL_GLOBAL T* as_global(const T* p) {
  return (const BL_GLOBAL T*)p;
}
template <typename T>
__device__ __forceinline__ BL_GLOBAL T* as_global(T* p) {
  return (BL_GLOBAL T*)p;
}

// Descriptor tables (tiles, boxes, face and fill records, members) are never
// written by a kernel; reading them through the constant address space lets a
// workgroup-uniform index become a scalar load.  Otherwise a store or an LDS
// load elsewhere in the kernel can turn them into vector loads, whose waits
// then also wait for every data load in flight.
#if defined(__HIP_DEVICE_COMPILE__)
#define BL_CONST __attribute__((address_space(4)))
#else
#define BL_CONST
#endif
template <typename T>
__device__ __forceinline__ T ldc(const T* p) {
  return *(const BL_CONST T*)p;
}

// Workgroup barrier ordering LDS only: waits for this wave's LDS accesses, not
// for its global stores (__syncthreads also drains those).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0); vmcnt and expcnt left open
  __builtin_amdgcn_s_barrier();
}

// forward Euler, second-order centred differences (Sec. 4.1 of the paper):
// u + c*(((xm+xp) + (ym+yp)) + (zm+zp) - 6u), c = dt/dx^2
template <typename T>
__device__ __forceinline__ T heat_cell(T uc, T xm, T xp, T ym, T yp, T zm, T zp, T c) {
  const T s = ((xm + xp) + (ym + yp)) + (zm + zp);
  return uc + c * (s - T(6) * uc);
}

// exact solve of one cell of -L_h phi = f from its six neighbours
template <typename T>
__device__ __forceinline__ T gsrb_cell(T xm, T xp, T ym, T yp, T zm, T zp, T fv, T h2, T inv6) {
  return ((((xm + xp) + (ym + yp)) + (zm + zp)) + h2 * fv) * inv6;
}

// Workgroups are dealt round-robin to the 8 XCDs; renumber them so that the
// tile list is cut into chunks of kXcdChunk consecutive tiles dealt to the XCDs
// in turn.  A chunk's tiles share one XCD's L2, and all XCDs move through the
// list together, so boxes next to each other in the list (and their shared
// faces) are worked on at about the same time.  On the 512^3 uneven level this
// ran at 70% of the HBM peak against 68% for one contiguous eighth per XCD and
// 64% for plain round-robin.  A launch of fewer than kXcdChunkedFrom
// workgroups (about two rounds of resident ones) runs nearly all at once, so
// only L2 reuse between neighbouring tiles matters: it keeps one contiguous
// eighth per XCD (one 128^3 box: 236 against 195 GCell/s chunked).  Past the
// last whole round of chunks, workgroups keep their numbers.  Bijective on
// [0, gridDim.x).  Chunks of 8 tiles since tiles take two z steps (16 tiles of
// one step before: the same planes per chunk); 8, 16, 32 measured 2.010, 2.031,
// 2.024 ms per step on the 512^3 uneven level.
constexpr int kXcdChunk = 8;
constexpr int kXcdChunkedFrom = 4096;
__device__ __forceinline__ int logical_block() {
  const int G = gridDim.x;
  const int x = blockIdx.x & 7, q = blockIdx.x >> 3;
  if (G < kXcdChunkedFrom) {
    const int per = G >> 3, rem = G & 7;
    return x * per + (x < rem ? x : rem) + q;
  }
  const int full = G / (8 * kXcdChunk) * (8 * kXcdChunk);
  if ((int)blockIdx.x >= full) return (int)blockIdx.x;
  return (q / kXcdChunk) * (8 * kXcdChunk) + x * kXcdChunk + q % kXcdChunk;
}

// Tiles of this workgroup: one tile, or (persistent grid) a contiguous range
// of near-equal length, the first ntiles % G workers one tile more.
__device__ __forceinline__ void tile_range(int ntiles, int persist, int& first, int& last) {
  const int w = logical_block();
  if (!persist) {
    first = w;
    last = w + 1;
    return;
  }
  const int G = gridDim.x;
  const int q = ntiles / G, r = ntiles % G;
  first = w * q + (w < r ? w : r);
  last = first + q + (w < r ? 1 : 0);
}

// Position of this lane in a tile.
struct TileLane {
  bool active;
  int lx, ty;  // x vector and row inside the tile
  int xv, y;   // box-local x vector and row
  int x0;      // box-local x of the first of the lane's V cells
};

template <int V>
__device__ __forceinline__ TileLane tile_lane(const DevTile& tl) {
  TileLane L;
  const int lane = (int)threadIdx.x;
  const int nvt = tl.nvt;
  L.ty = lane / nvt;
  L.lx = lane - L.ty * nvt;
  L.active = L.ty < tl.rows;
  L.xv = tl.xv0 + L.lx;
  L.y = tl.y0 + L.ty;
  L.x0 = L.xv * V;
  return L;
}

// Face sources.  The records of a face partition the one-cell layer outside it;
// the record covering tangential coordinates (t1, t2) names the source of that
// ghost value: a neighbour's valid cell, its periodic image, or the box's own
// ghost cell where no box covers the layer.  The loops below run in uniform
// control flow (every lane walks the same records, so the record reads are
// scalar loads) and select per lane with `want`.

// x and y faces (t2 = z): value at plane z is data[base + z*step] for the whole
// tile, since tiles never straddle a record's z boundary.
__device__ __forceinline__ void face_source_z(const DevFaceRec* __restrict__ recs, int start, int count, bool want,
                                              int t1, int t2, int comp, int64_t& base, int& step) {
  for (int r = start; r < start + count; ++r) {
    const DevFaceRec R = ldc(recs + r);
    const bool in = want & (t1 >= R.t1lo) & (t1 <= R.t1hi) & (t2 >= R.t2lo) & (t2 <= R.t2hi);
    const int64_t b = R.base + (int64_t)t1 * R.s1 + (int64_t)comp * R.sc;
    base = in ? b : base;
    step = in ? R.s2 : step;
  }
}

// z faces: the value next to (t1, t2) = (x, y).
__device__ __forceinline__ int64_t face_index_xy(const DevFaceRec* __restrict__ recs, int start, int count, int t1,
                                                 int t2, int comp, int64_t fallback) {
  int64_t idx = fallback;
  for (int r = start; r < start + count; ++r) {
    const DevFaceRec R = ldc(recs + r);
    const bool in = (t1 >= R.t1lo) & (t1 <= R.t1hi) & (t2 >= R.t2lo) & (t2 <= R.t2hi);
    const int64_t b = R.base + (int64_t)t1 * R.s1 + (int64_t)t2 * R.s2 + (int64_t)comp * R.sc;
    idx = in ? b : idx;
  }
  return idx;
}

template <typename T, int V>
struct EdgeVals {
  T left, right;
  Vec<T, V> ym, yp;
};

// ---------------------------------------------------------------- heat step
// One tile: lanes march z0..z1-1, keeping planes z-1, z, z+1 in registers with
// plane z+2 and the neighbour values of plane z+1 already in flight.  Every
// lane issues the same five loads per plane (the next plane of its column, the
// rows above and below, the x neighbours on either side) and one store; lanes
// on a box face (FUSED) only point those loads at the neighbouring box through
// the face records, and prefetches past the tile's end are clamped to a plane
// that exists.  The steady-state body is therefore straight-line code whose
// loads stay in flight across planes; it is unrolled four times so that the
// rotation of the plane registers is a renaming, not a copy of registers with
// loads pending.  Lanes beyond the tile's rows mirror row y0 and store the
// same values as its lanes.
// FVEC: every y- and z-face source row is vec-aligned, so face rows are one
// 16-byte load per lane; otherwise face cells are loaded one by one.
// ZB > 0 selects the block form for tiles of at most ZB planes: all of the
// tile's loads are issued first, then its updates (short, load-heavy waves).
template <typename T, int V, bool FUSED, bool FVEC, int ZB>
__global__ void __launch_bounds__(kStencilMaxThreads) __attribute__((amdgpu_waves_per_eu(ZB == 8 ? 2 : 4)))
    k_heat_rows(const DevTile* __restrict__ tiles, int ntiles, const DevBox* __restrict__ boxes,
                const DevFaceRec* __restrict__ recs, DevMember m0, const DevMember* __restrict__ members, int flip,
                int persist) {
  int first, last;
  tile_range(ntiles, persist, first, last);
  for (int t = first; t < last; ++t) {
    const DevTile tl = ldc(tiles + t);
    const DevBox B = ldc(boxes + tl.box);
    const DevMember M = members ? ldc(members + tl.member) : m0;
    const bool swap = ((flip + M.flip_offset) & 1) != 0;
    const BL_GLOBAL T* __restrict__ u = as_global(static_cast<const T*>(swap ? M.b : M.a));
    BL_GLOBAL T* __restrict__ w = as_global(static_cast<T*>(swap ? M.a : M.b));
    const T c = (T)M.c;
    const TileLane L = tile_lane<V>(tl);
    const int n = tl.comp;
    const int sy = B.sy, sz = B.sz;
    const int z0 = tl.z0, z1 = tl.z1;
    const int yy = L.active ? L.y : tl.y0;
    const int64_t cb = B.off + (int64_t)n * B.sc + L.x0 + (int64_t)yy * sy;  // cell (x0, y, z = 0)
    BL_GLOBAL T* wp = w + cb;
    BL_GLOBAL T* mir = w + B.mir + (int64_t)n * B.sc + yy;  // mirror column of row y (side 0, z = 0)

    // Neighbour sources as base + z*step: the own FAB (interior cells, ghost
    // rows, the x ghost slab for the row's first and last lanes), or on a box
    // face of the fused form the face record's source.
    const int64_t slab_lo = B.xs + (int64_t)n * B.sc + (int64_t)yy * B.ng;  // ghost x = -1 at z = 0
    const int64_t slab_hi = slab_lo + B.xs_side;                            // ghost x = ex at z = 0
    const bool xlo = L.xv == 0, xhi = L.xv == B.nvx - 1;
    int64_t lb = xlo ? slab_lo : cb - 1, rb = xhi ? slab_hi : cb + V, ymb = cb - sy, ypb = cb + sy;
    int ls = xlo ? B.xs_z : sz, rs = xhi ? B.xs_z : sz, yms = sz, yps = sz;
    // z-face planes: fixed sources (z = -1 and z = ez)
    int64_t zlo = cb - sz, zhi = cb + (int64_t)B.ez * sz;
    const bool zface_lo = FUSED && z0 == 0;
    const bool zface_hi = FUSED && z1 == B.ez;
    if (FUSED) {
      face_source_z(recs, B.face_start[0], B.face_count[0], xlo, yy, z0, n, lb, ls);
      face_source_z(recs, B.face_start[1], B.face_count[1], xhi, yy, z0, n, rb, rs);
      if (FVEC) {
        if (tl.y0 == 0) face_source_z(recs, B.face_start[2], B.face_count[2], yy == 0, L.x0, z0, n, ymb, yms);
        if (tl.y0 + tl.rows == B.ey)
          face_source_z(recs, B.face_start[3], B.face_count[3], yy == B.ey - 1, L.x0, z0, n, ypb, yps);
        if (zface_lo) zlo = face_index_xy(recs, B.face_start[4], B.face_count[4], L.x0, yy, n, zlo);
        if (zface_hi) zhi = face_index_xy(recs, B.face_start[5], B.face_count[5], L.x0, yy, n, zhi);
      }
    }
    // plane z of the lane's column, z in [z0-1, z1]
    auto plane = [&](int z) -> Vec<T, V> {
      if (!FUSED || FVEC) {
        int64_t a = cb + (int64_t)z * sz;
        if (FUSED) a = z < 0 ? zlo : (z >= B.ez ? zhi : a);
        return ldv<T, V>(u + a);
      }
      Vec<T, V> v;
      if (z >= 0 && z < B.ez) {
        v = ldv<T, V>(u + cb + (int64_t)z * sz);
      } else {
        const int f = z < 0 ? 4 : 5;
#pragma unroll
        for (int e = 0; e < V; ++e)
          v.v[e] = u[face_index_xy(recs, B.face_start[f], B.face_count[f], L.x0 + e, yy, n, cb + z * sz + e)];
      }
      return v;
    };
    auto edges = [&](int z, EdgeVals<T, V>& E) {
      E.left = u[lb + (int64_t)z * ls];
      E.right = u[rb + (int64_t)z * rs];
      if (!FUSED || FVEC) {
        E.ym = ldv<T, V>(u + ymb + (int64_t)z * yms);
        E.yp = ldv<T, V>(u + ypb + (int64_t)z * yps);
      } else {
#pragma unroll
        for (int e = 0; e < V; ++e) {
          int64_t bm = ymb + e, bp = ypb + e;
          int sm = yms, sp = yps;
          if (tl.y0 == 0)
            face_source_z(recs, B.face_start[2], B.face_count[2], yy == 0, L.x0 + e, z0, n, bm, sm);
          if (tl.y0 + tl.rows == B.ey)
            face_source_z(recs, B.face_start[3], B.face_count[3], yy == B.ey - 1, L.x0 + e, z0, n, bp, sp);
          E.ym.v[e] = u[bm + (int64_t)z * sm];
          E.yp.v[e] = u[bp + (int64_t)z * sp];
        }
      }
    };
    auto step = [&](int z, const Vec<T, V>& zm, const Vec<T, V>& cc, const Vec<T, V>& zp, Vec<T, V>& zq,
                    const EdgeVals<T, V>& ec, EdgeVals<T, V>& en) {
      zq = plane(z + 2 < z1 ? z + 2 : z1);        // clamped: always a plane that exists
      edges(z + 1 < z1 ? z + 1 : z1 - 1, en);
      Vec<T, V> o;
#pragma unroll
      for (int e = 0; e < V; ++e) {
        const T xm = e == 0 ? ec.left : cc.v[e - 1];
        const T xp = e == V - 1 ? ec.right : cc.v[e + 1];
        o.v[e] = heat_cell(cc.v[e], xm, xp, ec.ym.v[e], ec.yp.v[e], zm.v[e], zp.v[e], c);
      }
      stv<T, V>(wp + (int64_t)z * sz, o);
      if (FUSED) {  // the new state's edge columns, for the neighbours' next step
        if (xlo) mir[(int64_t)z * B.ey] = o.v[0];
        if (xhi) mir[B.mir_side + (int64_t)z * B.ey] = o.v[V - 1];
      }
    };

    if (ZB == 0) {  // march
      Vec<T, V> pa = plane(z0 - 1), pb = plane(z0), pc = plane(z0 + 1), pd;
      EdgeVals<T, V> e0, e1;
      edges(z0, e0);
      int z = z0;
      for (; z + 4 <= z1; z += 4) {
        step(z, pa, pb, pc, pd, e0, e1);
        step(z + 1, pb, pc, pd, pa, e1, e0);
        step(z + 2, pc, pd, pa, pb, e0, e1);
        step(z + 3, pd, pa, pb, pc, e1, e0);
      }
      if (z < z1) step(z, pa, pb, pc, pd, e0, e1);
      if (z + 1 < z1) step(z + 1, pb, pc, pd, pa, e1, e0);
      if (z + 2 < z1) step(z + 2, pc, pd, pa, pb, e0, e1);
    } else {  // block: every load of the tile (at most ZB planes) first, then the updates
      constexpr int NB = ZB > 0 ? ZB : 1;
      Vec<T, V> P[NB + 2];
      EdgeVals<T, V> E[NB];
#pragma unroll
      for (int k = 0; k < NB + 2; ++k) P[k] = plane(z0 - 1 + k < z1 ? z0 - 1 + k : z1);
#pragma unroll
      for (int k = 0; k < NB; ++k) edges(z0 + k < z1 ? z0 + k : z1 - 1, E[k]);
#pragma unroll
      for (int k = 0; k < NB; ++k) {
        if (z0 + k < z1) {
          Vec<T, V> o;
#pragma unroll
          for (int e = 0; e < V; ++e) {
            const T xm = e == 0 ? E[k].left : P[k + 1].v[e - 1];
            const T xp = e == V - 1 ? E[k].right : P[k + 1].v[e + 1];
            o.v[e] = heat_cell(P[k + 1].v[e], xm, xp, E[k].ym.v[e], E[k].yp.v[e], P[k].v[e], P[k + 2].v[e], c);
          }
          const int z = z0 + k;
          stv<T, V>(wp + (int64_t)z * sz, o);
          if (FUSED) {
            if (xlo) mir[(int64_t)z * B.ey] = o.v[0];
            if (xhi) mir[B.mir_side + (int64_t)z * B.ey] = o.v[V - 1];
          }
        }
      }
    }
  }
}

// ---------------------------------------------------------------- heat step, LDS block form
// Source (base + z*step) of face cell (t1, z) of an x or y face for lanes with
// `want`, from the tile's resolved record fr of that face (one record covers
// the tile's part of the face: a uniform scalar read) or, for kFaceMany, by
// search over the face's records [start, start+count).  Callers pick fr, start
// and count with constant indices: a variable index into the tile or box
// descriptor would move the descriptor to scratch memory.
__device__ __forceinline__ void tile_face_source(const DevFaceRec* __restrict__ recs, int32_t fr, int start,
                                                 int count, bool want, int t1, int z0, int comp, int64_t& base,
                                                 int& step) {
  if (fr >= 0) {
    const DevFaceRec R = ldc(recs + fr);
    base = want ? R.base + (int64_t)t1 * R.s1 + (int64_t)comp * R.sc : base;
    step = want ? R.s2 : step;
  } else if (fr == kFaceMany) {
    face_source_z(recs, start, count, want, t1, z0, comp, base, step);
  }
}

// Element index of z-face cell (t1, t2) = (x, y), as above.
__device__ __forceinline__ int64_t tile_face_index(const DevFaceRec* __restrict__ recs, int32_t fr, int start,
                                                   int count, int t1, int t2, int comp, int64_t fallback) {
  if (fr >= 0) {
    const DevFaceRec R = ldc(recs + fr);
    return R.base + (int64_t)t1 * R.s1 + (int64_t)t2 * R.s2 + (int64_t)comp * R.sc;
  }
  if (fr == kFaceMany) return face_index_xy(recs, start, count, t1, t2, comp, fallback);
  return fallback;
}

// Tiles of at most ZB planes.  Every lane loads its own ZB+2 planes; only the
// lanes on the tile's edges load what lies outside the tile (the rows above
// and below, the x neighbours at the row ends: from the FAB, or through the
// face records when FUSED).  The tile's planes then go through LDS, from which
// every lane takes its in-tile x and y neighbours.  One wait for all loads,
// one barrier, then the updates.  FUSED: the new edge columns are gathered in
// LDS and written to the mirror with one coalesced store.  Needs FVEC when FUSED.
// LDS: ZB*blockDim vectors of planes, then 2*ZB*rmax mirror values.
template <typename T, int V, bool FUSED, int ZB>
__global__ void __launch_bounds__(kStencilMaxThreads) __attribute__((amdgpu_waves_per_eu(ZB == 8 ? 2 : 4)))
    k_heat_lds(const DevTile* __restrict__ tiles, int ntiles, const DevBox* __restrict__ boxes,
               const DevFaceRec* __restrict__ recs, DevMember m0, const DevMember* __restrict__ members, int flip,
               int persist, int rmax) {
  extern __shared__ unsigned char smem_raw[];
  Vec<T, V>* sh = reinterpret_cast<Vec<T, V>*>(smem_raw);  // [ZB][blockDim.x]
  T* shm = reinterpret_cast<T*>(sh + ZB * blockDim.x);     // [2][ZB][rmax]
  int first, last;
  tile_range(ntiles, persist, first, last);
  for (int t = first; t < last; ++t) {
    const DevTile tl = ldc(tiles + t);
    const DevBox B = ldc(boxes + tl.box);
    const DevMember M = members ? ldc(members + tl.member) : m0;
    const bool swap = ((flip + M.flip_offset) & 1) != 0;
    const BL_GLOBAL T* __restrict__ u = as_global(static_cast<const T*>(swap ? M.b : M.a));
    BL_GLOBAL T* __restrict__ w = as_global(static_cast<T*>(swap ? M.a : M.b));
    const T c = (T)M.c;
    const TileLane L = tile_lane<V>(tl);
    const int n = tl.comp, nvt = tl.nvt, rows = tl.rows;
    const int sy = B.sy, sz = B.sz;
    const int z0 = tl.z0, z1 = tl.z1;
    const int yy = L.active ? L.y : tl.y0;
    const int64_t cb = B.off + (int64_t)n * B.sc + L.x0 + (int64_t)yy * sy;
    BL_GLOBAL T* wp = w + cb;

    // the lane's own planes first (z-face planes through the face records)
    int64_t zlo = cb - sz, zhi = cb + (int64_t)B.ez * sz;
    if (FUSED) {
      if (z0 == 0) zlo = tile_face_index(recs, tl.frec[4], B.face_start[4], B.face_count[4], L.x0, yy, n, zlo);
      if (z1 == B.ez) zhi = tile_face_index(recs, tl.frec[5], B.face_start[5], B.face_count[5], L.x0, yy, n, zhi);
    }
    Vec<T, V> P[ZB + 2];
#pragma unroll
    for (int k = 0; k < ZB + 2; ++k) {
      const int z = z0 - 1 + k < z1 ? z0 - 1 + k : z1;
      int64_t a = cb + (int64_t)z * sz;
      if (FUSED) a = z < 0 ? zlo : (z >= B.ez ? zhi : a);
      P[k] = ldv<T, V>(u + a);
    }

    // sources of what lies outside the tile
    const int64_t slab_lo = B.xs + (int64_t)n * B.sc + (int64_t)yy * B.ng;
    const bool xlo = L.xv == 0, xhi = L.xv == B.nvx - 1;
    int64_t lb = xlo ? slab_lo : cb - 1, rb = xhi ? slab_lo + B.xs_side : cb + V;
    int64_t ymb = cb - sy, ypb = cb + sy;
    int ls = xlo ? B.xs_z : sz, rs = xhi ? B.xs_z : sz, yms = sz, yps = sz;
    if (FUSED) {
      tile_face_source(recs, tl.frec[0], B.face_start[0], B.face_count[0], xlo, yy, z0, n, lb, ls);
      tile_face_source(recs, tl.frec[1], B.face_start[1], B.face_count[1], xhi, yy, z0, n, rb, rs);
      tile_face_source(recs, tl.frec[2], B.face_start[2], B.face_count[2], yy == 0, L.x0, z0, n, ymb, yms);
      tile_face_source(recs, tl.frec[3], B.face_start[3], B.face_count[3], yy == B.ey - 1, L.x0, z0, n, ypb, yps);
    }
    const bool eL = L.lx == 0, eR = L.lx == nvt - 1, eM = L.ty == 0, eP = L.ty == rows - 1;
    T hl[ZB], hr[ZB];
    Vec<T, V> hm[ZB], hp[ZB];
#pragma unroll
    for (int k = 0; k < ZB; ++k) {
      const int z = z0 + k < z1 ? z0 + k : z1 - 1;
      if (eL) hl[k] = u[lb + (int64_t)z * ls];
      if (eR) hr[k] = u[rb + (int64_t)z * rs];
      if (eM) hm[k] = ldv<T, V>(u + ymb + (int64_t)z * yms);
      if (eP) hp[k] = ldv<T, V>(u + ypb + (int64_t)z * yps);
    }
#pragma unroll
    for (int k = 0; k < ZB; ++k) sh[k * blockDim.x + threadIdx.x] = P[k + 1];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < ZB; ++k) {
      const Vec<T, V>* row = sh + k * blockDim.x + threadIdx.x;
      const T left = eL ? hl[k] : row[-1].v[V - 1];
      const T right = eR ? hr[k] : row[1].v[0];
      const Vec<T, V> ym = eM ? hm[k] : row[-nvt];
      const Vec<T, V> yp = eP ? hp[k] : row[nvt];
      Vec<T, V> o;
#pragma unroll
      for (int e = 0; e < V; ++e) {
        const T xm = e == 0 ? left : P[k + 1].v[e - 1];
        const T xp = e == V - 1 ? right : P[k + 1].v[e + 1];
        o.v[e] = heat_cell(P[k + 1].v[e], xm, xp, ym.v[e], yp.v[e], P[k].v[e], P[k + 2].v[e], c);
      }
      const int z = z0 + k;
      if (z < z1 && L.active) stv<T, V>(wp + (int64_t)z * sz, o);
      if (FUSED && L.active) {  // this tile's share of the new edge columns, staged in LDS
        if (xlo) shm[(0 * ZB + k) * rmax + L.ty] = o.v[0];
        if (xhi) shm[(1 * ZB + k) * rmax + L.ty] = o.v[V - 1];
      }
    }
    if (FUSED) {
      const bool has_lo = tl.xv0 == 0, has_hi = tl.xv0 + nvt == B.nvx;
      if (has_lo || has_hi) {
        lds_barrier();
        BL_GLOBAL T* mir = w + B.mir + (int64_t)n * B.sc + tl.y0;
        for (int q = threadIdx.x; q < 2 * ZB * rows; q += blockDim.x) {
          const int side = q / (ZB * rows), k = (q / rows) % ZB, r = q % rows;
          if (z0 + k < z1 && (side ? has_hi : has_lo))
            mir[side * B.mir_side + (int64_t)(z0 + k) * B.ey + r] = shm[(side * ZB + k) * rmax + r];
        }
      }
    }
    if (persist) __syncthreads();  // the next tile reuses the LDS buffers
  }
}

// ---------------------------------------------------------------- heat step, LDS block form, halos loaded into LDS
// Bytes from global memory straight into LDS (no registers): lane l's bytes
// land at dst + l*size; dst is the same for the whole wave.
#if defined(__HIP_DEVICE_COMPILE__)
#define BL_LDS __attribute__((address_space(3)))
__device__ __forceinline__ void lds_load16(const BL_GLOBAL void* src, void* dst) {
  __builtin_amdgcn_global_load_lds(src, (BL_LDS void*)dst, 16, 0, 0);
}
__device__ __forceinline__ void lds_load4(const BL_GLOBAL void* src, void* dst) {
  __builtin_amdgcn_global_load_lds(src, (BL_LDS void*)dst, 4, 0, 0);
}
#else
__device__ __forceinline__ void lds_load16(const void*, void*) {}
__device__ __forceinline__ void lds_load4(const void*, void*) {}
#endif


// The stencil forms with the halo in LDS work on linear tiles (DevLinTile): a
// run of nq consecutive x vectors of a plane (rows are contiguous, so a run
// may start and end inside a row), over up to ZB planes per z block and nzs z
// blocks per workgroup.  What lies outside the run (the nvx vectors before and
// after it, the values beyond its row ends) goes from memory straight into
// LDS, loaded by all waves in 64-lane pieces, so the registers hold only the
// lanes' own planes.  LDS: ZB*blockDim plane vectors `sh`; per z block, plane
// and side, nh = min(nvx, nq) vectors `shy` and nrows values `shx` (the fused
// forms then stage the new edge columns there, each slot written by the one
// lane that read it).
template <typename T, int V>
struct TileLds {
  Vec<T, V>* sh;
  Vec<T, V>* shy;
  T* shx;
  int nthr, wave, nwaves, lane;
};

template <typename T, int V, int ZB>
__device__ __forceinline__ TileLds<T, V> tile_lds(unsigned char* smem, int yhmax) {
  TileLds<T, V> S;
  S.nthr = blockDim.x;
  S.sh = reinterpret_cast<Vec<T, V>*>(smem);
  S.shy = S.sh + ZB * S.nthr;
  S.shx = reinterpret_cast<T*>(S.shy + ZB * 2 * yhmax);
  S.wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  S.nwaves = S.nthr >> 6;
  S.lane = (int)threadIdx.x & 63;
  return S;
}

// Position of this lane in a linear tile.
struct LinLane {
  bool active;
  int s, i;      // z block, index in the run
  int q, y, xv;  // plane vector, its row and x vector
  int x0;        // first x cell of the vector
  int zb0, zb1;  // the lane's planes [zb0, zb1)
  int nh;        // halo vectors per side: min(nvx, nq)
};

template <int V, int ZB>
__device__ __forceinline__ LinLane lin_lane(const DevLinTile& tl, int nvx) {
  LinLane L;
  const int l = (int)threadIdx.x;
  const int s = l / tl.nq;
  L.active = s < tl.nzs;
  L.s = L.active ? s : 0;  // idle lanes shadow block 0 so every address stays valid
  L.i = l - s * tl.nq;
  L.q = tl.q0 + L.i;
  L.y = L.q / nvx;
  L.xv = L.q - L.y * nvx;
  L.x0 = L.xv * V;
  L.zb0 = tl.z0 + L.s * ZB;
  L.zb1 = L.zb0 + ZB < tl.z1 ? L.zb0 + ZB : tl.z1;
  L.nh = nvx < tl.nq ? nvx : tl.nq;
  return L;
}

// Issue the loads of the tile's halo into LDS (no wait).
template <typename T, int V, bool FUSED, int ZB>
__device__ __forceinline__ void stage_halo(const TileLds<T, V>& S, const DevLinTile& tl, const DevBox& B,
                                           const DevFaceRec* __restrict__ recs, const BL_GLOBAL T* __restrict__ u,
                                           int64_t comp0) {
  using VT = Vec<T, V>;
  constexpr int DPV = (int)sizeof(T) / 4;  // dwords per value
  const int n = tl.comp, nvx = B.nvx, P = B.ey * nvx, sz = B.sz;
  const int nh = nvx < tl.nq ? nvx : tl.nq, nr = tl.nrows;
  // the nh vectors before the run (s = 0) and after it (s = 1): one 16-byte
  // vector per lane, or one dword per lane for narrower vectors
  constexpr int YW = sizeof(VT) == 16 ? 16 : 4;
  constexpr int YPER = (int)sizeof(VT) / YW;  // lanes per vector
  const int nyi = nh * YPER, nchy = (nyi + 63) >> 6;
  for (int q = S.wave; q < tl.nzs * ZB * 2 * nchy; q += S.nwaves) {
    const int ch = q % nchy, rest = q / nchy, side = rest & 1, k = (rest >> 1) % ZB, zs = (rest >> 1) / ZB;
    const int i = ch * 64 + S.lane;
    const int zz = tl.z0 + zs * ZB + k, z = zz < tl.z1 ? zz : tl.z1 - 1;
    if (i < nyi) {
      const int j = i / YPER, part = i - j * YPER;
      const int h = side ? tl.q0 + tl.nq - nh + nvx + j : tl.q0 - nvx + j;
      int64_t a = comp0 + (int64_t)h * V + (int64_t)z * sz;  // rows y = -1 and y = ey are the ghost rows
      if (FUSED && (h < 0 || h >= P)) {
        const int x0 = (h < 0 ? h + nvx : h - P) * V;
        int64_t base = a;
        int step = 0;
        const int32_t fr = side ? tl.frec[3] : tl.frec[2];
        const int fs = side ? B.face_start[3] : B.face_start[2], fc = side ? B.face_count[3] : B.face_count[2];
        tile_face_source(recs, fr, fs, fc, true, x0, tl.z0, n, base, step);
        a = base + (int64_t)z * step;
      }
      VT* dst = S.shy + ((zs * ZB + k) * 2 + side) * nh;
      if (YW == 16)
        lds_load16(u + a, dst + ch * 64);
      else
        lds_load4(reinterpret_cast<const BL_GLOBAL unsigned char*>(u + a) + part * 4,
                  reinterpret_cast<unsigned char*>(dst) + ch * 256);
    }
  }
  // the values left (side 0) and right (side 1) of each row of the run, one dword
  // per lane: the box face (x slab or face record) where the row's end lies in
  // the run, else the element next to the run in the same row
  const int nitems = nr * DPV, nchx = (nitems + 63) >> 6;
  const bool lo_inrow = tl.q0 % nvx != 0, hi_inrow = (tl.q0 + tl.nq) % nvx != 0;
  for (int q = S.wave; q < tl.nzs * ZB * 2 * nchx; q += S.nwaves) {
    const int ch = q % nchx, rest = q / nchx, side = rest & 1, k = (rest >> 1) % ZB, zs = (rest >> 1) / ZB;
    const int i = ch * 64 + S.lane;
    const int zz = tl.z0 + zs * ZB + k, z = zz < tl.z1 ? zz : tl.z1 - 1;
    if (i < nitems) {
      const int r = i / DPV, part = i - r * DPV;
      const int y = tl.y_first + r;
      int64_t a;
      if (side == 0 && r == 0 && lo_inrow) {
        a = comp0 + (int64_t)tl.q0 * V - 1 + (int64_t)z * sz;
      } else if (side == 1 && r == nr - 1 && hi_inrow) {
        a = comp0 + (int64_t)(tl.q0 + tl.nq) * V + (int64_t)z * sz;
      } else if (!FUSED) {
        a = B.xs + (int64_t)n * B.sc + (side ? B.xs_side : 0) + (int64_t)z * B.xs_z + (int64_t)y * B.ng;
      } else {
        int64_t base = 0;
        int step = 0;
        const int32_t fr = side ? tl.frec[1] : tl.frec[0];
        const int fs = side ? B.face_start[1] : B.face_start[0], fc = side ? B.face_count[1] : B.face_count[0];
        tile_face_source(recs, fr, fs, fc, true, y, tl.z0, n, base, step);
        a = base + (int64_t)z * step;
      }
      lds_load4(reinterpret_cast<const BL_GLOBAL unsigned char*>(u + a) + part * 4,
                reinterpret_cast<unsigned char*>(S.shx + ((zs * ZB + k) * 2 + side) * nr) + ch * 256);
    }
  }
}

// The lane's planes zb0-1+K0 .. zb0+ZB (P[K0] .. P[ZB+1]; clamped to zb1; z-face
// planes through the face records when FUSED) into registers.  K0 = 2 loads
// what a z step of a tile needs beyond the two planes carried from the step
// below it.
template <typename T, int V, bool FUSED, int ZB, int K0 = 0>
__device__ __forceinline__ void load_planes(Vec<T, V> (&P)[ZB + 2], const LinLane& L, const DevLinTile& tl,
                                            const DevBox& B, const DevFaceRec* __restrict__ recs,
                                            const BL_GLOBAL T* __restrict__ u, int64_t cb) {
  const int n = tl.comp, sz = B.sz;
  int64_t zlo = cb - sz, zhi = cb + (int64_t)B.ez * sz;
  if (FUSED) {
    if (K0 == 0 && tl.z0 == 0)
      zlo = tile_face_index(recs, tl.frec[4], B.face_start[4], B.face_count[4], L.x0, L.y, n, zlo);
    if (tl.z1 == B.ez) zhi = tile_face_index(recs, tl.frec[5], B.face_start[5], B.face_count[5], L.x0, L.y, n, zhi);
  }
#pragma unroll
  for (int k = K0; k < ZB + 2; ++k) {
    const int z = L.zb0 - 1 + k < L.zb1 ? L.zb0 - 1 + k : L.zb1;
    int64_t a = cb + (int64_t)z * sz;
    if (FUSED) a = z < 0 ? zlo : (z >= B.ez ? zhi : a);
    P[k] = ldv<T, V>(u + a);
  }
}

// Neighbours of the lane's vector in its plane k (after the barrier that follows
// the planes' LDS writes): the values left and right of it, the vectors of the
// rows below and above.
template <typename T, int V>
struct Nbr {
  T left, right;
  Vec<T, V> ym, yp;
};
// The value a neighbouring lane holds: from lane l-1 (WAVE_SHR1) or lane l+1
// (WAVE_SHL1) of the wave, by DPP; lanes with no such neighbour get 0.
constexpr int kDppWaveShl1 = 0x130, kDppWaveShr1 = 0x138;
#if defined(__HIP_DEVICE_COMPILE__)
template <int CTRL>
__device__ __forceinline__ float lane_shift(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double lane_shift(double v) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xF, 0xF, false);
  const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
#else
template <int CTRL, typename T>
__device__ __forceinline__ T lane_shift(T v) { return v; }
#endif

// own: the lane's vector of plane k.  DPP: the x neighbours inside the run come
// from the adjacent lanes by DPP, so LDS is read only at run and row ends and
// at the first and last lane of a wave (reading single elements of
// neighbouring vectors from LDS puts lanes 16 bytes apart and doubles the bank
// conflicts).  Measured on one GPU against LDS reads: the GSRB pass 5-6%
// faster (it takes DPP); the 7-point heat kernel 1% and the
// variable-coefficient kernel 2% slower (they keep the LDS reads).
template <typename T, int V, int ZB, bool DPP>
__device__ __forceinline__ Nbr<T, V> tile_neighbours(const TileLds<T, V>& S, const LinLane& L, const DevLinTile& tl,
                                                     int nvx, int k, const Vec<T, V>& own) {
  const Vec<T, V>* row = S.sh + k * S.nthr + threadIdx.x;
  const int slot = (L.s * ZB + k) * 2;
  const int r = L.y - tl.y_first;
  Nbr<T, V> N;
  if (DPP) {
    const int wl = (int)threadIdx.x & 63;
    const T from_left = lane_shift<kDppWaveShr1>(own.v[V - 1]);
    const T from_right = lane_shift<kDppWaveShl1>(own.v[0]);
    if (L.xv == 0 || L.i == 0)
      N.left = S.shx[slot * tl.nrows + r];
    else
      N.left = wl == 0 ? row[-1].v[V - 1] : from_left;
    if (L.xv == nvx - 1 || L.i == tl.nq - 1)
      N.right = S.shx[(slot + 1) * tl.nrows + r];
    else
      N.right = wl == 63 ? row[1].v[0] : from_right;
  } else {
    N.left = (L.xv == 0 || L.i == 0) ? S.shx[slot * tl.nrows + r] : row[-1].v[V - 1];
    N.right = (L.xv == nvx - 1 || L.i == tl.nq - 1) ? S.shx[(slot + 1) * tl.nrows + r] : row[1].v[0];
  }
  N.ym = L.i < nvx ? S.shy[slot * L.nh + L.i] : row[-nvx];
  N.yp = L.i + nvx >= tl.nq ? S.shy[(slot + 1) * L.nh + L.i - (tl.nq - L.nh)] : row[nvx];
  return N;
}

// A lane's new edge values into its own x-halo slots (the mirror staging).
template <typename T, int V, int ZB>
__device__ __forceinline__ void stage_edges(const TileLds<T, V>& S, const LinLane& L, const DevLinTile& tl, int nvx,
                                            int k, const Vec<T, V>& o) {
  const int slot = (L.s * ZB + k) * 2, r = L.y - tl.y_first;
  if (L.xv == 0) S.shx[slot * tl.nrows + r] = o.v[0];
  if (L.xv == nvx - 1) S.shx[(slot + 1) * tl.nrows + r] = o.v[V - 1];
}

// The staged edge columns of the run's rows whose ends lie in the run, stored
// as contiguous runs into the mirror.
template <typename T, int V, int ZB>
__device__ __forceinline__ void store_mirror(const TileLds<T, V>& S, const DevLinTile& tl, const DevBox& B,
                                             BL_GLOBAL T* __restrict__ w) {
  const int nvx = B.nvx, nr = tl.nrows;
  const bool lo_first = tl.q0 % nvx == 0, hi_last = (tl.q0 + tl.nq) % nvx == 0;
  if (nr == 1 && !lo_first && !hi_last) return;  // a run inside one row: no box face
  lds_barrier();
  BL_GLOBAL T* mir = w + B.mir + (int64_t)tl.comp * B.sc + tl.y_first;
  const int per = tl.nzs * ZB * 2 * nr;
  for (int q = threadIdx.x; q < per; q += S.nthr) {
    const int r = q % nr, rest = q / nr, side = rest & 1, k = (rest >> 1) % ZB, zs = (rest >> 1) / ZB;
    const int z = tl.z0 + zs * ZB + k;
    const bool has = side ? (r < nr - 1 || hi_last) : (r > 0 || lo_first);
    if (has && k < ZB && z < tl.z1 && z < tl.z0 + (zs + 1) * ZB)
      mir[side * B.mir_side + (int64_t)z * B.ey + r] = S.shx[((zs * ZB + k) * 2 + side) * nr + r];
  }
}

// z steps of a linear tile: a tile spans up to zsteps * ZB * nzs planes and is
// worked on in steps of ZB * nzs planes (nzs z blocks side by side, each ZB
// planes), bottom to top.  Step j is the tile cut to its planes.
template <int ZB>
__device__ __forceinline__ DevLinTile tile_zstep(const DevLinTile& tl, int j) {
  DevLinTile ts = tl;
  const int span = ZB * tl.nzs;
  ts.z0 = tl.z0 + j * span;
  ts.z1 = ts.z0 + span < tl.z1 ? ts.z0 + span : tl.z1;
  const int nb = (ts.z1 - ts.z0 + ZB - 1) / ZB;
  ts.nzs = nb < tl.nzs ? nb : tl.nzs;
  return ts;
}

// Heat step, block form with the halo in LDS: per z step of the tile, one wait
// for all loads, the lanes' planes into LDS, one barrier, the updates,
// full-vector stores.  With one z block per step (planes of a workgroup's size
// or more), the two planes above a step are carried in registers into the next
// step, which loads only its ZB new planes.  Both forms store the new edge
// columns into the output's edge mirror.
template <typename T, int V, bool FUSED, int ZB>
__global__ void __launch_bounds__(kStencilMaxThreads)
    __attribute__((amdgpu_waves_per_eu(ZB == 8 ? 4 : 6)))
    k_heat_dma(const DevLinTile* __restrict__ tiles, int ntiles, const DevBox* __restrict__ boxes,
               const DevFaceRec* __restrict__ recs, DevMember m0, const DevMember* __restrict__ members, int flip,
               int persist, int yhmax) {
  using VT = Vec<T, V>;
  extern __shared__ unsigned char smem_raw[];
  const TileLds<T, V> S = tile_lds<T, V, ZB>(smem_raw, yhmax);
  int first, last;
  tile_range(ntiles, persist, first, last);
  for (int t = first; t < last; ++t) {
    const DevLinTile tl = ldc(tiles + t);
    const DevBox B = ldc(boxes + tl.box);
    const DevMember M = members ? ldc(members + tl.member) : m0;
    const bool swap = ((flip + M.flip_offset) & 1) != 0;
    const BL_GLOBAL T* __restrict__ u = as_global(static_cast<const T*>(swap ? M.b : M.a));
    BL_GLOBAL T* __restrict__ w = as_global(static_cast<T*>(swap ? M.a : M.b));
    const T c = (T)M.c;
    const int nvx = B.nvx;
    const int64_t comp0 = B.off + (int64_t)tl.comp * B.sc;
    const int span = ZB * tl.nzs, nsteps = (tl.z1 - tl.z0 + span - 1) / span;
    const bool carry = tl.nzs == 1;

    VT P[ZB + 2];
    for (int j = 0; j < nsteps; ++j) {
      const DevLinTile ts = tile_zstep<ZB>(tl, j);
      const LinLane L = lin_lane<V, ZB>(ts, nvx);
      const int64_t cb = comp0 + (int64_t)L.q * V;
      if (j > 0 && carry) {
        P[0] = P[ZB];
        P[1] = P[ZB + 1];
        load_planes<T, V, FUSED, ZB, 2>(P, L, ts, B, recs, u, cb);
      } else {
        load_planes<T, V, FUSED, ZB>(P, L, ts, B, recs, u, cb);
      }
      stage_halo<T, V, FUSED, ZB>(S, ts, B, recs, u, comp0);
#pragma unroll
      for (int k = 0; k < ZB; ++k) S.sh[k * S.nthr + threadIdx.x] = P[k + 1];
      __syncthreads();
      BL_GLOBAL T* wp = w + cb;
#pragma unroll
      for (int k = 0; k < ZB; ++k) {
        const Nbr<T, V> N = tile_neighbours<T, V, ZB, false>(S, L, ts, nvx, k, P[k + 1]);
        VT o;
#pragma unroll
        for (int e = 0; e < V; ++e) {
          const T xm = e == 0 ? N.left : P[k + 1].v[e - 1];
          const T xp = e == V - 1 ? N.right : P[k + 1].v[e + 1];
          o.v[e] = heat_cell(P[k + 1].v[e], xm, xp, N.ym.v[e], N.yp.v[e], P[k].v[e], P[k + 2].v[e], c);
        }
        const int z = L.zb0 + k;
        if (z < L.zb1 && L.active) {
          stv_nt<T, V>(wp + (int64_t)z * B.sz, o);
          stage_edges<T, V, ZB>(S, L, ts, nvx, k, o);
        }
      }
      store_mirror<T, V, ZB>(S, ts, B, w);  // both forms leave the output's edge mirror current
      if (persist || j + 1 < nsteps) __syncthreads();  // the next step or tile reuses the LDS buffers
    }
  }
}

// ---------------------------------------------------------------- heat step with a variable coefficient, flux form
// Flux through the face between cells lo and hi: the mean of the two cells'
// coefficients times the difference quotient, the difference multiplied by 1/dx.
template <typename T>
__device__ __forceinline__ T face_flux(T ulo, T uhi, T blo, T bhi, T inv_dx) {
  const T b = (T)0.5 * (blo + bhi);
  return b * ((uhi - ulo) * inv_dx);
}

// du/dt = div(beta grad u), forward Euler in the flux form of Sec. 4.1: per
// cell the six face fluxes, their differences per direction times 1/dx, then
// u + dt*((dFx + dFy) + dFz).  The fluxes stay in registers; a face shared by
// two cells of one lane (neighbours in its vector, consecutive planes) is
// computed once.  u and beta are staged alike, each with its own LDS region of
// lds_half bytes: the lane's planes in registers and LDS, the tile's halo
// straight into LDS.  FUSED: neighbour boxes through the face records (the
// edge mirrors of u and beta current); otherwise the FABs' own filled ghosts.
// Both forms store the new u's edge columns into its mirror.
template <typename T, int V, bool FUSED, int ZB>
__global__ void __launch_bounds__(kStencilMaxThreads)
    __attribute__((amdgpu_waves_per_eu(ZB == 8 ? 2 : (ZB == 4 ? 3 : 5))))
    k_heat_vc_dma(const DevLinTile* __restrict__ tiles, int ntiles, const DevBox* __restrict__ boxes,
                  const DevFaceRec* __restrict__ recs, const T* u_, T* w_, const T* beta_, T dt, T inv_dx,
                  int yhmax, int lds_half) {
  using VT = Vec<T, V>;
  extern __shared__ unsigned char smem_raw[];
  const TileLds<T, V> S = tile_lds<T, V, ZB>(smem_raw, yhmax);
  const TileLds<T, V> Sb = tile_lds<T, V, ZB>(smem_raw + lds_half, yhmax);
  const BL_GLOBAL T* __restrict__ u = as_global(u_);
  const BL_GLOBAL T* __restrict__ bt = as_global(beta_);
  BL_GLOBAL T* __restrict__ w = as_global(w_);
  int first, last;
  tile_range(ntiles, 0, first, last);
  for (int t = first; t < last; ++t) {
    const DevLinTile tl = ldc(tiles + t);
    const DevBox B = ldc(boxes + tl.box);
    const int nvx = B.nvx;
    const int64_t comp0 = B.off + (int64_t)tl.comp * B.sc;
    const int span = ZB * tl.nzs, nsteps = (tl.z1 - tl.z0 + span - 1) / span;
    const bool carry = tl.nzs == 1;

    VT P[ZB + 2], Q[ZB + 2];  // u, beta
    for (int j = 0; j < nsteps; ++j) {  // z steps as in k_heat_dma, both fields carried
      const DevLinTile ts = tile_zstep<ZB>(tl, j);
      const LinLane L = lin_lane<V, ZB>(ts, nvx);
      const int64_t cb = comp0 + (int64_t)L.q * V;
      if (j > 0 && carry) {
        P[0] = P[ZB];
        P[1] = P[ZB + 1];
        Q[0] = Q[ZB];
        Q[1] = Q[ZB + 1];
        load_planes<T, V, FUSED, ZB, 2>(P, L, ts, B, recs, u, cb);
        load_planes<T, V, FUSED, ZB, 2>(Q, L, ts, B, recs, bt, cb);
      } else {
        load_planes<T, V, FUSED, ZB>(P, L, ts, B, recs, u, cb);
        load_planes<T, V, FUSED, ZB>(Q, L, ts, B, recs, bt, cb);
      }
      stage_halo<T, V, FUSED, ZB>(S, ts, B, recs, u, comp0);
      stage_halo<T, V, FUSED, ZB>(Sb, ts, B, recs, bt, comp0);
#pragma unroll
      for (int k = 0; k < ZB; ++k) {
        S.sh[k * S.nthr + threadIdx.x] = P[k + 1];
        Sb.sh[k * Sb.nthr + threadIdx.x] = Q[k + 1];
      }
      __syncthreads();
      BL_GLOBAL T* wp = w + cb;
      T fz[V];  // flux through the lower z face of the current plane
#pragma unroll
      for (int e = 0; e < V; ++e) fz[e] = face_flux(P[0].v[e], P[1].v[e], Q[0].v[e], Q[1].v[e], inv_dx);
#pragma unroll
      for (int k = 0; k < ZB; ++k) {
        const Nbr<T, V> N = tile_neighbours<T, V, ZB, false>(S, L, ts, nvx, k, P[k + 1]);
        const Nbr<T, V> NB = tile_neighbours<T, V, ZB, false>(Sb, L, ts, nvx, k, Q[k + 1]);
        const VT& c = P[k + 1];
        const VT& cbeta = Q[k + 1];
        T fx = face_flux(N.left, c.v[0], NB.left, cbeta.v[0], inv_dx);  // lower x face of element 0
        VT o;
#pragma unroll
        for (int e = 0; e < V; ++e) {
          const T uxp = e == V - 1 ? N.right : c.v[e + 1];
          const T bxp = e == V - 1 ? NB.right : cbeta.v[e + 1];
          const T fxp = face_flux(c.v[e], uxp, cbeta.v[e], bxp, inv_dx);
          const T fym = face_flux(N.ym.v[e], c.v[e], NB.ym.v[e], cbeta.v[e], inv_dx);
          const T fyp = face_flux(c.v[e], N.yp.v[e], cbeta.v[e], NB.yp.v[e], inv_dx);
          const T fzp = face_flux(c.v[e], P[k + 2].v[e], cbeta.v[e], Q[k + 2].v[e], inv_dx);
          const T dfx = (fxp - fx) * inv_dx, dfy = (fyp - fym) * inv_dx, dfz = (fzp - fz[e]) * inv_dx;
          o.v[e] = c.v[e] + dt * ((dfx + dfy) + dfz);
          fx = fxp;
          fz[e] = fzp;
        }
        const int z = L.zb0 + k;
        if (z < L.zb1 && L.active) {
          stv_nt<T, V>(wp + (int64_t)z * B.sz, o);
          stage_edges<T, V, ZB>(S, L, ts, nvx, k, o);
        }
      }
      store_mirror<T, V, ZB>(S, ts, B, w);  // both forms leave the output's edge mirror current
      if (j + 1 < nsteps) __syncthreads();  // the next step reuses the LDS buffers
    }
  }
}

// ---------------------------------------------------------------- multigrid grid transfers
// Both kernels run over the flattened items of a level (coarse cells, or x
// pairs of fine cells): item g belongs to the box b with pre[b] <= g <
// pre[b+1].  Workgroup w takes items [w*per, (w+1)*per) and wgbox[w] is the box
// of its first item.  A workgroup inside one box (every workgroup of a level of
// large boxes) reads that box's descriptors as scalars; one that spans boxes
// (tiny boxes near the bottom of a V-cycle) finds each item's box by bisection
// from wgbox[w], so a level of many tiny boxes still fills whole workgroups.
__device__ __forceinline__ int box_of_item(const int32_t* __restrict__ pre, int lo, int hi, int g) {
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (pre[mid] <= g) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Restriction of the residual of one coarse cell (I, J, K) (refinement ratio 2):
// its 8 fine cells are the x pair 2I, 2I+1 of rows 2J+b', planes 2K+c; each one's
// residual r = f + (s - 6 phi) / h2 is taken in FP64 from promoted values,
// summed in the order c, b', then x (lower first), and the sum times 1/8 is
// stored.  phi's ghosts must be filled (x neighbours at box faces come from the
// x ghost slab).
template <typename T>
__device__ __forceinline__ void restrict_cell(const DevBox& F, const DevBox& C, int q,
                                              const BL_GLOBAL T* __restrict__ phi, const BL_GLOBAL T* __restrict__ f,
                                              BL_GLOBAL T* __restrict__ fc, double h2) {
  const int I = q % C.ex;
  q /= C.ex;
  const int J = q % C.ey, K = q / C.ey;
  const int x0 = 2 * I;
  double acc = 0.0;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
#pragma unroll
    for (int bb = 0; bb < 2; ++bb) {
      const int y = 2 * J + bb, z = 2 * K + c;
      const int64_t row = F.off + (int64_t)y * F.sy + (int64_t)z * F.sz;
      const Vec<T, 2> ctr = ldv<T, 2>(phi + row + x0);
      const Vec<T, 2> ym = ldv<T, 2>(phi + row - F.sy + x0);
      const Vec<T, 2> yp = ldv<T, 2>(phi + row + F.sy + x0);
      const Vec<T, 2> zm = ldv<T, 2>(phi + row - F.sz + x0);
      const Vec<T, 2> zp = ldv<T, 2>(phi + row + F.sz + x0);
      const Vec<T, 2> fv = ldv<T, 2>(f + row + x0);
      const int64_t slab = F.xs + (int64_t)z * F.xs_z + (int64_t)y * F.ng;
      const double left = (double)(x0 == 0 ? phi[slab] : phi[row + x0 - 1]);
      const double right = (double)(x0 + 2 == F.ex ? phi[slab + F.xs_side] : phi[row + x0 + 2]);
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const double xm = a == 0 ? left : (double)ctr.v[0];
        const double xp = a == 0 ? (double)ctr.v[1] : right;
        const double sv = ((xm + xp) + ((double)ym.v[a] + (double)yp.v[a])) + ((double)zm.v[a] + (double)zp.v[a]);
        const double r = (double)fv.v[a] + (sv - 6.0 * (double)ctr.v[a]) / h2;
        acc = (c == 0 && bb == 0 && a == 0) ? r : acc + r;
      }
    }
  }
  fc[C.off + I + (int64_t)J * C.sy + (int64_t)K * C.sz] = (T)(acc * 0.125);
}

// One lane per coarse cell, kRestrictPerWG cells per workgroup.
template <typename T>
__global__ void __launch_bounds__(kRestrictPerWG)
    k_restrict_residual(const int32_t* __restrict__ cpre, const int32_t* __restrict__ wgbox, int nbox, int total,
                        const DevBox* __restrict__ fboxes, const DevBox* __restrict__ cboxes, const T* phi_,
                        const T* f_, T* fc_, double h2) {
  const BL_GLOBAL T* __restrict__ phi = as_global(phi_);
  const BL_GLOBAL T* __restrict__ f = as_global(f_);
  BL_GLOBAL T* __restrict__ fc = as_global(fc_);
  const int g0 = (int)blockIdx.x * kRestrictPerWG;
  const int end = g0 + kRestrictPerWG < total ? g0 + kRestrictPerWG : total;
  const int b0 = ldc(wgbox + blockIdx.x);
  const int g = g0 + (int)threadIdx.x;
  if (ldc(cpre + b0 + 1) >= end) {  // the whole workgroup in box b0
    if (g < end) restrict_cell<T>(ldc(fboxes + b0), ldc(cboxes + b0), g - ldc(cpre + b0), phi, f, fc, h2);
  } else if (g < end) {
    const int b = box_of_item(cpre, b0, nbox - 1, g);
    restrict_cell<T>(fboxes[b], cboxes[b], g - cpre[b], phi, f, fc, h2);
  }
}

// Prolongation, piecewise constant: an item is an x pair (2i', 2i'+1) of a fine
// row (y, z); both cells add the value of their coarse cell (i', y/2, z/2).
// Four items per lane (lanes, then lanes + blockDim, ...), all loads first.
template <typename T>
__global__ void __launch_bounds__(256)
    k_prolong_add(const int32_t* __restrict__ ppre, const int32_t* __restrict__ wgbox, int nbox, int total,
                  const DevBox* __restrict__ fboxes, const DevBox* __restrict__ cboxes, T* phi_, const T* pc_) {
  constexpr int K = kProlongPerWG / 256;
  BL_GLOBAL T* __restrict__ phi = as_global(phi_);
  const BL_GLOBAL T* __restrict__ pc = as_global(pc_);
  const int g0 = (int)blockIdx.x * kProlongPerWG;
  const int end = g0 + kProlongPerWG < total ? g0 + kProlongPerWG : total;
  const int b0 = ldc(wgbox + blockIdx.x);
  const bool one_box = ldc(ppre + b0 + 1) >= end;
  int64_t at[K];
  T v[K];
  Vec<T, 2> w[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int g = g0 + k * 256 + (int)threadIdx.x;
    at[k] = -1;
    if (g >= end) continue;
    int b = b0;
    if (!one_box) b = box_of_item(ppre, b0, nbox - 1, g);
    const DevBox F = one_box ? ldc(fboxes + b0) : fboxes[b];
    const DevBox C = one_box ? ldc(cboxes + b0) : cboxes[b];
    int q = g - (one_box ? ldc(ppre + b0) : ppre[b]);
    const int npx = F.ex >> 1;
    const int ip = q % npx;
    q /= npx;
    const int y = q % F.ey, z = q / F.ey;
    v[k] = pc[C.off + ip + (int64_t)(y >> 1) * C.sy + (int64_t)(z >> 1) * C.sz];
    at[k] = F.off + 2 * ip + (int64_t)y * F.sy + (int64_t)z * F.sz;
    w[k] = ldv<T, 2>(phi + at[k]);
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    if (at[k] < 0) continue;
    Vec<T, 2> o;
    o.v[0] = w[k].v[0] + v[k];
    o.v[1] = w[k].v[1] + v[k];
    stv<T, 2>(phi + at[k], o);
  }
}

// ---------------------------------------------------------------- multigrid bottom in one workgroup
// The coarse levels of a V-cycle where every level covers a fully periodic
// domain: each level is a dense periodic array in LDS (phi, then f), so a
// FillBoundary is the periodic wrap of the index and every pass is one
// barrier, not a launch.  The arithmetic is the launched passes' own: the GSRB
// cell update in T, the residual in FP64 from promoted values summed over the 8
// children in the order z, y, x (lower first) and times 1/8, piecewise constant
// prolongation in T.
struct MgLevelView {
  int nx, ny, nz, lo0, lo1, lo2;
  int off;
};

__device__ __forceinline__ MgLevelView mg_level(const MgBottom& m, int l) {
  MgLevelView v;
  v.nx = m.n[l][0];
  v.ny = m.n[l][1];
  v.nz = m.n[l][2];
  v.lo0 = m.lo[l][0];
  v.lo1 = m.lo[l][1];
  v.lo2 = m.lo[l][2];
  v.off = m.off[l];
  return v;
}

// nsweeps red-black sweeps (red = even global i+j+k first) of level v in LDS
template <typename T>
__device__ void mg_lds_smooth(T* lds, const MgLevelView& v, double h2, int nsweeps) {
  const int N = v.nx * v.ny * v.nz;
  T* phi = lds + v.off;
  const T* f = phi + N;
  const T h2t = (T)h2, inv6 = (T)(1.0 / 6.0);
  for (int s = 0; s < nsweeps; ++s)
    for (int color = 0; color < 2; ++color) {
      for (int q = (int)threadIdx.x; q < N; q += (int)blockDim.x) {
        const int i = q % v.nx, t = q / v.nx, j = t % v.ny, k = t / v.ny;
        if (((v.lo0 + i + v.lo1 + j + v.lo2 + k) & 1) != color) continue;
        const int im = i == 0 ? v.nx - 1 : i - 1, ip = i == v.nx - 1 ? 0 : i + 1;
        const int jm = j == 0 ? v.ny - 1 : j - 1, jp = j == v.ny - 1 ? 0 : j + 1;
        const int km = k == 0 ? v.nz - 1 : k - 1, kp = k == v.nz - 1 ? 0 : k + 1;
        const int row = k * v.ny, pl = v.nx;
        phi[q] = gsrb_cell(phi[(row + j) * pl + im], phi[(row + j) * pl + ip], phi[(row + jm) * pl + i],
                           phi[(row + jp) * pl + i], phi[(km * v.ny + j) * pl + i], phi[(kp * v.ny + j) * pl + i],
                           f[q], h2t, inv6);
      }
      __syncthreads();
    }
}

// f of level c = the restriction of the residual f + L_h phi of level v
template <typename T>
__device__ void mg_lds_restrict(T* lds, const MgLevelView& v, const MgLevelView& c, double h2) {
  const int N = v.nx * v.ny * v.nz, Nc = c.nx * c.ny * c.nz;
  const T* phi = lds + v.off;
  const T* f = phi + N;
  T* fc = lds + c.off + Nc;
  for (int q = (int)threadIdx.x; q < Nc; q += (int)blockDim.x) {
    const int I = q % c.nx, t = q / c.nx, J = t % c.ny, K = t / c.ny;
    double acc = 0.0;
    for (int cz = 0; cz < 2; ++cz)
      for (int by = 0; by < 2; ++by)
        for (int ax = 0; ax < 2; ++ax) {
          const int i = 2 * I + ax, j = 2 * J + by, k = 2 * K + cz;
          const int im = i == 0 ? v.nx - 1 : i - 1, ip = i == v.nx - 1 ? 0 : i + 1;
          const int jm = j == 0 ? v.ny - 1 : j - 1, jp = j == v.ny - 1 ? 0 : j + 1;
          const int km = k == 0 ? v.nz - 1 : k - 1, kp = k == v.nz - 1 ? 0 : k + 1;
          const int at = (k * v.ny + j) * v.nx + i;
          const double xm = (double)phi[(k * v.ny + j) * v.nx + im], xp = (double)phi[(k * v.ny + j) * v.nx + ip];
          const double ym = (double)phi[(k * v.ny + jm) * v.nx + i], yp = (double)phi[(k * v.ny + jp) * v.nx + i];
          const double zm = (double)phi[(km * v.ny + j) * v.nx + i], zp = (double)phi[(kp * v.ny + j) * v.nx + i];
          const double sv = ((xm + xp) + (ym + yp)) + (zm + zp);
          const double r = (double)f[at] + (sv - 6.0 * (double)phi[at]) / h2;
          acc = (cz == 0 && by == 0 && ax == 0) ? r : acc + r;
        }
    fc[q] = (T)(acc * 0.125);
  }
  T* pc = lds + c.off;
  for (int q = (int)threadIdx.x; q < Nc; q += (int)blockDim.x) pc[q] = (T)0;
  __syncthreads();
}

// phi of level v += phi of level c at each cell's parent
template <typename T>
__device__ void mg_lds_prolong(T* lds, const MgLevelView& v, const MgLevelView& c) {
  const int N = v.nx * v.ny * v.nz;
  T* phi = lds + v.off;
  const T* pc = lds + c.off;
  for (int q = (int)threadIdx.x; q < N; q += (int)blockDim.x) {
    const int i = q % v.nx, t = q / v.nx, j = t % v.ny, k = t / v.ny;
    phi[q] = phi[q] + pc[((k >> 1) * c.ny + (j >> 1)) * c.nx + (i >> 1)];
  }
  __syncthreads();
}

// Valid cell g of the level (its flattened index, boxes in order; cpre[b] = the
// first cell of box b): its element in the MultiFab and its dense index.
__device__ __forceinline__ void mg_cell(const DevBox* __restrict__ boxes, const int32_t* __restrict__ cpre, int nbox,
                                        const MgLevelView& top, int g, int64_t& at, int& dense) {
  const int b = box_of_item(cpre, 0, nbox - 1, g);
  const DevBox& B = boxes[b];
  const int q = g - cpre[b];
  const int i = q % B.ex, t = q / B.ex, j = t % B.ey, k = t / B.ey;
  dense = ((B.glo[2] + k - top.lo2) * top.ny + (B.glo[1] + j - top.lo1)) * top.nx + (B.glo[0] + i - top.lo0);
  at = B.off + i + (int64_t)j * B.sy + (int64_t)k * B.sz;
}

template <typename T>
__global__ void __launch_bounds__(1024)
    k_mg_bottom(const DevBox* __restrict__ boxes, const int32_t* __restrict__ cpre, int nbox, T* phi_, const T* f_,
                MgBottom m, double h2, int load_phi, int nu1, int nu2, int nub) {
  extern __shared__ unsigned char smem_raw[];
  T* lds = reinterpret_cast<T*>(smem_raw);
  BL_GLOBAL T* phiL = as_global(phi_);
  const BL_GLOBAL T* fL = as_global(f_);
  const MgLevelView top = mg_level(m, 0);
  const int N0 = top.nx * top.ny * top.nz;  // the boxes cover the domain: N0 valid cells
  // level L's valid cells into the dense arrays, every lane its own cells of any box
  for (int g = (int)threadIdx.x; g < N0; g += (int)blockDim.x) {
    int64_t a;
    int d;
    mg_cell(boxes, cpre, nbox, top, g, a, d);
    lds[top.off + N0 + d] = fL[a];
    lds[top.off + d] = load_phi ? phiL[a] : (T)0;
  }
  __syncthreads();
  // down: nu1 sweeps and restriction on every level but the coarsest
  double h = h2;
  for (int l = 0; l + 1 < m.nlev; ++l) {
    const MgLevelView v = mg_level(m, l), c = mg_level(m, l + 1);
    mg_lds_smooth<T>(lds, v, h, nu1);
    mg_lds_restrict<T>(lds, v, c, h);
    h *= 4.0;
  }
  mg_lds_smooth<T>(lds, mg_level(m, m.nlev - 1), h, nub);
  // up: prolongation and nu2 sweeps
  for (int l = m.nlev - 2; l >= 0; --l) {
    h *= 0.25;
    const MgLevelView v = mg_level(m, l), c = mg_level(m, l + 1);
    mg_lds_prolong<T>(lds, v, c);
    mg_lds_smooth<T>(lds, v, h, nu2);
  }
  for (int g = (int)threadIdx.x; g < N0; g += (int)blockDim.x) {
    int64_t a;
    int d;
    mg_cell(boxes, cpre, nbox, top, g, a, d);
    phiL[a] = lds[top.off + d];
  }
}

// ---------------------------------------------------------------- 8th-order heat step (9-cell span)
// Workgroup barrier with acquire/release ordering of LDS only: loads from global
// memory issued before it stay in flight.
__device__ __forceinline__ void lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Forward-Euler heat step with the 8th-order centred second difference (9
// cells per axis; the span of Sec. 4.2's stencils).  With p_m = u[-m] + u[+m]
// along an axis, D = ((A1*p1 + A2*p2) + A3*p3) + A4*p4 and
// u_new = u + c*(((Dx + Dy) + Dz) + A0X3*u); each coefficient rounded once.
constexpr double kH8A1 = 8.0 / 5.0, kH8A2 = -1.0 / 5.0, kH8A3 = 8.0 / 315.0, kH8A4 = -1.0 / 560.0;
constexpr double kH8A0X3 = -205.0 / 24.0;

// The segment of a face (segments [start, start + count)) that covers
// tangential coordinates (t1, t2).  The segments tile the face, so when none
// of the first count - 1 does, the last one does.
__device__ __forceinline__ DevH8Seg h8_find(const DevH8Seg* __restrict__ segs, int start, int count, int t1, int t2) {
  int i = start;
  for (; i < start + count - 1; ++i) {
    const DevH8Seg g = segs[i];
    if (t1 >= g.t1lo && t1 <= g.t1hi && t2 >= g.t2lo && t2 <= g.t2hi) break;
  }
  return segs[i];
}

// One workgroup per tile (x vectors xv0..xv0+nvt-1 of rows y0..y0+rows-1 over
// planes z0..z1-1, at most 256 lanes, rows <= 32, nvt <= 32), marching up z.
// Each lane keeps the 9 planes z-4..z+4 of its own vector column in registers.
// Plane z goes into one of two LDS buffers of ldh x ldw values together with
// its 4-wide x and y halo, so x and y neighbours come from LDS; the next
// plane's column value and halo are loaded before the barrier and stay in
// flight across it.  One barrier per plane.  Cells outside the box come from
// the FAB's filled ghosts (x: the x ghost slab), or, FUSED, straight from
// their source: each lane finds the segment of its face that covers its cell
// (h8_find) and finds the next one when its z leaves the segment.  FUSED with
// wmir: the lanes of the first and last 4 x columns (boxes at least 8 cells
// wide, 4 a multiple of V) also store their new values into w's 4-layer edge
// mirror, layer m of side s at mir + s*mir_side + m*ey*ez + z*ey + y, where
// the next step's neighbours read their x-face cells.
template <typename T, int V, bool FUSED>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
    k_heat8(const DevTile* __restrict__ tiles, const DevH8Seg* __restrict__ segs, const DevH8Face* __restrict__ faces,
            const DevBox* __restrict__ boxes, const T* u_, T* w_, T c, int ldw, int ldh, int wmir) {
  using VT = Vec<T, V>;
  extern __shared__ unsigned char smem_raw[];
  T* const lds = reinterpret_cast<T*>(smem_raw);
  const DevTile tl = ldc(tiles + logical_block());
  const DevBox B = ldc(boxes + tl.box);
  const DevH8Face F = FUSED ? ldc(faces + tl.box) : DevH8Face{};
  // the same record through memory, for faces chosen per lane (indexing F with
  // a lane's value would place it in scratch)
  const DevH8Face* __restrict__ Fp = faces + tl.box;
  const int64_t n = tl.comp;
  // address of cell (x, y, 0) of the tile's component through segment g
  auto seg_at = [&](const DevH8Seg& g, int x, int y) -> int64_t {
    return g.o + n * g.sc + (int64_t)x * g.sx + (int64_t)y * g.sy;
  };
  const BL_GLOBAL T* __restrict__ u = as_global(u_);
  BL_GLOBAL T* __restrict__ w = as_global(w_);
  const int l = (int)threadIdx.x;
  const int nvt = tl.nvt, rows = tl.rows, W = nvt * V, x0 = tl.xv0 * V;
  const int lx = l % nvt, ly = l / nvt;
  const bool active = ly < rows;
  const int lyc = active ? ly : 0;  // idle lanes shadow row 0, so every address stays valid
  const int64_t sz = B.sz;
  const int64_t comp0 = B.off + (int64_t)tl.comp * B.sc;
  const int64_t col = comp0 + x0 + lx * V + (int64_t)(tl.y0 + lyc) * B.sy;
  // y halo: 4 rows below and 4 above the tile, one vector per lane
  const bool hy = l < 8 * nvt;
  int64_t yh_at = col;
  int yh_step = B.sz;  // plane strides fit 32 bits (checked when the segments are made)
  int yh_slot = 0, yh_x = 0, yh_y = 0, yh_f = -1, yh_t2hi = 0;  // yh_f >= 0: a y face's segment
  if (hy) {
    const int r = l / nvt, xv = l % nvt;
    yh_y = r < 4 ? tl.y0 - 4 + r : tl.y0 + rows + r - 4;
    yh_x = x0 + xv * V;
    yh_at = comp0 + yh_x + (int64_t)yh_y * B.sy;
    if (FUSED && (yh_y < 0 || yh_y >= B.ey)) {
      yh_f = yh_y < 0 ? 2 : 3;
      const DevH8Seg g = h8_find(segs, Fp->start[yh_f], Fp->count[yh_f], yh_x, tl.z0);
      yh_at = seg_at(g, yh_x, yh_y);
      yh_step = (int)g.sz;
      yh_t2hi = g.t2hi;
    }
    yh_slot = (r < 4 ? r : rows + r) * ldw + 4 + xv * V;
  }
  // x halo: 4 values left and right of each row, one per lane, the 4 values of
  // a row side in 4 consecutive lanes (adjacent addresses, so a wave touches a
  // quarter of the lines it would with one row per lane); a value beyond the
  // box's x range comes from the x ghost slab (layer = distance from the face - 1)
  const bool hx = l < 8 * rows;
  int64_t xh_at = col;
  int xh_step = B.sz;
  int xh_slot = 0, xh_x = 0, xh_y = 0, xh_f = -1, xh_t2hi = 0;  // xh_f >= 0: an x face's segment
  if (hx) {
    const int side = l / (4 * rows), rem = l - side * 4 * rows, m = rem & 3, yr = rem >> 2;
    const int y = tl.y0 + yr;
    const int x = side ? x0 + W + m : x0 - 1 - m;
    xh_x = x;
    xh_y = y;
    if (FUSED && (x < 0 || x >= B.ex)) {
      xh_f = x < 0 ? 0 : 1;
      const DevH8Seg g = h8_find(segs, Fp->start[xh_f], Fp->count[xh_f], y, tl.z0);
      xh_at = seg_at(g, x, y);
      xh_step = (int)g.sz;
      xh_t2hi = g.t2hi;
    } else if (x < 0 || x >= B.ex) {
      xh_at = B.xs + (int64_t)tl.comp * B.sc + (x < 0 ? 0 : B.xs_side) + (int64_t)y * B.ng + (x < 0 ? -1 - x : x - B.ex);
      xh_step = B.xs_z;
    } else {
      xh_at = comp0 + x + (int64_t)y * B.sy;
    }
    xh_slot = (yr + 4) * ldw + (side ? 4 + W + m : 3 - m);
  }
  const T A1 = (T)kH8A1, A2 = (T)kH8A2, A3 = (T)kH8A3, A4 = (T)kH8A4, A0 = (T)kH8A0X3;
  // the mirror element of the lane's first cell at z = 0 (relative to the
  // component's mirror), or -1: side 0 layer = column, side 1 layer = ex-1-column
  const int mlay = B.ey * B.ez;
  int moff = -1;
  if (FUSED && wmir && active) {
    const int xc = x0 + lx * V;
    if (xc < 4) moff = xc * mlay + tl.y0 + ly;
    else if (xc >= B.ex - 4) moff = B.mir_side + (B.ex - 1 - xc) * mlay + tl.y0 + ly;
  }

  // the lane's column below and above the box (FUSED: planes z < 0 and z >= ez
  // through the z faces' segments, one each for the whole tile)
  int64_t czlo = col, czhi = col;
  int szlo = B.sz, szhi = B.sz;
  if (FUSED) {
    const int xc = x0 + lx * V, yc = tl.y0 + lyc;
    if (tl.z0 < 4) {
      const DevH8Seg g = h8_find(segs, F.start[4], F.count[4], xc, yc);
      czlo = seg_at(g, xc, yc);
      szlo = (int)g.sz;
    }
    if (tl.z1 + 4 > B.ez) {
      const DevH8Seg g = h8_find(segs, F.start[5], F.count[5], xc, yc);
      czhi = seg_at(g, xc, yc);
      szhi = (int)g.sz;
    }
  }
  auto column = [&](int zz) -> const BL_GLOBAL T* {
    if (FUSED && zz < 0) return u + czlo + (int64_t)zz * szlo;
    if (FUSED && zz >= B.ez) return u + czhi + (int64_t)zz * szhi;
    return u + col + (int64_t)zz * sz;
  };
  VT Q[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) Q[k] = ldv<T, V>(column(tl.z0 - 4 + k));
  VT yh = hy ? ldv<T, V>(u + yh_at + (int64_t)tl.z0 * yh_step) : Q[0];
  T xh = hx ? u[xh_at + (int64_t)tl.z0 * xh_step] : (T)0;
  const int own = (ly + 4) * ldw + 4 + lx * V;
  // running pointers, one plane further each step: the next plane's halo
  // values; the column's next plane and the output are formed from col each
  // step (col is made opaque, so they are not kept as two more 64-bit pointers)
  const BL_GLOBAL T* py = u + yh_at + (int64_t)(tl.z0 + 1) * yh_step;
  const BL_GLOBAL T* px = u + xh_at + (int64_t)(tl.z0 + 1) * xh_step;
  for (int z = tl.z0; z < tl.z1; ++z) {
    int64_t cz = col;
    asm volatile("" : "+v"(cz));
    const BL_GLOBAL T* pq = u + cz + (int64_t)(z + 5) * sz;
    BL_GLOBAL T* pw = w + cz + (int64_t)z * sz;
    T* buf = lds + ((z - tl.z0) & 1) * (ldw * ldh);
    if (active) *reinterpret_cast<VT*>(buf + own) = Q[4];
    if (hy) *reinterpret_cast<VT*>(buf + yh_slot) = yh;
    if (hx) buf[xh_slot] = xh;
    const bool more = z + 1 < tl.z1;
    VT qn = Q[8], yhn = yh;
    T xhn = xh;
    if (more) {
      // plane z + 5 > 0: only the box's planes and those above it
      qn = ldv<T, V>(FUSED ? (z + 5 >= B.ez ? u + czhi + (int64_t)(z + 5) * szhi : pq) : pq);
      if (hy) {
        if (FUSED && yh_f >= 0 && z + 1 > yh_t2hi) {  // the next plane lies in the face's next segment
          const DevH8Seg g = h8_find(segs, Fp->start[yh_f], Fp->count[yh_f], yh_x, z + 1);
          yh_at = seg_at(g, yh_x, yh_y);
          yh_step = (int)g.sz;
          yh_t2hi = g.t2hi;
          py = u + yh_at + (int64_t)(z + 1) * yh_step;
        }
        yhn = ldv<T, V>(py);
      }
      if (hx) {
        if (FUSED && xh_f >= 0 && z + 1 > xh_t2hi) {
          const DevH8Seg g = h8_find(segs, Fp->start[xh_f], Fp->count[xh_f], xh_y, z + 1);
          xh_at = seg_at(g, xh_x, xh_y);
          xh_step = (int)g.sz;
          xh_t2hi = g.t2hi;
          px = u + xh_at + (int64_t)(z + 1) * xh_step;
        }
        xhn = *px;
      }
    }
    py += FUSED ? yh_step : sz;
    px += xh_step;
    lds_sync();
    if (active) {
      // neighbours as whole aligned vectors (one 16-byte LDS read each: reading
      // single elements of neighbouring vectors makes lanes 16 bytes apart and
      // doubles the bank conflicts); x: the K vectors on each side, y: the
      // vectors of the rows 1..4 below and above
      const VT* rv = reinterpret_cast<const VT*>(buf + own);
      constexpr int K = (4 + V - 1) / V;
      const int lv = ldw / V;
      // the y neighbours' 8 reads first; FUSED: the x neighbours' 4 reads once
      // the rows 1 and 2 away are summed, into the registers those freed, so
      // that 4 waves per SIMD fit in the registers (mirror stores included)
      T py1[V], py2[V], py3[V], py4[V];
      {
        VT Ym[4], Yp[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          Ym[m] = rv[-(m + 1) * lv];
          Yp[m] = rv[(m + 1) * lv];
        }
#pragma unroll
        for (int e = 0; e < V; ++e) {
          py1[e] = Ym[0].v[e] + Yp[0].v[e];
          py2[e] = Ym[1].v[e] + Yp[1].v[e];
        }
        if (FUSED) {
#pragma unroll
          for (int e = 0; e < V; ++e) asm volatile("" ::"v"(py1[e]), "v"(py2[e]));
          asm volatile("" ::: "memory");
        }
#pragma unroll
        for (int e = 0; e < V; ++e) {
          py3[e] = Ym[2].v[e] + Yp[2].v[e];
          py4[e] = Ym[3].v[e] + Yp[3].v[e];
        }
      }
      VT X[2 * K + 1];
#pragma unroll
      for (int i = 0; i < 2 * K + 1; ++i) X[i] = i == K ? Q[4] : rv[i - K];
      auto xat = [&](int d) -> T { return X[(d + K * V) / V].v[(d + K * V) % V]; };  // cell d of the row
      VT o;
#pragma unroll
      for (int e = 0; e < V; ++e) {
        const T uc = Q[4].v[e];
        const T px1 = xat(e - 1) + xat(e + 1), px2 = xat(e - 2) + xat(e + 2);
        const T px3 = xat(e - 3) + xat(e + 3), px4 = xat(e - 4) + xat(e + 4);
        const T pz1 = Q[3].v[e] + Q[5].v[e], pz2 = Q[2].v[e] + Q[6].v[e];
        const T pz3 = Q[1].v[e] + Q[7].v[e], pz4 = Q[0].v[e] + Q[8].v[e];
        const T Dx = ((A1 * px1 + A2 * px2) + A3 * px3) + A4 * px4;
        const T Dy = ((A1 * py1[e] + A2 * py2[e]) + A3 * py3[e]) + A4 * py4[e];
        const T Dz = ((A1 * pz1 + A2 * pz2) + A3 * pz3) + A4 * pz4;
        o.v[e] = uc + c * (((Dx + Dy) + Dz) + A0 * uc);
      }
      stv_nt<T, V>(pw, o);
      if (FUSED && moff >= 0) {  // the cells of one vector: consecutive layers, forward on side 0
        // (mo is opaque to the compiler, so the addresses below are formed here
        // from one register rather than hoisted out of the loop as 64-bit values)
        int mo = moff;
        asm volatile("" : "+v"(mo));
        BL_GLOBAL T* pm = w + (B.mir + n * B.sc + (int64_t)z * B.ey);
        const int step = mo >= B.mir_side ? -mlay : mlay;
#pragma unroll
        for (int e = 0; e < V; ++e) pm[mo + e * step] = o.v[e];
      }
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) Q[k] = Q[k + 1];
    Q[8] = qn;
    yh = yhn;
    xh = xhn;
  }
}

__device__ double block_reduce(double v, int op);

// GSRB colour pass, fused with the ghost fill (neighbour boxes read through the
// face records), in place.  color 0 (red: even global i+j+k) or 1 (black)
// updates that colour's cells; every lane stores its whole vector, the other
// colour's cells with their unchanged values, so stores are full lines and a
// concurrent reader sees either value of a cell this pass does not change.
//
// RES: also accumulates r^2, r = f + (s - 6 phi)/h2 in FP64 from promoted
// values (the division taken as a product with 1/h2: the norm is held to
// 1e-13, not to the bit), over the valid cells of colour rescolor (2: all) into
// partials[workgroup].  Race-free pairs only: the black pass (color 1,
// rescolor 1) takes black cells after their update, whose red neighbours this
// pass does not change; the red pass (color 0, rescolor 0) takes red cells
// before their update, whose black neighbours it does not change.  Together
// they give the residual of the state between a black pass and the next red
// pass.  color -1 stores nothing and may take any rescolor.
template <typename T, int V, int ZB, bool RES>
__global__ void __launch_bounds__(kStencilMaxThreads)
    __attribute__((amdgpu_waves_per_eu(RES ? (ZB == 8 ? 2 : 4) : (ZB == 8 ? 3 : 5))))
    k_gsrb_dma(const DevLinTile* __restrict__ tiles, int ntiles, const DevBox* __restrict__ boxes,
               const DevFaceRec* __restrict__ recs, T* phi_, const T* __restrict__ f_, T h2, T inv6, int color,
               int rescolor, double inv_h2d, double* __restrict__ partials, int persist, int yhmax) {
  using VT = Vec<T, V>;
  extern __shared__ unsigned char smem_raw[];
  const TileLds<T, V> S = tile_lds<T, V, ZB>(smem_raw, yhmax);
  BL_GLOBAL T* phi = as_global(phi_);
  const BL_GLOBAL T* __restrict__ fq = as_global(f_);
  double acc = 0.0;
  int first, last;
  tile_range(ntiles, persist, first, last);
  for (int t = first; t < last; ++t) {
    const DevLinTile tl = ldc(tiles + t);
    const DevBox B = ldc(boxes + tl.box);
    const int nvx = B.nvx;
    const int64_t comp0 = B.off + (int64_t)tl.comp * B.sc;
    const int span = ZB * tl.nzs, nsteps = (tl.z1 - tl.z0 + span - 1) / span;
    const bool carry = tl.nzs == 1;

    // z steps as in k_heat_dma.  The two planes carried into a step hold the
    // values from before this pass; the one below the step is also the pass's
    // output there, but a cell of the colour this pass updates has z
    // neighbours of the other colour, which the pass leaves unchanged.
    VT P[ZB + 2], F[ZB];
    for (int j = 0; j < nsteps; ++j) {
      const DevLinTile ts = tile_zstep<ZB>(tl, j);
      const LinLane L = lin_lane<V, ZB>(ts, nvx);
      const int64_t cb = comp0 + (int64_t)L.q * V;
      const int par0 = (B.glo[0] + L.x0 + B.glo[1] + L.y + B.glo[2]) & 1;  // parity of (x0, y, z = 0)
      if (j > 0 && carry) {
        P[0] = P[ZB];
        P[1] = P[ZB + 1];
        load_planes<T, V, true, ZB, 2>(P, L, ts, B, recs, phi, cb);
      } else {
        load_planes<T, V, true, ZB>(P, L, ts, B, recs, phi, cb);
      }
#pragma unroll
      for (int k = 0; k < ZB; ++k) {
        const int z = L.zb0 + k < L.zb1 ? L.zb0 + k : L.zb1 - 1;
        F[k] = ldv<T, V>(fq + cb + (int64_t)z * B.sz);
      }
      stage_halo<T, V, true, ZB>(S, ts, B, recs, phi, comp0);
#pragma unroll
      for (int k = 0; k < ZB; ++k) S.sh[k * S.nthr + threadIdx.x] = P[k + 1];
      __syncthreads();
      BL_GLOBAL T* wp = phi + cb;
#pragma unroll
      for (int k = 0; k < ZB; ++k) {
        const Nbr<T, V> N = tile_neighbours<T, V, ZB, true>(S, L, ts, nvx, k, P[k + 1]);
        const int z = L.zb0 + k;
        const bool valid = z < L.zb1 && L.active;
        VT o = P[k + 1];
        if (color >= 0) {
#pragma unroll
          for (int e = 0; e < V; ++e) {
            const T xm = e == 0 ? N.left : P[k + 1].v[e - 1];
            const T xp = e == V - 1 ? N.right : P[k + 1].v[e + 1];
            const T nv = gsrb_cell(xm, xp, N.ym.v[e], N.yp.v[e], P[k].v[e], P[k + 2].v[e], F[k].v[e], h2, inv6);
            if (((par0 + z + e) & 1) == color) o.v[e] = nv;
          }
        }
        if (RES && valid) {
#pragma unroll
          for (int e = 0; e < V; ++e) {
            if (rescolor != 2 && ((par0 + z + e) & 1) != rescolor) continue;
            const double xm = e == 0 ? (double)N.left : (double)P[k + 1].v[e - 1];
            const double xp = e == V - 1 ? (double)N.right : (double)P[k + 1].v[e + 1];
            const double sv = ((xm + xp) + ((double)N.ym.v[e] + (double)N.yp.v[e])) +
                              ((double)P[k].v[e] + (double)P[k + 2].v[e]);
            // the cell's own value: after its update in the black pass, before it otherwise
            const double cv = color == 1 ? (double)o.v[e] : (double)P[k + 1].v[e];
            const double r = (double)F[k].v[e] + (sv - 6.0 * cv) * inv_h2d;
            acc += r * r;
          }
        }
        if (color < 0) continue;
        if (valid) {
          stv_nt<T, V>(wp + (int64_t)z * B.sz, o);
          stage_edges<T, V, ZB>(S, L, ts, nvx, k, o);
        }
      }
      if (color >= 0) store_mirror<T, V, ZB>(S, ts, B, phi);
      if (persist || j + 1 < nsteps) __syncthreads();  // the next step or tile reuses the LDS buffers
    }
  }
  if (RES) {
    const double r = block_reduce(acc, R_SUM);
    if (threadIdx.x == 0) partials[logical_block()] = r;
  }
}

// ---------------------------------------------------------------- FillBoundary
// One workgroup per chunk of a copy-plan record; bit copies (integer type of the element size).
template <typename I>
__global__ void __launch_bounds__(kFillChunk)
    k_fill(I* __restrict__ data, const DevFillRec* __restrict__ recs, const DevFillChunk* __restrict__ chunks,
           int scomp, int ncomp) {
  const DevFillChunk ch = ldc(chunks + blockIdx.x);
  const DevFillRec R = ldc(recs + ch.rec);
  const int cell = ch.start + (int)threadIdx.x;
  if (cell >= R.nx * R.ny * R.nz) return;
  const int x = cell % R.nx;
  const int t = cell / R.nx;
  const int y = t % R.ny;
  const int z = t / R.ny;
  const int64_t d = R.dst_base + (int64_t)x * R.dsx + (int64_t)y * R.dsy + (int64_t)z * R.dsz;
  const int64_t s = R.src_base + (int64_t)x * R.ssx + (int64_t)y * R.ssy + (int64_t)z * R.ssz;
  for (int n = scomp; n < scomp + ncomp; ++n) data[d + n * R.dsc] = data[s + n * R.ssc];
}

// ---------------------------------------------------------------- dense <-> MultiFab
template <typename T, int V>
__global__ void __launch_bounds__(1024)
    k_copy_global(T* __restrict__ data, T* __restrict__ g, const DevTile* __restrict__ tiles,
                  const DevBox* __restrict__ boxes, int scomp, int ncomp, int dlo0, int dlo1, int dlo2, int Nx, int Ny,
                  int Nz, int to_global) {
  const DevTile tl = ldc(tiles + blockIdx.x);
  const TileLane L = tile_lane<V>(tl);
  if (tl.comp < scomp || tl.comp >= scomp + ncomp || !L.active) return;
  const DevBox B = ldc(boxes + tl.box);
  const int y = L.y, x0 = L.x0;
  const int64_t cb = B.off + (int64_t)tl.comp * B.sc + x0 + (int64_t)y * B.sy;
  for (int z = tl.z0; z < tl.z1; ++z) {
    const int64_t gi = (((int64_t)(tl.comp - scomp) * Nz + (B.glo[2] + z - dlo2)) * Ny + (B.glo[1] + y - dlo1)) * Nx +
                       (B.glo[0] + x0 - dlo0);
    T* p = data + cb + (int64_t)z * B.sz;
#pragma unroll
    for (int e = 0; e < V; ++e) {
      if (to_global)
        g[gi + e] = p[e];
      else
        p[e] = g[gi + e];
    }
  }
}

template <typename T, int V>
__global__ void __launch_bounds__(1024)
    k_set_valid(T* __restrict__ data, T val, const DevTile* __restrict__ tiles, const DevBox* __restrict__ boxes,
                int scomp, int ncomp) {
  const DevTile tl = ldc(tiles + blockIdx.x);
  const TileLane L = tile_lane<V>(tl);
  if (tl.comp < scomp || tl.comp >= scomp + ncomp || !L.active) return;
  const DevBox B = ldc(boxes + tl.box);
  const int64_t cb = B.off + (int64_t)tl.comp * B.sc + L.x0 + (int64_t)L.y * B.sy;
  for (int z = tl.z0; z < tl.z1; ++z)
#pragma unroll
    for (int e = 0; e < V; ++e) data[cb + (int64_t)z * B.sz + e] = val;
}

// whole component blocks (rows with ghosts and padding, x slab, mirror) of components [scomp, scomp+ncomp)
template <typename T>
__global__ void __launch_bounds__(256)
    k_set_fab(T* __restrict__ data, T val, const DevBox* __restrict__ boxes, int scomp, int ncomp) {
  const DevBox B = ldc(boxes + blockIdx.y);
  const int64_t start = B.off - ((int64_t)B.ng * B.sy + (int64_t)B.ng * B.sz) + (int64_t)scomp * B.sc;
  const int64_t count = B.sc * ncomp;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    data[start + i] = val;
}

// ---------------------------------------------------------------- mirror and FAB copies
// The edge-column mirror of every box and component from the state itself
// (before the first fused step of a run).  One workgroup per (box, component).
template <typename T>
__global__ void __launch_bounds__(256)
    k_extract_mirror(T* __restrict__ data, const DevBox* __restrict__ boxes, int ncomp) {
  const DevBox B = ldc(boxes + blockIdx.x / ncomp);
  const int n = blockIdx.x % ncomp;
  const int64_t cnt = (int64_t)B.ey * B.ez;
  T* mir = data + B.mir + (int64_t)n * B.sc;
  const T* rows = data + B.off + (int64_t)n * B.sc;
  for (int64_t q = threadIdx.x; q < cnt; q += blockDim.x) {
    const int y = (int)(q % B.ey), z = (int)(q / B.ey);
    const T* r = rows + (int64_t)y * B.sy + (int64_t)z * B.sz;
    mir[q] = r[0];
    mir[B.mir_side + q] = r[B.ex - 1];
  }
}

// element index of box-local cell (i, j, k) of the grown box, component 0
__device__ __forceinline__ int64_t cell_index(const DevBox& B, int i, int j, int k) {
  if (i >= 0 && i < B.ex) return B.off + i + (int64_t)j * B.sy + (int64_t)k * B.sz;
  const int side = i < 0 ? 0 : 1;
  const int layer = i < 0 ? -1 - i : i - B.ex;
  return B.xs + (int64_t)side * B.xs_side + (int64_t)k * B.xs_z + (int64_t)j * B.ng + layer;
}

// FAB `box` (grown box, components [scomp, scomp+ncomp)) <-> dense (ncomp, nz, ny, nx) array
template <typename I>
__global__ void __launch_bounds__(256)
    k_copy_fab(I* __restrict__ data, I* __restrict__ dense, const DevBox* __restrict__ boxes, int box, int scomp,
               int ncomp, int to_dense) {
  const DevBox B = ldc(boxes + box);
  const int g = B.ng;
  const int nx = B.ex + 2 * g, ny = B.ey + 2 * g, nz = B.ez + 2 * g;
  const int64_t total = (int64_t)ncomp * nz * ny * nx;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(q % nx) - g;
    int64_t r = q / nx;
    const int j = (int)(r % ny) - g;
    r /= ny;
    const int k = (int)(r % nz) - g;
    const int n = (int)(r / nz) + scomp;
    const int64_t e = cell_index(B, i, j, k) + (int64_t)n * B.sc;
    if (to_dense)
      dense[q] = data[e];
    else
      data[e] = dense[q];
  }
}

// ---------------------------------------------------------------- reductions
__device__ __forceinline__ double r_identity(int op) {
  if (op == R_MAX) return -INFINITY;
  if (op == R_MIN) return INFINITY;
  return 0.0;
}
__device__ __forceinline__ double r_term(double v, int op) {
  if (op == R_NORM0 || op == R_NORM1) return fabs(v);
  if (op == R_NORM2) return v * v;
  return v;
}
__device__ __forceinline__ double r_combine(double a, double b, int op) {
  if (op == R_MAX || op == R_NORM0) return fmax(a, b);
  if (op == R_MIN) return fmin(a, b);
  return a + b;
}

// Fixed-shape reduction of one value per thread: wave64 butterfly, then the
// wave results in order.  Deterministic for a given block size.
__device__ double block_reduce(double v, int op) {
  __shared__ double wsum[16];
  for (int off = 32; off > 0; off >>= 1) v = r_combine(v, __shfl_xor(v, off, 64), op);
  const int wave = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  if ((threadIdx.x & 63) == 0) wsum[wave] = v;
  __syncthreads();
  double r = r_identity(op);
  if (threadIdx.x == 0)
    for (int i = 0; i < nw; ++i) r = r_combine(r, wsum[i], op);
  __syncthreads();
  return r;  // valid in thread 0
}

// Reduction over the valid cells of one component: a workgroup per chunk
// (planes z0..z1-1 of one box), each plane one contiguous run read with four
// independent vector loads per lane in flight.
template <typename T, int V>
__global__ void __launch_bounds__(256)
    k_reduce_chunks(const T* __restrict__ data_, const DevRedChunk* __restrict__ chunks,
                    const DevBox* __restrict__ boxes, int comp, int op, double* __restrict__ partials) {
  const DevRedChunk ch = ldc(chunks + blockIdx.x);
  const DevBox B = ldc(boxes + ch.box);
  const BL_GLOBAL T* data = as_global(data_);
  const int nv = B.ex * B.ey / V;
  const int bd = (int)blockDim.x;
  double acc = r_identity(op);
  for (int z = ch.z0; z < ch.z1; ++z) {
    const BL_GLOBAL T* run = data + B.off + (int64_t)comp * B.sc + (int64_t)z * B.sz;
    for (int i = threadIdx.x; i < nv; i += 4 * bd) {
      Vec<T, V> v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int j = i + u * bd < nv ? i + u * bd : i;
        v[u] = ldv<T, V>(run + (int64_t)j * V);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (i + u * bd < nv)
#pragma unroll
          for (int e = 0; e < V; ++e) acc = r_combine(acc, r_term((double)v[u].v[e], op), op);
    }
  }
  const double r = block_reduce(acc, op);
  if (threadIdx.x == 0) partials[blockIdx.x] = r;
}

template <typename T, int V>
__global__ void __launch_bounds__(1024)
    k_reduce_tiles(const T* __restrict__ data, const DevTile* __restrict__ tiles, const DevBox* __restrict__ boxes,
                   int comp, int op, double* __restrict__ partials) {
  const DevTile tl = ldc(tiles + blockIdx.x);
  const TileLane L = tile_lane<V>(tl);
  double acc = r_identity(op);
  if (tl.comp == comp && L.active) {
    const DevBox B = ldc(boxes + tl.box);
    const T* p = data + B.off + (int64_t)comp * B.sc + L.x0 + (int64_t)L.y * B.sy;
    for (int z = tl.z0; z < tl.z1; ++z) {
      const Vec<T, V> v = ldv<T, V>(p + (int64_t)z * B.sz);
#pragma unroll
      for (int e = 0; e < V; ++e) acc = r_combine(acc, r_term((double)v.v[e], op), op);
    }
  }
  const double r = block_reduce(acc, op);
  if (threadIdx.x == 0) partials[blockIdx.x] = r;
}

__global__ void __launch_bounds__(1024)
    k_reduce_final(const double* __restrict__ partials, int n, int op, int take_sqrt, double* __restrict__ out) {
  double acc = r_identity(op);
  for (int i = threadIdx.x; i < n; i += blockDim.x) acc = r_combine(acc, partials[i], op);
  const double r = block_reduce(acc, op);
  if (threadIdx.x == 0) *out = take_sqrt ? sqrt(r) : r;
}

// ---------------------------------------------------------------- red-black Gauss-Seidel
// One colour, in place, reading phi's filled ghosts.  Cells of the colour read
// only cells of the other colour, which no lane writes during this pass.
template <typename T, int V>
__global__ void __launch_bounds__(1024)
    k_gsrb(const DevTile* __restrict__ tiles, const DevBox* __restrict__ boxes, T* __restrict__ phi,
           const T* __restrict__ f, T h2, T inv6, int color) {
  const DevTile tl = ldc(tiles + blockIdx.x);
  const TileLane L = tile_lane<V>(tl);
  if (!L.active) return;
  const DevBox B = ldc(boxes + tl.box);
  const int y = L.y, x0 = L.x0;
  const int64_t cb = B.off + x0 + (int64_t)y * B.sy;
  T* pp = phi + cb;
  const T* fp = f + cb;
  const int sy = B.sy, sz = B.sz;
  const int par0 = (B.glo[0] + x0 + B.glo[1] + y + B.glo[2]) & 1;
  const int64_t lb = L.xv == 0 ? B.xs + (int64_t)y * B.ng : cb - 1;
  const int64_t rb = L.xv == B.nvx - 1 ? B.xs + B.xs_side + (int64_t)y * B.ng : cb + V;
  const int ls = L.xv == 0 ? B.xs_z : sz, rs = L.xv == B.nvx - 1 ? B.xs_z : sz;
  for (int z = tl.z0; z < tl.z1; ++z) {
    T* pz = pp + z * sz;
    const Vec<T, V> cc = ldv<T, V>(pz);
    const Vec<T, V> zm = ldv<T, V>(pz - sz);
    const Vec<T, V> zp = ldv<T, V>(pz + sz);
    const Vec<T, V> ym = ldv<T, V>(pz - sy);
    const Vec<T, V> yp = ldv<T, V>(pz + sy);
    const Vec<T, V> fv = ldv<T, V>(fp + z * sz);
    const T left = phi[lb + (int64_t)z * ls], right = phi[rb + (int64_t)z * rs];
#pragma unroll
    for (int e = 0; e < V; ++e) {
      if (((par0 + z + e) & 1) != color) continue;
      const T xm = e == 0 ? left : cc.v[e - 1];
      const T xp = e == V - 1 ? right : cc.v[e + 1];
      pz[e] = gsrb_cell(xm, xp, ym.v[e], yp.v[e], zm.v[e], zp.v[e], fv.v[e], h2, inv6);
    }
  }
}

// r = f + (s - 6 phi)/h2 in FP64 from promoted values; per-tile sums of r^2
template <typename T, int V>
__global__ void __launch_bounds__(1024)
    k_residual(const DevTile* __restrict__ tiles, const DevBox* __restrict__ boxes, const T* __restrict__ phi,
               const T* __restrict__ f, double h2, double* __restrict__ partials) {
  const DevTile tl = ldc(tiles + blockIdx.x);
  const TileLane L = tile_lane<V>(tl);
  double acc = 0.0;
  if (L.active) {
    const DevBox B = ldc(boxes + tl.box);
    const int64_t cb = B.off + L.x0 + (int64_t)L.y * B.sy;
    const T* pp = phi + cb;
    const T* fp = f + cb;
    const int sy = B.sy, sz = B.sz;
    const int64_t lb = L.xv == 0 ? B.xs + (int64_t)L.y * B.ng : cb - 1;
    const int64_t rb = L.xv == B.nvx - 1 ? B.xs + B.xs_side + (int64_t)L.y * B.ng : cb + V;
    const int ls = L.xv == 0 ? B.xs_z : sz, rs = L.xv == B.nvx - 1 ? B.xs_z : sz;
    for (int z = tl.z0; z < tl.z1; ++z) {
      const T* pz = pp + z * sz;
      const Vec<T, V> cc = ldv<T, V>(pz);
      const Vec<T, V> zm = ldv<T, V>(pz - sz);
      const Vec<T, V> zp = ldv<T, V>(pz + sz);
      const Vec<T, V> ym = ldv<T, V>(pz - sy);
      const Vec<T, V> yp = ldv<T, V>(pz + sy);
      const Vec<T, V> fv = ldv<T, V>(fp + z * sz);
      const double left = (double)phi[lb + (int64_t)z * ls], right = (double)phi[rb + (int64_t)z * rs];
#pragma unroll
      for (int e = 0; e < V; ++e) {
        const double xm = e == 0 ? left : (double)cc.v[e - 1];
        const double xp = e == V - 1 ? right : (double)cc.v[e + 1];
        const double s = ((xm + xp) + ((double)ym.v[e] + (double)yp.v[e])) + ((double)zm.v[e] + (double)zp.v[e]);
        const double r = (double)fv.v[e] + (s - 6.0 * (double)cc.v[e]) / h2;
        acc += r * r;
      }
    }
  }
  const double r = block_reduce(acc, R_SUM);
  if (threadIdx.x == 0) partials[blockIdx.x] = r;
}

template <typename T, int V, int ZB>
hipError_t heat_dispatch_zb(bool fused, const HeatArgs& a, int g, int block, int persist, hipStream_t s) {
#define BL_LAUNCH_ROWS(F, Y)                                                                                     \
  hipLaunchKernelGGL((k_heat_rows<T, V, F, Y, ZB>), dim3(g), dim3(block), 0, s, a.tiles, a.ntiles, a.boxes, a.recs, \
                     a.m0, a.members, a.flip, persist)
  if (!fused) BL_LAUNCH_ROWS(false, true);
  else if (a.fvec) BL_LAUNCH_ROWS(true, true);
  else BL_LAUNCH_ROWS(true, false);
#undef BL_LAUNCH_ROWS
  return hipGetLastError();
}

template <typename T, int V, int ZB>
hipError_t heat_dispatch_lds(bool fused, const HeatArgs& a, int g, int block, int persist, hipStream_t s) {
  const int rmax = a.rmax > 0 ? a.rmax : block;
  const size_t lds = (size_t)ZB * block * sizeof(Vec<T, V>) + (fused ? (size_t)2 * ZB * rmax * sizeof(T) : 0);
  if (fused)
    hipLaunchKernelGGL((k_heat_lds<T, V, true, ZB>), dim3(g), dim3(block), lds, s, a.tiles, a.ntiles, a.boxes, a.recs,
                       a.m0, a.members, a.flip, persist, rmax);
  else
    hipLaunchKernelGGL((k_heat_lds<T, V, false, ZB>), dim3(g), dim3(block), lds, s, a.tiles, a.ntiles, a.boxes,
                       a.recs, a.m0, a.members, a.flip, persist, rmax);
  return hipGetLastError();
}

template <typename T, int V, int ZB>
size_t dma_lds_bytes(int yhmax, int xhmax, int block) {
  return (size_t)ZB * block * sizeof(Vec<T, V>) + (size_t)ZB * 2 * yhmax * sizeof(Vec<T, V>) +
         (size_t)ZB * 2 * xhmax * sizeof(T);
}

template <typename T, int V, int ZB>
hipError_t heat_dispatch_dma(bool fused, const HeatArgs& a, int block, int grid, hipStream_t s) {
  const int persist = grid > 0 ? 1 : 0;
  const int g = persist ? (grid < a.nlin ? grid : a.nlin) : a.nlin;
  const size_t lds = dma_lds_bytes<T, V, ZB>(a.yhmax, a.xhmax, block);
  if (fused)
    hipLaunchKernelGGL((k_heat_dma<T, V, true, ZB>), dim3(g), dim3(block), lds, s, a.lin, a.nlin, a.boxes, a.recs,
                       a.m0, a.members, a.flip, persist, a.yhmax);
  else
    hipLaunchKernelGGL((k_heat_dma<T, V, false, ZB>), dim3(g), dim3(block), lds, s, a.lin, a.nlin, a.boxes, a.recs,
                       a.m0, a.members, a.flip, persist, a.yhmax);
  return hipGetLastError();
}

template <typename T, int V>
hipError_t heat_dispatch(bool fused, const HeatArgs& a, int grid, int block, hipStream_t s) {
  const int persist = grid > 0 ? 1 : 0;
  const int g = persist ? (grid < a.ntiles ? grid : a.ntiles) : a.ntiles;
  // the halo-in-LDS form over the linear tiles (its LDS is checked when the plan is made)
  if (a.form == 3 && a.lin && (!fused || a.fvec)) {
    switch (a.zblock) {
      case 2: return heat_dispatch_dma<T, V, 2>(fused, a, block, grid, s);
      case 8: return heat_dispatch_dma<T, V, 8>(fused, a, block, grid, s);
      default: return heat_dispatch_dma<T, V, 4>(fused, a, block, grid, s);
    }
  }
  if (a.form >= 2 && (!fused || a.fvec)) {
    switch (a.zblock) {
      case 2: return heat_dispatch_lds<T, V, 2>(fused, a, g, block, persist, s);
      case 4: return heat_dispatch_lds<T, V, 4>(fused, a, g, block, persist, s);
      case 8: return heat_dispatch_lds<T, V, 8>(fused, a, g, block, persist, s);
      default: break;
    }
  }
  switch (a.zblock) {
    case 2: return heat_dispatch_zb<T, V, 2>(fused, a, g, block, persist, s);
    case 4: return heat_dispatch_zb<T, V, 4>(fused, a, g, block, persist, s);
    case 8: return heat_dispatch_zb<T, V, 8>(fused, a, g, block, persist, s);
    default: return heat_dispatch_zb<T, V, 0>(fused, a, g, block, persist, s);
  }
}

// ---------------------------------------------------------------- red-black sweep in one pass
// A sweep is a red pass then a black pass; a black cell's neighbours are all
// red and a red cell's all black, so one launch can do both if it has, for
// every black cell, the new values of its six red neighbours.  Inside a box
// they are computed one plane ahead; next to a face they are the neighbour
// box's new red values at its own face cells, which the ring kernel computes
// beforehand into the box's ghost layer, at the red positions only (the black
// positions keep the old values that the red update of the box's own face
// cells needs).  Both kernels evaluate every cell with gsrb_cell on the same
// operands as the two-pass form, so FP64 results are the same bits.

// Value of source box-local cell (i, j, k) of phi.  XF (the cell lies on the
// box's low or high x column, the source of an x face): valid cells of columns
// 0 and ex-1 from the edge mirror and of columns 1 and ex-2 from the second
// edge-column copy m2 (2*ey*ez values: side 0 then side 1), so that a wave's
// lanes, which run along y, read contiguous values; any other cell from the
// FAB (rows or x ghost slab).
template <typename T>
__device__ __forceinline__ T ring_val(const BL_GLOBAL T* __restrict__ phi, const BL_GLOBAL T* __restrict__ m2,
                                      const DevBox& S, int i, int j, int k, bool xf) {
  if (xf && j >= 0 && j < S.ey && k >= 0 && k < S.ez) {
    const int64_t yz = (int64_t)k * S.ey + j;
    if (i == 0) return phi[S.mir + yz];
    if (i == S.ex - 1) return phi[S.mir + S.mir_side + yz];
    if (i == 1) return m2[yz];
    if (i == S.ex - 2) return m2[(int64_t)S.ey * S.ez + yz];
  }
  return phi[cell_index(S, i, j, k)];
}

// The new red values of every covered face ghost cell, written into the ghost
// layer at the red positions: the red update of the source box's cell, from its
// six neighbours in the source FAB (whose face ghosts hold the old values) and
// f.  One workgroup per record, a lane per red cell (h1 = red cells per row
// at most, rows along t2).  Reads only black positions and writes only red
// ones, through separate views.
template <typename T>
__global__ void __launch_bounds__(256)
    k_gsrb_ring(T* phi_, const T* __restrict__ f_, const DevBox* __restrict__ boxes,
                const DevRingRec* __restrict__ recs, const T* __restrict__ mir2_,
                const int64_t* __restrict__ mir2off, T h2, T inv6) {
  const DevRingRec R = ldc(recs + blockIdx.x);
  const int h1 = (R.n1 + 1) / 2, ncell = h1 * R.n2;
  const DevBox D = ldc(boxes + R.box);
  const DevBox S = ldc(boxes + R.src);
  const BL_GLOBAL T* __restrict__ phi = as_global(static_cast<const T*>(phi_));
  BL_GLOBAL T* __restrict__ out = as_global(phi_);
  const BL_GLOBAL T* f = as_global(f_);
  const BL_GLOBAL T* m2 = as_global(mir2_) + mir2off[R.src];
  const int a = R.face >> 1;
  const bool xf = a == 0;
  const int par00 = (D.glo[0] + R.lo[0] + D.glo[1] + R.lo[1] + D.glo[2] + R.lo[2]) & 1;
  for (int c = (int)threadIdx.x; c < ncell; c += (int)blockDim.x) {
    const int u2 = c / h1;
    const int u1 = 2 * (c - u2 * h1) + ((par00 + u2) & 1);  // the red cell: (par00 + u1 + u2) even
    if (u1 >= R.n1) continue;
    int q0 = R.lo[0], q1 = R.lo[1], q2 = R.lo[2];
    if (a == 0) {
      q1 += u1;
      q2 += u2;
    } else if (a == 1) {
      q0 += u1;
      q2 += u2;
    } else {
      q0 += u1;
      q1 += u2;
    }
    const int i = q0 + R.d[0], j = q1 + R.d[1], k = q2 + R.d[2];
    const T xm = ring_val(phi, m2, S, i - 1, j, k, xf), xp = ring_val(phi, m2, S, i + 1, j, k, xf);
    const T ym = ring_val(phi, m2, S, i, j - 1, k, xf), yp = ring_val(phi, m2, S, i, j + 1, k, xf);
    const T zm = ring_val(phi, m2, S, i, j, k - 1, xf), zp = ring_val(phi, m2, S, i, j, k + 1, xf);
    const T fv =
        xf ? f[S.mir + (i == 0 ? 0 : (int64_t)S.mir_side) + (int64_t)k * S.ey + j] : f[cell_index(S, i, j, k)];
    out[cell_index(D, q0, q1, q2)] = gsrb_cell(xm, xp, ym, yp, zm, zp, fv, h2, inv6);
  }
}

// Both edge-column copies of component 0: columns 0 and ex-1 into the edge
// mirror, columns 1 and ex-2 into m2 (as read by ring_val).
template <typename T>
__global__ void __launch_bounds__(256)
    k_extract_edges2(T* __restrict__ data, const DevBox* __restrict__ boxes, T* __restrict__ mir2,
                     const int64_t* __restrict__ mir2off) {
  const DevBox B = ldc(boxes + blockIdx.x);
  const int64_t cnt = (int64_t)B.ey * B.ez;
  T* mir = data + B.mir;
  T* m2 = mir2 + mir2off[blockIdx.x];
  for (int64_t q = threadIdx.x; q < cnt; q += blockDim.x) {
    const int y = (int)(q % B.ey), z = (int)(q / B.ey);
    const T* r = data + B.off + (int64_t)y * B.sy + (int64_t)z * B.sz;
    mir[q] = r[0];
    mir[B.mir_side + q] = r[B.ex - 1];
    m2[q] = r[1];
    m2[cnt + q] = r[B.ex - 2];
  }
}

// Value at x cell e of vector v, or the plane's neighbour values at the ends.
template <typename T, int V>
struct PlaneNbr {
  T left, right;
  Vec<T, V> ym, yp;
};

// In-plane neighbours of a lane's vector (row y, first cell x0) from an LDS
// plane buffer: (ey + 2) rows of ex values (ghost row y = -1, the valid rows,
// ghost row y = ey), then the ey low-x and ey high-x ghost values.
template <typename T, int V>
__device__ __forceinline__ PlaneNbr<T, V> plane_nbr(const T* pb, int ex, int ey, int nvx, int y, int xv) {
  PlaneNbr<T, V> N;
  const int x0 = xv * V, rowsz = (ey + 2) * ex;
  const T* row = pb + (y + 1) * ex + x0;
  N.ym = ldv<T, V>(row - ex);
  N.yp = ldv<T, V>(row + ex);
  N.left = xv > 0 ? row[-1] : pb[rowsz + y];
  N.right = xv < nvx - 1 ? row[V] : pb[rowsz + ey + y];
  return N;
}

// A box's new face cells into the face ghost cells of the boxes they border
// (push records of one face of the box).  x faces: the value of cell (y, z);
// y and z faces: the V values of x cells x0.. of row t2 (z, or y for z faces).
template <typename T>
__device__ __forceinline__ void push_x(BL_GLOBAL T* out, const DevPushRec* __restrict__ recs, int start, int count,
                                       int y, int z, T v) {
  for (int r = start; r < start + count; ++r) {
    const DevPushRec Q = ldc(recs + r);
    if (y >= Q.t1lo && y <= Q.t1hi && z >= Q.t2lo && z <= Q.t2hi)
      out[Q.base + (int64_t)y * Q.s1 + (int64_t)z * Q.s2] = v;
  }
}
template <typename T, int V>
__device__ __forceinline__ void push_row(BL_GLOBAL T* out, const DevPushRec* __restrict__ recs, int start, int count,
                                         int x0, int t2, const Vec<T, V>& o) {
  for (int r = start; r < start + count; ++r) {
    const DevPushRec Q = ldc(recs + r);
    if (t2 < Q.t2lo || t2 > Q.t2hi) continue;
    const int64_t b = Q.base + (int64_t)t2 * Q.s2 + x0;
    if (x0 >= Q.t1lo && x0 + V - 1 <= Q.t1hi && b % V == 0) {  // the whole vector, aligned
      stv<T, V>(out + b, o);
      continue;
    }
#pragma unroll
    for (int e = 0; e < V; ++e)
      if (x0 + e >= Q.t1lo && x0 + e <= Q.t1hi) out[b + e] = o.v[e];
  }
}

// The cells of one colour in a lane's vector c (the colour of cell e is that of
// e + q, q = 0 or 1 per lane): cells e = 2k + q, k < V/2, each solved from its
// six neighbours (the values left and right of the vector, the vectors of the
// rows and planes around it) and f, the other cells kept.  Operands picked by
// selects, so a lane computes V/2 updates whatever its parity.  RES: r^2 with
// r = f + (s - 6v)/h2 in FP64 from promoted values, v the cell's old value
// (AFTER false) or new one (AFTER true), added to acc.
// (The vectors come by value: a select between two elements of a vector behind
// a reference becomes one load at a variable index, which puts the caller's
// vectors in scratch memory.)
template <typename T, int V, bool AFTER, int QS>
__device__ __forceinline__ Vec<T, V> colour_update_t(Vec<T, V> c, T left, T right, Vec<T, V> ym, Vec<T, V> yp,
                                                     Vec<T, V> zm, Vec<T, V> zp, Vec<T, V> fv, int q, T h2, T inv6,
                                                     bool res, double inv_h2d, double& acc) {
  Vec<T, V> o = c;
  const bool s = QS >= 0 ? QS != 0 : q != 0;
#pragma unroll
  for (int k = 0; k < V / 2; ++k) {
    const int e0 = 2 * k, e1 = 2 * k + 1;
    const T own = s ? c.v[e1] : c.v[e0];
    const T xm = s ? c.v[e0] : (e0 == 0 ? left : c.v[e0 - 1]);
    const T xp = s ? (e1 == V - 1 ? right : c.v[e1 + 1]) : c.v[e1];
    const T a = s ? ym.v[e1] : ym.v[e0], b = s ? yp.v[e1] : yp.v[e0];
    const T cz = s ? zm.v[e1] : zm.v[e0], dz = s ? zp.v[e1] : zp.v[e0];
    const T ff = s ? fv.v[e1] : fv.v[e0];
    const T nv = gsrb_cell(xm, xp, a, b, cz, dz, ff, h2, inv6);
    o.v[e0] = s ? c.v[e0] : nv;
    o.v[e1] = s ? nv : c.v[e1];
    if (res) {
      const double sv = ((double)xm + (double)xp) + ((double)a + (double)b);
      const double sum = sv + ((double)cz + (double)dz);
      const double v = AFTER ? (double)nv : (double)own;
      const double rr = (double)ff + (sum - 6.0 * v) * inv_h2d;
      acc += rr * rr;
    }
  }
  return o;
}

// The same with the parity taken as a branch into one of two select-free
// bodies: where all lanes of a wave share q (the sweep lays out its lanes so
// that they do), the wave runs one body only.
template <typename T, int V, bool AFTER>
__device__ __forceinline__ Vec<T, V> colour_update(Vec<T, V> c, T left, T right, Vec<T, V> ym, Vec<T, V> yp,
                                                   Vec<T, V> zm, Vec<T, V> zp, Vec<T, V> fv, int q, T h2, T inv6,
                                                   bool res, double inv_h2d, double& acc) {
  if (q == 0) return colour_update_t<T, V, AFTER, 0>(c, left, right, ym, yp, zm, zp, fv, q, h2, inv6, res, inv_h2d, acc);
  return colour_update_t<T, V, AFTER, 1>(c, left, right, ym, yp, zm, zp, fv, q, h2, inv6, res, inv_h2d, acc);
}

// One red-black sweep of the valid planes z0..z1-1 of one box per workgroup
// (DevRedChunk), from phi into out (another buffer of the same layout).  phi's
// face ghosts hold the old values at black positions and the new red values at
// red positions (FillBoundary, then k_gsrb_ring).  The workgroup marches up z:
// at plane i it computes the new red values of plane i from the old planes
// i-1..i+1, then the new black values of plane i-1 from the red values of
// planes i-2..i, and stores plane i-1: its cells, its four edge columns (the
// edge mirror and the second copy; staged in LDS and stored by a few lanes one
// plane later) and its face cells into the face ghost cells of out that they
// fill (push records), so that out needs no FillBoundary before the next sweep.  It starts one plane below z0 and ends one
// above z1 (red values only there); the planes outside the box are phi's
// ghost planes as they stand.  Lane l takes plane vectors l + m*blockDim.x,
// m < K; each plane passes through one of three LDS buffers (old values, then
// the red values written over them in place: a cell's red update reads only
// black cells, which keep their values), one barrier per plane; other lanes
// read a buffer only while it holds plane i or i-1.  Plane i+2 and f of plane
// i+1 are loaded during plane i.
//
// Norms (partials per workgroup, FP64 from promoted values, as the two-pass
// form): red_part takes r^2 at the red cells of phi (the state before the
// sweep), black_part at the black cells of the result; the sum of the black
// part of one sweep and the red part of the next is the squared residual norm
// of the state between them.
template <typename T, int V, int K>
__global__ void __launch_bounds__(1024)
    k_gsrb_sweep(const DevBox* __restrict__ boxes, const DevRedChunk* __restrict__ work, const T* phi_, T* out_,
                 const T* __restrict__ f_, T* omir2_, const int64_t* __restrict__ mir2off,
                 const DevPushRec* __restrict__ push, const DevPushFace* __restrict__ pface, T h2, T inv6,
                 double inv_h2d, double* __restrict__ red_part, double* __restrict__ black_part) {
  using VT = Vec<T, V>;
  extern __shared__ unsigned char smem_raw[];
  const int wg = (int)blockIdx.x;
  const DevRedChunk W = ldc(work + wg);
  const DevBox B = ldc(boxes + W.box);
  const BL_GLOBAL T* phi = as_global(phi_);
  const BL_GLOBAL T* fq = as_global(f_);
  BL_GLOBAL T* out = as_global(out_);
  BL_GLOBAL T* omir2 = as_global(omir2_) + mir2off[W.box];
  const int ex = B.ex, ey = B.ey, ez = B.ez, nvx = B.nvx, P = ey * nvx;
  const int nthr = (int)blockDim.x, tid = (int)threadIdx.x;
  const int z0 = W.z0, z1 = W.z1;
  const int rowsz = (ey + 2) * ex, bufsz = (rowsz + 2 * ey + V - 1) / V * V;
  T* lds = reinterpret_cast<T*>(smem_raw);
  // the four edge columns of a stored plane (x = 0, 1, ex-2, ex-1), staged for
  // coalesced stores one plane later: two sets of 4*ey values
  T* stg = lds + 3 * bufsz;
  const int64_t sz = B.sz;
  const int gpar = B.glo[0] + B.glo[1] + B.glo[2];
  const DevPushFace PF = ldc(pface + W.box);

  // the lane's vectors: row, x vector, offset (plane 0) and parity of their
  // first cell at z = 0.  Vector index q runs over the even rows first, then the
  // odd rows, so that the lanes of a wave share their colour pattern (x
  // vectors start at even x).
  bool act[K];
  int yv[K], xvv[K], par[K];
  int64_t go[K];
  const int neven = (ey + 1) / 2 * nvx;
#pragma unroll
  for (int m = 0; m < K; ++m) {
    const int q = tid + m * nthr;
    act[m] = q < P;
    const int qq = act[m] ? q : P - 1;
    const int odd = qq >= neven ? 1 : 0, qr = qq - odd * neven, rr = qr / nvx;
    yv[m] = 2 * rr + odd;
    xvv[m] = qr - rr * nvx;
    go[m] = B.off + (int64_t)yv[m] * B.sy + (int64_t)xvv[m] * V;
    par[m] = (gpar + xvv[m] * V + yv[m]) & 1;
  }
  // the lane's ghost item of each plane: a vector of the ghost rows, or an x ghost value
  const int nyr = 2 * nvx, nring = nyr + 2 * ey;
  int64_t ra;
  int64_t rstep;
  int rl;  // LDS offset in a plane buffer
  if (tid < nyr) {
    const int side = tid / nvx, xv = tid - side * nvx;
    ra = B.off + (int64_t)(side ? ey : -1) * B.sy + (int64_t)xv * V;
    rstep = sz;
    rl = (side ? ey + 1 : 0) * ex + xv * V;
  } else {
    const int t = tid < nring ? tid - nyr : 0, side = t / ey, yy = t - side * ey;
    ra = B.xs + (int64_t)side * B.xs_side + (int64_t)yy * B.ng;
    rstep = B.xs_z;
    rl = rowsz + side * ey + yy;
  }
  auto ring_load = [&](int z, VT& h) {
    if (tid < nyr)
      h = ldv<T, V>(phi + ra + (int64_t)z * rstep);
    else if (tid < nring)
      h.v[0] = phi[ra + (int64_t)z * rstep];
  };
  auto ring_store = [&](T* pb, const VT& h) {
    if (tid < nyr)
      stv<T, V>(pb + rl, h);
    else if (tid < nring)
      pb[rl] = h.v[0];
  };
  auto plane_at = [&](int m, int z) -> VT {  // z in [-1, ez]
    return ldv<T, V>(phi + go[m] + (int64_t)z * sz);
  };
  auto f_at = [&](int m, int z) -> VT { return ldv<T, V>(fq + go[m] + (int64_t)z * sz); };
  auto clampz = [&](int z) { return z < -1 ? -1 : (z > ez ? ez : z); };
  auto clampf = [&](int z) { return z < 0 ? 0 : (z > ez - 1 ? ez - 1 : z); };

  // registers: plane i+1 (Gp) and i+2 (Gn, in flight) at the lane's vectors, f
  // of planes i-1..i+1, the new red vector of plane i; planes i-2..i are read
  // back from their LDS buffers at the lane's own position
  VT Gp[K], Gn[K], Fm[K], Fc[K], Fn[K], Rc[K];
  VT H, Hn;
  const int i0 = z0 - 1;
  auto own = [&](int m) { return (yv[m] + 1) * ex + xvv[m] * V; };
  // planes i0-1 and i0 into buffers 2 and 0 (the ghost items of plane i0 when it
  // is a valid plane), plane i0+1 into registers
  ring_load(clampf(i0), H);
#pragma unroll
  for (int m = 0; m < K; ++m) {
    const VT a = plane_at(m, clampz(i0 - 1)), b = plane_at(m, clampz(i0));
    Gp[m] = plane_at(m, clampz(i0 + 1));
    Fc[m] = f_at(m, clampf(i0));
    Fm[m] = Fc[m];
    if (act[m]) {
      stv<T, V>(lds + 2 * bufsz + own(m), a);
      stv<T, V>(lds + own(m), b);
    }
  }
  if (i0 >= 0 && i0 < ez) ring_store(lds, H);
  // the staged edge columns of plane zz (set sidx) into out's edge mirror, the
  // second copy and the x-face ghosts of the neighbours: lane t < 4*ey takes
  // column t / ey, row t % ey
  auto flush_edges = [&](int sidx, int zz) {
    if (tid < 4 * ey) {
      const int c = tid / ey, y = tid - c * ey;
      const T v = stg[sidx * 4 * ey + tid];
      const int64_t yz = (int64_t)zz * ey + y;
      if (c == 0) {
        out[B.mir + yz] = v;
        push_x(out, push, PF.start[0], PF.count[0], y, zz, v);
      } else if (c == 1) {
        omir2[yz] = v;
      } else if (c == 2) {
        omir2[(int64_t)ey * ez + yz] = v;
      } else {
        out[B.mir + B.mir_side + yz] = v;
        push_x(out, push, PF.start[1], PF.count[1], y, zz, v);
      }
    }
  };
  double accr = 0.0, accb = 0.0;
  for (int i = i0; i <= z1; ++i) {
    const int r = i - i0, bc = r % 3, bm = (r + 2) % 3, bn = (r + 1) % 3;
    T* pc = lds + bc * bufsz;  // plane i
    T* pm = lds + bm * bufsz;  // plane i-1 (new red values)
    T* pn = lds + bn * bufsz;  // plane i-2 (new red values), then plane i+1
    lds_barrier();  // LDS only: the global stores need no wait, the loads are waited for where used
    // loads for the next planes: the ghost item first, so that waiting for it
    // at the end of this plane leaves the plane loads in flight
    const bool next_in = i + 1 <= ez && i + 1 <= z1;
    if (i + 1 < ez && i + 1 <= z1) ring_load(i + 1, Hn);
#pragma unroll
    for (int m = 0; m < K; ++m) {
      Gn[m] = plane_at(m, clampz(i + 2));
      Fn[m] = f_at(m, clampf(i + 1));
    }
    if (i - 2 >= z0) flush_edges((i - 1) & 1, i - 2);  // the plane stored one step ago
    // red values of plane i
    if (i >= 0 && i < ez) {
      const bool resr = red_part && i >= z0 && i < z1;
#pragma unroll
      for (int m = 0; m < K; ++m) {
        const PlaneNbr<T, V> N = plane_nbr<T, V>(pc, ex, ey, nvx, yv[m], xvv[m]);
        const VT g = ldv<T, V>(pc + own(m));
        const VT gm = ldv<T, V>(pm + own(m));  // plane i-1: old values at its black cells
        const VT o = colour_update<T, V, false>(g, N.left, N.right, N.ym, N.yp, gm, Gp[m], Fc[m], (par[m] + i) & 1,
                                                h2, inv6, resr && act[m], inv_h2d, accr);
        Rc[m] = o;
        if (act[m]) stv<T, V>(pc + own(m), o);
      }
    } else {
#pragma unroll
      for (int m = 0; m < K; ++m) Rc[m] = ldv<T, V>(pc + own(m));  // a ghost plane as it stands
    }
    // black values of plane i-1, stored: its cells, its edge columns, its face
    // cells into the neighbours' face ghosts of out
    if (i - 1 >= z0) {
      const int z = i - 1;
#pragma unroll
      for (int m = 0; m < K; ++m) {
        const PlaneNbr<T, V> N = plane_nbr<T, V>(pm, ex, ey, nvx, yv[m], xvv[m]);
        const VT rm1 = ldv<T, V>(pm + own(m));
        const VT rm2 = ldv<T, V>(pn + own(m));
        const VT o = colour_update<T, V, true>(rm1, N.left, N.right, N.ym, N.yp, rm2, Rc[m], Fm[m],
                                               (par[m] + z + 1) & 1, h2, inv6, black_part && act[m], inv_h2d, accb);
        if (!act[m]) continue;
        stv<T, V>(out + go[m] + (int64_t)z * sz, o);
        T* sg = stg + (i & 1) * 4 * ey;
        if (xvv[m] == 0) {
          sg[yv[m]] = o.v[0];
          sg[ey + yv[m]] = o.v[1];
        }
        if (xvv[m] == nvx - 1) {
          sg[2 * ey + yv[m]] = o.v[V - 2];
          sg[3 * ey + yv[m]] = o.v[V - 1];
        }
        if (yv[m] == 0) push_row<T, V>(out, push, PF.start[2], PF.count[2], xvv[m] * V, z, o);
        if (yv[m] == ey - 1) push_row<T, V>(out, push, PF.start[3], PF.count[3], xvv[m] * V, z, o);
        if (z == 0) push_row<T, V>(out, push, PF.start[4], PF.count[4], xvv[m] * V, yv[m], o);
        if (z == ez - 1) push_row<T, V>(out, push, PF.start[5], PF.count[5], xvv[m] * V, yv[m], o);
      }
    }
    // plane i+1 into the buffer that plane i-2 used (each lane reads and writes
    // only its own slots there)
    if (next_in) {
#pragma unroll
      for (int m = 0; m < K; ++m)
        if (act[m]) stv<T, V>(pn + own(m), Gp[m]);
      if (i + 1 < ez) ring_store(pn, Hn);
    }
#pragma unroll
    for (int m = 0; m < K; ++m) {
      Gp[m] = Gn[m];
      Fm[m] = Fc[m];
      Fc[m] = Fn[m];
    }
  }
  lds_barrier();
  flush_edges(z1 & 1, z1 - 1);  // the last plane
  if (red_part) {
    const double v = block_reduce(accr, R_SUM);
    if (threadIdx.x == 0) red_part[wg] = v;
  }
  if (black_part) {
    const double v = block_reduce(accb, R_SUM);
    if (threadIdx.x == 0) black_part[wg] = v;
  }
}

}  // namespace

int device_cu_count() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (!cached[dev]) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
    cached[dev] = n;
  }
  return cached[dev];
}

hipError_t launch_heat(int dtype, int vec, bool fused, const HeatArgs& a, int grid, int block, hipStream_t s) {
  if ((a.form == 3 && a.lin ? a.nlin : a.ntiles) <= 0) return hipSuccess;
  if (dtype == BL_F64) return vec == 2 ? heat_dispatch<double, 2>(fused, a, grid, block, s)
                                       : heat_dispatch<double, 1>(fused, a, grid, block, s);
  return vec == 4 ? heat_dispatch<float, 4>(fused, a, grid, block, s) : heat_dispatch<float, 1>(fused, a, grid, block, s);
}

hipError_t launch_fill(const Plan& p, void* data, int scomp, int ncomp, hipStream_t s, bool from_mirror) {
  const int n = (int)p.hfillchunks.size();
  if (n == 0 || ncomp <= 0) return hipSuccess;
  const DevFillRec* recs = from_mirror && p.dfillrecs_mir ? p.dfillrecs_mir : p.dfillrecs;
  if (p.esize == 8)
    hipLaunchKernelGGL(k_fill<unsigned long long>, dim3(n), dim3(kFillChunk), 0, s, (unsigned long long*)data, recs,
                       p.dfillchunks, scomp, ncomp);
  else
    hipLaunchKernelGGL(k_fill<unsigned int>, dim3(n), dim3(kFillChunk), 0, s, (unsigned int*)data, recs,
                       p.dfillchunks, scomp, ncomp);
  return hipGetLastError();
}

template <typename T, int V>
static void copy_global_t(const Plan& p, void* data, void* g, int scomp, int ncomp, int to_global, int block,
                          hipStream_t s) {
  const int Nx = p.domain.len(0), Ny = p.domain.len(1), Nz = p.domain.len(2);
  hipLaunchKernelGGL((k_copy_global<T, V>), dim3((unsigned)p.htiles.size()), dim3(block), 0, s, (T*)data, (T*)g,
                     p.dtiles, p.dboxes, scomp, ncomp, p.domain.lo[0], p.domain.lo[1], p.domain.lo[2], Nx, Ny, Nz,
                     to_global);
}

hipError_t launch_copy_global(const Plan& p, void* data, void* global, int scomp, int ncomp, int to_global, int block,
                              hipStream_t s) {
  if (p.htiles.empty() || ncomp <= 0) return hipSuccess;
  if (p.dtype == BL_F64) {
    if (p.vec == 2) copy_global_t<double, 2>(p, data, global, scomp, ncomp, to_global, block, s);
    else copy_global_t<double, 1>(p, data, global, scomp, ncomp, to_global, block, s);
  } else {
    if (p.vec == 4) copy_global_t<float, 4>(p, data, global, scomp, ncomp, to_global, block, s);
    else copy_global_t<float, 1>(p, data, global, scomp, ncomp, to_global, block, s);
  }
  return hipGetLastError();
}

hipError_t launch_set_val(const Plan& p, void* data, double val, int scomp, int ncomp, int with_ghosts, int block,
                          hipStream_t s) {
  if (p.htiles.empty() || ncomp <= 0) return hipSuccess;
  const unsigned nt = (unsigned)p.htiles.size();
  const unsigned nb = (unsigned)p.hboxes.size();
  if (with_ghosts) {
    if (p.dtype == BL_F64)
      hipLaunchKernelGGL(k_set_fab<double>, dim3(64, nb), dim3(256), 0, s, (double*)data, val, p.dboxes, scomp, ncomp);
    else
      hipLaunchKernelGGL(k_set_fab<float>, dim3(64, nb), dim3(256), 0, s, (float*)data, (float)val, p.dboxes, scomp,
                         ncomp);
  } else if (p.dtype == BL_F64) {
    if (p.vec == 2)
      hipLaunchKernelGGL((k_set_valid<double, 2>), dim3(nt), dim3(block), 0, s, (double*)data, val, p.dtiles, p.dboxes,
                         scomp, ncomp);
    else
      hipLaunchKernelGGL((k_set_valid<double, 1>), dim3(nt), dim3(block), 0, s, (double*)data, val, p.dtiles, p.dboxes,
                         scomp, ncomp);
  } else {
    if (p.vec == 4)
      hipLaunchKernelGGL((k_set_valid<float, 4>), dim3(nt), dim3(block), 0, s, (float*)data, (float)val, p.dtiles,
                         p.dboxes, scomp, ncomp);
    else
      hipLaunchKernelGGL((k_set_valid<float, 1>), dim3(nt), dim3(block), 0, s, (float*)data, (float)val, p.dtiles,
                         p.dboxes, scomp, ncomp);
  }
  return hipGetLastError();
}

hipError_t launch_extract_mirror(const Plan& p, void* data, hipStream_t s) {
  const unsigned nb = (unsigned)(p.hboxes.size() * p.ncomp);
  if (!nb) return hipSuccess;
  if (p.dtype == BL_F64)
    hipLaunchKernelGGL(k_extract_mirror<double>, dim3(nb), dim3(256), 0, s, (double*)data, p.dboxes, p.ncomp);
  else
    hipLaunchKernelGGL(k_extract_mirror<float>, dim3(nb), dim3(256), 0, s, (float*)data, p.dboxes, p.ncomp);
  return hipGetLastError();
}

hipError_t launch_copy_fab(const Plan& p, void* data, void* dense, int box, int scomp, int ncomp, int to_dense,
                           hipStream_t s) {
  if (p.esize == 8)
    hipLaunchKernelGGL(k_copy_fab<unsigned long long>, dim3(256), dim3(256), 0, s, (unsigned long long*)data,
                       (unsigned long long*)dense, p.dboxes, box, scomp, ncomp, to_dense);
  else
    hipLaunchKernelGGL(k_copy_fab<unsigned int>, dim3(256), dim3(256), 0, s, (unsigned int*)data,
                       (unsigned int*)dense, p.dboxes, box, scomp, ncomp, to_dense);
  return hipGetLastError();
}

hipError_t launch_reduce(const Plan& p, const void* data, int comp, int op, double* partials, double* out, int block,
                         hipStream_t s) {
  if (p.dred) {  // chunks of whole planes
    const unsigned nc = (unsigned)p.hred.size();
    if (p.dtype == BL_F64) {
      if (p.vec == 2)
        hipLaunchKernelGGL((k_reduce_chunks<double, 2>), dim3(nc), dim3(256), 0, s, (const double*)data, p.dred,
                           p.dboxes, comp, op, partials);
      else
        hipLaunchKernelGGL((k_reduce_chunks<double, 1>), dim3(nc), dim3(256), 0, s, (const double*)data, p.dred,
                           p.dboxes, comp, op, partials);
    } else {
      if (p.vec == 4)
        hipLaunchKernelGGL((k_reduce_chunks<float, 4>), dim3(nc), dim3(256), 0, s, (const float*)data, p.dred,
                           p.dboxes, comp, op, partials);
      else
        hipLaunchKernelGGL((k_reduce_chunks<float, 1>), dim3(nc), dim3(256), 0, s, (const float*)data, p.dred,
                           p.dboxes, comp, op, partials);
    }
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(1024), 0, s, partials, (int)nc, op, op == R_NORM2 ? 1 : 0, out);
    return hipGetLastError();
  }
  const unsigned nt = (unsigned)p.htiles.size();
  if (p.dtype == BL_F64) {
    if (p.vec == 2)
      hipLaunchKernelGGL((k_reduce_tiles<double, 2>), dim3(nt), dim3(block), 0, s, (const double*)data, p.dtiles,
                         p.dboxes, comp, op, partials);
    else
      hipLaunchKernelGGL((k_reduce_tiles<double, 1>), dim3(nt), dim3(block), 0, s, (const double*)data, p.dtiles,
                         p.dboxes, comp, op, partials);
  } else {
    if (p.vec == 4)
      hipLaunchKernelGGL((k_reduce_tiles<float, 4>), dim3(nt), dim3(block), 0, s, (const float*)data, p.dtiles,
                         p.dboxes, comp, op, partials);
    else
      hipLaunchKernelGGL((k_reduce_tiles<float, 1>), dim3(nt), dim3(block), 0, s, (const float*)data, p.dtiles,
                         p.dboxes, comp, op, partials);
  }
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(1024), 0, s, partials, (int)nt, op, op == R_NORM2 ? 1 : 0, out);
  return hipGetLastError();
}

// ------------------------------------------------- reduction without allocation
// The partial results of one reduction (one double per reduction chunk) in a
// fixed device array instead of memory the library allocates.  Each GPU the
// library runs on holds its own copy at its own address until the process ends;
// host code uses only the address hipGetSymbolAddress returns for the current
// device, never the array's name.  Nothing in it must start at zero: every
// chunk writes its own slot before the final pass reads it.  Calls that overlap
// on one GPU share the array and race.
static __device__ __align__(256) double scratch[kNoAllocPartials];

static std::mutex g_scratch_mu;
static double* g_scratch_ptr[kMaxDevices];

hipError_t noalloc_partials(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

hipError_t launch_reduce_noalloc(const Plan& p, const void* data, int comp, int op, double* out, hipStream_t s) {
  double* partials = nullptr;
  hipError_t e = noalloc_partials(&partials);
  if (e != hipSuccess) return e;
  return launch_reduce(p, data, comp, op, partials, out, 256, s);
}

hipError_t launch_gsrb(const Plan& p, void* phi, const void* f, double h2, int color, int block, hipStream_t s) {
  const unsigned nt = (unsigned)p.htiles.size();
  if (nt == 0) return hipSuccess;
  if (p.dtype == BL_F64) {
    const double inv6 = 1.0 / 6.0;
    if (p.vec == 2)
      hipLaunchKernelGGL((k_gsrb<double, 2>), dim3(nt), dim3(block), 0, s, p.dtiles, p.dboxes, (double*)phi,
                         (const double*)f, h2, inv6, color);
    else
      hipLaunchKernelGGL((k_gsrb<double, 1>), dim3(nt), dim3(block), 0, s, p.dtiles, p.dboxes, (double*)phi,
                         (const double*)f, h2, inv6, color);
  } else {
    const float h2f = (float)h2, inv6f = (float)(1.0 / 6.0);
    if (p.vec == 4)
      hipLaunchKernelGGL((k_gsrb<float, 4>), dim3(nt), dim3(block), 0, s, p.dtiles, p.dboxes, (float*)phi,
                         (const float*)f, h2f, inv6f, color);
    else
      hipLaunchKernelGGL((k_gsrb<float, 1>), dim3(nt), dim3(block), 0, s, p.dtiles, p.dboxes, (float*)phi,
                         (const float*)f, h2f, inv6f, color);
  }
  return hipGetLastError();
}

hipError_t launch_residual(const Plan& p, const void* phi, const void* f, double h2, double* partials, double* out,
                           int block, hipStream_t s) {
  const unsigned nt = (unsigned)p.htiles.size();
  if (p.dtype == BL_F64) {
    if (p.vec == 2)
      hipLaunchKernelGGL((k_residual<double, 2>), dim3(nt), dim3(block), 0, s, p.dtiles, p.dboxes, (const double*)phi,
                         (const double*)f, h2, partials);
    else
      hipLaunchKernelGGL((k_residual<double, 1>), dim3(nt), dim3(block), 0, s, p.dtiles, p.dboxes, (const double*)phi,
                         (const double*)f, h2, partials);
  } else {
    if (p.vec == 4)
      hipLaunchKernelGGL((k_residual<float, 4>), dim3(nt), dim3(block), 0, s, p.dtiles, p.dboxes, (const float*)phi,
                         (const float*)f, h2, partials);
    else
      hipLaunchKernelGGL((k_residual<float, 1>), dim3(nt), dim3(block), 0, s, p.dtiles, p.dboxes, (const float*)phi,
                         (const float*)f, h2, partials);
  }
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(1024), 0, s, partials, (int)nt, (int)R_SUM, 1, out);
  return hipGetLastError();
}

// Fused GSRB colour pass / residual (k_gsrb_dma) over the whole level; the
// grid is one workgroup per tile or, persistent, `grid` workgroups; with
// `partials` the per-workgroup sums of r^2 of the cells of colour rescolor.
template <typename T, int V, int ZB>
static hipError_t gsrb_dma_zb(const Plan& p, void* phi, const void* f, double h2, int color, int rescolor,
                              double* partials, int g, int persist, int block, hipStream_t s, bool rows) {
  const DevFaceRec* recs = rows ? p.dfacerecs_rows : p.dfacerecs;
  const size_t lds = dma_lds_bytes<T, V, ZB>(p.yhmax, p.xhmax, block);
  const T h2t = (T)h2, inv6 = (T)(1.0 / 6.0);
  if (partials)
    hipLaunchKernelGGL((k_gsrb_dma<T, V, ZB, true>), dim3(g), dim3(block), lds, s, p.dlin, (int)p.hlin.size(),
                       p.dboxes, recs, (T*)phi, (const T*)f, h2t, inv6, color, rescolor, 1.0 / h2, partials,
                       persist, p.yhmax);
  else
    hipLaunchKernelGGL((k_gsrb_dma<T, V, ZB, false>), dim3(g), dim3(block), lds, s, p.dlin, (int)p.hlin.size(),
                       p.dboxes, recs, (T*)phi, (const T*)f, h2t, inv6, color, rescolor, 1.0 / h2, partials,
                       persist, p.yhmax);
  return hipGetLastError();
}

template <typename T, int V>
static hipError_t gsrb_dma_v(const Plan& p, void* phi, const void* f, double h2, int color, int rescolor,
                             double* partials, int g, int persist, int block, hipStream_t s, bool rows) {
  switch (p.cfg.zchunk) {
    case 2: return gsrb_dma_zb<T, V, 2>(p, phi, f, h2, color, rescolor, partials, g, persist, block, s, rows);
    case 8: return gsrb_dma_zb<T, V, 8>(p, phi, f, h2, color, rescolor, partials, g, persist, block, s, rows);
    default: return gsrb_dma_zb<T, V, 4>(p, phi, f, h2, color, rescolor, partials, g, persist, block, s, rows);
  }
}

bool gsrb_fused_ok(const Plan& p, int block) {
  (void)block;
  return p.cfg.block == 3 && p.fvec && !p.hlin.empty();  // linear tiles exist only where their LDS fits
}

int gsrb_fused_grid(const Plan& p, int grid) {
  const int nt = (int)p.hlin.size();
  return grid > 0 ? (grid < nt ? grid : nt) : nt;
}

hipError_t launch_gsrb_fused(const Plan& p, void* phi, const void* f, double h2, int color, int rescolor,
                             double* partials, int grid, int block, hipStream_t s, bool rows) {
  if (p.hlin.empty()) return hipSuccess;
  const int g = gsrb_fused_grid(p, grid), persist = grid > 0 ? 1 : 0;
  if (p.dtype == BL_F64)
    return p.vec == 2 ? gsrb_dma_v<double, 2>(p, phi, f, h2, color, rescolor, partials, g, persist, block, s, rows)
                      : gsrb_dma_v<double, 1>(p, phi, f, h2, color, rescolor, partials, g, persist, block, s, rows);
  return p.vec == 4 ? gsrb_dma_v<float, 4>(p, phi, f, h2, color, rescolor, partials, g, persist, block, s, rows)
                    : gsrb_dma_v<float, 1>(p, phi, f, h2, color, rescolor, partials, g, persist, block, s, rows);
}

// One-pass red-black sweep: the ring kernel, the edge-column copies, the sweep.
hipError_t launch_gsrb_ring(const Plan& p, void* phi, const void* f, const void* mir2, double h2, hipStream_t s) {
  const unsigned nr = (unsigned)p.hringrecs.size();
  if (nr == 0) return hipSuccess;
  if (p.dtype == BL_F64)
    hipLaunchKernelGGL(k_gsrb_ring<double>, dim3(nr), dim3(256), 0, s, (double*)phi, (const double*)f, p.dboxes,
                       p.dringrecs, (const double*)mir2, p.dmir2off, h2, 1.0 / 6.0);
  else
    hipLaunchKernelGGL(k_gsrb_ring<float>, dim3(nr), dim3(256), 0, s, (float*)phi, (const float*)f, p.dboxes,
                       p.dringrecs, (const float*)mir2, p.dmir2off, (float)h2, (float)(1.0 / 6.0));
  return hipGetLastError();
}

hipError_t launch_extract_edges2(const Plan& p, void* data, void* mir2, hipStream_t s) {
  const unsigned nb = (unsigned)p.hboxes.size();
  if (nb == 0) return hipSuccess;
  if (p.dtype == BL_F64)
    hipLaunchKernelGGL(k_extract_edges2<double>, dim3(nb), dim3(256), 0, s, (double*)data, p.dboxes, (double*)mir2,
                       p.dmir2off);
  else
    hipLaunchKernelGGL(k_extract_edges2<float>, dim3(nb), dim3(256), 0, s, (float*)data, p.dboxes, (float*)mir2,
                       p.dmir2off);
  return hipGetLastError();
}

size_t gsrb_sweep_lds(int ex, int ey, int vec, int esize) {
  const size_t rowsz = (size_t)(ey + 2) * ex, bufsz = (rowsz + 2 * (size_t)ey + vec - 1) / vec * vec;
  return (3 * bufsz + 8 * (size_t)ey) * (size_t)esize;
}

template <typename T, int V, int K>
static hipError_t gsrb_sweep_t(const Plan& p, const DevRedChunk* work, int nwork, int block, size_t lds,
                               const void* phi, void* out, const void* f, void* omir2, double h2, double* red,
                               double* black, hipStream_t s) {
  if (lds > 65536) {  // more than the default dynamic LDS of a launch
    hipError_t e = hipFuncSetAttribute((const void*)k_gsrb_sweep<T, V, K>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_gsrb_sweep<T, V, K>), dim3(nwork), dim3(block), lds, s, p.dboxes, work, (const T*)phi,
                     (T*)out, (const T*)f, (T*)omir2, p.dmir2off, p.dpushrecs, p.dpushface, (T)h2, (T)(1.0 / 6.0),
                     1.0 / h2, red, black);
  return hipGetLastError();
}

hipError_t launch_gsrb_sweep(const Plan& p, const DevRedChunk* work, int nwork, int block, int k, size_t lds,
                             const void* phi, void* out, const void* f, void* omir2, double h2, double* red,
                             double* black, hipStream_t s) {
  if (nwork <= 0) return hipSuccess;
  if (p.dtype == BL_F64)
    return k == 2 ? gsrb_sweep_t<double, 2, 2>(p, work, nwork, block, lds, phi, out, f, omir2, h2, red, black, s)
                  : gsrb_sweep_t<double, 2, 1>(p, work, nwork, block, lds, phi, out, f, omir2, h2, red, black, s);
  return k == 2 ? gsrb_sweep_t<float, 4, 2>(p, work, nwork, block, lds, phi, out, f, omir2, h2, red, black, s)
                : gsrb_sweep_t<float, 4, 1>(p, work, nwork, block, lds, phi, out, f, omir2, h2, red, black, s);
}

// Variable-coefficient heat step (k_heat_vc_dma) over the whole level, one
// workgroup per linear tile.
size_t vc_lds_half(int dtype, int vec, int zchunk, int yhmax, int xhmax, int block) {
  const size_t es = dtype == BL_F64 ? 8 : 4, vb = es * (size_t)vec, zb = (size_t)zchunk;
  const size_t b = zb * block * vb + zb * 2 * yhmax * vb + zb * 2 * xhmax * es;
  return (b + 15) & ~(size_t)15;
}

template <typename T, int V, int ZB>
static hipError_t vc_zb(const VcArgs& a, hipStream_t s) {
  const size_t half = vc_lds_half(sizeof(T) == 8 ? BL_F64 : BL_F32, V, ZB, a.yhmax, a.xhmax, a.block);
  if (a.fused)
    hipLaunchKernelGGL((k_heat_vc_dma<T, V, true, ZB>), dim3(a.nlin), dim3(a.block), 2 * half, s, a.lin, a.nlin,
                       a.boxes, a.recs, (const T*)a.u, (T*)a.w, (const T*)a.beta, (T)a.dt, (T)a.inv_dx, a.yhmax,
                       (int)half);
  else
    hipLaunchKernelGGL((k_heat_vc_dma<T, V, false, ZB>), dim3(a.nlin), dim3(a.block), 2 * half, s, a.lin, a.nlin,
                       a.boxes, a.recs, (const T*)a.u, (T*)a.w, (const T*)a.beta, (T)a.dt, (T)a.inv_dx, a.yhmax,
                       (int)half);
  return hipGetLastError();
}

template <typename T, int V>
static hipError_t vc_v(const VcArgs& a, hipStream_t s) {
  switch (a.zchunk) {
    case 2: return vc_zb<T, V, 2>(a, s);
    case 8: return vc_zb<T, V, 8>(a, s);
    default: return vc_zb<T, V, 4>(a, s);
  }
}

hipError_t launch_heat_varcoef(int dtype, int vec, const VcArgs& a, hipStream_t s) {
  if (a.nlin <= 0) return hipSuccess;
  if (dtype == BL_F64) return vec == 2 ? vc_v<double, 2>(a, s) : vc_v<double, 1>(a, s);
  return vec == 4 ? vc_v<float, 4>(a, s) : vc_v<float, 1>(a, s);
}

hipError_t launch_restrict_residual(const Plan& fine, const Plan& coarse, const void* phi, const void* f, void* fc,
                                    double h2, hipStream_t s) {
  const int total = coarse.hcellpre.empty() ? 0 : coarse.hcellpre.back();
  if (total <= 0) return hipSuccess;
  const int nb = (int)coarse.hboxes.size(), g = (int)coarse.hcellwg.size();
  if (fine.dtype == BL_F64)
    hipLaunchKernelGGL(k_restrict_residual<double>, dim3(g), dim3(kRestrictPerWG), 0, s, coarse.dcellpre,
                       coarse.dcellwg, nb, total, fine.dboxes, coarse.dboxes, (const double*)phi, (const double*)f,
                       (double*)fc, h2);
  else
    hipLaunchKernelGGL(k_restrict_residual<float>, dim3(g), dim3(kRestrictPerWG), 0, s, coarse.dcellpre,
                       coarse.dcellwg, nb, total, fine.dboxes, coarse.dboxes, (const float*)phi, (const float*)f,
                       (float*)fc, h2);
  return hipGetLastError();
}

hipError_t launch_prolong_add(const Plan& fine, const Plan& coarse, void* phi, const void* pc, hipStream_t s) {
  const int total = fine.hpairpre.empty() ? 0 : fine.hpairpre.back();
  if (total <= 0) return hipSuccess;
  const int nb = (int)fine.hboxes.size(), g = (int)fine.hpairwg.size();
  if (fine.dtype == BL_F64)
    hipLaunchKernelGGL(k_prolong_add<double>, dim3(g), dim3(256), 0, s, fine.dpairpre, fine.dpairwg, nb, total,
                       fine.dboxes, coarse.dboxes, (double*)phi, (const double*)pc);
  else
    hipLaunchKernelGGL(k_prolong_add<float>, dim3(g), dim3(256), 0, s, fine.dpairpre, fine.dpairwg, nb, total,
                       fine.dboxes, coarse.dboxes, (float*)phi, (const float*)pc);
  return hipGetLastError();
}

size_t mg_bottom_lds(const MgBottom& m, int esize) {
  size_t n = 0;
  for (int l = 0; l < m.nlev; ++l) n += 2 * (size_t)m.n[l][0] * m.n[l][1] * m.n[l][2];
  return n * (size_t)esize;
}

size_t mg_bottom_lds_limit() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
    return 65536;
  return (size_t)v < kMgBottomLds ? (size_t)v : kMgBottomLds;
}

hipError_t launch_mg_bottom(const Plan& pl, void* phi, const void* f, const MgBottom& m, double h2, int load_phi,
                            int nu1, int nu2, int nu_bottom, hipStream_t s) {
  const int nb = (int)pl.hboxes.size();
  const size_t lds = mg_bottom_lds(m, pl.esize);
  if (lds > 65536) {  // more than the default dynamic LDS of a launch
    hipError_t e = pl.dtype == BL_F64
                       ? hipFuncSetAttribute((const void*)k_mg_bottom<double>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)
                       : hipFuncSetAttribute((const void*)k_mg_bottom<float>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  if (pl.dtype == BL_F64)
    hipLaunchKernelGGL(k_mg_bottom<double>, dim3(1), dim3(1024), lds, s, pl.dboxes, pl.dcellpre, nb, (double*)phi,
                       (const double*)f, m, h2, load_phi, nu1, nu2, nu_bottom);
  else
    hipLaunchKernelGGL(k_mg_bottom<float>, dim3(1), dim3(1024), lds, s, pl.dboxes, pl.dcellpre, nb, (float*)phi,
                       (const float*)f, m, h2, load_phi, nu1, nu2, nu_bottom);
  return hipGetLastError();
}

// 8th-order heat step over the tiles of k_heat8: with segs and faces, the
// fused form (write_mirror: which also writes w's 4-layer edge mirror);
// without, u's ghosts must have been filled.
template <typename T, int V>
static void heat8_t(const DevTile* tiles, const DevH8Seg* segs, const DevH8Face* faces, int ntiles,
                    const DevBox* boxes, const void* u, void* w, double c, int ldw, int ldh, int wmir, size_t lds,
                    hipStream_t s) {
  if (segs)
    hipLaunchKernelGGL((k_heat8<T, V, true>), dim3(ntiles), dim3(256), lds, s, tiles, segs, faces, boxes,
                       (const T*)u, (T*)w, (T)c, ldw, ldh, wmir);
  else
    hipLaunchKernelGGL((k_heat8<T, V, false>), dim3(ntiles), dim3(256), lds, s, tiles, segs, faces, boxes,
                       (const T*)u, (T*)w, (T)c, ldw, ldh, 0);
}

hipError_t launch_heat8(int dtype, int vec, const DevTile* tiles, const DevH8Seg* segs, const DevH8Face* faces,
                        int ntiles, const DevBox* boxes, const void* u, void* w, double c, int rmax, int nvtmax,
                        bool write_mirror, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (segs && !faces) return hipErrorInvalidValue;
  if (write_mirror && !segs) return hipErrorInvalidValue;
  if (write_mirror && 4 % vec) return hipErrorInvalidValue;  // a vector lies in one side's 4 columns
  const int ldw = ((nvtmax * vec + 8) + 3) & ~3, ldh = rmax + 8;
  const size_t lds = 2 * (size_t)ldw * ldh * (dtype == BL_F64 ? 8 : 4);
  const int wm = write_mirror ? 1 : 0;
  if (dtype == BL_F64) {
    if (vec == 2) heat8_t<double, 2>(tiles, segs, faces, ntiles, boxes, u, w, c, ldw, ldh, wm, lds, s);
    else heat8_t<double, 1>(tiles, segs, faces, ntiles, boxes, u, w, c, ldw, ldh, wm, lds, s);
  } else {
    if (vec == 4) heat8_t<float, 4>(tiles, segs, faces, ntiles, boxes, u, w, c, ldw, ldh, wm, lds, s);
    else heat8_t<float, 1>(tiles, segs, faces, ntiles, boxes, u, w, c, ldw, ldh, wm, lds, s);
  }
  return hipGetLastError();
}

// Plain device copy of nvec 16-byte vectors: one 4 KB chunk per workgroup, one
// vector per lane (the shape that reached the highest copy bandwidth here).
__global__ void __launch_bounds__(256) k_copy16(const Vec<double, 2>* src_, Vec<double, 2>* dst_, int64_t nvec) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < nvec) as_global(dst_)[i] = as_global(src_)[i];
}

hipError_t launch_copy16(void* dst, const void* src, size_t bytes, hipStream_t s) {
  const int64_t nvec = (int64_t)(bytes / 16);
  if (nvec == 0) return hipSuccess;
  const int64_t g = (nvec + 255) / 256;
  hipLaunchKernelGGL(k_copy16, dim3((unsigned)g), dim3(256), 0, s, (const Vec<double, 2>*)src, (Vec<double, 2>*)dst,
                     nvec);
  return hipGetLastError();
}

hipError_t launch_reduce_partials(const double* partials, int n, int take_sqrt, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(1024), 0, s, partials, n, (int)R_SUM, take_sqrt, out);
  return hipGetLastError();
}

}  // namespace bl
