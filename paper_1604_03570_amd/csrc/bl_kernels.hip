// gfx950 kernels of libboxtile: FillBoundary copy, the 7-point heat step
// (per-box and fused forms), red-black Gauss-Seidel colour passes, the FP64
// residual, reductions and data movement between MultiFabs and dense arrays.
//
// Thread mapping shared by the stencil kernels: a workgroup takes one tile
// (box, component, a run of lanes over the box's x-y plane, a z range).  Each
// lane owns `V` consecutive x cells of one row (V*sizeof(T) = 16 bytes when all
// x extents allow it, so every row access is one aligned 16-byte load) and
// marches up the z range keeping the planes z-1, z, z+1 in registers; x and y
// neighbours come from the neighbouring lanes' rows through the caches.
//
// Every cell update is one fixed expression (heat_cell / gsrb_cell), compiled
// without FMA contraction, so the per-box, fused and batched forms produce
// bit-identical results.
#include <hip/hip_runtime.h>

#include <cmath>
#include <limits>

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

// Workgroups are dealt round-robin to the 8 XCDs; renumber them so that each
// XCD's workgroups take one contiguous eighth of the tile list (neighbouring
// tiles then share that XCD's L2).  Bijective on [0, gridDim.x).
__device__ __forceinline__ int logical_block() {
  const int G = gridDim.x;
  const int x = blockIdx.x & 7, q = blockIdx.x >> 3;
  const int per = G >> 3, rem = G & 7;
  return x * per + (x < rem ? x : rem) + q;
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

template <typename T>
__device__ __forceinline__ T qnan() {
  return std::numeric_limits<T>::quiet_NaN();
}

// Value in the ghost layer next to face `face` at tangential coordinates (t1, t2):
// the record covering them gives its source (a neighbour's valid cell, its
// periodic image, or the box's own ghost cell where no box covers the layer).
template <typename T>
__device__ __forceinline__ T face_load(const T* __restrict__ u, const DevFaceRec* __restrict__ recs, int start,
                                       int count, int t1, int t2, int comp) {
  for (int r = start; r < start + count; ++r) {
    const DevFaceRec R = recs[r];
    if (t1 >= R.t1lo && t1 <= R.t1hi && t2 >= R.t2lo && t2 <= R.t2hi)
      return u[R.base + (int64_t)t1 * R.s1 + (int64_t)t2 * R.s2 + (int64_t)comp * R.sc];
  }
  return qnan<T>();  // records partition every face; not reached
}

// ---------------------------------------------------------------- heat step
template <typename T, int V, bool FUSED>
__global__ void __launch_bounds__(1024)
    k_heat(const DevTile* __restrict__ tiles, int ntiles, const DevBox* __restrict__ boxes,
           const DevFaceRec* __restrict__ recs, DevMember m0, const DevMember* __restrict__ members, int flip,
           int persist) {
  int first, last;
  tile_range(ntiles, persist, first, last);
  for (int t = first; t < last; ++t) {
    const DevTile tl = tiles[t];
    if ((int)threadIdx.x >= tl.nl) continue;
    const DevBox B = boxes[tl.box];
    const DevMember M = members ? members[tl.member] : m0;
    const bool swap = ((flip + M.flip_offset) & 1) != 0;
    const T* __restrict__ u = static_cast<const T*>(swap ? M.b : M.a);
    T* __restrict__ w = static_cast<T*>(swap ? M.a : M.b);
    const T c = (T)M.c;
    const int n = tl.comp;
    const int l = tl.l0 + (int)threadIdx.x;
    const int y = l / B.nvx;
    const int xv = l - y * B.nvx;
    const int x0 = xv * V;
    const int64_t cb = B.off + (int64_t)n * B.sc + x0 + (int64_t)y * B.sy;
    const T* up = u + cb;
    T* wp = w + cb;
    const int sy = B.sy, sz = B.sz;
    int z = tl.z0;
    Vec<T, V> zm, cc, zp, ym, yp, o;
    if (!FUSED || z > 0) {
      zm = ldv<T, V>(up + (z - 1) * sz);
    } else {
#pragma unroll
      for (int e = 0; e < V; ++e) zm.v[e] = face_load(u, recs, B.face_start[4], B.face_count[4], x0 + e, y, n);
    }
    cc = ldv<T, V>(up + z * sz);
    for (; z < tl.z1; ++z) {
      const T* pz = up + z * sz;
      if (!FUSED || z + 1 < B.ez) {
        zp = ldv<T, V>(pz + sz);
      } else {
#pragma unroll
        for (int e = 0; e < V; ++e) zp.v[e] = face_load(u, recs, B.face_start[5], B.face_count[5], x0 + e, y, n);
      }
      T left, right;
      if (!FUSED || xv > 0)
        left = pz[-1];
      else
        left = face_load(u, recs, B.face_start[0], B.face_count[0], y, z, n);
      if (!FUSED || xv + 1 < B.nvx)
        right = pz[V];
      else
        right = face_load(u, recs, B.face_start[1], B.face_count[1], y, z, n);
      if (!FUSED || y > 0) {
        ym = ldv<T, V>(pz - sy);
      } else {
#pragma unroll
        for (int e = 0; e < V; ++e) ym.v[e] = face_load(u, recs, B.face_start[2], B.face_count[2], x0 + e, z, n);
      }
      if (!FUSED || y + 1 < B.ey) {
        yp = ldv<T, V>(pz + sy);
      } else {
#pragma unroll
        for (int e = 0; e < V; ++e) yp.v[e] = face_load(u, recs, B.face_start[3], B.face_count[3], x0 + e, z, n);
      }
#pragma unroll
      for (int e = 0; e < V; ++e) {
        const T xm = e == 0 ? left : cc.v[e - 1];
        const T xp = e == V - 1 ? right : cc.v[e + 1];
        o.v[e] = heat_cell(cc.v[e], xm, xp, ym.v[e], yp.v[e], zm.v[e], zp.v[e], c);
      }
      stv<T, V>(wp + z * sz, o);
      zm = cc;
      cc = zp;
    }
  }
}

// ---------------------------------------------------------------- FillBoundary
// One workgroup per chunk of a copy-plan record; bit copies (integer type of the element size).
template <typename I>
__global__ void __launch_bounds__(kFillChunk)
    k_fill(I* __restrict__ data, const DevFillRec* __restrict__ recs, const DevFillChunk* __restrict__ chunks,
           int scomp, int ncomp) {
  const DevFillChunk ch = chunks[blockIdx.x];
  const DevFillRec R = recs[ch.rec];
  const int cell = ch.start + (int)threadIdx.x;
  if (cell >= R.nx * R.ny * R.nz) return;
  const int x = cell % R.nx;
  const int t = cell / R.nx;
  const int y = t % R.ny;
  const int z = t / R.ny;
  const int64_t d = R.dst_base + x + (int64_t)y * R.dsy + (int64_t)z * R.dsz;
  const int64_t s = R.src_base + x + (int64_t)y * R.ssy + (int64_t)z * R.ssz;
  for (int n = scomp; n < scomp + ncomp; ++n) data[d + n * R.dsc] = data[s + n * R.ssc];
}

// ---------------------------------------------------------------- dense <-> MultiFab
template <typename T, int V>
__global__ void __launch_bounds__(1024)
    k_copy_global(T* __restrict__ data, T* __restrict__ g, const DevTile* __restrict__ tiles,
                  const DevBox* __restrict__ boxes, int scomp, int ncomp, int dlo0, int dlo1, int dlo2, int Nx, int Ny,
                  int Nz, int to_global) {
  const DevTile tl = tiles[blockIdx.x];
  if (tl.comp < scomp || tl.comp >= scomp + ncomp || (int)threadIdx.x >= tl.nl) return;
  const DevBox B = boxes[tl.box];
  const int l = tl.l0 + (int)threadIdx.x;
  const int y = l / B.nvx;
  const int x0 = (l - y * B.nvx) * V;
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
  const DevTile tl = tiles[blockIdx.x];
  if (tl.comp < scomp || tl.comp >= scomp + ncomp || (int)threadIdx.x >= tl.nl) return;
  const DevBox B = boxes[tl.box];
  const int l = tl.l0 + (int)threadIdx.x;
  const int y = l / B.nvx;
  const int x0 = (l - y * B.nvx) * V;
  const int64_t cb = B.off + (int64_t)tl.comp * B.sc + x0 + (int64_t)y * B.sy;
  for (int z = tl.z0; z < tl.z1; ++z)
#pragma unroll
    for (int e = 0; e < V; ++e) data[cb + (int64_t)z * B.sz + e] = val;
}

// whole FAB blocks (valid, ghost and row padding) of components [scomp, scomp+ncomp)
template <typename T>
__global__ void __launch_bounds__(256)
    k_set_fab(T* __restrict__ data, T val, const DevBox* __restrict__ boxes, int scomp, int ncomp, int xlead, int ng) {
  const DevBox B = boxes[blockIdx.y];
  const int64_t start = B.off - (xlead + (int64_t)ng * B.sy + (int64_t)ng * B.sz) + (int64_t)scomp * B.sc;
  const int64_t count = B.sc * ncomp;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    data[start + i] = val;
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

template <typename T, int V>
__global__ void __launch_bounds__(1024)
    k_reduce_tiles(const T* __restrict__ data, const DevTile* __restrict__ tiles, const DevBox* __restrict__ boxes,
                   int comp, int op, double* __restrict__ partials) {
  const DevTile tl = tiles[blockIdx.x];
  double acc = r_identity(op);
  if (tl.comp == comp && (int)threadIdx.x < tl.nl) {
    const DevBox B = boxes[tl.box];
    const int l = tl.l0 + (int)threadIdx.x;
    const int y = l / B.nvx;
    const int x0 = (l - y * B.nvx) * V;
    const T* p = data + B.off + (int64_t)comp * B.sc + x0 + (int64_t)y * B.sy;
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
  const DevTile tl = tiles[blockIdx.x];
  if ((int)threadIdx.x >= tl.nl) return;
  const DevBox B = boxes[tl.box];
  const int l = tl.l0 + (int)threadIdx.x;
  const int y = l / B.nvx;
  const int x0 = (l - y * B.nvx) * V;
  const int64_t cb = B.off + x0 + (int64_t)y * B.sy;
  T* pp = phi + cb;
  const T* fp = f + cb;
  const int sy = B.sy, sz = B.sz;
  const int par0 = (B.glo[0] + x0 + B.glo[1] + y + B.glo[2]) & 1;
  for (int z = tl.z0; z < tl.z1; ++z) {
    T* pz = pp + z * sz;
    const Vec<T, V> cc = ldv<T, V>(pz);
    const Vec<T, V> zm = ldv<T, V>(pz - sz);
    const Vec<T, V> zp = ldv<T, V>(pz + sz);
    const Vec<T, V> ym = ldv<T, V>(pz - sy);
    const Vec<T, V> yp = ldv<T, V>(pz + sy);
    const Vec<T, V> fv = ldv<T, V>(fp + z * sz);
    const T left = pz[-1], right = pz[V];
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
  const DevTile tl = tiles[blockIdx.x];
  double acc = 0.0;
  if ((int)threadIdx.x < tl.nl) {
    const DevBox B = boxes[tl.box];
    const int l = tl.l0 + (int)threadIdx.x;
    const int y = l / B.nvx;
    const int x0 = (l - y * B.nvx) * V;
    const int64_t cb = B.off + x0 + (int64_t)y * B.sy;
    const T* pp = phi + cb;
    const T* fp = f + cb;
    const int sy = B.sy, sz = B.sz;
    for (int z = tl.z0; z < tl.z1; ++z) {
      const T* pz = pp + z * sz;
      const Vec<T, V> cc = ldv<T, V>(pz);
      const Vec<T, V> zm = ldv<T, V>(pz - sz);
      const Vec<T, V> zp = ldv<T, V>(pz + sz);
      const Vec<T, V> ym = ldv<T, V>(pz - sy);
      const Vec<T, V> yp = ldv<T, V>(pz + sy);
      const Vec<T, V> fv = ldv<T, V>(fp + z * sz);
      const double left = (double)pz[-1], right = (double)pz[V];
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

template <typename T, int V>
hipError_t heat_dispatch(bool fused, const HeatArgs& a, int grid, int block, hipStream_t s) {
  const int persist = grid > 0 ? 1 : 0;
  const int g = persist ? (grid < a.ntiles ? grid : a.ntiles) : a.ntiles;
  if (fused)
    hipLaunchKernelGGL((k_heat<T, V, true>), dim3(g), dim3(block), 0, s, a.tiles, a.ntiles, a.boxes, a.recs, a.m0,
                       a.members, a.flip, persist);
  else
    hipLaunchKernelGGL((k_heat<T, V, false>), dim3(g), dim3(block), 0, s, a.tiles, a.ntiles, a.boxes, a.recs, a.m0,
                       a.members, a.flip, persist);
  return hipGetLastError();
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
  if (a.ntiles <= 0) return hipSuccess;
  if (dtype == BL_F64) return vec == 2 ? heat_dispatch<double, 2>(fused, a, grid, block, s)
                                       : heat_dispatch<double, 1>(fused, a, grid, block, s);
  return vec == 4 ? heat_dispatch<float, 4>(fused, a, grid, block, s) : heat_dispatch<float, 1>(fused, a, grid, block, s);
}

hipError_t launch_fill(const Plan& p, void* data, int scomp, int ncomp, hipStream_t s) {
  const int n = (int)p.hfillchunks.size();
  if (n == 0 || ncomp <= 0) return hipSuccess;
  if (p.esize == 8)
    hipLaunchKernelGGL(k_fill<unsigned long long>, dim3(n), dim3(kFillChunk), 0, s, (unsigned long long*)data,
                       p.dfillrecs, p.dfillchunks, scomp, ncomp);
  else
    hipLaunchKernelGGL(k_fill<unsigned int>, dim3(n), dim3(kFillChunk), 0, s, (unsigned int*)data, p.dfillrecs,
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
      hipLaunchKernelGGL(k_set_fab<double>, dim3(64, nb), dim3(256), 0, s, (double*)data, val, p.dboxes, scomp, ncomp,
                         p.xlead, p.ng);
    else
      hipLaunchKernelGGL(k_set_fab<float>, dim3(64, nb), dim3(256), 0, s, (float*)data, (float)val, p.dboxes, scomp,
                         ncomp, p.xlead, p.ng);
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

hipError_t launch_reduce(const Plan& p, const void* data, int comp, int op, double* partials, double* out, int block,
                         hipStream_t s) {
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

}  // namespace bl
