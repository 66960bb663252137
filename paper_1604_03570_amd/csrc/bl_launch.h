// Host-side launchers of the gfx950 kernels (bl_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "bl_internal.h"

namespace bl {

enum ReduceOp { R_SUM = 0, R_MAX = 1, R_MIN = 2, R_NORM0 = 3, R_NORM1 = 4, R_NORM2 = 5 };

struct HeatArgs {
  const DevTile* tiles;        // first tile of the launch
  int ntiles;
  const DevBox* boxes;
  const DevFaceRec* recs;
  DevMember m0;                // used when members == nullptr
  const DevMember* members;
  int flip;
  int fvec;                    // 1: every y- and z-face source row allows aligned vector loads
  int zblock;                  // 2, 4, 8: block form (tiles of at most that many planes); else the march
  int form;                    // 0 march, 1 block, 2 block with LDS neighbours, 3 as 2 with halos loaded into LDS
  int rmax;                    // most rows of any tile of the launch
  int nvtmax;                  // most x vectors of any tile of the launch
  // form 3: the linear tiles (when null, form 3 runs as form 2 on `tiles`)
  const DevLinTile* lin;
  int nlin;
  int yhmax, xhmax;            // LDS sizing: most halo vectors / row ends of a linear tile
};

// Stencil over `ntiles` tiles.  fused: tiles at box faces read neighbour boxes
// through the face records; otherwise they read the FAB's own (filled) ghosts.
// grid == 0: one workgroup per tile; else `grid` persistent workgroups each
// taking a contiguous range of tiles.
hipError_t launch_heat(int dtype, int vec, bool fused, const HeatArgs& a, int grid, int block, hipStream_t s);

// FillBoundary of components [scomp, scomp+ncomp); from_mirror: one-column
// sources at a box's x face are read from its edge mirror (which must be current)
hipError_t launch_fill(const Plan& p, void* data, int scomp, int ncomp, hipStream_t s, bool from_mirror = false);

hipError_t launch_copy_global(const Plan& p, void* data, void* global, int scomp, int ncomp, int to_global,
                              int block, hipStream_t s);

hipError_t launch_set_val(const Plan& p, void* data, double val, int scomp, int ncomp, int with_ghosts, int block,
                          hipStream_t s);

// Fill every box's edge-column mirror from the state in `data` (one launch).
hipError_t launch_extract_mirror(const Plan& p, void* data, hipStream_t s);

// FAB `box`, grown box, components [scomp, scomp+ncomp) <-> dense (ncomp, nz, ny, nx) device array.
hipError_t launch_copy_fab(const Plan& p, void* data, void* dense, int box, int scomp, int ncomp, int to_dense,
                           hipStream_t s);

// partials must hold p.htiles.size() doubles; the result lands in *out (device).
hipError_t launch_reduce(const Plan& p, const void* data, int comp, int op, double* partials, double* out, int block,
                         hipStream_t s);

// launch_reduce with the partials in the library's fixed device array of
// kNoAllocPartials doubles (no allocation): needs p.dred and at most that many
// chunks.  Calls that overlap on one GPU race on the array.
constexpr int kNoAllocPartials = 65536;
constexpr int kMaxDevices = 64;
hipError_t launch_reduce_noalloc(const Plan& p, const void* data, int comp, int op, double* out, hipStream_t s);

hipError_t launch_gsrb(const Plan& p, void* phi, const void* f, double h2, int color, int block, hipStream_t s);

// The bottom of a V-cycle in one workgroup: levels L..L+nlev-1 of a hierarchy
// whose levels from L down each cover a fully periodic domain, held as dense
// periodic arrays in LDS (phi and f of every level).  Takes f of level L from
// its MultiFab (and phi if load_phi, else phi = 0), runs the cycle's part from
// level L down and back (nu1 sweeps, restriction, ..., nu_bottom sweeps on the
// coarsest, ..., prolongation, nu2 sweeps) and stores phi's valid cells of
// level L.  h2 is level L's spacing squared (times 4 per level below).
constexpr int kMgBottomMaxLevels = 16;
constexpr size_t kMgBottomLds = 163840;  // at most; the device's per-workgroup LDS if smaller
size_t mg_bottom_lds_limit();
struct MgBottom {
  int nlev;
  int n[kMgBottomMaxLevels][3];   // domain extents per level
  int lo[kMgBottomMaxLevels][3];  // domain lower corners
  int off[kMgBottomMaxLevels];    // LDS element offset of phi (f follows it)
};
size_t mg_bottom_lds(const MgBottom& m, int esize);
hipError_t launch_mg_bottom(const Plan& pl, void* phi, const void* f, const MgBottom& m, double h2, int load_phi,
                            int nu1, int nu2, int nu_bottom, hipStream_t s);

// ||f + L_h phi||_2 in FP64 into *out (device); reads phi's ghosts (fill first).
hipError_t launch_residual(const Plan& p, const void* phi, const void* f, double h2, double* partials, double* out,
                           int block, hipStream_t s);

// Fused GSRB (no fill: neighbour boxes through the face records, edge mirrors
// current): colour pass color (0 red, 1 black; -1 none) in place; with
// partials, per-workgroup sums of r^2 over the cells of colour rescolor (2: all)
// into partials[0 .. gsrb_fused_grid).  Usable when gsrb_fused_ok.
bool gsrb_fused_ok(const Plan& p, int block);
int gsrb_fused_grid(const Plan& p, int grid);
// rows: x-face neighbours from the neighbour boxes' rows, not their edge-column
// mirrors (a first pass, when phi's mirror is not current).  Only colour passes
// (color >= 0) rewrite the mirror; a norm-only pass (color -1) leaves it as it
// was, so every caller that reads the mirror afterwards either refreshes it or
// reads rows first.
hipError_t launch_gsrb_fused(const Plan& p, void* phi, const void* f, double h2, int color, int rescolor,
                             double* partials, int grid, int block, hipStream_t s, bool rows = false);
// *out = sum (sqrt of it if take_sqrt) of partials[0..n)
hipError_t launch_reduce_partials(const double* partials, int n, int take_sqrt, double* out, hipStream_t s);
// One-pass red-black sweep.  launch_gsrb_ring: the new red values of every
// covered face ghost cell into phi's ghost layer (red positions); mir2: phi's
// second edge-column copy.  launch_extract_edges2: both edge-column copies of
// data (the mirror and mir2) from its rows.  launch_gsrb_sweep: the sweep of
// the work chunks (box, planes) from phi into out, with out's edge columns;
// red / black (may be NULL): per-workgroup partials of the squared residual at
// phi's red cells and at out's black cells.  gsrb_sweep_lds: the LDS of a
// workgroup for a box of ex x ey planes (3 plane buffers with their ghost items).
hipError_t launch_gsrb_ring(const Plan& p, void* phi, const void* f, const void* mir2, double h2, hipStream_t s);
hipError_t launch_extract_edges2(const Plan& p, void* data, void* mir2, hipStream_t s);
size_t gsrb_sweep_lds(int ex, int ey, int vec, int esize);
hipError_t launch_gsrb_sweep(const Plan& p, const DevRedChunk* work, int nwork, int block, int k, size_t lds,
                             const void* phi, void* out, const void* f, void* omir2, double h2, double* red,
                             double* black, hipStream_t s);

// Variable-coefficient heat step in the flux form, u -> w with coefficient beta
// (same layout), over linear tiles built for zchunk and block; LDS 2*vc_lds_half.
struct VcArgs {
  const DevLinTile* lin;
  int nlin;
  const DevBox* boxes;
  const DevFaceRec* recs;
  int yhmax, xhmax, zchunk, block;
  int fused;                   // 1: neighbour boxes through the face records; 0: filled ghosts
  const void* u;
  void* w;
  const void* beta;
  double dt, inv_dx;
};
size_t vc_lds_half(int dtype, int vec, int zchunk, int yhmax, int xhmax, int block);
hipError_t launch_heat_varcoef(int dtype, int vec, const VcArgs& a, hipStream_t s);

// Multigrid transfers between a level and its coarsening by 2 (box b of
// `coarse` is box b of `fine` coarsened; every fine box has even lo and
// extents).  Restriction: fc = mean of the 8 fine residuals f + L_h phi of each
// coarse cell (phi's ghosts filled).  Prolongation: phi += parent value.
hipError_t launch_restrict_residual(const Plan& fine, const Plan& coarse, const void* phi, const void* f, void* fc,
                                    double h2, hipStream_t s);
hipError_t launch_prolong_add(const Plan& fine, const Plan& coarse, void* phi, const void* pc, hipStream_t s);

// 8th-order heat step (9-cell span) over tiles built for it (build_h8_tiles):
// at most 256 lanes, rows <= rmax <= 32, nvt <= nvtmax <= 32.  segs == nullptr:
// u's ghosts (>= 4 layers) filled; else the fused form, cells outside a box
// read through the face segments of build_h8_segments, no fill needed.
hipError_t launch_heat8(int dtype, int vec, const DevTile* tiles, const DevH8Seg* segs, const DevH8Face* faces,
                        int ntiles, const DevBox* boxes, const void* u, void* w, double c, int rmax, int nvtmax,
                        bool write_mirror, hipStream_t s);

// dst[0..bytes) = src[0..bytes): 16-byte aligned, bytes a multiple of 16.
hipError_t launch_copy16(void* dst, const void* src, size_t bytes, hipStream_t s);

int device_cu_count();

}  // namespace bl
