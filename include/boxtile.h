/*
 * boxtile: the single-level hot path of "BoxLib with Tiling: An AMR Software
 * Framework" on AMD MI355X (gfx950).
 *
 * The calls follow the paper's own objects:
 *   Box          a rectangle in index space held as six integers (Sec. 3.1);
 *   BoxArray     the non-intersecting grids of one level, a copy of which every
 *                process holds (Sec. 3, Sec. 3.1);
 *   DistributionMapping  which process (here: which GPU) owns each grid (Sec. 3.1);
 *   MultiFab     the FArrayBoxes of one level: per grid, multi-component data on
 *                the grid grown by ghost cells (Sec. 3.1);
 *   FillBoundary the ghost-cell fill between the grids of one level, including
 *                periodic images (Sec. 3.1, Sec. 3.3, Sec. 4.1);
 *   heat step    forward Euler with second-order centred differences (Sec. 4.1);
 *   reductions   e.g. the maximum of one component over the level (Sec. 3.1).
 * The red-black Gauss-Seidel smoother and its residual norm are the textbook
 * smoother of the multigrid solvers the paper names (Sec. 1, Sec. 3.3); the
 * paper does not write them out.
 *
 * Conventions
 *   - Every call returns a bl_status: BL_OK (0) or a negative error code; no
 *     exception crosses this interface.  bl_last_error() returns a message for
 *     the calling thread's most recent failure.
 *   - Boxes hold inclusive cell indices.  A domain box is [lo, hi] per axis.
 *   - Handles (bl_boxarray, bl_distmap, bl_multifab, bl_batch) are created and
 *     destroyed by the library.  They are not thread-safe; distinct handles
 *     may be used from distinct threads.
 *   - Field data lives in device memory owned by the CALLER (for example a
 *     torch tensor); it must outlive every MultiFab made on it.  The library
 *     owns only its metadata (host and device).
 *   - Work is enqueued asynchronously on the hipStream_t passed in (0 is the
 *     null stream).  Calls that return a scalar to a host pointer synchronise
 *     that stream before returning.
 *   - Data layout of a MultiFab: FAB b is one contiguous block per component:
 *     its rows (valid x cells of every row of the grown box, x fastest, then
 *     y, then z; the rows of a plane are contiguous and each plane starts on
 *     a 128-byte boundary), then an "x
 *     ghost slab" holding the ghost cells left and right of the rows
 *     (contiguous along y), then a copy of the box's own first and last valid
 *     x columns that the fused stencil keeps for its neighbours.
 *     bl_multifab_layout and bl_multifab_xghost_layout give exact offsets and
 *     strides; bl_multifab_copy_fab moves a whole FAB to or from a dense array.
 */
#ifndef BOXTILE_H
#define BOXTILE_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t bl_status;
#define BL_OK 0
#define BL_EINVAL (-1)   /* an argument is out of range */
#define BL_EOVERLAP (-2) /* two boxes of a BoxArray intersect */
#define BL_EDOMAIN (-3)  /* a box leaves the domain */
#define BL_ESHAPE (-4)   /* MultiFabs disagree in BoxArray, ncomp or nghost */
#define BL_EDTYPE (-5)   /* MultiFabs disagree in dtype, or the dtype is unknown */
#define BL_ENOMEM (-6)   /* a buffer is too small, or host/device metadata allocation failed */
#define BL_EHIP (-7)     /* a HIP runtime call failed; the message names it */

typedef struct {
  int32_t lo[3], hi[3];
} bl_box; /* inclusive cell indices (Sec. 3.1: six integers) */

typedef enum { BL_F64 = 0, BL_F32 = 1 } bl_dtype;

typedef enum {
  BL_SUM = 0,   /* sum of the component over valid cells, FP64 accumulation */
  BL_MAX = 1,   /* maximum (Sec. 3.1: mf.max(comp)) */
  BL_MIN = 2,   /* minimum */
  BL_NORM0 = 3, /* max |u| */
  BL_NORM1 = 4, /* sum |u|, FP64 accumulation */
  BL_NORM2 = 5  /* sqrt(sum u^2), FP64 accumulation */
} bl_reduce_op;

typedef struct bl_boxarray bl_boxarray;
typedef struct bl_distmap bl_distmap;
typedef struct bl_multifab bl_multifab;
typedef struct bl_batch bl_batch;

/* Message for the calling thread's last failed call ("" if none). */
const char* bl_last_error(void);
/* Library version string. */
const char* bl_version(void);

/* ---------------------------------------------------------------- BoxArray */

/*
 * A level's grids (Sec. 3, Sec. 3.1): nboxes >= 1 boxes that must be non-empty,
 * pairwise disjoint (else BL_EOVERLAP) and inside `domain` (else BL_EDOMAIN).
 * They need not cover the domain.  periodic[d] != 0 makes axis d periodic for
 * FillBoundary.  The boxes are copied; *out is owned by the caller and freed
 * with bl_boxarray_destroy.
 */
bl_status bl_boxarray_create(const bl_box* boxes, int32_t nboxes, const bl_box* domain,
                             const int32_t periodic[3], bl_boxarray** out);

/*
 * Regular chop of `domain` into boxes of edge max_edge[d] along axis d, cut
 * from the low end, the remainder (if any) as the last box of the axis; boxes
 * listed x fastest, then y, then z.  max_edge[d] >= 1, else BL_EINVAL.
 */
bl_status bl_boxarray_chop(const bl_box* domain, const int32_t periodic[3], const int32_t max_edge[3],
                           bl_boxarray** out);

/*
 * Seeded recursive chop into uneven boxes.  Depth first, low half first: a box
 * whose longest edge m is <= max_edge is kept if m < 2*min_edge, or else if a
 * uniform draw in [0,1) is below 1/2; otherwise its longest axis (lowest on
 * ties) is cut at offset min_edge + align*(draw mod ((m - 2*min_edge)/align + 1))
 * from the box's low end.  Draw n of the stream is SplitMix64 (Steele, Lea and
 * Flood, 2014) of seed + (n+1)*0x9E3779B97F4A7C15; a uniform draw uses its top
 * 53 bits.  Requires min_edge % align == 0 and max_edge >= 2*min_edge
 * (else BL_EINVAL).
 */
bl_status bl_boxarray_chop_random(const bl_box* domain, const int32_t periodic[3], int32_t min_edge,
                                  int32_t max_edge, int32_t align, uint64_t seed, bl_boxarray** out);

/*
 * The BoxArray coarsened by `ratio` (Sec. 1's multigrid levels): box i becomes
 * lo/ratio .. (hi+1)/ratio - 1, the domain likewise, same periodic flags, same
 * box order.  Every box corner and extent, and the domain's, must be divisible
 * by ratio (else BL_EINVAL).  The result is a new BoxArray owned by the caller.
 */
bl_status bl_boxarray_coarsen(const bl_boxarray* ba, int32_t ratio, bl_boxarray** out);

/* Number of boxes, and (if boxes != NULL) the boxes themselves, in order. */
bl_status bl_boxarray_get(const bl_boxarray* ba, int32_t* nboxes, bl_box* boxes);
/* Domain box and periodic flags. */
bl_status bl_boxarray_domain(const bl_boxarray* ba, bl_box* domain, int32_t periodic[3]);
void bl_boxarray_destroy(bl_boxarray* ba);

/* ------------------------------------------------------ DistributionMapping */

/*
 * Owner of each box (Sec. 3.1: the data of a MultiFab are distributed among
 * processes).  This build runs on one GPU: ndevices must be 1 and owner, if
 * given, must hold nboxes zeros; other values give BL_EINVAL.
 */
bl_status bl_distmap_create(const bl_boxarray* ba, int32_t ndevices, const int32_t* owner,
                            bl_distmap** out);
void bl_distmap_destroy(bl_distmap* dm);

/* ----------------------------------------------------------------- MultiFab */

/*
 * Device bytes a MultiFab of this shape needs (ncomp >= 1, nghost >= 0).
 */
bl_status bl_multifab_bytes(const bl_boxarray* ba, int32_t ncomp, int32_t nghost, bl_dtype dtype,
                            size_t* bytes);

/*
 * A MultiFab (Sec. 3.1) on caller-owned device memory dev_ptr of `bytes` bytes
 * (BL_ENOMEM if fewer than bl_multifab_bytes; dev_ptr must be 256-byte
 * aligned, else BL_EINVAL).  The memory is not initialised.  dm may be NULL
 * (all boxes on this GPU).  Stencil calls need nghost >= 1.
 */
bl_status bl_multifab_create(const bl_boxarray* ba, const bl_distmap* dm, int32_t ncomp, int32_t nghost,
                             bl_dtype dtype, void* dev_ptr, size_t bytes, bl_multifab** out);

/*
 * Layout of the rows of FAB `box`: its grown box, the element offset (from
 * dev_ptr) of the row cell (valid lo x, grown lo y, grown lo z), component 0,
 * and element strides {x, y, z, comp}.  Cell (i,j,k), component n, with i in
 * the box's valid x range and j, k in the grown range, is at
 *   offset + (i - box.lo[0]) + (j - grown.lo[1])*stride[1]
 *          + (k - grown.lo[2])*stride[2] + n*stride[3]
 * in elements of the MultiFab's dtype.  Planes are padded so that each
 * starts on a 128-byte boundary.  Ghost cells outside the valid x range
 * live in the x ghost slab (bl_multifab_xghost_layout).
 */
bl_status bl_multifab_layout(const bl_multifab* mf, int32_t box, bl_box* grown, size_t* offset_elems,
                             int64_t stride[4]);

/*
 * Layout of the x ghost slab of FAB `box` (nghost >= 1): the element offset of
 * the ghost cell (box.lo[0]-1, grown lo y, grown lo z), component 0, and
 * strides {layer, y, z, side, comp}.  Ghost cell (i,j,k), component n, with
 * i < box.lo[0] (side 0, layer box.lo[0]-1-i) or i > box.hi[0] (side 1, layer
 * i-box.hi[0]-1), is at offset + layer*stride[0] + (j - grown.lo[1])*stride[1]
 * + (k - grown.lo[2])*stride[2] + side*stride[3] + n*stride[4].
 */
bl_status bl_multifab_xghost_layout(const bl_multifab* mf, int32_t box, size_t* offset_elems, int64_t stride[5]);

/*
 * Copy FAB `box` (its whole grown box, valid and ghost cells, components
 * [scomp, scomp+ncomp)) to (to_dense != 0) or from a dense device array of
 * shape (ncomp, nz, ny, nx) over the grown box, x fastest, of the MultiFab's
 * dtype.  Bit copies.
 */
bl_status bl_multifab_copy_fab(bl_multifab* mf, int32_t box, int32_t scomp, int32_t ncomp, void* dense_dev,
                               int32_t to_dense, hipStream_t stream);

/* Shape query: number of boxes, ncomp, nghost, dtype. */
bl_status bl_multifab_info(const bl_multifab* mf, int32_t* nboxes, int32_t* ncomp, int32_t* nghost,
                           int32_t* dtype);
/* Frees the handle and its metadata; does not free dev_ptr. */
void bl_multifab_destroy(bl_multifab* mf);

/*
 * Next to each box's valid cells the storage holds a copy of the box's first
 * and last valid x column, contiguous along y (its edge mirror; with nghost
 * >= 4, of its first and last 4 columns).  Reading a neighbour box's x face
 * from that copy costs a few contiguous lines instead of one line per row.
 * The library remembers, per MultiFab, whether the copy is current: the calls
 * that write it with the state they produce (the fused heat, GSRB and
 * variable-coefficient steps, the 8th-order mirror form, the unfused heat
 * step's stencil) mark it so, every other write by the library marks it
 * stale, and later calls read the copy only where it is current (the first
 * step of an advance, FillBoundary, the first GSRB pass).  A caller who writes
 * a MultiFab's storage without the library (through its own kernels or
 * copies) must call bl_multifab_modified before the MultiFab's next use;
 * otherwise a later call may read a stale copy.  BL_EINVAL for NULL.
 */
bl_status bl_multifab_modified(bl_multifab* mf);

/*
 * Copy between the valid cells of components [scomp, scomp+ncomp) and a dense
 * device array `global_dev` of shape (ncomp, Nz, Ny, Nx) over the domain, x
 * fastest, of the MultiFab's dtype.  to_global != 0 copies MultiFab -> array
 * (cells no box covers are not written); 0 copies array -> MultiFab.  Ghost
 * cells are not touched.
 */
bl_status bl_multifab_copy_global(bl_multifab* mf, int32_t scomp, int32_t ncomp, void* global_dev,
                                  int32_t to_global, hipStream_t stream);

/* Set components [scomp, scomp+ncomp) to val on valid cells, and on ghost cells too if with_ghosts. */
bl_status bl_multifab_set_val(bl_multifab* mf, double val, int32_t scomp, int32_t ncomp, int32_t with_ghosts,
                              hipStream_t stream);

/* ------------------------------------------------------------ FillBoundary */

/*
 * FillBoundary (Sec. 3.1, Sec. 3.3, Sec. 4.1): for components [scomp,
 * scomp+ncomp), every ghost cell of every FAB takes the valid value at its
 * index wrapped along the periodic axes, if that index lies in the domain and
 * in some box; other ghost cells keep their value.  Valid cells are only read.
 */
bl_status bl_fill_boundary(bl_multifab* mf, int32_t scomp, int32_t ncomp, hipStream_t stream);

/* ---------------------------------------------------------------- heat step */

/*
 * One forward-Euler heat step with second-order centred differences
 * (Sec. 4.1), the plain per-box form: optionally FillBoundary(u_old) first
 * (fill_first != 0), then one kernel launch per box:
 *   u_new = u + c*( ((u[i-1]+u[i+1]) + (u[j-1]+u[j+1])) + (u[k-1]+u[k+1]) - 6u ),
 *   c = dt/dx^2 (diffusivity 1), for every component, on valid cells.
 * Ghost cells of u_new are not written.  u_old and u_new must share BoxArray,
 * ncomp and nghost (BL_ESHAPE) and dtype (BL_EDTYPE); nghost >= 1 (BL_EINVAL).
 */
bl_status bl_heat_step(bl_multifab* u_old, bl_multifab* u_new, double c, int32_t fill_first,
                       hipStream_t stream);

/*
 * nsteps heat steps, ping-ponging u[0] -> u[1] -> u[0] ...; the result is in
 * u[nsteps % 2].  Each step is ONE launch of the fused kernel over the
 * flattened tile list of all boxes and components: tiles next to a box face
 * read the neighbouring box's valid cells (or their periodic image) directly,
 * which is the value FillBoundary would have put in the ghost cell; x
 * neighbours come from the copy of each box's edge columns that every step
 * writes with the new state (the first step reads them from the neighbours'
 * rows in the default tile form; the other forms run a first kernel that makes
 * the copy for u[0]).  The launches
 * are captured once in a HIP graph and replayed.  Ghost
 * cells are neither read where a box covers them nor written.  Results are
 * bit-identical to bl_heat_step with fill_first = 1.
 */
bl_status bl_heat_advance(bl_multifab* u[2], int32_t nsteps, double c, hipStream_t stream);

/*
 * nsteps forward-Euler heat steps with the 8th-order centred second difference
 * (9 cells per axis: the stencil span of Sec. 4.2's application, applied to the
 * heat equation), ping-ponging u[0] -> u[1] -> ...; result in u[nsteps % 2].
 * With p_m = u[-m] + u[+m] along an axis (m = 1..4),
 *   D = ((A1*p1 + A2*p2) + A3*p3) + A4*p4,   u_new = u + c*(((Dx + Dy) + Dz) + A0X3*u),
 * A1 = 8/5, A2 = -1/5, A3 = 8/315, A4 = -1/560, A0X3 = 3*(-205/72), each rounded
 * once (to the storage type for FP32); c = dt/dx^2.  nghost >= 4 (BL_EINVAL);
 * shapes as bl_heat_step.  Forward Euler with this stencil is stable for
 * c <= 0.1025.  Each step is one stencil launch over all boxes and components,
 * in one of two forms with bit-identical results:
 *   BL_H8_FILL   FillBoundary(u_old), then the stencil reads u_old's ghosts;
 *   BL_H8_FUSED  no FillBoundary: cells outside a box are read from the
 *                neighbour box (periodic image included) that FillBoundary would
 *                copy them from, or from the box's own ghost cells where no box
 *                covers them; each lane finds its source among the face's
 *                segments.  Applies where every neighbour across a face is at
 *                least 4 cells thick, plane strides fit in 32 bits and, with
 *                vectors of more than one cell, neighbour boundaries fall on
 *                x-vector edges (bl_heat8_fused_ok); else BL_EINVAL.
 *   BL_H8_AUTO   the fused form where it applies, else the fill form.
 *   BL_H8_FUSED_MIRROR  the fused form that also writes u_new's 4-layer edge
 *                mirror (copies of the first and last 4 valid x columns,
 *                contiguous along y; see bl_multifab_modified) and, where its
 *                input's mirror is current, reads the x-face cells a neighbour
 *                covers from that neighbour's mirror instead of its rows (a few
 *                contiguous lines per face plane instead of one line per row).
 *                The first step of a call reads the rows unless the previous
 *                call left u[0]'s mirror current.  Needs every box at least 8
 *                cells wide in x (BL_EINVAL).  Fewer bytes fetched, more
 *                written; BL_H8_AUTO does not pick it.
 * The fill form writes u_old's ghost cells each step; the fused forms write no
 * ghost cell.  bl_heat8_advance is bl_heat8_advance_form with BL_H8_AUTO.
 */
typedef enum { BL_H8_AUTO = 0, BL_H8_FILL = 1, BL_H8_FUSED = 2, BL_H8_FUSED_MIRROR = 3 } bl_h8_form;
bl_status bl_heat8_advance(bl_multifab* u[2], int32_t nsteps, double c, hipStream_t stream);
bl_status bl_heat8_advance_form(bl_multifab* u[2], int32_t nsteps, double c, int32_t form, hipStream_t stream);
/* *ok = 1 where the fused form applies to mf's layout, else 0 (also for
 * nghost < 4).  Builds and caches its face segments (host work and a device
 * upload, once per layout). */
bl_status bl_heat8_fused_ok(const bl_multifab* mf, int32_t* ok);

/*
 * Host-only views of the metadata above, for checking it without a GPU (no
 * device memory is touched).  bl_heat8_fused_layout: the face segments the
 * fused 8th-order form would use for a MultiFab of this shape (from_mirror = 0:
 * those of a step that reads neighbour rows; 1: those of a step whose input's
 * 4-layer mirror is current, BL_EINVAL where a box is narrower than 8 cells in
 * x); *nsegs their count; with segs non-NULL, 12 int64 per segment {box, face (2*axis + side),
 * t1lo, t1hi, t2lo, t2hi, o, sc, sx, sy, sz, vec}: the segment covers the 4 cell
 * layers of that face over box-local tangential coordinates (t1, t2) in
 * [t1lo, t1hi] x [t2lo, t2hi] ((y, z) for x faces, (x, z) for y faces, (x, y)
 * for z faces), and cell (x, y, z) of component n there is element
 * o + n*sc + x*sx + y*sy + z*sz; *total_elems (nullable) the MultiFab's
 * element count.  BL_EINVAL (reason in bl_last_error) where the fused form
 * does not apply.  bl_layout_index: element index of cell (global indices,
 * inside box's grown box) of component comp in a MultiFab of this shape.
 * bl_layout_mirror_index: element index of row j, plane k (global indices,
 * inside box's valid box) of layer `layer` of side `side` (0 low x, 1 high x)
 * of box's edge mirror, the copy of valid column `layer` (side 0) or
 * ex-1-layer (side 1); 4 layers with nghost >= 4, else 1 (BL_EINVAL beyond).
 */
bl_status bl_heat8_fused_layout(const bl_boxarray* ba, int32_t ncomp, int32_t nghost, int32_t dtype,
                                int32_t from_mirror, int32_t* nsegs, int64_t* segs, int64_t* total_elems);
bl_status bl_layout_index(const bl_boxarray* ba, int32_t ncomp, int32_t nghost, int32_t dtype, int32_t box,
                          const int32_t cell[3], int32_t comp, int64_t* index);
bl_status bl_layout_mirror_index(const bl_boxarray* ba, int32_t ncomp, int32_t nghost, int32_t dtype, int32_t box,
                                 int32_t side, int32_t layer, int32_t j, int32_t k, int32_t comp, int64_t* index);

/*
 * nsteps forward-Euler steps of du/dt = div(beta grad u) in the flux form
 * (Sec. 4.1's face-flux loops, here with a coefficient per cell), ping-ponging
 * u[0] -> u[1] -> u[0] ...; the result is in u[nsteps % 2].  Per valid cell
 * and component n, with b the mean of the two cells' beta on each face:
 *   F(i-1/2) = (0.5*(beta[i-1] + beta[i])) * ((u[i] - u[i-1]) * inv_dx)   (and y, z),
 *   u_new = u + dt*((dFx + dFy) + dFz),   dFx = (F(i+1/2) - F(i-1/2)) * inv_dx.
 * inv_dx is 1/dx, formed by the caller.  beta (component n: the coefficient of
 * u's component n) shares BoxArray, ncomp, nghost and dtype with u (BL_ESHAPE,
 * BL_EDTYPE) and its own storage (BL_EINVAL); its valid cells are only read.
 * Neighbour values are those FillBoundary would put in the ghost cells of u
 * and of beta.  Each step is ONE launch over the flattened tile list: where
 * every face source allows aligned vector loads, tiles next to a box face read
 * the neighbouring boxes directly, and a first kernel writes the edge-column
 * copies of beta and u[0] (beta's ghost cells are not written); otherwise
 * beta's ghosts are filled once and u's before each step.  The stream is not
 * synchronised; stability (dt <= dx^2 / (6 max beta)) is the caller's.
 */
bl_status bl_heat_varcoef_advance(bl_multifab* u[2], bl_multifab* beta, int32_t nsteps, double dt,
                                  double inv_dx, hipStream_t stream);

/*
 * One step of the unfused batched form: FillBoundary(u_old) as one copy
 * kernel, then one stencil kernel over all tiles reading the filled ghosts.
 * Same result as bl_heat_step; kept to measure the fill fraction.
 */
bl_status bl_heat_step_unfused(bl_multifab* u_old, bl_multifab* u_new, double c, hipStream_t stream);

/* ------------------------------------------------------ red-black Gauss-Seidel */

/*
 * nsweeps red-black Gauss-Seidel sweeps on -L_h phi = f, L_h the 7-point
 * Laplacian (L_h phi = (sum of 6 neighbours - 6 phi)/h2), in place on phi
 * (component 0).  Colour = parity of i+j+k in global indices, red (even)
 * first; FillBoundary(phi) runs before each colour, and each cell of the
 * colour is solved exactly:
 *   phi = ((((phi[i-1]+phi[i+1]) + (phi[j-1]+phi[j+1])) + (phi[k-1]+phi[k+1])) + h2*f) * (1/6).
 * If resnorm_host != NULL, after each sweep the FP64 residual norm
 * ||f + L_h phi||_2 over valid cells is written to resnorm_host[s] (the stream
 * is synchronised once at the end).  phi and f share BoxArray, dtype and
 * nghost >= 1.  Every periodic axis needs an even extent (else BL_EINVAL:
 * the colouring would not match across the wrap).
 *
 * Where it applies (bl_gsrb_one_pass_applies), each sweep is one pass over
 * the level: FillBoundary, then the new red values of the face ghost cells
 * computed from the neighbouring boxes, then one launch that computes each
 * box's red values a plane ahead of its black ones, into a second state
 * buffer of phi's size (allocated on first use and kept with phi; phi holds
 * the result when the call returns).  The cell values are those of the
 * two-pass form to the bit; phi's ghost cells that a box covers are left
 * with unspecified values (the two-pass form leaves them as they were), those
 * no box covers keep theirs.  Writes f's edge mirror if it is not current.
 */
bl_status bl_gsrb_sweeps(bl_multifab* phi, const bl_multifab* f, double h2, int32_t nsweeps,
                         double* resnorm_host, hipStream_t stream);

/*
 * Configuration of bl_gsrb_sweeps (process-wide): one_pass = 1 (default)
 * takes the one-pass sweep where it applies, 0 always the two colour passes;
 * zchunk (>= 0): planes of one box per workgroup of the one-pass sweep (0,
 * the default: 32, halved down to 8 while the level would have fewer than 256
 * workgroups); vectors_per_lane: 16-byte plane vectors per lane (1 or 2; 0, the
 * default: 1 for planes of at most 512 vectors, else 2).  BL_EINVAL for
 * other values.
 */
bl_status bl_set_gsrb_config(int32_t one_pass, int32_t zchunk, int32_t vectors_per_lane);
bl_status bl_get_gsrb_config(int32_t* one_pass, int32_t* zchunk, int32_t* vectors_per_lane);

/*
 * *applies = 1 if bl_gsrb_sweeps on phi takes the one-pass sweep under the
 * current configuration: every box's x extent a whole number of 16-byte
 * vectors (vec = 4 FP32 or 2 FP64 values), planes of at most 1024 lanes'
 * vectors, at least as many lanes as ghost items around a plane (2*ex/vec
 * ghost-row vectors + 2*ey x ghost values) and as 4*ey, three plane buffers
 * within one workgroup's LDS (160 KiB on MI355X).  Otherwise 0.
 */
bl_status bl_gsrb_one_pass_applies(const bl_multifab* phi, int32_t* applies);

/* ||f + L_h phi||_2 over valid cells in FP64 (fills phi's ghosts first); synchronises. */
bl_status bl_residual_norm(bl_multifab* phi, const bl_multifab* f, double h2, double* out_host,
                           hipStream_t stream);

/* ---------------------------------------------------------------- multigrid */

/*
 * Geometric multigrid for -L_h phi = f (Sec. 1 names the multilevel multigrid
 * solvers; Sec. 3.3 their coarse levels of small grids), cell-centred,
 * refinement ratio 2, single-component MultiFabs.  Box b of a coarse level is
 * box b of the level above coarsened (bl_boxarray_coarsen with ratio 2).
 *
 * Restriction of the residual: FillBoundary(phi), then every valid cell
 * (I,J,K) of fc takes the mean of the residuals r = f + (s - 6 phi)/h2 of its
 * 8 cells (2I+a, 2J+b, 2K+c) on phi's level (s as in the GSRB residual),
 * computed in FP64 from promoted values, summed in the order c, b, a (lower
 * child first), times 0.125, stored in fc's dtype.  phi and f share a shape;
 * fc lives on the coarsened BoxArray (BL_ESHAPE otherwise), same dtype
 * (BL_EDTYPE), its own storage.  fc's ghost cells are not written.
 */
bl_status bl_mg_restrict_residual(bl_multifab* phi, const bl_multifab* f, double h2, bl_multifab* fc,
                                  hipStream_t stream);

/*
 * Prolongation, piecewise constant: every valid cell (i,j,k) of phi adds the
 * value of cell (floor(i/2), floor(j/2), floor(k/2)) of pc (on the coarsened
 * BoxArray).  Ghost cells of phi are not written.
 */
bl_status bl_mg_prolong_add(bl_multifab* phi, const bl_multifab* pc, hipStream_t stream);

/*
 * The hierarchy.  Level 0 is `ba`; level l+1 is level l coarsened by 2, made
 * while every box and the domain have even corners and extents and every
 * periodic axis of the coarse domain keeps an even extent (red-black colouring
 * across the wrap), up to max_levels levels in all (>= 1).  Coarse levels hold
 * phi and f with one ghost layer in a caller-owned, 256-byte aligned device
 * workspace of bl_mg_workspace_bytes bytes (0 for a single level), which must
 * outlive the hierarchy.  nlevels (may be NULL) receives the level count.
 */
typedef struct bl_mg bl_mg;
bl_status bl_mg_workspace_bytes(const bl_boxarray* ba, bl_dtype dtype, int32_t max_levels, size_t* bytes,
                                int32_t* nlevels);
bl_status bl_mg_create(const bl_boxarray* ba, bl_dtype dtype, int32_t max_levels, void* work_dev, size_t bytes,
                       bl_mg** out);
bl_status bl_mg_levels(const bl_mg* mg, int32_t* nlevels);
/*
 * First level of the hierarchy's fused bottom, or -1: from that level down,
 * every level covers a fully periodic domain and all of them fit one
 * workgroup's LDS (phi and f of each; 160 KiB on MI355X), and bl_mg_vcycles runs that part
 * of each cycle as one launch (the same arithmetic as the level-by-level
 * passes, so the same bits).
 */
bl_status bl_mg_bottom_level(const bl_mg* mg, int32_t* level);
void bl_mg_destroy(bl_mg* mg);

/*
 * ncycles V-cycles on -L_h phi = f, phi (on the hierarchy's level-0 BoxArray,
 * its dtype, nghost 1) updated in place.  On level l, with h^2 = 4^l h2:
 * nu1 GSRB sweeps (as bl_gsrb_sweeps), the residual restricted into level
 * l+1's f, level l+1's phi set to 0 (ghost cells too), the cycle on level
 * l+1, its phi added back by prolongation, nu2 sweeps; the coarsest level takes
 * nu_bottom sweeps.  Ghost cells that no box covers keep the caller's values
 * on level 0 and are 0 on coarse levels.  If resnorm_host != NULL,
 * resnorm_host[c] = ||f + L_h phi||_2 over level 0's valid cells after cycle c
 * (FP64; the stream is synchronised once at the end).  Every periodic axis of
 * level 0 needs an even extent.
 */
bl_status bl_mg_vcycles(bl_mg* mg, bl_multifab* phi, const bl_multifab* f, double h2, int32_t ncycles,
                        int32_t nu1, int32_t nu2, int32_t nu_bottom, double* resnorm_host, hipStream_t stream);

/* ---------------------------------------------------------------- reductions */

/* Reduction of component comp over valid cells (Sec. 3.1); result to host; synchronises. */
bl_status bl_reduce(const bl_multifab* mf, int32_t comp, bl_reduce_op op, double* out_host,
                    hipStream_t stream);
/* Same, result written to device memory out_dev (one double); does not synchronise. */
bl_status bl_reduce_async(const bl_multifab* mf, int32_t comp, bl_reduce_op op, double* out_dev,
                          hipStream_t stream);

/*
 * For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): bl_reduce_async with the
 * same kernels and the same result, bit for bit, but its partial results (one
 * double per reduction chunk of about 32K values of the component) go to a
 * fixed device array of the library's, 65536 doubles (512 KiB) per GPU, held
 * from the first call on that GPU until the process ends.  It calls no
 * hipMalloc, hipFree or allocating library routine.  BL_EINVAL if the
 * MultiFab has more chunks than that (about 2^31 valid cells per component),
 * or for a NULL argument, a component out of range or an unknown op.
 * Asynchronous on `stream`; out_dev (one double, device memory) is written by
 * the stream.  Every call on one GPU shares that GPU's array: calls that
 * overlap on one GPU (two streams, or two threads) race and must be ordered
 * by the caller.
 */
bl_status bl_reduce_async_noalloc(const bl_multifab* mf, int32_t comp, bl_reduce_op op, double* out_dev,
                                  hipStream_t stream);

/* ------------------------------------------------------------ device copy */

/*
 * dst[0..bytes) = src[0..bytes) on the device, one 16-byte vector per lane and
 * one 4 KB chunk per workgroup: the plain streaming copy that serves as the
 * attainable-bandwidth line for the stencils.  dst, src and bytes must be
 * multiples of 16 and the ranges must not overlap (BL_EINVAL).  Asynchronous.
 */
bl_status bl_device_copy(void* dst, const void* src, size_t bytes, hipStream_t stream);

/* ------------------------------------------------------------ launch tuning */

/*
 * Tile shape of the stencil kernels: zchunk = most z planes per tile (1..16384),
 * waves = 64-lane waves per workgroup (1..4), persist = workgroups per CU of
 * the persistent grid (0: one workgroup per tile), block = 1 for the block
 * form (each tile issues all of its loads before its updates), 2 for the
 * block form exchanging in-tile neighbours through LDS, 3 for that form with
 * the tile's halo loaded from memory straight into LDS (zchunk 2, 4 or 8 for
 * the block forms), 0 for the z march.  zsteps (1..64, form 3 only): z steps
 * per tile; a workgroup takes its tile's planes zchunk at a time, bottom to
 * top, and carries the two planes above a step into the next one, so the
 * planes between steps are read once, not twice.  Default: zchunk 4, waves 4,
 * persist 0, block 3, zsteps 2.  Applies to MultiFabs created afterwards and to
 * bl_batch objects at their next rebuild; results do not depend on it.  The
 * configuration is one setting of the whole process, shared by every thread:
 * set it before creating MultiFabs, not while other threads create them.
 */
bl_status bl_set_tile_config(int32_t zchunk, int32_t waves, int32_t persist, int32_t block, int32_t zsteps);
bl_status bl_get_tile_config(int32_t* zchunk, int32_t* waves, int32_t* persist, int32_t* block, int32_t* zsteps);

/*
 * Autotuner of the tile shape (the paper tunes tile sizes per loop and
 * machine, Sec. 3.2 and Sec. 4.1; here the shape is picked by timing on the
 * device).  Times the fused heat step (bl_heat_advance's kernel) of u0/u1 on
 * `stream` for every candidate shape: block forms 3 and 2, zchunk 2, 4 and 8,
 * waves 2, 3 and 4, zsteps 1, 2, 4 and 8 for form 3 (persist as set by
 * bl_set_tile_config), 2 warm-up steps
 * then 2*trial_steps timed steps each (1 <= trial_steps <= 1000), and keeps
 * the fastest: MultiFabs of this (BoxArray, ncomp, nghost, dtype) created
 * afterwards use it, and u0 and u1 are switched to it now.  A later
 * bl_set_tile_config drops every autotuned choice.
 *
 * The contents of u0 and u1 are overwritten (the trial steps advance them):
 * tune before loading initial data, or on scratch MultiFabs.  Synchronises
 * `stream`.  Optional outputs: the first max_results candidates' shapes
 * (configs[5*i .. 5*i+4] = zchunk, waves, persist, block, zsteps) and their
 * mean milliseconds per step, their count in *nresults, the chosen shape in
 * best[5].
 * Errors: ESHAPE/EDTYPE as bl_heat_step, ESHAPE if u0 is not on ba, EINVAL
 * for trial_steps or max_results out of range, EHIP.
 */
bl_status bl_autotune(const bl_boxarray* ba, bl_multifab* u0, bl_multifab* u1, double c, int32_t trial_steps,
                      int32_t max_results, int32_t* nresults, int32_t* configs, float* ms_per_step,
                      int32_t best[5], hipStream_t stream);

/* ------------------------------------------------------------------- batching */

/*
 * A set of independent heat problems advanced together: every bl_batch_step
 * advances each member by one step with one fused launch per dtype over the
 * concatenated tile lists.  Members may be added and removed between steps.
 * u0/u1 are the member's ping-pong pair (same shape and dtype, nghost >= 1);
 * its current state is u0 after an even number of its steps, u1 after an odd
 * number (bl_batch_parity).  The MultiFabs must outlive their membership.
 * The paper's collapsed (grid, tile) loop (Sec. 3.3) spans every member here.
 *
 * Issue every bl_batch_step of one batch on the same stream: after an add or
 * remove, the next step refills the batch's device tables with copies ordered
 * on that stream (no device synchronisation), building each member's tile
 * list once, when it is first stepped.  Only a newly joined member's edge
 * mirror is extracted; the fused kernel keeps the others current.
 */
bl_status bl_batch_create(bl_batch** out);
bl_status bl_batch_add(bl_batch* b, bl_multifab* u0, bl_multifab* u1, double c, int32_t* member_id);
bl_status bl_batch_remove(bl_batch* b, int32_t member_id);
bl_status bl_batch_parity(const bl_batch* b, int32_t member_id, int32_t* steps_done);
bl_status bl_batch_step(bl_batch* b, hipStream_t stream);
/*
 * nsteps consecutive bl_batch_step calls in one (nsteps >= 0; EINVAL below):
 * the same launches in the same order, issued from the library, so that a
 * serving loop pays its own per-step host work once per call.  Members join and
 * leave only between calls.
 */
bl_status bl_batch_steps(bl_batch* b, int32_t nsteps, hipStream_t stream);
void bl_batch_destroy(bl_batch* b);

/* ------------------------------------------------------- metadata inspection */

/*
 * FillBoundary copy plan of a BoxArray for ghost width nghost: number of
 * records, and if rec != NULL the records as 11 int32 each: {dst box, src box,
 * lo[3], hi[3] of the destination ghost region (global indices), shift[3]},
 * the source cell being destination + shift.  Every ghost cell that some box
 * covers (after periodic wrap) lies in exactly one record.  Host metadata
 * only (no device work); for tests and inspection.
 */
bl_status bl_fill_plan(const bl_boxarray* ba, int32_t nghost, int32_t* nrec, int32_t* rec);

/*
 * Logical tiles of every box (Sec. 3.2's tiling of a box for one loop): along
 * each axis, tiles of tile_size[d] cells from the box's low corner, the last
 * one taking what remains; listed box by box, then by z, y and x (x fastest).
 * 7 int32 per tile {box, lo[3], hi[3]} (inclusive, global index space):
 *   BL_TILE_CELL   the tile's cells (arg ignored); the tiles of a box partition it;
 *   BL_TILE_NODAL  faces normal to axis arg (face i lies between cells i-1 and i):
 *                  the tile's lower faces, plus face hi+1 where the tile ends at the
 *                  box's high side, so the face tiles of a box partition its faces;
 *   BL_TILE_GROWN  the tile grown by arg cells on the sides where it meets the box
 *                  boundary only, so grown tiles still do not overlap.
 * With out == NULL only *ntiles is set.  tile_size[d] >= 1, 0 <= arg <= 2 for
 * NODAL, arg >= 0 for GROWN (else BL_EINVAL).  Host metadata only.
 */
typedef enum { BL_TILE_CELL = 0, BL_TILE_NODAL = 1, BL_TILE_GROWN = 2 } bl_tile_kind;
bl_status bl_tile_boxes(const bl_boxarray* ba, const int32_t tile_size[3], bl_tile_kind kind, int32_t arg,
                        int32_t* ntiles, int32_t* out);

/*
 * Face-source records of the fused stencil: for each box and face (2*axis +
 * side, side 1 = high), the one-cell layer just outside the face split into
 * rectangles, each read from one source box (src) at destination + shift; a
 * part no box covers has src = the box itself and shift 0 (its own ghost
 * cells).  12 int32 per record: {box, face, src, lo[3], hi[3], shift[3]}.
 * Host metadata only.
 */
bl_status bl_face_plan(const bl_boxarray* ba, int32_t* nrec, int32_t* rec);

/*
 * Flattened tile list of the stencil kernels for a MultiFab of this shape
 * under the current tile configuration: number of tiles and, if tiles != NULL,
 * 9 int32 per tile {box, comp, xv0, nvt, y0, rows, z0, z1, vec}: x vectors
 * xv0..xv0+nvt-1 (each vec consecutive x cells, box-local) of rows
 * y0..y0+rows-1 over box-local z planes z0..z1-1.  Host metadata only.
 */
bl_status bl_tile_list(const bl_boxarray* ba, int32_t ncomp, int32_t nghost, bl_dtype dtype, int32_t* ntiles,
                       int32_t* tiles);

/*
 * Tiles of the stencil forms with the halo in LDS (block form 3; empty under
 * other forms) for a MultiFab of this shape under the current tile
 * configuration: 11 int32 per tile {box, comp, q0, nq, nzs, z0, z1, zchunk,
 * vec, lanes, zsteps}: the run of x vectors q0..q0+nq-1 of the box's plane
 * (vector q is row q / nvx, x vector q % nvx, nvx = x extent / vec) over planes
 * z0..z1-1, taken in z steps of nzs z blocks of zchunk planes each (at most
 * zsteps steps); nzs*nq <= lanes.  Where the configured shape gives fewer than
 * 1024 tiles, every tile takes one z step, and if still fewer, one z block per
 * step (more, shorter workgroups for a small level).  Host metadata only.
 */
bl_status bl_stencil_tiles(const bl_boxarray* ba, int32_t ncomp, int32_t nghost, bl_dtype dtype, int32_t* ntiles,
                           int32_t* tiles);

/*
 * Static partition of a tile list over nworkers, as the paper's tile-level
 * threading shares the collapsed (grid, tile) loop (Sec. 3.3): worker w gets
 * the contiguous range [first[w], first[w+1]) of near-equal length, the
 * first (ntiles mod nworkers) workers one tile more.  first has nworkers+1
 * entries.
 */
bl_status bl_static_partition(int32_t ntiles, int32_t nworkers, int32_t* first);

#ifdef __cplusplus
}
#endif

#endif /* BOXTILE_H */
