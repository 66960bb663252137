// Internal declarations of libboxtile: host metadata and device descriptors.
#pragma once

#include <cstdint>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/boxtile.h"

namespace bl {

// ---------------------------------------------------------------- errors
bl_status fail(bl_status code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();
bl_status hip_fail(int err, const char* what);

#define BL_HIP(expr)                                   \
  do {                                                 \
    hipError_t e_ = (expr);                            \
    if (e_ != hipSuccess) return ::bl::hip_fail(e_, #expr); \
  } while (0)

// ---------------------------------------------------------------- boxes
struct Box {
  int lo[3], hi[3];
  int len(int d) const { return hi[d] - lo[d] + 1; }
  bool empty() const { return hi[0] < lo[0] || hi[1] < lo[1] || hi[2] < lo[2]; }
  int64_t volume() const { return empty() ? 0 : (int64_t)len(0) * len(1) * len(2); }
  bool contains(const Box& o) const {
    for (int d = 0; d < 3; ++d)
      if (o.lo[d] < lo[d] || o.hi[d] > hi[d]) return false;
    return true;
  }
  Box grow(int n) const {
    Box b = *this;
    for (int d = 0; d < 3; ++d) { b.lo[d] -= n; b.hi[d] += n; }
    return b;
  }
  Box shift(const int s[3]) const {
    Box b = *this;
    for (int d = 0; d < 3; ++d) { b.lo[d] += s[d]; b.hi[d] += s[d]; }
    return b;
  }
  static Box intersect(const Box& a, const Box& b) {
    Box r;
    for (int d = 0; d < 3; ++d) {
      r.lo[d] = a.lo[d] > b.lo[d] ? a.lo[d] : b.lo[d];
      r.hi[d] = a.hi[d] < b.hi[d] ? a.hi[d] : b.hi[d];
    }
    return r;
  }
};

inline Box from_c(const bl_box& b) {
  Box r;
  for (int d = 0; d < 3; ++d) { r.lo[d] = b.lo[d]; r.hi[d] = b.hi[d]; }
  return r;
}
inline bl_box to_c(const Box& b) {
  bl_box r;
  for (int d = 0; d < 3; ++d) { r.lo[d] = b.lo[d]; r.hi[d] = b.hi[d]; }
  return r;
}

// Uniform bins over the domain for box-intersection queries.
class BoxBins {
 public:
  void build(const std::vector<Box>& boxes, const Box& domain);
  // indices of boxes that may intersect q (q in domain coordinates, clipped)
  void query(const Box& q, std::vector<int>& out) const;

 private:
  Box dom_{};
  int bin_[3] = {1, 1, 1}, nb_[3] = {1, 1, 1};
  std::vector<std::vector<int>> cells_;
  mutable std::vector<int> mark_;
  mutable int stamp_ = 0;
};

// ---------------------------------------------------------------- level geometry
struct FillRecord {   // FillBoundary copy plan entry
  int dst, src;       // box indices
  Box region;         // destination ghost cells, global indices
  int shift[3];       // source cell = destination cell + shift
};

struct FaceRecord {   // one source rectangle of one face layer of a box
  int box, face;      // face = 2*axis + side (side 1 = high)
  int src;            // source box (== box for an uncovered part: own ghost cells)
  Box region;         // destination ghost cells (one cell thick), global indices
  int shift[3];
};

}  // namespace bl

// Opaque handle types of the C interface.
struct bl_boxarray {
  std::vector<bl::Box> boxes;
  bl::Box domain;
  int periodic[3];
  uint64_t uid;
  bl::BoxBins bins;
  // plans computed lazily per ghost width
  std::mutex mu;
  std::vector<std::pair<int, std::shared_ptr<const std::vector<bl::FillRecord>>>> fill_plans;
  std::vector<std::pair<int, std::shared_ptr<const std::vector<bl::FaceRecord>>>> face_plans;
};

struct bl_distmap {
  std::vector<int> owner;
  uint64_t ba_uid;
};

namespace bl {

// ---------------------------------------------------------------- device descriptors
// Per box of a MultiFab layout.  Offsets and strides are in elements.
//
// FAB layout, per component block (comp stride sc):
//   rows:   the grown box in y and z, valid x only: cell (i, j, k) (box-local,
//           i in [0, ex), j and k in [-ng, e+ng)) at off + i + j*sy + k*sz;
//           rows of a plane are contiguous (sy = ex) and every plane starts
//           on a 128-byte boundary, so whole rows form one contiguous span;
//   x slab: the x ghost cells, contiguous along y: ghost layer l (0 = next to
//           the box) of side s (0 = low x, 1 = high x) at
//           xs + s*xs_side + k*xs_z + j*ng + l  (j, k grown range);
//   mirror: a copy of the box's own first (s = 0) and last (s = 1) valid x
//           column, contiguous along y: mir + s*mir_side + k*ey + j.  The fused
//           stencil writes it with each new state; neighbours read their x
//           face values from it.  With nghost >= 4 it holds 4 layers per side,
//           layer m (m = 0..3: column m, or column ex-1-m on side 1) at
//           mir + s*mir_side + m*ey*ez + k*ey + j, so layer 0 is where the
//           1-layer copy is; the fused 8th-order step writes all 4.
struct DevBox {
  int64_t off;       // row cell (0,0,0), component 0
  int64_t sc;        // component stride
  int64_t xs;        // x slab cell (side 0, j = 0, k = 0, l = 0), component 0
  int64_t mir;       // mirror (side 0, j = 0, k = 0), component 0
  int32_t sy, sz;    // row and plane strides
  int32_t xs_side, xs_z, mir_side;
  int32_t ex, ey, ez;
  int32_t nvx;       // x vectors per row (ex / vec)
  int32_t ng;
  int32_t glo[3];    // global index of valid cell (0,0,0)
  int32_t face_start[6];
  int16_t face_count[6];
  int32_t pad_[2];
};
static_assert(sizeof(DevBox) % 16 == 0, "DevBox alignment");

// Source of the ghost layer next to one face, over a rectangle of the face:
// the value next to box-local tangential coordinates (t1, t2) of component n is
// data[base + t1*s1 + t2*s2 + n*sc].  Tangential axes of an x face are (y, z),
// of a y face (x, z), of a z face (x, y).
struct DevFaceRec {
  int64_t base;
  int64_t sc;
  int32_t s1, s2;
  int16_t t1lo, t1hi, t2lo, t2hi;
};
static_assert(sizeof(DevFaceRec) == 32, "DevFaceRec size");

// A unit of stencil work: x vectors xv0..xv0+nvt-1 (each vec cells) of rows
// y0..y0+rows-1 of one box and component, over box-local z planes z0..z1-1.
// Lane l of the workgroup takes x vector xv0 + l % nvt of row y0 + l / nvt.
// Tiles never straddle a z boundary of the box's x- or y-face records, so
// each lane's face sources are fixed for the whole tile.
// frec[f]: for each face f of the box that the tile touches, the index of the
// one face record that covers the tile's part of that face, kFaceMany if
// several records do (the kernel then searches), kFaceNone if the tile does
// not touch face f.
// Where the fused 8th-order stencil reads the cells next to one face of a box:
// the face's 4 cell layers are tiled by segments, each a rectangle of the
// face's tangential coordinates (t1, t2) = (y, z) for x faces, (x, z) for y
// faces, (x, y) for z faces (box-local), over all 4 layers.  Cell (x, y, z) of
// component n (box-local indices of the face's box) in a segment is
// data[o + n*sc + x*sx + y*sy + z*sz].  The source is one neighbour box (through
// its FillBoundary record, periodic shift included) or the box's own ghost
// cells where no box covers that part of the face (x faces: the x ghost slab,
// sx = -1 on the low side).
struct DevH8Seg {
  int64_t o, sc, sz;
  int32_t sx, sy;
  int32_t t1lo, t1hi, t2lo, t2hi;
};
static_assert(sizeof(DevH8Seg) == 48, "DevH8Seg size");
struct DevH8Face {  // the segments of face f of a box: [start[f], start[f] + count[f])
  int32_t start[6];
  int32_t count[6];
};

constexpr int32_t kFaceNone = -1;
constexpr int32_t kFaceMany = -2;
struct DevTile {    // 32-bit fields only: each one is a plain scalar load
  int32_t box;
  int32_t member;
  int32_t comp;
  int32_t xv0, nvt;
  int32_t y0, rows;
  int32_t z0, z1;
  int32_t frec[6];
  int32_t pad_;
};
static_assert(sizeof(DevTile) == 64, "DevTile size");

// A unit of work of the stencil forms with the halo in LDS: a run of nq
// consecutive x vectors of a plane (the valid rows of a plane are contiguous,
// so vector q is row q / nvx, x vector q % nvx, and a run may start or end
// inside a row), over planes z0..z1-1 split into nzs z blocks of zchunk planes.
// Lane l takes vector q0 + l % nq of block l / nq.  rows spanned: y_first ..
// y_first + nrows - 1.  frec as for DevTile, over the tile's bounding rows.
struct DevLinTile {
  int32_t box;
  int32_t member;
  int32_t comp;
  int32_t q0, nq, nzs;
  int32_t z0, z1;
  int32_t y_first, nrows;
  int32_t frec[6];
};
static_assert(sizeof(DevLinTile) == 64, "DevLinTile size");

// A reduction chunk: valid planes z0..z1-1 of one box (any one component).  The
// valid cells of a plane are one contiguous run (rows are contiguous), so a
// chunk is z1-z0 runs of ex*ey values.
struct DevRedChunk {
  int32_t box, z0, z1, pad_;
};

// One heat problem of a launch: at launch flip f it reads a and writes b when
// (f + flip_offset) is even, and the reverse when it is odd.
struct DevMember {
  void* a;
  void* b;
  double c;
  int32_t flip_offset;
  int32_t pad_;
};

// FillBoundary copy record: a box of destination ghost cells, one class of
// storage (rows or one side of the x slab), and its source valid cells; both
// addresses are affine in the cell's offset (x, y, z) from the region's low corner.
struct DevFillRec {
  int64_t dst_base;  // element index of the region's low cell, comp 0
  int64_t src_base;  // element index of its source cell, comp 0
  int64_t dsc, ssc;  // component strides
  int32_t dsx, dsy, dsz;
  int32_t ssx, ssy, ssz;
  int32_t nx, ny, nz;
  int32_t pad_[3];
};
struct DevFillChunk {
  int32_t rec;
  int32_t start;     // first cell (linear x-fastest index inside the region)
};
// The one-pass red-black sweep: one covered part of one face ghost layer of a
// box, whose new red values are computed from the source box's data.
// Destination ghost cell (t1, t2) of the region (box-local coordinates of the
// destination, the face coordinate fixed) is source box-local cell
// (destination + d); t1 is the fastest of the face's tangential axes (y for
// x faces, x for y and z faces).
struct DevRingRec {
  int32_t box, src, face;
  int32_t lo[3];   // destination box-local cell at the region's low corner
  int32_t n1, n2;  // region extents along t1 and t2
  int32_t d[3];
  int32_t pad_;
};
static_assert(sizeof(DevRingRec) == 48, "DevRingRec size");
// Where the one-pass sweep writes a box's new face cells so that they land in
// the neighbours' face ghost cells (the FillBoundary of its output, pushed by
// the source): face cell (t1, t2) of the source box (box-local tangential
// coordinates, t1lo..t1hi x t2lo..t2hi) goes to element base + t1*s1 + t2*s2.
struct DevPushRec {
  int64_t base;
  int32_t s1, s2;
  int32_t t1lo, t1hi, t2lo, t2hi;
};
static_assert(sizeof(DevPushRec) == 32, "DevPushRec size");
struct DevPushFace {  // the push records of face f of a box: [start[f], start[f] + count[f])
  int32_t start[6];
  int32_t count[6];
};
constexpr int kFillChunk = 256;
constexpr size_t kLatencyTiles = 1024;  // below this many linear tiles, shorter tiles (build_lin_tiles)
constexpr size_t kRingRecs = 2048;      // below this many one-pass ring records, records split along t2
constexpr int kStencilMaxThreads = 256;  // workgroup size limit of the stencil kernels (waves <= 4)
constexpr int kRestrictPerWG = 256;     // coarse cells per workgroup of the restriction (one per lane)
constexpr int kProlongPerWG = 1024;     // x pairs per workgroup of the prolongation (four per lane)
constexpr size_t kDmaLdsMax = 65536;     // LDS of one workgroup of the halo-in-LDS stencil form, at most

// ---------------------------------------------------------------- layout + plans
struct TileConfig {
  int zchunk = 4;     // z planes per tile at most
  int waves = 4;      // 64-lane waves per workgroup
  int persist = 0;    // workgroups per CU for the persistent grid (0: one workgroup per tile)
  int block = 3;      // 0: z march; 1: block form; 2: block form with LDS neighbours; 3: as 2, halos
                      // loaded straight into LDS (block forms: zchunk 2, 4 or 8)
  int zsteps = 2;     // form 3: z steps per linear tile (a tile spans up to zsteps * zchunk planes
                      // per z block; a workgroup carries the planes between its steps)
};
TileConfig& tile_config();

struct FabGeom {
  Box valid, grown;
  int64_t fab;        // first element of the FAB
  int64_t off;        // row cell (0,0,0), component 0 (as DevBox::off)
  int64_t sy, sz, sc;
  int64_t xs, xs_side, xs_z;
  int64_t mir, mir_side;
  int mir_layers;     // 4 with nghost >= 4, else 1 (layer stride ey*ez)
  int ng;
  // element index (component 0) of any cell of the grown box, global indices
  int64_t index(int i, int j, int k) const {
    const int li = i - valid.lo[0], lj = j - valid.lo[1], lk = k - valid.lo[2];
    const int ex = valid.len(0);
    if (li >= 0 && li < ex) return off + li + lj * sy + lk * sz;
    const int side = li < 0 ? 0 : 1;
    const int layer = li < 0 ? -1 - li : li - ex;
    return xs + side * xs_side + lk * xs_z + (int64_t)lj * ng + layer;
  }
};

// Everything that depends on (BoxArray, ncomp, nghost, dtype) only; shared by
// every MultiFab of that shape, so records hold offsets relative to the data pointer.
struct Plan {
  uint64_t ba_uid = 0;
  std::vector<Box> boxes;
  Box domain{};
  int periodic[3] = {0, 0, 0};
  int ncomp = 0, ng = 0, dtype = 0, esize = 8, vec = 1;
  int fvec = 1;  // every y- and z-face record's source rows are vec-aligned (one 16-byte load per lane)
  std::vector<FabGeom> fabs;
  size_t total_elems = 0;

  // host copies
  std::vector<DevBox> hboxes;
  std::vector<DevFaceRec> hfacerecs;
  // the same records with every covered x face read from the source box's rows
  // instead of its edge-column mirror: the first fused step of a run, whose
  // input has no current mirror
  std::vector<DevFaceRec> hfacerecs_rows;
  std::vector<DevTile> htiles;            // all components
  std::vector<int> box_tile_start;        // tiles of box b = [start[b], start[b+1])
  int rmax = 1;                           // most rows of any tile
  int nvtmax = 1;                         // most x vectors of any tile
  std::vector<DevLinTile> hlin;           // the stencil's tiles (forms with the halo in LDS)
  std::vector<DevRedChunk> hred;          // reduction chunks
  int yhmax = 1;                          // most halo row vectors (nzs * min(nvx, nq)) of a linear tile
  int xhmax = 1;                          // most halo row ends (nzs * nrows) of a linear tile
  std::vector<int32_t> hcellpre;         // flattened valid cells: box b holds [hcellpre[b], hcellpre[b+1])
  std::vector<int32_t> hpairpre;         // the same in pairs of x cells (boxes of even x extent)
  std::vector<int32_t> hcellwg;          // first box of each workgroup of kRestrictPerWG cells
  std::vector<int32_t> hpairwg;          // first box of each workgroup of kProlongPerWG pairs
  std::vector<DevFillRec> hfillrecs;
  // the same records, except that a one-column source at a box's x face is read
  // from the source box's edge mirror (contiguous along y) instead of its rows
  std::vector<DevFillRec> hfillrecs_mir;
  std::vector<DevFillChunk> hfillchunks;
  std::shared_ptr<const std::vector<FillRecord>> fill;
  // one-pass red-black sweep: covered face parts, the same parts as push
  // records grouped by source box and face, and each box's offset into the second edge-column copy (columns 1 and
  // ex-2: 2*ey*ez values per box)
  std::vector<DevRingRec> hringrecs;
  std::vector<DevPushRec> hpushrecs;
  std::vector<DevPushFace> hpushface;
  std::vector<int64_t> hmir2off;
  int64_t mir2_total = 0;
  bool faces_covered = false;  // no box has a face ghost cell that no box covers
  // the sweep's work chunks (box, planes), made on first use for one
  // (planes per chunk, vectors per lane); block: lanes per workgroup
  std::vector<DevRedChunk> hsweep;
  DevRedChunk* dsweep = nullptr;
  int sweep_zc = 0, sweep_k = 0, sweep_block = 0;
  int sweep_req_zc = -1, sweep_req_k = -1, sweep_ok = 0;  // the configuration it was made for
  size_t sweep_lds = 0;

  // device copies (owned), made by upload_plan
  DevBox* dboxes = nullptr;
  DevFaceRec* dfacerecs = nullptr;
  DevFaceRec* dfacerecs_rows = nullptr;
  DevTile* dtiles = nullptr;
  DevLinTile* dlin = nullptr;
  DevRedChunk* dred = nullptr;
  DevFillRec* dfillrecs = nullptr;
  DevFillRec* dfillrecs_mir = nullptr;
  DevFillChunk* dfillchunks = nullptr;
  int32_t* dcellpre = nullptr;
  int32_t* dpairpre = nullptr;
  int32_t* dcellwg = nullptr;
  int32_t* dpairwg = nullptr;
  DevRingRec* dringrecs = nullptr;
  DevPushRec* dpushrecs = nullptr;
  DevPushFace* dpushface = nullptr;
  int64_t* dmir2off = nullptr;
  bool uploaded = false;
  TileConfig cfg;

  // linear tiles of the variable-coefficient flux-form kernel, which stages two
  // fields: made on first use when the stencil's own would not fit its LDS
  std::vector<DevLinTile> hvlin;
  DevLinTile* dvlin = nullptr;
  int vyhmax = 1, vxhmax = 1, vzchunk = 0;

  // tiles of the 8th-order stencil (made on first use)
  std::vector<DevTile> hh8;
  DevTile* dh8 = nullptr;
  int h8rmax = 1, h8nvtmax = 1;
  bool h8built = false;
  // the fused form's face segments (made on first use); h8fused: -1 not tried,
  // 0 not possible (h8why), 1 built
  std::vector<DevH8Seg> hh8seg;
  std::vector<DevH8Face> hh8face;
  DevH8Seg* dh8seg = nullptr;
  DevH8Face* dh8face = nullptr;
  int h8fused = -1;
  std::string h8why;
  // the same segments with every x-face segment a neighbour covers reading
  // that neighbour's 4-layer edge mirror instead of its rows; h8mirror: the
  // fused form writes its output's 4-layer mirror and may read them (every
  // box at least 8 cells wide in x)
  std::vector<DevH8Seg> hh8segm;
  DevH8Seg* dh8segm = nullptr;
  bool h8mirror = false;

  ~Plan();
};

bl_status build_plan(const bl_boxarray* ba, int ncomp, int ng, int dtype, const TileConfig& cfg,
                     std::shared_ptr<Plan>* out);
bl_status upload_plan(Plan& p);  // allocates and copies device metadata (once)
std::shared_ptr<const std::vector<FillRecord>> fill_plan(bl_boxarray* ba, int ng);
std::shared_ptr<const std::vector<FaceRecord>> face_plan(bl_boxarray* ba, int ng);
void build_tiles(const Plan& p, const TileConfig& cfg, int member, int box_base, int rec_base,
                 std::vector<DevTile>& tiles, std::vector<int>* box_tile_start);

// Linear tiles of the stencil for every box and component: runs of at most
// 64*cfg.waves vectors (plane split evenly), or whole planes stacked in
// several z blocks when a plane holds fewer vectors than the workgroup.
void build_lin_tiles(const Plan& p, const TileConfig& cfg, int member, int box_base, int rec_base,
                     std::vector<DevLinTile>& tiles, int* yhmax, int* xhmax);
// LDS bytes of one workgroup of the linear-tile stencil forms.
size_t lin_lds_bytes(const TileConfig& cfg, int esize, int vec, int yhmax, int xhmax);
// Tiles of the 8th-order stencil: per box and component, x vectors in groups of
// at most 16, rows in groups of at most min(32, 256 / group width), z in chunks
// of 32 planes; memory order (z chunk, then y, then x).
void build_h8_tiles(const Plan& p, std::vector<DevTile>& tiles, int* rmax, int* nvtmax);
// Face segments of the fused 8th-order stencil (no FillBoundary) for every box.
// False (reason in *why) where the form does not apply: a neighbour thinner
// than the 4 layers across a face, or (vectors of more than one cell) a y- or
// z-face segment edge inside an x vector or a source row not vector-aligned.
// With msegs: also the segments that read x faces from the neighbours' 4-layer
// edge mirrors (same order and tangential ranges; left empty where some box is
// narrower than 8 cells in x, whose two mirror sides would share columns).
bool build_h8_segments(const Plan& p, std::vector<DevH8Seg>& segs, std::vector<DevH8Face>& faces, std::string* why,
                       std::vector<DevH8Seg>* msegs = nullptr);

}  // namespace bl

struct bl_multifab {
  std::shared_ptr<bl::Plan> plan;
  void* data = nullptr;
  size_t bytes = 0;
  // every box's edge mirror holds its current first and last valid x column:
  // set by the library's calls that write the mirror of the state they produce,
  // cleared by every other write (and by bl_multifab_modified for writes made
  // outside the library)
  bool mirror_current = false;
  // layers 1..3 of the 4-layer mirror (nghost >= 4) are current too: set only
  // by the fused 8th-order step, which writes all 4
  bool mirror4_current = false;
  // every write by the library but that step: layer 0 current or not, and the
  // other layers stale
  void mark_mirror(bool layer0_current) {
    mirror_current = layer0_current;
    mirror4_current = false;
  }
  // the one-pass red-black sweep's second edge-column copy (columns 1 and ex-2
  // of component 0), allocated on first use
  void* dmir2 = nullptr;
  void* dtwin = nullptr;  // the one-pass sweep's second state buffer (same layout)
  double* dscratch = nullptr;   // reduction partials + results (device), grown on demand
  size_t nscratch = 0;
  double* hres = nullptr;       // pinned host landing slots for scalar results
  size_t nhres = 0;
  ~bl_multifab();
};
