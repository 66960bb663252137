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
struct DevBox {
  int64_t off;       // element offset of valid cell (0,0,0) (box-local), component 0
  int64_t sc;        // component stride
  int32_t sy, sz;    // row and plane strides
  int32_t ex, ey, ez;
  int32_t nvx;       // x vectors per row (ex / vec)
  int32_t glo[3];    // global index of valid cell (0,0,0)
  int32_t face_start[6];
  int16_t face_count[6];
  int32_t pad_[1];
};
static_assert(sizeof(DevBox) % 8 == 0, "DevBox alignment");

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

// A unit of stencil work: lanes l0..l0+nl-1 of the box's plane (plane index =
// x-vector + row * vectors-per-row), z planes z0..z1-1, one component.
struct DevTile {
  int32_t box;
  int32_t comp;
  int32_t member;
  int32_t l0;
  int32_t nl;
  int32_t z0, z1;
  int32_t work;      // cells (nl * vec * (z1 - z0)), for static partitions
};
static_assert(sizeof(DevTile) == 32, "DevTile size");

// One heat problem of a launch: at launch flip f it reads a and writes b when
// (f + flip_offset) is even, and the reverse when it is odd.
struct DevMember {
  void* a;
  void* b;
  double c;
  int32_t flip_offset;
  int32_t pad_;
};

// FillBoundary copy chunk: up to kFillChunk cells of one record.
struct DevFillRec {
  int64_t dst_base;  // element offset of the region's low cell in the destination, comp 0
  int64_t src_base;  // element offset of its source cell, comp 0
  int64_t dsc, ssc;  // component strides
  int32_t dsy, dsz, ssy, ssz;
  int32_t nx, ny, nz;
  int32_t pad_;
};
struct DevFillChunk {
  int32_t rec;
  int32_t start;     // first cell (linear x-fastest index inside the region)
};
constexpr int kFillChunk = 256;

// ---------------------------------------------------------------- layout + plans
struct TileConfig {
  int zchunk = 1024;  // z planes per tile
  int waves = 4;      // 64-lane waves per workgroup
  int persist = 0;    // workgroups per CU for the persistent grid (0: one workgroup per tile)
};
TileConfig& tile_config();

struct FabGeom {
  Box grown;
  int64_t off_valid;  // element offset of valid cell (0,0,0), comp 0
  int64_t off_grown;  // element offset of the grown box's low cell, comp 0
  int64_t sy, sz, sc;
};

// Everything that depends on (BoxArray, ncomp, nghost, dtype) only; shared by
// every MultiFab of that shape, so records hold offsets relative to the data pointer.
struct Plan {
  uint64_t ba_uid = 0;
  std::vector<Box> boxes;
  Box domain{};
  int periodic[3] = {0, 0, 0};
  int ncomp = 0, ng = 0, dtype = 0, esize = 8, vec = 1, xlead = 0;
  std::vector<FabGeom> fabs;
  size_t total_elems = 0;

  // host copies
  std::vector<DevBox> hboxes;
  std::vector<DevFaceRec> hfacerecs;
  std::vector<DevTile> htiles;            // all components
  std::vector<int> box_tile_start;        // tiles of box b = [start[b], start[b+1])
  std::vector<DevFillRec> hfillrecs;
  std::vector<DevFillChunk> hfillchunks;
  std::shared_ptr<const std::vector<FillRecord>> fill;

  // device copies (owned), made by upload_plan
  DevBox* dboxes = nullptr;
  DevFaceRec* dfacerecs = nullptr;
  DevTile* dtiles = nullptr;
  DevFillRec* dfillrecs = nullptr;
  DevFillChunk* dfillchunks = nullptr;
  bool uploaded = false;
  TileConfig cfg;

  ~Plan();
};

bl_status build_plan(const bl_boxarray* ba, int ncomp, int ng, int dtype, std::shared_ptr<Plan>* out);
bl_status upload_plan(Plan& p);  // allocates and copies device metadata (once)
std::shared_ptr<const std::vector<FillRecord>> fill_plan(bl_boxarray* ba, int ng);
std::shared_ptr<const std::vector<FaceRecord>> face_plan(bl_boxarray* ba, int ng);
void build_tiles(const Plan& p, const TileConfig& cfg, int member, int box_base,
                 std::vector<DevTile>& tiles, std::vector<int>* box_tile_start);

}  // namespace bl

struct bl_multifab {
  std::shared_ptr<bl::Plan> plan;
  void* data = nullptr;
  size_t bytes = 0;
  double* dscratch = nullptr;   // reduction partials + results (device), grown on demand
  size_t nscratch = 0;
  double* hres = nullptr;       // pinned host landing slots for scalar results
  size_t nhres = 0;
  ~bl_multifab();
};
