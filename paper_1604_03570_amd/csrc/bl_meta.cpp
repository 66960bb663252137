// Host metadata of libboxtile: errors, BoxArray / DistributionMapping, the
// FillBoundary copy plan, the per-face source records of the fused stencil,
// the FAB layout and the flattened tile list.  No device code here.
#include <algorithm>
#include <array>
#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>

#include "bl_internal.h"

namespace bl {

// ---------------------------------------------------------------- errors
static thread_local std::string g_err;

bl_status fail(bl_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

void clear_error() { g_err.clear(); }

TileConfig& tile_config() {
  static TileConfig cfg;
  return cfg;
}

// ---------------------------------------------------------------- bins
void BoxBins::build(const std::vector<Box>& boxes, const Box& domain) {
  dom_ = domain;
  int maxlen = 1;
  for (const Box& b : boxes)
    for (int d = 0; d < 3; ++d) maxlen = std::max(maxlen, b.len(d));
  for (int d = 0; d < 3; ++d) {
    bin_[d] = std::max(1, maxlen);
    nb_[d] = (domain.len(d) + bin_[d] - 1) / bin_[d];
  }
  cells_.assign((size_t)nb_[0] * nb_[1] * nb_[2], {});
  for (int i = 0; i < (int)boxes.size(); ++i) {
    const Box& b = boxes[i];
    int l[3], h[3];
    for (int d = 0; d < 3; ++d) {
      l[d] = (b.lo[d] - dom_.lo[d]) / bin_[d];
      h[d] = (b.hi[d] - dom_.lo[d]) / bin_[d];
    }
    for (int z = l[2]; z <= h[2]; ++z)
      for (int y = l[1]; y <= h[1]; ++y)
        for (int x = l[0]; x <= h[0]; ++x) cells_[((size_t)z * nb_[1] + y) * nb_[0] + x].push_back(i);
  }
  mark_.assign(boxes.size(), 0);
  stamp_ = 0;
}

void BoxBins::query(const Box& q0, std::vector<int>& out) const {
  out.clear();
  Box q = Box::intersect(q0, dom_);
  if (q.empty()) return;
  if (++stamp_ == 0) {
    std::fill(mark_.begin(), mark_.end(), 0);
    stamp_ = 1;
  }
  int l[3], h[3];
  for (int d = 0; d < 3; ++d) {
    l[d] = (q.lo[d] - dom_.lo[d]) / bin_[d];
    h[d] = (q.hi[d] - dom_.lo[d]) / bin_[d];
  }
  for (int z = l[2]; z <= h[2]; ++z)
    for (int y = l[1]; y <= h[1]; ++y)
      for (int x = l[0]; x <= h[0]; ++x)
        for (int i : cells_[((size_t)z * nb_[1] + y) * nb_[0] + x])
          if (mark_[i] != stamp_) {
            mark_[i] = stamp_;
            out.push_back(i);
          }
  std::sort(out.begin(), out.end());
}

// ---------------------------------------------------------------- SplitMix64
static uint64_t splitmix64(uint64_t seed, uint64_t n) {
  uint64_t z = seed + (n + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static std::atomic<uint64_t> g_uid{1};

static bl_status make_boxarray(std::vector<Box>&& boxes, const Box& domain, const int32_t periodic[3],
                               bl_boxarray** out) {
  if (!out) return fail(BL_EINVAL, "out is NULL");
  *out = nullptr;
  if (boxes.empty()) return fail(BL_EINVAL, "a BoxArray needs at least one box");
  if (domain.empty()) return fail(BL_EINVAL, "empty domain");
  for (size_t i = 0; i < boxes.size(); ++i) {
    const Box& b = boxes[i];
    if (b.empty()) return fail(BL_EINVAL, "box %zu is empty", i);
    if (!domain.contains(b))
      return fail(BL_EDOMAIN, "box %zu [%d,%d,%d]-[%d,%d,%d] leaves the domain", i, b.lo[0], b.lo[1], b.lo[2],
                  b.hi[0], b.hi[1], b.hi[2]);
  }
  bl_boxarray* ba = new (std::nothrow) bl_boxarray;
  if (!ba) return fail(BL_ENOMEM, "host allocation");
  ba->boxes = std::move(boxes);
  ba->domain = domain;
  for (int d = 0; d < 3; ++d) ba->periodic[d] = periodic ? (periodic[d] != 0) : 0;
  ba->uid = g_uid.fetch_add(1);
  ba->bins.build(ba->boxes, domain);
  // pairwise disjointness through the bins
  std::vector<int> cand;
  for (size_t i = 0; i < ba->boxes.size(); ++i) {
    ba->bins.query(ba->boxes[i], cand);
    for (int j : cand)
      if (j != (int)i && !Box::intersect(ba->boxes[i], ba->boxes[j]).empty()) {
        delete ba;
        return fail(BL_EOVERLAP, "boxes %zu and %d intersect", i, j);
      }
  }
  *out = ba;
  return BL_OK;
}

}  // namespace bl

using namespace bl;

extern "C" {

const char* bl_last_error(void) { return g_err.c_str(); }
const char* bl_version(void) { return "boxtile 0.1 (gfx950)"; }

bl_status bl_boxarray_create(const bl_box* boxes, int32_t nboxes, const bl_box* domain,
                             const int32_t periodic[3], bl_boxarray** out) {
  clear_error();
  if (!boxes || !domain || nboxes < 1) return fail(BL_EINVAL, "need boxes, nboxes >= 1 and a domain");
  std::vector<Box> v(nboxes);
  for (int i = 0; i < nboxes; ++i) v[i] = from_c(boxes[i]);
  return make_boxarray(std::move(v), from_c(*domain), periodic, out);
}

bl_status bl_boxarray_coarsen(const bl_boxarray* ba, int32_t ratio, bl_boxarray** out) {
  clear_error();
  if (!ba || !out) return fail(BL_EINVAL, "NULL argument");
  if (ratio < 1) return fail(BL_EINVAL, "ratio %d < 1", ratio);
  auto coarsen = [ratio](const Box& b, Box& c) {
    for (int d = 0; d < 3; ++d) {
      if (b.lo[d] % ratio != 0 || b.len(d) % ratio != 0) return false;
      c.lo[d] = b.lo[d] / ratio;
      c.hi[d] = (b.hi[d] + 1) / ratio - 1;
    }
    return true;
  };
  Box dom{};
  if (!coarsen(ba->domain, dom)) return fail(BL_EINVAL, "the domain's corner or extent is not divisible by %d", ratio);
  std::vector<Box> v(ba->boxes.size());
  for (size_t i = 0; i < v.size(); ++i)
    if (!coarsen(ba->boxes[i], v[i])) return fail(BL_EINVAL, "box %zu's corner or extent is not divisible by %d", i, ratio);
  return make_boxarray(std::move(v), dom, ba->periodic, out);
}

bl_status bl_boxarray_chop(const bl_box* domain, const int32_t periodic[3], const int32_t max_edge[3],
                           bl_boxarray** out) {
  clear_error();
  if (!domain || !max_edge) return fail(BL_EINVAL, "NULL argument");
  Box dom = from_c(*domain);
  if (dom.empty()) return fail(BL_EINVAL, "empty domain");
  std::vector<std::pair<int, int>> cuts[3];
  for (int d = 0; d < 3; ++d) {
    if (max_edge[d] < 1) return fail(BL_EINVAL, "max_edge[%d] = %d < 1", d, max_edge[d]);
    int e = std::min(max_edge[d], dom.len(d));
    for (int a = dom.lo[d]; a <= dom.hi[d]; a += e) cuts[d].push_back({a, std::min(a + e - 1, dom.hi[d])});
  }
  std::vector<Box> v;
  for (auto& z : cuts[2])
    for (auto& y : cuts[1])
      for (auto& x : cuts[0]) v.push_back(Box{{x.first, y.first, z.first}, {x.second, y.second, z.second}});
  return make_boxarray(std::move(v), dom, periodic, out);
}

bl_status bl_boxarray_chop_random(const bl_box* domain, const int32_t periodic[3], int32_t min_edge,
                                  int32_t max_edge, int32_t align, uint64_t seed, bl_boxarray** out) {
  clear_error();
  if (!domain) return fail(BL_EINVAL, "NULL domain");
  if (min_edge < 1 || align < 1 || min_edge % align != 0 || max_edge < 2 * min_edge)
    return fail(BL_EINVAL, "need min_edge %% align == 0 and max_edge >= 2*min_edge");
  Box dom = from_c(*domain);
  if (dom.empty()) return fail(BL_EINVAL, "empty domain");
  uint64_t counter = 0;
  std::vector<Box> v, stack{dom};
  while (!stack.empty()) {
    Box b = stack.back();
    stack.pop_back();
    int m = std::max(b.len(0), std::max(b.len(1), b.len(2)));
    if (m <= max_edge) {
      if (m < 2 * min_edge) {
        v.push_back(b);
        continue;
      }
      double u = (double)(splitmix64(seed, counter++) >> 11) * (1.0 / 9007199254740992.0);
      if (u < 0.5) {
        v.push_back(b);
        continue;
      }
    }
    int axis = b.len(0) == m ? 0 : (b.len(1) == m ? 1 : 2);
    uint64_t nchoice = (uint64_t)((m - 2 * min_edge) / align + 1);
    int off = min_edge + align * (int)(splitmix64(seed, counter++) % nchoice);
    Box lo = b, hi = b;
    lo.hi[axis] = b.lo[axis] + off - 1;
    hi.lo[axis] = b.lo[axis] + off;
    stack.push_back(hi);
    stack.push_back(lo);
  }
  return make_boxarray(std::move(v), dom, periodic, out);
}

bl_status bl_boxarray_get(const bl_boxarray* ba, int32_t* nboxes, bl_box* boxes) {
  clear_error();
  if (!ba || !nboxes) return fail(BL_EINVAL, "NULL argument");
  *nboxes = (int32_t)ba->boxes.size();
  if (boxes)
    for (size_t i = 0; i < ba->boxes.size(); ++i) boxes[i] = to_c(ba->boxes[i]);
  return BL_OK;
}

bl_status bl_boxarray_domain(const bl_boxarray* ba, bl_box* domain, int32_t periodic[3]) {
  clear_error();
  if (!ba) return fail(BL_EINVAL, "NULL BoxArray");
  if (domain) *domain = to_c(ba->domain);
  if (periodic)
    for (int d = 0; d < 3; ++d) periodic[d] = ba->periodic[d];
  return BL_OK;
}

void bl_boxarray_destroy(bl_boxarray* ba) { delete ba; }

bl_status bl_distmap_create(const bl_boxarray* ba, int32_t ndevices, const int32_t* owner, bl_distmap** out) {
  clear_error();
  if (!ba || !out) return fail(BL_EINVAL, "NULL argument");
  *out = nullptr;
  if (ndevices != 1) return fail(BL_EINVAL, "the library runs on one GPU: ndevices must be 1, got %d", ndevices);
  if (owner)
    for (size_t i = 0; i < ba->boxes.size(); ++i)
      if (owner[i] != 0) return fail(BL_EINVAL, "box %zu owned by device %d; only device 0 exists", i, owner[i]);
  bl_distmap* dm = new (std::nothrow) bl_distmap;
  if (!dm) return fail(BL_ENOMEM, "host allocation");
  dm->owner.assign(ba->boxes.size(), 0);
  dm->ba_uid = ba->uid;
  *out = dm;
  return BL_OK;
}

void bl_distmap_destroy(bl_distmap* dm) { delete dm; }

bl_status bl_static_partition(int32_t ntiles, int32_t nworkers, int32_t* first) {
  clear_error();
  if (ntiles < 0 || nworkers < 1 || !first) return fail(BL_EINVAL, "need ntiles >= 0, nworkers >= 1, first");
  int q = ntiles / nworkers, r = ntiles % nworkers;
  for (int w = 0; w <= nworkers; ++w) first[w] = w * q + std::min(w, r);
  return BL_OK;
}

}  // extern "C"

namespace bl {

// ---------------------------------------------------------------- copy plans
static void periodic_shifts(const bl_boxarray* ba, std::vector<std::array<int, 3>>& out) {
  out.clear();
  int n[3];
  for (int d = 0; d < 3; ++d) n[d] = ba->domain.len(d);
  for (int sz = -1; sz <= 1; ++sz)
    for (int sy = -1; sy <= 1; ++sy)
      for (int sx = -1; sx <= 1; ++sx) {
        int s[3] = {sx, sy, sz};
        bool ok = true;
        for (int d = 0; d < 3; ++d)
          if (s[d] != 0 && !ba->periodic[d]) ok = false;
        if (ok) out.push_back({sx * n[0], sy * n[1], sz * n[2]});
      }
}

static std::shared_ptr<std::vector<FillRecord>> compute_fill_plan(const bl_boxarray* ba, int ng) {
  auto plan = std::make_shared<std::vector<FillRecord>>();
  std::vector<std::array<int, 3>> shifts;
  periodic_shifts(ba, shifts);
  std::vector<int> cand;
  for (int b = 0; b < (int)ba->boxes.size(); ++b) {
    Box g = ba->boxes[b].grow(ng);
    for (auto& s : shifts) {
      Box gs = g.shift(s.data());
      ba->bins.query(gs, cand);
      for (int b2 : cand) {
        bool zero = s[0] == 0 && s[1] == 0 && s[2] == 0;
        if (zero && b2 == b) continue;
        Box I = Box::intersect(gs, ba->boxes[b2]);
        if (I.empty()) continue;
        int neg[3] = {-s[0], -s[1], -s[2]};
        FillRecord r;
        r.dst = b;
        r.src = b2;
        r.region = I.shift(neg);
        for (int d = 0; d < 3; ++d) r.shift[d] = s[d];
        plan->push_back(r);
      }
    }
  }
  return plan;
}

static std::shared_ptr<std::vector<FaceRecord>> compute_face_plan(const bl_boxarray* ba, int ng) {
  (void)ng;
  auto plan = std::make_shared<std::vector<FaceRecord>>();
  std::vector<std::array<int, 3>> shifts;
  periodic_shifts(ba, shifts);
  std::vector<int> cand;
  for (int b = 0; b < (int)ba->boxes.size(); ++b) {
    const Box& bx = ba->boxes[b];
    for (int face = 0; face < 6; ++face) {
      int a = face / 2, side = face % 2;
      Box layer = bx;
      layer.lo[a] = layer.hi[a] = side ? bx.hi[a] + 1 : bx.lo[a] - 1;
      size_t first = plan->size();
      for (auto& s : shifts) {
        Box ls = layer.shift(s.data());
        ba->bins.query(ls, cand);
        for (int b2 : cand) {
          Box I = Box::intersect(ls, ba->boxes[b2]);
          if (I.empty()) continue;
          int neg[3] = {-s[0], -s[1], -s[2]};
          FaceRecord r;
          r.box = b;
          r.face = face;
          r.src = b2;
          r.region = I.shift(neg);
          for (int d = 0; d < 3; ++d) r.shift[d] = s[d];
          plan->push_back(r);
        }
      }
      // the uncovered part of the layer reads the box's own ghost cells
      int t1 = a == 0 ? 1 : 0, t2 = a == 2 ? 1 : 2;
      std::vector<int> c1{layer.lo[t1], layer.hi[t1] + 1}, c2{layer.lo[t2], layer.hi[t2] + 1};
      for (size_t i = first; i < plan->size(); ++i) {
        const Box& R = (*plan)[i].region;
        c1.push_back(R.lo[t1]);
        c1.push_back(R.hi[t1] + 1);
        c2.push_back(R.lo[t2]);
        c2.push_back(R.hi[t2] + 1);
      }
      std::sort(c1.begin(), c1.end());
      c1.erase(std::unique(c1.begin(), c1.end()), c1.end());
      std::sort(c2.begin(), c2.end());
      c2.erase(std::unique(c2.begin(), c2.end()), c2.end());
      size_t covered_end = plan->size();
      for (size_t j = 0; j + 1 < c2.size(); ++j) {
        int run_lo = 0, run_on = 0;
        for (size_t i = 0; i + 1 < c1.size(); ++i) {
          bool cov = false;
          for (size_t r = first; r < covered_end && !cov; ++r) {
            const Box& R = (*plan)[r].region;
            cov = c1[i] >= R.lo[t1] && c1[i] <= R.hi[t1] && c2[j] >= R.lo[t2] && c2[j] <= R.hi[t2];
          }
          if (!cov && !run_on) {
            run_on = 1;
            run_lo = c1[i];
          }
          bool end_run = run_on && (cov || i + 2 == c1.size());
          if (end_run) {
            int run_hi = cov ? c1[i] - 1 : c1[i + 1] - 1;
            FaceRecord r;
            r.box = b;
            r.face = face;
            r.src = b;
            r.region = layer;
            r.region.lo[t1] = run_lo;
            r.region.hi[t1] = run_hi;
            r.region.lo[t2] = c2[j];
            r.region.hi[t2] = c2[j + 1] - 1;
            r.shift[0] = r.shift[1] = r.shift[2] = 0;
            plan->push_back(r);
            run_on = 0;
          }
        }
      }
    }
  }
  return plan;
}

std::shared_ptr<const std::vector<FillRecord>> fill_plan(bl_boxarray* ba, int ng) {
  std::lock_guard<std::mutex> lk(ba->mu);
  for (auto& e : ba->fill_plans)
    if (e.first == ng) return e.second;
  ba->fill_plans.push_back({ng, compute_fill_plan(ba, ng)});
  return ba->fill_plans.back().second;
}

std::shared_ptr<const std::vector<FaceRecord>> face_plan(bl_boxarray* ba, int ng) {
  std::lock_guard<std::mutex> lk(ba->mu);
  for (auto& e : ba->face_plans)
    if (e.first == ng) return e.second;
  ba->face_plans.push_back({ng, compute_face_plan(ba, ng)});
  return ba->face_plans.back().second;
}

// ---------------------------------------------------------------- layout, records, tiles
static int64_t round_up(int64_t a, int64_t m) { return (a + m - 1) / m * m; }

// Index of the face record of box B, face f, covering the tangential
// rectangle [a1, b1] x [a2, b2] (box-local) entirely, or kFaceMany.
static int32_t covering_record(const Plan& p, const DevBox& B, int f, int a1, int b1, int a2, int b2) {
  int32_t found = kFaceMany;
  for (int r = B.face_start[f]; r < B.face_start[f] + B.face_count[f]; ++r) {
    const DevFaceRec& R = p.hfacerecs[r];
    const bool overlap = !(b1 < R.t1lo || a1 > R.t1hi || b2 < R.t2lo || a2 > R.t2hi);
    if (!overlap) continue;
    const bool covers = a1 >= R.t1lo && b1 <= R.t1hi && a2 >= R.t2lo && b2 <= R.t2hi;
    if (!covers) return kFaceMany;
    found = r;
  }
  return found;
}

void build_tiles(const Plan& p, const TileConfig& cfg, int member, int box_base, int rec_base,
                 std::vector<DevTile>& tiles, std::vector<int>* box_tile_start) {
  const int lanes = 64 * cfg.waves;
  if (box_tile_start) box_tile_start->clear();
  std::vector<int> zc;
  for (int b = 0; b < (int)p.hboxes.size(); ++b) {
    const DevBox& B = p.hboxes[b];
    if (box_tile_start) box_tile_start->push_back((int)tiles.size());
    // z cuts: chunk boundaries and every z boundary of the x- and y-face records
    zc.clear();
    for (int z = 0; z < B.ez; z += cfg.zchunk) zc.push_back(z);
    zc.push_back(B.ez);
    for (int f = 0; f < 4; ++f)
      for (int r = B.face_start[f]; r < B.face_start[f] + B.face_count[f]; ++r) {
        zc.push_back(std::max(0, std::min<int>(B.ez, p.hfacerecs[r].t2lo)));
        zc.push_back(std::max(0, std::min<int>(B.ez, p.hfacerecs[r].t2hi + 1)));
      }
    std::sort(zc.begin(), zc.end());
    zc.erase(std::unique(zc.begin(), zc.end()), zc.end());
    const int nvt_full = std::min(B.nvx, lanes);
    const int rows_full = std::max(1, std::min(B.ey, lanes / nvt_full));
    // consecutive tiles cover consecutive memory: the row groups of one z range
    // come together, then the next z range
    for (int n = 0; n < p.ncomp; ++n)
      for (size_t k = 0; k + 1 < zc.size(); ++k)
        for (int xv0 = 0; xv0 < B.nvx; xv0 += nvt_full)
          for (int y0 = 0; y0 < B.ey; y0 += rows_full) {
            DevTile t;
            std::memset(&t, 0, sizeof t);
            t.box = box_base + b;
            t.member = member;
            t.comp = n;
            t.xv0 = xv0;
            t.nvt = std::min(nvt_full, B.nvx - xv0);
            t.y0 = y0;
            t.rows = std::min(rows_full, B.ey - y0);
            t.z0 = zc[k];
            t.z1 = zc[k + 1];
            const int x0 = xv0 * p.vec, x1 = (xv0 + t.nvt) * p.vec - 1;
            const int y1 = y0 + t.rows - 1, z1 = t.z1 - 1;
            const bool touch[6] = {xv0 == 0, xv0 + t.nvt == B.nvx, y0 == 0, y0 + t.rows == B.ey, t.z0 == 0,
                                   t.z1 == B.ez};
            const int rect[6][4] = {{y0, y1, t.z0, z1}, {y0, y1, t.z0, z1}, {x0, x1, t.z0, z1},
                                    {x0, x1, t.z0, z1}, {x0, x1, y0, y1},   {x0, x1, y0, y1}};
            for (int f = 0; f < 6; ++f) {
              t.frec[f] = kFaceNone;
              if (!touch[f]) continue;
              const int32_t r = covering_record(p, B, f, rect[f][0], rect[f][1], rect[f][2], rect[f][3]);
              t.frec[f] = r >= 0 ? r + rec_base : r;
            }
            tiles.push_back(t);
          }
  }
  if (box_tile_start) box_tile_start->push_back((int)tiles.size());
}

void build_h8_tiles(const Plan& p, std::vector<DevTile>& tiles, int* rmax, int* nvtmax) {
  tiles.clear();
  for (int b = 0; b < (int)p.hboxes.size(); ++b) {
    const DevBox& B = p.hboxes[b];
    const int nvt_full = std::min(B.nvx, 16);
    const int rows_full = std::max(1, std::min({B.ey, 32, 256 / nvt_full}));
    for (int n = 0; n < p.ncomp; ++n)
      for (int z0 = 0; z0 < B.ez; z0 += 32)
        for (int y0 = 0; y0 < B.ey; y0 += rows_full)
          for (int xv0 = 0; xv0 < B.nvx; xv0 += nvt_full) {
            DevTile t;
            std::memset(&t, 0, sizeof t);
            t.box = b;
            t.comp = n;
            t.xv0 = xv0;
            t.nvt = std::min(nvt_full, B.nvx - xv0);
            t.y0 = y0;
            t.rows = std::min(rows_full, B.ey - y0);
            t.z0 = z0;
            t.z1 = std::min(z0 + 32, B.ez);
            for (int f = 0; f < 6; ++f) t.frec[f] = kFaceNone;
            *rmax = std::max(*rmax, t.rows);
            *nvtmax = std::max(*nvtmax, t.nvt);
            tiles.push_back(t);
          }
  }
}

bool build_h8_segments(const Plan& p, std::vector<DevH8Seg>& segs, std::vector<DevH8Face>& faces, std::string* why,
                       std::vector<DevH8Seg>* msegs) {
  segs.clear();
  faces.clear();
  if (msegs) msegs->clear();
  if (p.ng < 4 || !p.fill) {
    *why = "nghost < 4";
    return false;
  }
  const int V = p.vec, nb = (int)p.hboxes.size();
  bool mir = msegs != nullptr;  // the mirror form: every box at least 8 cells wide in x
  for (const Box& b : p.boxes)
    if (b.len(0) < 8) mir = false;
  std::vector<std::vector<int>> byd(nb);
  for (int i = 0; i < (int)p.fill->size(); ++i) byd[(*p.fill)[i].dst].push_back(i);
  faces.resize(nb);
  for (int b = 0; b < nb; ++b) {
    const DevBox& B = p.hboxes[b];
    const Box& bx = p.boxes[b];
    const FabGeom& df = p.fabs[b];
    const int e[3] = {B.ex, B.ey, B.ez};
    for (int f = 0; f < 6; ++f) {
      const int a = f / 2, side = f % 2;
      const int u1 = a == 0 ? 1 : 0, u2 = a == 2 ? 1 : 2;  // tangential axes
      const int nlo = side ? e[a] : -4, nhi = side ? e[a] + 3 : -1;  // the face's 4 layers
      faces[b].start[f] = (int32_t)segs.size();
      std::vector<int> c1{0, e[u1]}, c2{0, e[u2]};
      std::vector<std::array<int, 4>> rects;  // covered (t1lo, t1hi, t2lo, t2hi)
      // checks segment g over (t1, t2) and appends it (with gm, the mirror
      // form's segment over the same cells, to the mirror form's list)
      auto check = [&](DevH8Seg& g, int t1lo, int t1hi, int t2lo, int t2hi) -> bool {
        g.t1lo = t1lo;
        g.t1hi = t1hi;
        g.t2lo = t2lo;
        g.t2hi = t2hi;
        if (g.sz > INT32_MAX || g.sy > INT32_MAX) {  // the kernel keeps plane strides in 32 bits
          *why = "a plane stride exceeds 32 bits";
          return false;
        }
        if (V > 1 && a > 0) {  // y and z faces: a lane's vector of x cells lies in one segment
          if (t1lo % V || (t1hi + 1) % V || g.o % V || g.sc % V || g.sy % V || g.sz % V) {
            *why = "a y- or z-face segment is not vector-aligned";
            return false;
          }
        }
        for (int c = 0; c < 16; ++c) {  // the affine address is extreme at the corners
          int q[3];
          q[a] = c & 1 ? nhi : nlo;
          q[u1] = c & 2 ? t1hi : t1lo;
          q[u2] = c & 4 ? t2hi : t2lo;
          const int64_t n = c & 8 ? p.ncomp - 1 : 0;
          const int len = a > 0 ? V : 1;
          if (a > 0 && (c & 2)) q[0] = t1hi - V + 1;  // vectors start at multiples of V
          const int64_t at = g.o + n * g.sc + (int64_t)q[0] * g.sx + (int64_t)q[1] * g.sy + (int64_t)q[2] * g.sz;
          if (at < 0 || at + len > (int64_t)p.total_elems) {
            *why = "internal error: a segment address leaves the MultiFab";
            return false;
          }
        }
        return true;
      };
      auto add = [&](DevH8Seg g, DevH8Seg gm, int t1lo, int t1hi, int t2lo, int t2hi) -> bool {
        if (!check(g, t1lo, t1hi, t2lo, t2hi)) return false;
        segs.push_back(g);
        if (mir) {
          if (!check(gm, t1lo, t1hi, t2lo, t2hi)) return false;
          msegs->push_back(gm);
        }
        return true;
      };
      for (int ri : byd[b]) {
        const FillRecord& r = (*p.fill)[ri];
        int lo[3], hi[3];
        bool meets = true;
        for (int d = 0; d < 3; ++d) {
          lo[d] = r.region.lo[d] - bx.lo[d];
          hi[d] = r.region.hi[d] - bx.lo[d];
          const int slo = d == a ? nlo : 0, shi = d == a ? nhi : e[d] - 1;
          lo[d] = std::max(lo[d], slo);
          hi[d] = std::min(hi[d], shi);
          if (lo[d] > hi[d]) meets = false;
        }
        if (!meets) continue;
        if (lo[a] != nlo || hi[a] != nhi) {
          *why = "a neighbour is thinner than the 4 ghost layers across a face";
          return false;
        }
        const FabGeom& sf = p.fabs[r.src];
        DevH8Seg g;
        std::memset(&g, 0, sizeof g);
        g.o = sf.off + (int64_t)(bx.lo[0] + r.shift[0] - sf.valid.lo[0]) +
              (int64_t)(bx.lo[1] + r.shift[1] - sf.valid.lo[1]) * sf.sy +
              (int64_t)(bx.lo[2] + r.shift[2] - sf.valid.lo[2]) * sf.sz;
        g.sc = sf.sc;
        g.sx = 1;
        g.sy = (int32_t)sf.sy;
        g.sz = sf.sz;
        DevH8Seg gm = g;
        if (mir && a == 0) {
          // source column cx = X0 + x of the neighbour (ex_s wide), a copy of
          // which is mirror layer cx on its side 0 (high face: cx = 0..3) or
          // ex_s-1-cx on its side 1 (low face); rows j = Y0 + y, planes k = Z0 + z
          const Box& sb = p.boxes[r.src];
          const int64_t exs = sb.len(0), eys = sb.len(1), L = eys * sb.len(2);
          const int64_t X0 = bx.lo[0] + r.shift[0] - sf.valid.lo[0];
          const int64_t Y0 = bx.lo[1] + r.shift[1] - sf.valid.lo[1], Z0 = bx.lo[2] + r.shift[2] - sf.valid.lo[2];
          const int64_t c0 = X0 + nlo, c1 = X0 + nhi;  // the source columns of the face's layers
          const bool ok = side ? (c0 == 0 && c1 == 3) : (c0 == exs - 4 && c1 == exs - 1);
          if (!ok || sf.mir_layers != 4 || L > INT32_MAX) {
            *why = "internal error: an x face's neighbour columns are not its mirror layers";
            return false;
          }
          gm.sy = 1;
          gm.sz = eys;
          if (side) {  // layer = X0 + x on side 0
            gm.o = sf.mir + X0 * L + Y0 + Z0 * eys;
            gm.sx = (int32_t)L;
          } else {     // layer = exs - 1 - X0 - x on side 1
            gm.o = sf.mir + sf.mir_side + (exs - 1 - X0) * L + Y0 + Z0 * eys;
            gm.sx = (int32_t)-L;
          }
        }
        if (!add(g, gm, lo[u1], hi[u1], lo[u2], hi[u2])) return false;
        rects.push_back({lo[u1], hi[u1], lo[u2], hi[u2]});
        c1.push_back(lo[u1]);
        c1.push_back(hi[u1] + 1);
        c2.push_back(lo[u2]);
        c2.push_back(hi[u2] + 1);
      }
      // the parts of the face no box covers: the box's own ghost cells
      std::sort(c1.begin(), c1.end());
      c1.erase(std::unique(c1.begin(), c1.end()), c1.end());
      std::sort(c2.begin(), c2.end());
      c2.erase(std::unique(c2.begin(), c2.end()), c2.end());
      DevH8Seg own;
      std::memset(&own, 0, sizeof own);
      own.sc = df.sc;
      if (a == 0) {  // x ghost slab: layer -1-x (low side) or x-ex (high side)
        own.o = side ? df.xs + df.xs_side - B.ex : df.xs - 1;
        own.sx = side ? 1 : -1;
        own.sy = (int32_t)df.ng;
        own.sz = df.xs_z;
      } else {       // rows of the grown box
        own.o = df.off;
        own.sx = 1;
        own.sy = (int32_t)df.sy;
        own.sz = df.sz;
      }
      for (size_t i1 = 0; i1 + 1 < c1.size(); ++i1)
        for (size_t i2 = 0; i2 + 1 < c2.size(); ++i2) {
          const int t1 = c1[i1], t2 = c2[i2];
          bool covered = false;
          for (const auto& R : rects)
            if (t1 >= R[0] && t1 <= R[1] && t2 >= R[2] && t2 <= R[3]) covered = true;
          if (!covered && !add(own, own, c1[i1], c1[i1 + 1] - 1, c2[i2], c2[i2 + 1] - 1)) return false;
        }
      faces[b].count[f] = (int32_t)segs.size() - faces[b].start[f];
    }
  }
  return true;
}

size_t lin_lds_bytes(const TileConfig& cfg, int esize, int vec, int yhmax, int xhmax) {
  const size_t zb = (size_t)cfg.zchunk, vb = (size_t)esize * vec;
  return zb * 64 * cfg.waves * vb + zb * 2 * yhmax * vb + zb * 2 * xhmax * esize;
}

// The linear tiles of p with at most zsteps z steps of at most nzs_cap z blocks each.
static void lin_tiles_pass(const Plan& p, const TileConfig& cfg, int zsteps, int nzs_cap, int member, int box_base,
                           int rec_base, std::vector<DevLinTile>& tiles, int* yhmax, int* xhmax) {
  const int lanes = 64 * cfg.waves;
  const int zb = std::max(1, cfg.zchunk);
  std::vector<int> zc;
  for (int b = 0; b < (int)p.hboxes.size(); ++b) {
    const DevBox& B = p.hboxes[b];
    const int nvx = B.nvx, P = B.ey * nvx;
    int nq, nzs, ntq;
    if (P >= lanes) {  // the plane split into ntq near-equal runs of at most `lanes` vectors
      ntq = (P + lanes - 1) / lanes;
      nq = (P + ntq - 1) / ntq;
      nzs = 1;
    } else {           // whole planes, as many z blocks as fill the workgroup
      ntq = 1;
      nq = P;
      nzs = std::max(1, std::min({lanes / P, (B.ez + zb - 1) / zb, nzs_cap}));
    }
    const int zlen = zb * nzs * std::max(1, zsteps);
    // z cuts: multiples of zlen and every z boundary of the x- and y-face records
    zc.clear();
    for (int z = 0; z < B.ez; z += zlen) zc.push_back(z);
    zc.push_back(B.ez);
    for (int f = 0; f < 4; ++f)
      for (int r = B.face_start[f]; r < B.face_start[f] + B.face_count[f]; ++r) {
        zc.push_back(std::max(0, std::min<int>(B.ez, p.hfacerecs[r].t2lo)));
        zc.push_back(std::max(0, std::min<int>(B.ez, p.hfacerecs[r].t2hi + 1)));
      }
    std::sort(zc.begin(), zc.end());
    zc.erase(std::unique(zc.begin(), zc.end()), zc.end());
    for (int n = 0; n < p.ncomp; ++n)
      for (size_t k = 0; k + 1 < zc.size(); ++k)
        for (int tq = 0; tq < ntq; ++tq) {
          DevLinTile t;
          std::memset(&t, 0, sizeof t);
          t.box = box_base + b;
          t.member = member;
          t.comp = n;
          t.q0 = tq * nq;
          t.nq = std::min(nq, P - t.q0);
          t.z0 = zc[k];
          t.z1 = zc[k + 1];
          t.nzs = std::min(nzs, (t.z1 - t.z0 + zb - 1) / zb);
          t.y_first = t.q0 / nvx;
          const int y_last = (t.q0 + t.nq - 1) / nvx;
          t.nrows = y_last - t.y_first + 1;
          const int x1 = B.ex - 1, z1 = t.z1 - 1;
          const bool touch[6] = {true, true, t.q0 < nvx, t.q0 + t.nq > P - nvx, t.z0 == 0, t.z1 == B.ez};
          const int rect[6][4] = {{t.y_first, y_last, t.z0, z1}, {t.y_first, y_last, t.z0, z1}, {0, x1, t.z0, z1},
                                  {0, x1, t.z0, z1},              {0, x1, t.y_first, y_last},   {0, x1, t.y_first, y_last}};
          for (int f = 0; f < 6; ++f) {
            t.frec[f] = kFaceNone;
            if (!touch[f]) continue;
            const int32_t r = covering_record(p, B, f, rect[f][0], rect[f][1], rect[f][2], rect[f][3]);
            t.frec[f] = r >= 0 ? r + rec_base : r;
          }
          if (yhmax) *yhmax = std::max(*yhmax, t.nzs * std::min(nvx, t.nq));
          if (xhmax) *xhmax = std::max(*xhmax, t.nzs * t.nrows);
          tiles.push_back(t);
        }
  }
}

void build_lin_tiles(const Plan& p, const TileConfig& cfg, int member, int box_base, int rec_base,
                     std::vector<DevLinTile>& tiles, int* yhmax, int* xhmax) {
  // A small level (few cells per box or few boxes) is latency-bound: a launch
  // takes about as long as its workgroups' chains of z steps.  Where the
  // configured shape gives fewer than kLatencyTiles tiles, one z step per tile,
  // then one z block per step, give more and shorter workgroups.
  const size_t first = tiles.size();
  const int yh0 = yhmax ? *yhmax : 0, xh0 = xhmax ? *xhmax : 0;
  const int zs[3] = {std::max(1, cfg.zsteps), 1, 1}, cap[3] = {1 << 30, 1 << 30, 1};
  for (int k = 0; k < 3; ++k) {
    if (k > 0 && zs[k] == zs[k - 1] && cap[k] == cap[k - 1]) continue;
    tiles.resize(first);
    if (yhmax) *yhmax = yh0;
    if (xhmax) *xhmax = xh0;
    lin_tiles_pass(p, cfg, zs[k], cap[k], member, box_base, rec_base, tiles, yhmax, xhmax);
    if (tiles.size() - first >= kLatencyTiles) break;
  }
}

// Layout of one FAB whose first element is `fab` (a multiple of A elements,
// A = 128 bytes / element size).  Returns its size in elements.
static int64_t layout_fab(const Box& b, int ng, int ncomp, int64_t A, int64_t fab, FabGeom& f) {
  const int64_t ex = b.len(0), ey = b.len(1), ez = b.len(2);
  const int64_t nyg = ey + 2 * ng, nzg = ez + 2 * ng;
  // rows of one plane are contiguous (pitch = x extent); planes start on
  // 128-byte boundaries, so a run of whole rows is one contiguous span
  const int64_t px = ex;
  const int64_t plane = round_up(nyg * px, A);
  const int64_t rows = nzg * plane;
  const int64_t slab = round_up(2 * nzg * nyg * ng, A);
  const int64_t layers = ng >= 4 ? 4 : 1;
  const int64_t mirror = round_up(2 * layers * ez * ey, A);
  f.valid = b;
  f.grown = b.grow(ng);
  f.ng = ng;
  f.fab = fab;
  f.sy = px;
  f.sz = plane;
  f.sc = rows + slab + mirror;
  f.off = fab + ng * f.sz + ng * f.sy;
  f.xs_side = nzg * nyg * ng;
  f.xs_z = nyg * ng;
  f.xs = fab + rows + ng * f.xs_z + (int64_t)ng * ng;
  f.mir_side = layers * ez * ey;
  f.mir_layers = (int)layers;
  f.mir = fab + rows + slab;
  return f.sc * ncomp;
}

static int64_t elem_align(int esize) { return 128 / esize; }

bl_status build_plan(const bl_boxarray* cba, int ncomp, int ng, int dtype, const TileConfig& cfg,
                     std::shared_ptr<Plan>* out) {
  bl_boxarray* ba = const_cast<bl_boxarray*>(cba);
  auto p = std::make_shared<Plan>();
  p->ba_uid = ba->uid;
  p->boxes = ba->boxes;
  p->domain = ba->domain;
  for (int d = 0; d < 3; ++d) p->periodic[d] = ba->periodic[d];
  p->ncomp = ncomp;
  p->ng = ng;
  p->dtype = dtype;
  p->esize = dtype == BL_F64 ? 8 : 4;
  const int v16 = 16 / p->esize;
  bool all_div = true;
  for (const Box& b : ba->boxes) {
    if (b.len(0) % v16) all_div = false;
    for (int d = 0; d < 3; ++d)
      if (b.len(d) > 16384) return fail(BL_EINVAL, "box edge %d above 16384", b.len(d));
  }
  p->vec = all_div ? v16 : 1;
  const int64_t A = elem_align(p->esize);
  int64_t off = 0;
  p->fabs.resize(ba->boxes.size());
  for (size_t i = 0; i < ba->boxes.size(); ++i) {
    const int64_t size = layout_fab(ba->boxes[i], ng, ncomp, A, off, p->fabs[i]);
    if (size >= ((int64_t)1 << 31))
      return fail(BL_EINVAL, "box %zu is too large for one FAB (%lld elements)", i, (long long)size);
    off = round_up(off + size, A);
  }
  p->total_elems = (size_t)off;

  // per-box descriptors
  p->hboxes.resize(ba->boxes.size());
  for (size_t i = 0; i < ba->boxes.size(); ++i) {
    const Box& b = ba->boxes[i];
    const FabGeom& f = p->fabs[i];
    DevBox& B = p->hboxes[i];
    std::memset(&B, 0, sizeof B);
    B.off = f.off;
    B.sc = f.sc;
    B.xs = f.xs;
    B.mir = f.mir;
    B.sy = (int32_t)f.sy;
    B.sz = (int32_t)f.sz;
    B.xs_side = (int32_t)f.xs_side;
    B.xs_z = (int32_t)f.xs_z;
    B.mir_side = (int32_t)f.mir_side;
    B.ex = b.len(0);
    B.ey = b.len(1);
    B.ez = b.len(2);
    B.nvx = B.ex / p->vec;
    B.ng = ng;
    for (int d = 0; d < 3; ++d) B.glo[d] = b.lo[d];
  }

  // Face records (fused stencil), grouped by (box, face) in order.  The value
  // next to tangential coordinates (t1, t2) of a face is read at
  // base + t1*s1 + t2*s2 (+ comp*sc): for a covered x face from the source
  // box's mirror of its edge column, for a covered y or z face from the
  // source's valid rows, for an uncovered part from the box's own ghost cells.
  const auto face_ptr = face_plan(ba, ng);
  const auto& faces = *face_ptr;
  p->hfacerecs.clear();
  p->hfacerecs_rows.clear();
  size_t k = 0;
  for (size_t i = 0; i < ba->boxes.size(); ++i) {
    const Box& bx = ba->boxes[i];
    for (int face = 0; face < 6; ++face) {
      DevBox& B = p->hboxes[i];
      B.face_start[face] = (int32_t)p->hfacerecs.size();
      int cnt = 0;
      while (k < faces.size() && faces[k].box == (int)i && faces[k].face == face) {
        const FaceRecord& r = faces[k++];
        const int a = face / 2, side = face % 2;
        const int t1 = a == 0 ? 1 : 0, t2 = a == 2 ? 1 : 2;
        const bool uncovered = r.src == (int)i && r.shift[0] == 0 && r.shift[1] == 0 && r.shift[2] == 0;
        const FabGeom& sf = p->fabs[r.src];
        const Box& sb = ba->boxes[r.src];
        // ghost-layer cell at the record's low tangential corner
        int q[3];
        for (int d = 0; d < 3; ++d) q[d] = r.region.lo[d];
        const int lo1 = r.region.lo[t1] - bx.lo[t1], lo2 = r.region.lo[t2] - bx.lo[t2];
        int64_t addr, s1, s2;
        if (uncovered) {
          const FabGeom& f = p->fabs[i];
          addr = f.index(q[0], q[1], q[2]);
          if (a == 0) {
            s1 = f.ng;    // along y in the x slab
            s2 = f.xs_z;  // along z
          } else {
            s1 = 1;
            s2 = a == 1 ? f.sz : f.sy;
          }
        } else if (a == 0) {
          // source cell: the source's last (for our low face) or first x column
          const int sside = side ? 0 : 1;
          const int j = q[1] + r.shift[1] - sb.lo[1], kk = q[2] + r.shift[2] - sb.lo[2];
          addr = sf.mir + sside * sf.mir_side + (int64_t)kk * sb.len(1) + j;
          s1 = 1;
          s2 = sb.len(1);
        } else {
          addr = sf.index(q[0] + r.shift[0], q[1] + r.shift[1], q[2] + r.shift[2]);
          s1 = 1;
          s2 = a == 1 ? sf.sz : sf.sy;
        }
        DevFaceRec R;
        R.base = addr - lo1 * s1 - lo2 * s2;
        R.sc = sf.sc;
        R.s1 = (int32_t)s1;
        R.s2 = (int32_t)s2;
        R.t1lo = (int16_t)lo1;
        R.t1hi = (int16_t)(r.region.hi[t1] - bx.lo[t1]);
        R.t2lo = (int16_t)lo2;
        R.t2hi = (int16_t)(r.region.hi[t2] - bx.lo[t2]);
        if (a >= 1 && p->vec > 1 &&
            (((R.base % p->vec) + p->vec) % p->vec != 0 || R.t1lo % p->vec != 0 || (R.t1hi + 1) % p->vec != 0))
          p->fvec = 0;
        p->hfacerecs.push_back(R);
        if (a == 0 && !uncovered) {  // the source's edge column in its own rows
          const int64_t ra = sf.index(q[0] + r.shift[0], q[1] + r.shift[1], q[2] + r.shift[2]);
          R.base = ra - lo1 * sf.sy - lo2 * sf.sz;
          R.s1 = (int32_t)sf.sy;
          R.s2 = (int32_t)sf.sz;
        }
        p->hfacerecs_rows.push_back(R);
        ++cnt;
      }
      if (cnt > 32767) return fail(BL_EINVAL, "too many neighbours on one face of box %zu", i);
      B.face_count[face] = (int16_t)cnt;
    }
  }

  // One-pass red-black sweep: every covered part of a face ghost layer, with
  // the offset from destination to source box-local cells, chunked; and the
  // offsets of each box's second edge-column copy.
  p->hringrecs.clear();
  p->hpushrecs.clear();
  p->hpushface.assign(ba->boxes.size(), DevPushFace{});
  p->faces_covered = true;
  // push records, per (source box, source face)
  std::vector<std::vector<DevPushRec>> push(6 * ba->boxes.size());
  for (const FaceRecord& r : faces) {
    const bool uncovered = r.src == r.box && r.shift[0] == 0 && r.shift[1] == 0 && r.shift[2] == 0;
    if (uncovered) {
      p->faces_covered = false;
      continue;
    }
    const Box& db = ba->boxes[r.box];
    const Box& sb = ba->boxes[r.src];
    const int a = r.face / 2;
    const int t1 = a == 0 ? 1 : 0, t2 = a == 2 ? 1 : 2;
    DevRingRec R{};
    R.box = r.box;
    R.src = r.src;
    R.face = r.face;
    for (int d = 0; d < 3; ++d) {
      R.lo[d] = r.region.lo[d] - db.lo[d];
      R.d[d] = db.lo[d] + r.shift[d] - sb.lo[d];
    }
    R.n1 = r.region.len(t1);
    R.n2 = r.region.len(t2);
    p->hringrecs.push_back(R);
    // the same part seen from the source: its face cells (the face opposite to
    // the destination's) and the destination ghost cells they fill
    const FabGeom& df = p->fabs[r.box];
    DevPushRec Q{};
    Q.t1lo = r.region.lo[t1] + r.shift[t1] - sb.lo[t1];
    Q.t1hi = r.region.hi[t1] + r.shift[t1] - sb.lo[t1];
    Q.t2lo = r.region.lo[t2] + r.shift[t2] - sb.lo[t2];
    Q.t2hi = r.region.hi[t2] + r.shift[t2] - sb.lo[t2];
    int64_t s1, s2;
    if (a == 0) {
      s1 = df.ng;
      s2 = df.xs_z;
    } else {
      s1 = 1;
      s2 = a == 1 ? df.sz : df.sy;
    }
    Q.s1 = (int32_t)s1;
    Q.s2 = (int32_t)s2;
    Q.base = df.index(r.region.lo[0], r.region.lo[1], r.region.lo[2]) - Q.t1lo * s1 - Q.t2lo * s2;
    const int sface = 2 * a + (1 - r.face % 2);
    push[6 * (size_t)r.src + sface].push_back(Q);
  }
  // few faces (a level of few boxes): each ring record split along t2 into
  // near-equal parts of at least 4 rows, so the ring launch has about
  // kRingRecs workgroups instead of one per face
  if (!p->hringrecs.empty() && p->hringrecs.size() < kRingRecs) {
    const int parts = (int)((kRingRecs + p->hringrecs.size() - 1) / p->hringrecs.size());
    std::vector<DevRingRec> split;
    for (const DevRingRec& R : p->hringrecs) {
      const int t2 = R.face / 2 == 2 ? 1 : 2;
      const int k = std::max(1, std::min(parts, R.n2 / 4));
      for (int q = 0; q < k; ++q) {
        const int a0 = (int)((int64_t)R.n2 * q / k), a1 = (int)((int64_t)R.n2 * (q + 1) / k);
        DevRingRec P = R;
        P.lo[t2] = R.lo[t2] + a0;
        P.n2 = a1 - a0;
        split.push_back(P);
      }
    }
    p->hringrecs.swap(split);
  }
  for (size_t i = 0; i < ba->boxes.size(); ++i)
    for (int f = 0; f < 6; ++f) {
      auto& v = push[6 * i + f];
      p->hpushface[i].start[f] = (int32_t)p->hpushrecs.size();
      p->hpushface[i].count[f] = (int32_t)v.size();
      p->hpushrecs.insert(p->hpushrecs.end(), v.begin(), v.end());
    }
  p->hmir2off.assign(ba->boxes.size(), 0);
  p->mir2_total = 0;
  for (size_t i = 0; i < ba->boxes.size(); ++i) {
    p->hmir2off[i] = p->mir2_total;
    p->mir2_total += 2 * (int64_t)ba->boxes[i].len(1) * ba->boxes[i].len(2);
  }

  // FillBoundary records: each plan region split by the destination's
  // storage class along x (low x slab, rows, high x slab), chunked.
  p->fill = fill_plan(ba, ng);
  p->hfillrecs.clear();
  p->hfillrecs_mir.clear();
  p->hfillchunks.clear();
  for (const FillRecord& r : *p->fill) {
    const Box& db = ba->boxes[r.dst];
    const FabGeom& df = p->fabs[r.dst];
    const FabGeom& sf = p->fabs[r.src];
    const int xs[3][2] = {{r.region.lo[0], std::min(r.region.hi[0], db.lo[0] - 1)},
                          {std::max(r.region.lo[0], db.lo[0]), std::min(r.region.hi[0], db.hi[0])},
                          {std::max(r.region.lo[0], db.hi[0] + 1), r.region.hi[0]}};
    for (int part = 0; part < 3; ++part) {
      if (xs[part][0] > xs[part][1]) continue;
      Box R0 = r.region;
      R0.lo[0] = xs[part][0];
      R0.hi[0] = xs[part][1];
      DevFillRec R;
      std::memset(&R, 0, sizeof R);
      const int *lo = R0.lo, *sh = r.shift;
      R.dst_base = df.index(lo[0], lo[1], lo[2]);
      R.dsx = R0.len(0) > 1 ? (int32_t)(df.index(lo[0] + 1, lo[1], lo[2]) - R.dst_base) : 0;
      R.dsy = R0.len(1) > 1 ? (int32_t)(df.index(lo[0], lo[1] + 1, lo[2]) - R.dst_base) : 0;
      R.dsz = R0.len(2) > 1 ? (int32_t)(df.index(lo[0], lo[1], lo[2] + 1) - R.dst_base) : 0;
      R.src_base = sf.index(lo[0] + sh[0], lo[1] + sh[1], lo[2] + sh[2]);
      R.ssx = 1;
      R.ssy = (int32_t)sf.sy;
      R.ssz = (int32_t)sf.sz;
      R.dsc = df.sc;
      R.ssc = sf.sc;
      R.nx = R0.len(0);
      R.ny = R0.len(1);
      R.nz = R0.len(2);
      const int rid = (int)p->hfillrecs.size();
      p->hfillrecs.push_back(R);
      // one source column at the source box's low or high x face: its edge mirror
      const Box& sb = ba->boxes[r.src];
      const int sx = lo[0] + sh[0];
      if (R.nx == 1 && (sx == sb.lo[0] || sx == sb.hi[0])) {
        const int side = sx == sb.lo[0] ? 0 : 1;  // a one-cell-wide source box: its low-side copy
        R.src_base = sf.mir + (int64_t)side * sf.mir_side + (int64_t)(lo[2] + sh[2] - sb.lo[2]) * sb.len(1) +
                     (lo[1] + sh[1] - sb.lo[1]);
        R.ssx = 0;
        R.ssy = 1;
        R.ssz = sb.len(1);
      }
      p->hfillrecs_mir.push_back(R);
      const int64_t vol = R0.volume();
      for (int64_t c0 = 0; c0 < vol; c0 += kFillChunk) p->hfillchunks.push_back(DevFillChunk{rid, (int32_t)c0});
    }
  }

  p->cfg = cfg;
  build_tiles(*p, p->cfg, 0, 0, 0, p->htiles, &p->box_tile_start);
  for (const DevTile& t : p->htiles) {
    p->rmax = std::max<int>(p->rmax, t.rows);
    p->nvtmax = std::max<int>(p->nvtmax, t.nvt);
  }
  // flattened cell and x-pair counts (grid transfers between multigrid levels)
  {
    int64_t nc = 0, np2 = 0;
    p->hcellpre.assign(1, 0);
    p->hpairpre.assign(1, 0);
    for (const DevBox& B : p->hboxes) {
      nc += (int64_t)B.ex * B.ey * B.ez;
      np2 += (int64_t)(B.ex / 2) * B.ey * B.ez;
      if (nc > INT32_MAX) {  // too large for the grid transfers, which then refuse this shape
        p->hcellpre.clear();
        p->hpairpre.clear();
        break;
      }
      p->hcellpre.push_back((int32_t)nc);
      p->hpairpre.push_back((int32_t)np2);
    }
    // the box holding the first item of each workgroup
    auto first_boxes = [](const std::vector<int32_t>& pre, int per, std::vector<int32_t>& out) {
      out.clear();
      if (pre.empty()) return;
      size_t b = 0;
      for (int64_t g = 0; g < pre.back(); g += per) {
        while (pre[b + 1] <= g) ++b;
        out.push_back((int32_t)b);
      }
    };
    first_boxes(p->hcellpre, kRestrictPerWG, p->hcellwg);
    first_boxes(p->hpairpre, kProlongPerWG, p->hpairwg);
  }
  // reduction chunks of about 32K values
  for (int b = 0; b < (int)p->hboxes.size(); ++b) {
    const DevBox& B = p->hboxes[b];
    const int64_t P = (int64_t)B.ex * B.ey;
    const int per = (int)std::max<int64_t>(1, std::min<int64_t>(B.ez, (32768 + P - 1) / P));
    for (int z = 0; z < B.ez; z += per) p->hred.push_back(DevRedChunk{b, z, std::min(B.ez, z + per), 0});
  }
  if (cfg.block == 3) {
    build_lin_tiles(*p, cfg, 0, 0, 0, p->hlin, &p->yhmax, &p->xhmax);
    if (lin_lds_bytes(cfg, p->esize, p->vec, p->yhmax, p->xhmax) > kDmaLdsMax) p->hlin.clear();  // form 2 instead
  }
  *out = p;
  return BL_OK;
}

}  // namespace bl

extern "C" {

static bl_status host_plan(const bl_boxarray* ba, int32_t ncomp, int32_t nghost, int32_t dtype,
                           std::shared_ptr<Plan>* out) {
  if (!ba) return fail(BL_EINVAL, "NULL BoxArray");
  if (dtype != BL_F64 && dtype != BL_F32) return fail(BL_EDTYPE, "unknown dtype %d", (int)dtype);
  if (ncomp < 1 || nghost < 0) return fail(BL_EINVAL, "ncomp %d, nghost %d", (int)ncomp, (int)nghost);
  return build_plan(ba, ncomp, nghost, dtype, tile_config(), out);
}

bl_status bl_heat8_fused_layout(const bl_boxarray* ba, int32_t ncomp, int32_t nghost, int32_t dtype,
                                int32_t from_mirror, int32_t* nsegs, int64_t* segs, int64_t* total_elems) {
  clear_error();
  if (!nsegs) return fail(BL_EINVAL, "NULL argument");
  std::shared_ptr<Plan> p;
  bl_status st = host_plan(ba, ncomp, nghost, dtype, &p);
  if (st != BL_OK) return st;
  std::vector<DevH8Seg> rv, mv;
  std::vector<DevH8Face> fv;
  std::string why;
  if (!build_h8_segments(*p, rv, fv, &why, &mv)) return fail(BL_EINVAL, "%s", why.c_str());
  if (from_mirror && mv.empty()) return fail(BL_EINVAL, "a box is narrower than 8 cells in x: no 4-layer mirror form");
  const std::vector<DevH8Seg>& sv = from_mirror ? mv : rv;
  *nsegs = (int32_t)sv.size();
  if (total_elems) *total_elems = (int64_t)p->total_elems;
  if (segs)
    for (size_t b = 0; b < fv.size(); ++b)
      for (int f = 0; f < 6; ++f)
        for (int i = fv[b].start[f]; i < fv[b].start[f] + fv[b].count[f]; ++i) {
          const DevH8Seg& g = sv[i];
          const int64_t row[12] = {(int64_t)b, f, g.t1lo, g.t1hi, g.t2lo, g.t2hi, g.o, g.sc, g.sx, g.sy, g.sz, p->vec};
          std::memcpy(segs + 12 * (int64_t)i, row, sizeof row);
        }
  return BL_OK;
}

bl_status bl_layout_index(const bl_boxarray* ba, int32_t ncomp, int32_t nghost, int32_t dtype, int32_t box,
                          const int32_t cell[3], int32_t comp, int64_t* index) {
  clear_error();
  if (!cell || !index) return fail(BL_EINVAL, "NULL argument");
  std::shared_ptr<Plan> p;
  bl_status st = host_plan(ba, ncomp, nghost, dtype, &p);
  if (st != BL_OK) return st;
  if (box < 0 || box >= (int32_t)p->fabs.size()) return fail(BL_EINVAL, "box %d out of range", (int)box);
  if (comp < 0 || comp >= ncomp) return fail(BL_EINVAL, "component %d out of range", (int)comp);
  const FabGeom& g = p->fabs[box];
  for (int d = 0; d < 3; ++d)
    if (cell[d] < g.grown.lo[d] || cell[d] > g.grown.hi[d])
      return fail(BL_EINVAL, "cell outside box %d's grown box", (int)box);
  *index = g.index(cell[0], cell[1], cell[2]) + (int64_t)comp * g.sc;
  return BL_OK;
}

bl_status bl_layout_mirror_index(const bl_boxarray* ba, int32_t ncomp, int32_t nghost, int32_t dtype, int32_t box,
                                 int32_t side, int32_t layer, int32_t j, int32_t k, int32_t comp, int64_t* index) {
  clear_error();
  if (!index) return fail(BL_EINVAL, "NULL argument");
  std::shared_ptr<Plan> p;
  bl_status st = host_plan(ba, ncomp, nghost, dtype, &p);
  if (st != BL_OK) return st;
  if (box < 0 || box >= (int32_t)p->fabs.size()) return fail(BL_EINVAL, "box %d out of range", (int)box);
  if (comp < 0 || comp >= ncomp) return fail(BL_EINVAL, "component %d out of range", (int)comp);
  const FabGeom& g = p->fabs[box];
  if (side < 0 || side > 1 || layer < 0 || layer >= g.mir_layers)
    return fail(BL_EINVAL, "side %d layer %d: the mirror has 2 sides of %d layers", (int)side, (int)layer, g.mir_layers);
  const Box& b = g.valid;
  if (j < b.lo[1] || j > b.hi[1] || k < b.lo[2] || k > b.hi[2]) return fail(BL_EINVAL, "row outside box %d", (int)box);
  const int64_t ey = b.len(1), ez = b.len(2);
  *index = g.mir + side * g.mir_side + layer * ey * ez + (int64_t)(k - b.lo[2]) * ey + (j - b.lo[1]) +
           (int64_t)comp * g.sc;
  return BL_OK;
}

bl_status bl_tile_boxes(const bl_boxarray* ba, const int32_t tile_size[3], bl_tile_kind kind, int32_t arg,
                        int32_t* ntiles, int32_t* out) {
  clear_error();
  if (!ba || !tile_size || !ntiles) return fail(BL_EINVAL, "NULL argument");
  for (int d = 0; d < 3; ++d)
    if (tile_size[d] < 1) return fail(BL_EINVAL, "tile_size[%d] = %d < 1", d, tile_size[d]);
  if (kind == BL_TILE_NODAL && (arg < 0 || arg > 2)) return fail(BL_EINVAL, "nodal direction %d not in 0..2", arg);
  if (kind == BL_TILE_GROWN && arg < 0) return fail(BL_EINVAL, "grow width %d < 0", arg);
  if (kind != BL_TILE_CELL && kind != BL_TILE_NODAL && kind != BL_TILE_GROWN)
    return fail(BL_EINVAL, "unknown tile kind %d", (int)kind);
  int64_t n = 0;
  for (size_t b = 0; b < ba->boxes.size(); ++b) {
    const Box& B = ba->boxes[b];
    int cnt[3];
    for (int d = 0; d < 3; ++d) cnt[d] = (B.len(d) + tile_size[d] - 1) / tile_size[d];
    for (int tz = 0; tz < cnt[2]; ++tz)
      for (int ty = 0; ty < cnt[1]; ++ty)
        for (int tx = 0; tx < cnt[0]; ++tx, ++n) {
          if (!out) continue;
          const int t[3] = {tx, ty, tz};
          int32_t* r = out + 7 * n;
          r[0] = (int32_t)b;
          for (int d = 0; d < 3; ++d) {
            int lo = B.lo[d] + t[d] * tile_size[d];
            int hi = std::min(B.hi[d], lo + tile_size[d] - 1);
            if (kind == BL_TILE_NODAL && d == arg && hi == B.hi[d]) hi += 1;  // the box's last face
            if (kind == BL_TILE_GROWN) {
              if (lo == B.lo[d]) lo -= arg;
              if (hi == B.hi[d]) hi += arg;
            }
            r[1 + d] = lo;
            r[4 + d] = hi;
          }
        }
  }
  if (n > INT32_MAX) return fail(BL_EINVAL, "more than 2^31 tiles");
  *ntiles = (int32_t)n;
  return BL_OK;
}

bl_status bl_multifab_bytes(const bl_boxarray* ba, int32_t ncomp, int32_t nghost, bl_dtype dtype, size_t* bytes) {
  clear_error();
  if (!ba || !bytes) return fail(BL_EINVAL, "NULL argument");
  if (ncomp < 1 || nghost < 0) return fail(BL_EINVAL, "need ncomp >= 1 and nghost >= 0");
  if (dtype != BL_F64 && dtype != BL_F32) return fail(BL_EDTYPE, "unknown dtype %d", (int)dtype);
  const int esize = dtype == BL_F64 ? 8 : 4;
  const int64_t A = elem_align(esize);
  int64_t off = 0;
  FabGeom f;
  for (const Box& b : ba->boxes) off = round_up(off + layout_fab(b, nghost, ncomp, A, off, f), A);
  *bytes = (size_t)off * esize;
  return BL_OK;
}

}  // extern "C"
