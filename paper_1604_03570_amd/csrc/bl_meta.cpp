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
  if (ndevices != 1) return fail(BL_EINVAL, "this build runs on one GPU: ndevices must be 1, got %d", ndevices);
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

void build_tiles(const Plan& p, const TileConfig& cfg, int member, int box_base, std::vector<DevTile>& tiles,
                 std::vector<int>* box_tile_start) {
  const int lanes = 64 * cfg.waves;
  if (box_tile_start) box_tile_start->clear();
  for (int b = 0; b < (int)p.hboxes.size(); ++b) {
    const DevBox& B = p.hboxes[b];
    if (box_tile_start) box_tile_start->push_back((int)tiles.size());
    int nplane = B.nvx * B.ey;
    for (int n = 0; n < p.ncomp; ++n)
      for (int l0 = 0; l0 < nplane; l0 += lanes)
        for (int z0 = 0; z0 < B.ez; z0 += cfg.zchunk) {
          DevTile t;
          t.box = box_base + b;
          t.comp = n;
          t.member = member;
          t.l0 = l0;
          t.nl = std::min(lanes, nplane - l0);
          t.z0 = z0;
          t.z1 = std::min(B.ez, z0 + cfg.zchunk);
          t.work = t.nl * p.vec * (t.z1 - t.z0);
          tiles.push_back(t);
        }
  }
  if (box_tile_start) box_tile_start->push_back((int)tiles.size());
}

bl_status build_plan(const bl_boxarray* cba, int ncomp, int ng, int dtype, std::shared_ptr<Plan>* out) {
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
  for (const Box& b : ba->boxes)
    if (b.len(0) % v16) all_div = false;
  p->vec = all_div ? v16 : 1;
  const int xlead = (int)round_up(ng, p->vec);
  p->xlead = xlead;
  const int64_t fab_align = 128 / p->esize;
  int64_t off = 0;
  p->fabs.resize(ba->boxes.size());
  for (size_t i = 0; i < ba->boxes.size(); ++i) {
    const Box& b = ba->boxes[i];
    FabGeom& f = p->fabs[i];
    f.grown = b.grow(ng);
    int64_t px = round_up(xlead + b.len(0) + ng, p->vec);
    f.sy = px;
    f.sz = px * (b.len(1) + 2 * ng);
    f.sc = f.sz * (b.len(2) + 2 * ng);
    if (f.sc * ncomp >= ((int64_t)1 << 31))
      return fail(BL_EINVAL, "box %zu is too large for one FAB (%lld elements)", i, (long long)(f.sc * ncomp));
    off = round_up(off, fab_align);
    f.off_valid = off + xlead + ng * f.sy + ng * f.sz;
    f.off_grown = off + (xlead - ng);
    off += f.sc * ncomp;
  }
  p->total_elems = (size_t)round_up(off, fab_align);

  // per-box descriptors and face records
  const auto face_ptr = face_plan(ba, ng);
  const auto& faces = *face_ptr;
  p->hboxes.resize(ba->boxes.size());
  for (size_t i = 0; i < ba->boxes.size(); ++i) {
    const Box& b = ba->boxes[i];
    const FabGeom& f = p->fabs[i];
    DevBox& B = p->hboxes[i];
    std::memset(&B, 0, sizeof B);
    B.off = f.off_valid;
    B.sc = f.sc;
    B.sy = (int32_t)f.sy;
    B.sz = (int32_t)f.sz;
    B.ex = b.len(0);
    B.ey = b.len(1);
    B.ez = b.len(2);
    B.nvx = B.ex / p->vec;
    for (int d = 0; d < 3; ++d) B.glo[d] = b.lo[d];
  }
  // face records arrive grouped by (box, face) in order
  p->hfacerecs.clear();
  size_t k = 0;
  for (size_t i = 0; i < ba->boxes.size(); ++i) {
    for (int face = 0; face < 6; ++face) {
      DevBox& B = p->hboxes[i];
      B.face_start[face] = (int32_t)p->hfacerecs.size();
      int cnt = 0;
      while (k < faces.size() && faces[k].box == (int)i && faces[k].face == face) {
        const FaceRecord& r = faces[k++];
        const Box& bx = ba->boxes[i];
        const Box& sb = ba->boxes[r.src];
        const FabGeom& sf = p->fabs[r.src];
        int a = face / 2, side = face % 2;
        int t1 = a == 0 ? 1 : 0, t2 = a == 2 ? 1 : 2;
        int64_t sstride[3] = {1, sf.sy, sf.sz};
        int lfix[3] = {0, 0, 0};
        lfix[a] = side ? bx.len(a) - 1 : 0;
        int nrm[3] = {0, 0, 0};
        nrm[a] = side ? 1 : -1;
        int64_t base = sf.off_valid;
        for (int d = 0; d < 3; ++d) base += (int64_t)(bx.lo[d] + lfix[d] + nrm[d] + r.shift[d] - sb.lo[d]) * sstride[d];
        DevFaceRec R;
        R.base = base;
        R.sc = sf.sc;
        R.s1 = (int32_t)sstride[t1];
        R.s2 = (int32_t)sstride[t2];
        R.t1lo = (int16_t)(r.region.lo[t1] - bx.lo[t1]);
        R.t1hi = (int16_t)(r.region.hi[t1] - bx.lo[t1]);
        R.t2lo = (int16_t)(r.region.lo[t2] - bx.lo[t2]);
        R.t2hi = (int16_t)(r.region.hi[t2] - bx.lo[t2]);
        p->hfacerecs.push_back(R);
        ++cnt;
      }
      if (cnt > 32767) return fail(BL_EINVAL, "too many neighbours on one face of box %zu", i);
      B.face_count[face] = (int16_t)cnt;
    }
  }
  for (const Box& b : ba->boxes)
    for (int d = 0; d < 3; ++d)
      if (b.len(d) > 32767) return fail(BL_EINVAL, "box edge above 32767");

  // FillBoundary records and chunks
  p->fill = fill_plan(ba, ng);
  const auto& fill = *p->fill;
  p->hfillrecs.clear();
  p->hfillchunks.clear();
  for (const FillRecord& r : fill) {
    const Box& db = ba->boxes[r.dst];
    const Box& sb = ba->boxes[r.src];
    const FabGeom& df = p->fabs[r.dst];
    const FabGeom& sf = p->fabs[r.src];
    DevFillRec R;
    std::memset(&R, 0, sizeof R);
    R.dst_base = df.off_valid + (r.region.lo[0] - db.lo[0]) + (r.region.lo[1] - db.lo[1]) * df.sy +
                 (r.region.lo[2] - db.lo[2]) * df.sz;
    R.src_base = sf.off_valid + (r.region.lo[0] + r.shift[0] - sb.lo[0]) +
                 (r.region.lo[1] + r.shift[1] - sb.lo[1]) * sf.sy + (r.region.lo[2] + r.shift[2] - sb.lo[2]) * sf.sz;
    R.dsc = df.sc;
    R.ssc = sf.sc;
    R.dsy = (int32_t)df.sy;
    R.dsz = (int32_t)df.sz;
    R.ssy = (int32_t)sf.sy;
    R.ssz = (int32_t)sf.sz;
    R.nx = r.region.len(0);
    R.ny = r.region.len(1);
    R.nz = r.region.len(2);
    int rid = (int)p->hfillrecs.size();
    p->hfillrecs.push_back(R);
    int64_t vol = r.region.volume();
    for (int64_t s = 0; s < vol; s += kFillChunk) p->hfillchunks.push_back(DevFillChunk{rid, (int32_t)s});
  }

  p->cfg = tile_config();
  build_tiles(*p, p->cfg, 0, 0, p->htiles, &p->box_tile_start);
  *out = p;
  return BL_OK;
}

}  // namespace bl

extern "C" {

bl_status bl_multifab_bytes(const bl_boxarray* ba, int32_t ncomp, int32_t nghost, bl_dtype dtype, size_t* bytes) {
  clear_error();
  if (!ba || !bytes) return fail(BL_EINVAL, "NULL argument");
  if (ncomp < 1 || nghost < 0) return fail(BL_EINVAL, "need ncomp >= 1 and nghost >= 0");
  if (dtype != BL_F64 && dtype != BL_F32) return fail(BL_EDTYPE, "unknown dtype %d", (int)dtype);
  int esize = dtype == BL_F64 ? 8 : 4;
  int v16 = 16 / esize;
  bool all_div = true;
  for (const Box& b : ba->boxes)
    if (b.len(0) % v16) all_div = false;
  int vec = all_div ? v16 : 1;
  int64_t xlead = round_up(nghost, vec);
  int64_t fab_align = 128 / esize, off = 0;
  for (const Box& b : ba->boxes) {
    int64_t px = round_up(xlead + b.len(0) + nghost, vec);
    int64_t sc = px * (b.len(1) + 2 * nghost) * (b.len(2) + 2 * nghost);
    off = round_up(off, fab_align) + sc * ncomp;
  }
  *bytes = (size_t)round_up(off, fab_align) * esize;
  return BL_OK;
}

}  // extern "C"
