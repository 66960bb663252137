// C interface of libboxtile: MultiFab handles, FillBoundary, heat step
// (per-box, unfused batched and fused/graph forms), red-black Gauss-Seidel,
// reductions, batching of independent problems and metadata inspection.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <tuple>

#include "bl_internal.h"
#include "bl_launch.h"

namespace bl {

bl_status hip_fail(int err, const char* what) {
  return fail(BL_EHIP, "%s failed: %s", what, hipGetErrorString((hipError_t)err));
}

Plan::~Plan() {
  (void)hipFree(dboxes);
  (void)hipFree(dfacerecs);
  (void)hipFree(dfacerecs_rows);
  (void)hipFree(dtiles);
  (void)hipFree(dlin);
  (void)hipFree(dred);
  (void)hipFree(dfillrecs);
  (void)hipFree(dfillrecs_mir);
  (void)hipFree(dfillchunks);
  (void)hipFree(dvlin);
  (void)hipFree(dcellpre);
  (void)hipFree(dpairpre);
  (void)hipFree(dh8);
  (void)hipFree(dh8seg);
  (void)hipFree(dh8segm);
  (void)hipFree(dh8face);
  (void)hipFree(dcellwg);
  (void)hipFree(dpairwg);
  (void)hipFree(dringrecs);
  (void)hipFree(dpushrecs);
  (void)hipFree(dpushface);
  (void)hipFree(dmir2off);
  (void)hipFree(dsweep);
}

template <typename T>
static bl_status upload(T** dst, const std::vector<T>& src, const char* what) {
  if (src.empty()) return BL_OK;
  hipError_t e = hipMalloc((void**)dst, sizeof(T) * src.size());
  if (e != hipSuccess) return hip_fail(e, what);
  e = hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, what);
  return BL_OK;
}

bl_status upload_plan(Plan& p) {
  if (p.uploaded) return BL_OK;
  bl_status st;
  if ((st = upload(&p.dboxes, p.hboxes, "hipMalloc/hipMemcpy(boxes)")) != BL_OK) return st;
  if ((st = upload(&p.dfacerecs, p.hfacerecs, "hipMalloc/hipMemcpy(face records)")) != BL_OK) return st;
  if ((st = upload(&p.dfacerecs_rows, p.hfacerecs_rows, "hipMalloc/hipMemcpy(face records, rows)")) != BL_OK)
    return st;
  if ((st = upload(&p.dtiles, p.htiles, "hipMalloc/hipMemcpy(tiles)")) != BL_OK) return st;
  if ((st = upload(&p.dlin, p.hlin, "hipMalloc/hipMemcpy(stencil tiles)")) != BL_OK) return st;
  if ((st = upload(&p.dred, p.hred, "hipMalloc/hipMemcpy(reduction chunks)")) != BL_OK) return st;
  if ((st = upload(&p.dfillrecs, p.hfillrecs, "hipMalloc/hipMemcpy(fill records)")) != BL_OK) return st;
  if ((st = upload(&p.dfillrecs_mir, p.hfillrecs_mir, "hipMalloc/hipMemcpy(fill records, mirrors)")) != BL_OK)
    return st;
  if ((st = upload(&p.dfillchunks, p.hfillchunks, "hipMalloc/hipMemcpy(fill chunks)")) != BL_OK) return st;
  if ((st = upload(&p.dcellpre, p.hcellpre, "hipMalloc/hipMemcpy(cell counts)")) != BL_OK) return st;
  if ((st = upload(&p.dpairpre, p.hpairpre, "hipMalloc/hipMemcpy(pair counts)")) != BL_OK) return st;
  if ((st = upload(&p.dcellwg, p.hcellwg, "hipMalloc/hipMemcpy(cell workgroups)")) != BL_OK) return st;
  if ((st = upload(&p.dpairwg, p.hpairwg, "hipMalloc/hipMemcpy(pair workgroups)")) != BL_OK) return st;
  if ((st = upload(&p.dringrecs, p.hringrecs, "hipMalloc/hipMemcpy(ring records)")) != BL_OK) return st;
  if ((st = upload(&p.dpushrecs, p.hpushrecs, "hipMalloc/hipMemcpy(push records)")) != BL_OK) return st;
  if ((st = upload(&p.dpushface, p.hpushface, "hipMalloc/hipMemcpy(push faces)")) != BL_OK) return st;
  if ((st = upload(&p.dmir2off, p.hmir2off, "hipMalloc/hipMemcpy(inner mirror offsets)")) != BL_OK) return st;
  p.uploaded = true;
  return BL_OK;
}

// Plans are shared by every MultiFab of one shape and tile configuration.
static std::mutex g_plan_mu;
static std::map<std::tuple<uint64_t, int, int, int, int, int, int, int>, std::weak_ptr<Plan>> g_plans;
static constexpr size_t kPlansKept = 64;
static std::deque<std::shared_ptr<Plan>> g_plan_keep;

// Tile configurations chosen by bl_autotune, per (BoxArray, ncomp, nghost, dtype);
// they take precedence over the global configuration until bl_set_tile_config.
static std::map<std::tuple<uint64_t, int, int, int>, TileConfig> g_tuned;

static TileConfig config_for(const bl_boxarray* ba, int ncomp, int ng, int dtype) {
  auto it = g_tuned.find(std::make_tuple(ba->uid, ncomp, ng, dtype));
  return it != g_tuned.end() ? it->second : tile_config();
}

static bl_status get_plan_cfg(const bl_boxarray* ba, int ncomp, int ng, int dtype, const TileConfig& cfg,
                              bool to_device, std::shared_ptr<Plan>* out) {
  auto key = std::make_tuple(ba->uid, ncomp, ng, dtype, cfg.zchunk, cfg.waves, cfg.block, cfg.zsteps);
  std::lock_guard<std::mutex> lk(g_plan_mu);
  auto it = g_plans.find(key);
  std::shared_ptr<Plan> p;
  if (it != g_plans.end()) p = it->second.lock();
  if (!p) {
    bl_status st = build_plan(ba, ncomp, ng, dtype, cfg, &p);
    if (st != BL_OK) return st;
    // drop the entries of plans that no MultiFab holds any more
    for (auto e = g_plans.begin(); e != g_plans.end();) e = e->second.expired() ? g_plans.erase(e) : std::next(e);
    g_plans[key] = p;
    // the most recent plans stay alive after their last MultiFab goes, so a
    // shape that comes back (a serving loop) reuses its tables
    g_plan_keep.push_back(p);
    if (g_plan_keep.size() > kPlansKept) g_plan_keep.pop_front();
  }
  if (to_device) {
    bl_status st = upload_plan(*p);
    if (st != BL_OK) return st;
  }
  *out = p;
  return BL_OK;
}

static bl_status get_plan(const bl_boxarray* ba, int ncomp, int ng, int dtype, bool to_device,
                          std::shared_ptr<Plan>* out) {
  TileConfig cfg;
  {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    cfg = config_for(ba, ncomp, ng, dtype);
  }
  return get_plan_cfg(ba, ncomp, ng, dtype, cfg, to_device, out);
}

static int block_of(const Plan& p) { return 64 * p.cfg.waves; }

// partial results of a reduction or residual norm: one per reduction chunk,
// tile or linear tile, whichever launch writes them
static size_t reduce_slots(const Plan& p) { return std::max({p.hred.size(), p.htiles.size(), p.hlin.size()}); }

static int persistent_grid(int persist) { return persist > 0 ? device_cu_count() * persist : 0; }

static bl_status same_shape(const bl_multifab* a, const bl_multifab* b) {
  if (!a || !b) return fail(BL_EINVAL, "NULL MultiFab");
  if (a->plan->dtype != b->plan->dtype) return fail(BL_EDTYPE, "MultiFabs differ in dtype");
  if (a->plan->ba_uid != b->plan->ba_uid || a->plan->ncomp != b->plan->ncomp || a->plan->ng != b->plan->ng)
    return fail(BL_ESHAPE, "MultiFabs differ in BoxArray, ncomp or nghost");
  return BL_OK;  // the FAB layout does not depend on the tile configuration
}

static bl_status ensure_scratch(bl_multifab* mf, size_t ndev, size_t nhost) {
  if (mf->nscratch < ndev) {
    (void)hipFree(mf->dscratch);
    mf->dscratch = nullptr;
    mf->nscratch = 0;
    BL_HIP(hipMalloc((void**)&mf->dscratch, ndev * sizeof(double)));
    mf->nscratch = ndev;
  }
  if (mf->nhres < nhost) {
    (void)hipHostFree(mf->hres);
    mf->hres = nullptr;
    mf->nhres = 0;
    BL_HIP(hipHostMalloc((void**)&mf->hres, nhost * sizeof(double), hipHostMallocDefault));
    mf->nhres = nhost;
  }
  return BL_OK;
}

// Stream used only to capture graphs (default priority, non-blocking).
static hipStream_t capture_stream() {
  static std::mutex mu;
  static std::map<int, hipStream_t> streams;
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lk(mu);
  auto it = streams.find(dev);
  if (it != streams.end()) return it->second;
  hipStream_t s = nullptr;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return nullptr;
  streams[dev] = s;
  return s;
}

struct GraphKey {
  const bl_multifab* u0;
  const bl_multifab* u1;
  void* d0;
  void* d1;
  int nsteps;
  uint64_t cbits;
  int persist;
  int device;
  bool start_mirror;
  bool operator==(const GraphKey& o) const {
    return u0 == o.u0 && u1 == o.u1 && d0 == o.d0 && d1 == o.d1 && nsteps == o.nsteps && cbits == o.cbits &&
           persist == o.persist && device == o.device && start_mirror == o.start_mirror;
  }
};
static std::mutex g_graph_mu;
static std::vector<std::pair<GraphKey, hipGraphExec_t>> g_graphs;

static void forget_graphs(const bl_multifab* mf) {
  std::lock_guard<std::mutex> lk(g_graph_mu);
  for (size_t i = 0; i < g_graphs.size();) {
    if (g_graphs[i].first.u0 == mf || g_graphs[i].first.u1 == mf) {
      (void)hipGraphExecDestroy(g_graphs[i].second);
      g_graphs.erase(g_graphs.begin() + i);
    } else {
      ++i;
    }
  }
}

}  // namespace bl

using namespace bl;

bl_multifab::~bl_multifab() {
  forget_graphs(this);
  (void)hipFree(dtwin);
  (void)hipFree(dmir2);
  (void)hipFree(dscratch);
  (void)hipHostFree(hres);
}

extern "C" {

bl_status bl_multifab_create(const bl_boxarray* ba, const bl_distmap* dm, int32_t ncomp, int32_t nghost,
                             bl_dtype dtype, void* dev_ptr, size_t bytes, bl_multifab** out) {
  clear_error();
  if (!ba || !out) return fail(BL_EINVAL, "NULL argument");
  *out = nullptr;
  if (dm && dm->ba_uid != ba->uid) return fail(BL_ESHAPE, "DistributionMapping belongs to another BoxArray");
  if (ncomp < 1 || nghost < 0) return fail(BL_EINVAL, "need ncomp >= 1 and nghost >= 0");
  if (dtype != BL_F64 && dtype != BL_F32) return fail(BL_EDTYPE, "unknown dtype %d", (int)dtype);
  for (int d = 0; d < 3; ++d)
    if (ba->periodic[d] && nghost > ba->domain.len(d))
      return fail(BL_EINVAL, "nghost %d exceeds the periodic extent %d of axis %d", nghost, ba->domain.len(d), d);
  size_t need = 0;
  bl_status st = bl_multifab_bytes(ba, ncomp, nghost, dtype, &need);
  if (st != BL_OK) return st;
  if (!dev_ptr) return fail(BL_EINVAL, "NULL device pointer");
  if (((uintptr_t)dev_ptr) % 256 != 0) return fail(BL_EINVAL, "device pointer is not 256-byte aligned");
  if (bytes < need) return fail(BL_ENOMEM, "buffer of %zu bytes, MultiFab needs %zu", bytes, need);
  std::shared_ptr<Plan> plan;
  if ((st = get_plan(ba, ncomp, nghost, dtype, true, &plan)) != BL_OK) return st;
  bl_multifab* mf = new (std::nothrow) bl_multifab;
  if (!mf) return fail(BL_ENOMEM, "host allocation");
  mf->plan = plan;
  mf->data = dev_ptr;
  mf->bytes = bytes;
  *out = mf;
  return BL_OK;
}

bl_status bl_multifab_layout(const bl_multifab* mf, int32_t box, bl_box* grown, size_t* offset_elems,
                             int64_t stride[4]) {
  clear_error();
  if (!mf) return fail(BL_EINVAL, "NULL MultiFab");
  const Plan& p = *mf->plan;
  if (box < 0 || box >= (int)p.fabs.size()) return fail(BL_EINVAL, "box %d out of range", box);
  const FabGeom& f = p.fabs[box];
  if (grown) *grown = to_c(f.grown);
  if (offset_elems) *offset_elems = (size_t)f.index(f.valid.lo[0], f.grown.lo[1], f.grown.lo[2]);
  if (stride) {
    stride[0] = 1;
    stride[1] = f.sy;
    stride[2] = f.sz;
    stride[3] = f.sc;
  }
  return BL_OK;
}

bl_status bl_multifab_xghost_layout(const bl_multifab* mf, int32_t box, size_t* offset_elems, int64_t stride[5]) {
  clear_error();
  if (!mf) return fail(BL_EINVAL, "NULL MultiFab");
  const Plan& p = *mf->plan;
  if (box < 0 || box >= (int)p.fabs.size()) return fail(BL_EINVAL, "box %d out of range", box);
  if (p.ng < 1) return fail(BL_EINVAL, "the MultiFab has no ghost cells");
  const FabGeom& f = p.fabs[box];
  if (offset_elems) *offset_elems = (size_t)f.index(f.valid.lo[0] - 1, f.grown.lo[1], f.grown.lo[2]);
  if (stride) {
    stride[0] = 1;
    stride[1] = f.ng;
    stride[2] = f.xs_z;
    stride[3] = f.xs_side;
    stride[4] = f.sc;
  }
  return BL_OK;
}

bl_status bl_multifab_copy_fab(bl_multifab* mf, int32_t box, int32_t scomp, int32_t ncomp, void* dense_dev,
                               int32_t to_dense, hipStream_t stream) {
  clear_error();
  if (!mf || !dense_dev) return fail(BL_EINVAL, "NULL argument");
  const Plan& p = *mf->plan;
  if (box < 0 || box >= (int)p.fabs.size()) return fail(BL_EINVAL, "box %d out of range", box);
  if (scomp < 0 || ncomp < 1 || scomp + ncomp > p.ncomp) return fail(BL_EINVAL, "component range out of bounds");
  if (!to_dense) mf->mark_mirror(false);
  BL_HIP(launch_copy_fab(p, mf->data, dense_dev, box, scomp, ncomp, to_dense, stream));
  return BL_OK;
}

bl_status bl_multifab_modified(bl_multifab* mf) {
  clear_error();
  if (!mf) return fail(BL_EINVAL, "NULL MultiFab");
  mf->mark_mirror(false);
  return BL_OK;
}

bl_status bl_multifab_info(const bl_multifab* mf, int32_t* nboxes, int32_t* ncomp, int32_t* nghost, int32_t* dtype) {
  clear_error();
  if (!mf) return fail(BL_EINVAL, "NULL MultiFab");
  if (nboxes) *nboxes = (int32_t)mf->plan->fabs.size();
  if (ncomp) *ncomp = mf->plan->ncomp;
  if (nghost) *nghost = mf->plan->ng;
  if (dtype) *dtype = mf->plan->dtype;
  return BL_OK;
}

void bl_multifab_destroy(bl_multifab* mf) { delete mf; }

bl_status bl_multifab_copy_global(bl_multifab* mf, int32_t scomp, int32_t ncomp, void* global_dev, int32_t to_global,
                                  hipStream_t stream) {
  clear_error();
  if (!mf || !global_dev) return fail(BL_EINVAL, "NULL argument");
  const Plan& p = *mf->plan;
  if (scomp < 0 || ncomp < 1 || scomp + ncomp > p.ncomp) return fail(BL_EINVAL, "component range out of bounds");
  if (!to_global) mf->mark_mirror(false);
  BL_HIP(launch_copy_global(p, mf->data, global_dev, scomp, ncomp, to_global, block_of(p), stream));
  return BL_OK;
}

bl_status bl_multifab_set_val(bl_multifab* mf, double val, int32_t scomp, int32_t ncomp, int32_t with_ghosts,
                              hipStream_t stream) {
  clear_error();
  if (!mf) return fail(BL_EINVAL, "NULL MultiFab");
  const Plan& p = *mf->plan;
  if (scomp < 0 || ncomp < 1 || scomp + ncomp > p.ncomp) return fail(BL_EINVAL, "component range out of bounds");
  mf->mark_mirror(false);
  BL_HIP(launch_set_val(p, mf->data, val, scomp, ncomp, with_ghosts, block_of(p), stream));
  return BL_OK;
}

bl_status bl_fill_boundary(bl_multifab* mf, int32_t scomp, int32_t ncomp, hipStream_t stream) {
  clear_error();
  if (!mf) return fail(BL_EINVAL, "NULL MultiFab");
  const Plan& p = *mf->plan;
  if (scomp < 0 || ncomp < 1 || scomp + ncomp > p.ncomp) return fail(BL_EINVAL, "component range out of bounds");
  BL_HIP(launch_fill(p, mf->data, scomp, ncomp, stream, mf->mirror_current));
  return BL_OK;
}

static bl_status check_heat(bl_multifab* a, bl_multifab* b) {
  bl_status st = same_shape(a, b);
  if (st != BL_OK) return st;
  if (a->plan->ng < 1) return fail(BL_EINVAL, "the stencil needs nghost >= 1");
  if (a->data == b->data) return fail(BL_EINVAL, "u_old and u_new share storage");
  return BL_OK;
}

static DevMember member_of(bl_multifab* a, bl_multifab* b, double c) {
  DevMember m;
  std::memset(&m, 0, sizeof m);
  m.a = a->data;
  m.b = b->data;
  m.c = c;
  m.flip_offset = 0;
  return m;
}

bl_status bl_heat_step(bl_multifab* u_old, bl_multifab* u_new, double c, int32_t fill_first, hipStream_t stream) {
  clear_error();
  bl_status st = check_heat(u_old, u_new);
  if (st != BL_OK) return st;
  const Plan& p = *u_old->plan;
  if (fill_first) BL_HIP(launch_fill(p, u_old->data, 0, p.ncomp, stream, u_old->mirror_current));
  u_new->mark_mirror(false);  // the per-box kernels do not write the edge mirror
  HeatArgs a{};
  a.fvec = p.fvec;
  a.zblock = p.cfg.block ? p.cfg.zchunk : 0;
  a.form = p.cfg.block;
  a.rmax = p.rmax;
  a.nvtmax = p.nvtmax;
  a.boxes = p.dboxes;
  a.recs = p.dfacerecs;
  a.m0 = member_of(u_old, u_new, c);
  a.members = nullptr;
  a.flip = 0;
  for (size_t b = 0; b < p.hboxes.size(); ++b) {  // one launch per box
    a.tiles = p.dtiles + p.box_tile_start[b];
    a.ntiles = p.box_tile_start[b + 1] - p.box_tile_start[b];
    BL_HIP(launch_heat(p.dtype, p.vec, false, a, 0, block_of(p), stream));
  }
  return BL_OK;
}

bl_status bl_heat_step_unfused(bl_multifab* u_old, bl_multifab* u_new, double c, hipStream_t stream) {
  clear_error();
  bl_status st = check_heat(u_old, u_new);
  if (st != BL_OK) return st;
  const Plan& p = *u_old->plan;
  BL_HIP(launch_fill(p, u_old->data, 0, p.ncomp, stream, u_old->mirror_current));
  HeatArgs a{p.dtiles, (int)p.htiles.size(), p.dboxes, p.dfacerecs, member_of(u_old, u_new, c), nullptr, 0,
             p.fvec, p.cfg.block ? p.cfg.zchunk : 0, p.cfg.block, p.rmax, p.nvtmax,
             p.dlin, (int)p.hlin.size(), p.yhmax, p.xhmax};
  // the halo-in-LDS kernel over linear tiles writes the output's edge mirror, the others do not
  u_new->mark_mirror(p.cfg.block == 3 && p.dlin != nullptr);
  BL_HIP(launch_heat(p.dtype, p.vec, false, a, persistent_grid(tile_config().persist), block_of(p), stream));
  return BL_OK;
}

bl_status bl_heat_advance(bl_multifab* u[2], int32_t nsteps, double c, hipStream_t stream) {
  clear_error();
  if (!u) return fail(BL_EINVAL, "NULL MultiFab array");
  bl_status st = check_heat(u[0], u[1]);
  if (st != BL_OK) return st;
  if (nsteps < 0) return fail(BL_EINVAL, "nsteps < 0");
  if (nsteps == 0) return BL_OK;
  const Plan& p = *u[0]->plan;
  const int persist = tile_config().persist;
  int dev = 0;
  BL_HIP(hipGetDevice(&dev));
  uint64_t cbits;
  std::memcpy(&cbits, &c, sizeof cbits);
  // the first step reads the starting state's x faces from its edge mirror when
  // the library knows that mirror to be current, else from the neighbours' rows
  // (form 3) or from a mirror extracted first (the other forms)
  const bool start_mirror = u[0]->mirror_current;
  const bool rows_first = !start_mirror && p.cfg.block == 3 && p.dlin && p.fvec && p.dfacerecs_rows;
  GraphKey key{u[0], u[1], u[0]->data, u[1]->data, nsteps, cbits, persist, dev, start_mirror};
  hipGraphExec_t exec = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_graph_mu);
    for (auto& e : g_graphs)
      if (e.first == key) exec = e.second;
  }
  if (!exec) {
    hipStream_t cs = capture_stream();
    if (!cs) return fail(BL_EHIP, "could not create the capture stream");
    HeatArgs a{p.dtiles, (int)p.htiles.size(), p.dboxes, p.dfacerecs, member_of(u[0], u[1], c), nullptr, 0,
               p.fvec, p.cfg.block ? p.cfg.zchunk : 0, p.cfg.block, p.rmax, p.nvtmax,
               p.dlin, (int)p.hlin.size(), p.yhmax, p.xhmax};
    BL_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    // The fused steps read x neighbours from the edge-column mirror that each
    // step writes for its output.  Without a current mirror of the starting
    // state, the halo-in-LDS form reads the first step's from the neighbours'
    // rows instead; the other forms get one made first.
    hipError_t le = rows_first || start_mirror ? hipSuccess : launch_extract_mirror(p, u[0]->data, cs);
    for (int s = 0; s < nsteps && le == hipSuccess; ++s) {
      a.flip = s & 1;
      a.recs = rows_first && s == 0 ? p.dfacerecs_rows : p.dfacerecs;
      le = launch_heat(p.dtype, p.vec, true, a, persistent_grid(persist), block_of(p), cs);
    }
    hipGraph_t graph = nullptr;
    hipError_t ee = hipStreamEndCapture(cs, &graph);
    if (le != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return hip_fail(le, "kernel launch during graph capture");
    }
    if (ee != hipSuccess) return hip_fail(ee, "hipStreamEndCapture");
    hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) return hip_fail(ie, "hipGraphInstantiate");
    std::lock_guard<std::mutex> lk(g_graph_mu);
    g_graphs.push_back({key, exec});
  }
  BL_HIP(hipGraphLaunch(exec, stream));
  if (nsteps >= 2 || !rows_first) u[0]->mark_mirror(true);  // written by step 1, extracted or kept
  u[1]->mark_mirror(true);                                    // written by step 0
  return BL_OK;
}

// Tiles for the variable-coefficient kernel: 2 planes per z block (measured on
// the 512^3 uneven level: 3.53 ms per step against 4.06 for 4 planes; twice the
// stencil's LDS leaves room for fewer workgroups) in kVcZsteps z steps, the
// plan's own linear tiles when they are of that shape, else tiles built once per
// plan.
static constexpr int kVcZsteps = 8;
static std::mutex g_vc_mu;

static bl_status vc_tiles(Plan& p, VcArgs* a) {
  a->block = 64 * p.cfg.waves;
  if (p.cfg.block == 3 && p.cfg.zchunk == 2 && p.cfg.zsteps == kVcZsteps && !p.hlin.empty() &&
      2 * vc_lds_half(p.dtype, p.vec, 2, p.yhmax, p.xhmax, a->block) <= kDmaLdsMax) {
    a->lin = p.dlin;
    a->nlin = (int)p.hlin.size();
    a->yhmax = p.yhmax;
    a->xhmax = p.xhmax;
    a->zchunk = 2;
    return BL_OK;
  }
  std::lock_guard<std::mutex> lk(g_vc_mu);
  if (!p.vzchunk) {
    TileConfig c = p.cfg;
    c.block = 3;
    c.zchunk = 2;
    c.persist = 0;
    c.zsteps = kVcZsteps;
    std::vector<DevLinTile> t;
    int yh = 1, xh = 1;
    build_lin_tiles(p, c, 0, 0, 0, t, &yh, &xh);
    if (2 * vc_lds_half(p.dtype, p.vec, 2, yh, xh, a->block) > kDmaLdsMax)
      return fail(BL_EINVAL, "the boxes' planes are too wide for the flux-form kernel's LDS staging at %d waves",
                  p.cfg.waves);
    bl_status st = upload(&p.dvlin, t, "hipMalloc/hipMemcpy(flux-form tiles)");
    if (st != BL_OK) return st;
    p.hvlin.swap(t);
    p.vyhmax = yh;
    p.vxhmax = xh;
    p.vzchunk = 2;
  }
  a->lin = p.dvlin;
  a->nlin = (int)p.hvlin.size();
  a->yhmax = p.vyhmax;
  a->xhmax = p.vxhmax;
  a->zchunk = p.vzchunk;
  return BL_OK;
}

bl_status bl_heat_varcoef_advance(bl_multifab* u[2], bl_multifab* beta, int32_t nsteps, double dt, double inv_dx,
                                  hipStream_t stream) {
  clear_error();
  if (!u) return fail(BL_EINVAL, "NULL MultiFab array");
  bl_status st = check_heat(u[0], u[1]);
  if (st != BL_OK) return st;
  if ((st = same_shape(u[0], beta)) != BL_OK) return st;
  if (beta->data == u[0]->data || beta->data == u[1]->data) return fail(BL_EINVAL, "beta shares storage with u");
  if (nsteps < 0) return fail(BL_EINVAL, "nsteps < 0");
  if (nsteps == 0) return BL_OK;
  Plan& p = *u[0]->plan;
  VcArgs a{};
  if ((st = vc_tiles(p, &a)) != BL_OK) return st;
  a.boxes = p.dboxes;
  a.recs = p.dfacerecs;
  a.fused = p.fvec;
  a.beta = beta->data;
  a.dt = dt;
  a.inv_dx = inv_dx;
  if (a.fused) {  // neighbour values from the neighbour boxes' faces and edge mirrors
    if (!beta->mirror_current) BL_HIP(launch_extract_mirror(p, beta->data, stream));
    if (!u[0]->mirror_current) BL_HIP(launch_extract_mirror(p, u[0]->data, stream));
    beta->mark_mirror(true);
  } else {
    BL_HIP(launch_fill(p, beta->data, 0, p.ncomp, stream, beta->mirror_current));
  }
  for (int s = 0; s < nsteps; ++s) {
    a.u = u[s & 1]->data;
    a.w = u[(s + 1) & 1]->data;
    if (!a.fused) BL_HIP(launch_fill(p, u[s & 1]->data, 0, p.ncomp, stream, s > 0 || u[0]->mirror_current));
    BL_HIP(launch_heat_varcoef(p.dtype, p.vec, a, stream));
  }
  // the kernel writes its output's edge mirror (both forms)
  u[0]->mark_mirror(a.fused || nsteps >= 2 || u[0]->mirror_current);
  u[1]->mark_mirror(true);
  return BL_OK;
}

// The fused 8th-order form's face segments of p, made on first use; *ok false
// (reason in p.h8why) where the layout does not allow the form.  Caller holds
// g_vc_mu.
static bl_status h8_segments(Plan& p, bool* ok) {
  if (p.h8fused < 0) {
    std::vector<DevH8Seg> sv, mv;
    std::vector<DevH8Face> fv;
    std::string why;
    if (build_h8_segments(p, sv, fv, &why, &mv)) {
      bl_status st = upload(&p.dh8seg, sv, "hipMalloc/hipMemcpy(8th-order face segments)");
      if (st == BL_OK) st = upload(&p.dh8face, fv, "hipMalloc/hipMemcpy(8th-order faces)");
      if (st == BL_OK && !mv.empty()) st = upload(&p.dh8segm, mv, "hipMalloc/hipMemcpy(8th-order mirror segments)");
      if (st != BL_OK) {
        (void)hipFree(p.dh8seg);
        (void)hipFree(p.dh8face);
        (void)hipFree(p.dh8segm);
        p.dh8seg = nullptr;
        p.dh8face = nullptr;
        p.dh8segm = nullptr;
        return st;
      }
      p.hh8seg.swap(sv);
      p.hh8face.swap(fv);
      p.h8mirror = !mv.empty();
      p.hh8segm.swap(mv);
      p.h8fused = 1;
    } else {
      p.h8why = why;
      p.h8fused = 0;
    }
  }
  *ok = p.h8fused == 1;
  return BL_OK;
}

bl_status bl_heat8_advance_form(bl_multifab* u[2], int32_t nsteps, double c, int32_t form, hipStream_t stream) {
  clear_error();
  if (!u) return fail(BL_EINVAL, "NULL MultiFab array");
  bl_status st = check_heat(u[0], u[1]);
  if (st != BL_OK) return st;
  Plan& p = *u[0]->plan;
  if (p.ng < 4) return fail(BL_EINVAL, "the 8th-order stencil needs nghost >= 4, not %d", p.ng);
  if (nsteps < 0) return fail(BL_EINVAL, "nsteps < 0");
  if (form < BL_H8_AUTO || form > BL_H8_FUSED_MIRROR)
    return fail(BL_EINVAL, "unknown 8th-order form %d", (int)form);
  bool fused = false;
  {
    std::lock_guard<std::mutex> lk(g_vc_mu);
    if (form != BL_H8_FILL) {
      if ((st = h8_segments(p, &fused)) != BL_OK) return st;
      if (!fused && (form == BL_H8_FUSED || form == BL_H8_FUSED_MIRROR))
        return fail(BL_EINVAL, "the fused 8th-order form does not apply to this layout: %s", p.h8why.c_str());
      if (form == BL_H8_FUSED_MIRROR && !p.h8mirror)
        return fail(BL_EINVAL, "the 4-layer mirror form needs every box at least 8 cells wide in x");
    }
    if (!p.h8built) {  // both forms run over the same tiles
      std::vector<DevTile> t;
      int rm = 1, nv = 1;
      build_h8_tiles(p, t, &rm, &nv);
      if ((st = upload(&p.dh8, t, "hipMalloc/hipMemcpy(8th-order tiles)")) != BL_OK) return st;
      p.hh8.swap(t);
      p.h8rmax = rm;
      p.h8nvtmax = nv;
      p.h8built = true;
    }
  }
  // the mirror form writes every output's 4-layer mirror, and reads its
  // input's where that is current: from step 1 on, and at step 0 where the
  // last write to u[0] was such a step
  const bool mir = form == BL_H8_FUSED_MIRROR;
  const bool start_mirror = u[0]->mirror4_current;
  // the MultiFabs the steps write are stale until the last step is launched
  // (an error in between leaves them so)
  for (int s = 0; s < nsteps && s < 2; ++s) u[(s + 1) & 1]->mark_mirror(false);
  for (int s = 0; s < nsteps; ++s) {
    void* src = u[s & 1]->data;
    void* dst = u[(s + 1) & 1]->data;
    if (!fused) BL_HIP(launch_fill(p, src, 0, p.ncomp, stream));
    const DevH8Seg* segs = !fused ? nullptr : (mir && (s > 0 || start_mirror)) ? p.dh8segm : p.dh8seg;
    BL_HIP(launch_heat8(p.dtype, p.vec, p.dh8, segs, fused ? p.dh8face : nullptr, (int)p.hh8.size(), p.dboxes, src,
                        dst, c, p.h8rmax, p.h8nvtmax, mir, stream));
  }
  for (int s = 0; s < nsteps && s < 2; ++s) {  // the MultiFabs steps s and s+2, ... wrote
    bl_multifab* out = u[(s + 1) & 1];
    out->mark_mirror(mir);
    out->mirror4_current = mir;
  }
  return BL_OK;
}

bl_status bl_heat8_advance(bl_multifab* u[2], int32_t nsteps, double c, hipStream_t stream) {
  return bl_heat8_advance_form(u, nsteps, c, BL_H8_AUTO, stream);
}

bl_status bl_heat8_fused_ok(const bl_multifab* mf, int32_t* ok) {
  clear_error();
  if (!mf || !ok) return fail(BL_EINVAL, "NULL argument");
  Plan& p = *mf->plan;
  if (p.ng < 4) {
    *ok = 0;
    return BL_OK;
  }
  std::lock_guard<std::mutex> lk(g_vc_mu);
  bool f = false;
  bl_status st = h8_segments(p, &f);
  if (st != BL_OK) return st;
  *ok = f ? 1 : 0;
  return BL_OK;
}

bl_status bl_reduce_async(const bl_multifab* cmf, int32_t comp, bl_reduce_op op, double* out_dev, hipStream_t stream) {
  clear_error();
  bl_multifab* mf = const_cast<bl_multifab*>(cmf);
  if (!mf || !out_dev) return fail(BL_EINVAL, "NULL argument");
  const Plan& p = *mf->plan;
  if (comp < 0 || comp >= p.ncomp) return fail(BL_EINVAL, "component %d out of range", comp);
  if ((int)op < 0 || (int)op > 5) return fail(BL_EINVAL, "unknown reduction %d", (int)op);
  bl_status st = ensure_scratch(mf, reduce_slots(p) + 8, 8);
  if (st != BL_OK) return st;
  BL_HIP(launch_reduce(p, mf->data, comp, (int)op, mf->dscratch, out_dev, block_of(p), stream));
  return BL_OK;
}

bl_status bl_reduce_async_noalloc(const bl_multifab* mf, int32_t comp, bl_reduce_op op, double* out_dev,
                                  hipStream_t stream) {
  clear_error();
  if (!mf || !out_dev) return fail(BL_EINVAL, "NULL argument");
  const Plan& p = *mf->plan;
  if (comp < 0 || comp >= p.ncomp) return fail(BL_EINVAL, "component %d out of range", comp);
  if ((int)op < 0 || (int)op > 5) return fail(BL_EINVAL, "unknown reduction %d", (int)op);
  if (!p.dred || p.hred.empty()) return fail(BL_EINVAL, "the MultiFab has no reduction chunks");
  if (p.hred.size() > (size_t)kNoAllocPartials)
    return fail(BL_EINVAL,
                "the MultiFab has %zu reduction chunks (about 32K values each); the no-allocation form holds at "
                "most %d partial results",
                p.hred.size(), kNoAllocPartials);
  BL_HIP(launch_reduce_noalloc(p, mf->data, comp, (int)op, out_dev, stream));
  return BL_OK;
}

bl_status bl_reduce(const bl_multifab* cmf, int32_t comp, bl_reduce_op op, double* out_host, hipStream_t stream) {
  clear_error();
  bl_multifab* mf = const_cast<bl_multifab*>(cmf);
  if (!mf || !out_host) return fail(BL_EINVAL, "NULL argument");
  const Plan& p = *mf->plan;
  bl_status st = ensure_scratch(mf, reduce_slots(p) + 8, 8);
  if (st != BL_OK) return st;
  double* dout = mf->dscratch + reduce_slots(p);
  if ((st = bl_reduce_async(mf, comp, op, dout, stream)) != BL_OK) return st;
  BL_HIP(hipMemcpyAsync(mf->hres, dout, sizeof(double), hipMemcpyDeviceToHost, stream));
  BL_HIP(hipStreamSynchronize(stream));
  *out_host = mf->hres[0];
  return BL_OK;
}

static bl_status check_gsrb(bl_multifab* phi, const bl_multifab* f) {
  bl_status st = same_shape(phi, f);
  if (st != BL_OK) return st;
  const Plan& p = *phi->plan;
  if (p.ncomp != 1) return fail(BL_EINVAL, "GSRB acts on single-component MultiFabs");
  if (p.ng < 1) return fail(BL_EINVAL, "the stencil needs nghost >= 1");
  for (int d = 0; d < 3; ++d)
    if (p.periodic[d] && p.domain.len(d) % 2)
      return fail(BL_EINVAL, "periodic axis %d has odd extent %d: red-black colouring breaks across the wrap", d,
                  p.domain.len(d));
  if (phi->data == f->data) return fail(BL_EINVAL, "phi and f share storage");
  return BL_OK;
}

// ||f + L_h phi||_2 into dout (device): the fused read-only pass where the plan
// allows it (neighbour values straight from the neighbour boxes), else
// FillBoundary and the residual kernel.  partials: reduce_slots(p) doubles.
static hipError_t residual_norm_dev(const Plan& p, bl_multifab* phi, const bl_multifab* f, double h2,
                                    double* partials, double* dout, hipStream_t stream) {
  hipError_t e;
  const int grid = persistent_grid(tile_config().persist);
  if (gsrb_fused_ok(p, block_of(p))) {
    e = launch_gsrb_fused(p, phi->data, f->data, h2, -1, 2, partials, grid, block_of(p), stream, !phi->mirror_current);
    if (e != hipSuccess) return e;
    return launch_reduce_partials(partials, gsrb_fused_grid(p, grid), 1, dout, stream);
  }
  e = launch_fill(p, phi->data, 0, 1, stream, phi->mirror_current);
  if (e != hipSuccess) return e;
  return launch_residual(p, phi->data, f->data, h2, partials, dout, block_of(p), stream);
}

bl_status bl_residual_norm(bl_multifab* phi, const bl_multifab* f, double h2, double* out_host, hipStream_t stream) {
  clear_error();
  bl_status st = check_gsrb(phi, f);
  if (st != BL_OK) return st;
  if (!out_host) return fail(BL_EINVAL, "NULL output");
  const Plan& p = *phi->plan;
  if ((st = ensure_scratch(phi, reduce_slots(p) + 8, 8)) != BL_OK) return st;
  double* dout = phi->dscratch + reduce_slots(p);
  BL_HIP(residual_norm_dev(p, phi, f, h2, phi->dscratch, dout, stream));
  BL_HIP(hipMemcpyAsync(phi->hres, dout, sizeof(double), hipMemcpyDeviceToHost, stream));
  BL_HIP(hipStreamSynchronize(stream));
  *out_host = phi->hres[0];
  return BL_OK;
}

// nsweeps red-black sweeps of phi in place, no norms: the fused passes where the
// plan allows them (the first reads x-face neighbours from the neighbours' rows
// and leaves the edge mirrors current), else a fill before each colour.
static hipError_t gsrb_smooth(const Plan& p, void* phi, const void* f, double h2, int nsweeps, hipStream_t stream) {
  if (nsweeps <= 0) return hipSuccess;
  hipError_t e = hipSuccess;
  if (gsrb_fused_ok(p, block_of(p))) {
    const int grid = persistent_grid(tile_config().persist);
    for (int s = 0; s < nsweeps && e == hipSuccess; ++s) {
      e = launch_gsrb_fused(p, phi, f, h2, 0, 0, nullptr, grid, block_of(p), stream, s == 0);
      if (e == hipSuccess) e = launch_gsrb_fused(p, phi, f, h2, 1, 1, nullptr, grid, block_of(p), stream);
    }
    return e;
  }
  for (int s = 0; s < nsweeps && e == hipSuccess; ++s)
    for (int color = 0; color < 2 && e == hipSuccess; ++color) {
      e = launch_fill(p, phi, 0, 1, stream);
      if (e == hipSuccess) e = launch_gsrb(p, phi, f, h2, color, block_of(p), stream);
    }
  return e;
}

// ||f + L_h phi||_2 of the level into *out (device); partials needs
// max(#linear tiles, #tiles) doubles.
static hipError_t residual_norm_dev(const Plan& p, void* phi, const void* f, double h2, double* partials,
                                    double* out, hipStream_t stream) {
  hipError_t e;
  if (gsrb_fused_ok(p, block_of(p))) {
    const int grid = persistent_grid(tile_config().persist);
    if ((e = launch_gsrb_fused(p, phi, f, h2, -1, 2, partials, grid, block_of(p), stream, true)) != hipSuccess)
      return e;
    return launch_reduce_partials(partials, gsrb_fused_grid(p, grid), 1, out, stream);
  }
  if ((e = launch_fill(p, phi, 0, 1, stream)) != hipSuccess) return e;
  return launch_residual(p, phi, f, h2, partials, out, block_of(p), stream);
}

// The red-black sweep's form: the one-pass sweep where it applies (default) or
// always the two colour passes; planes per workgroup (0: 32, halved down to 8
// while the level has fewer than 256 chunks) and vectors per lane (0: chosen
// from the largest plane) of the one-pass sweep.
static std::atomic<int> g_gsrb_one_pass{1}, g_gsrb_zchunk{0}, g_gsrb_vpl{0};

// The one-pass sweep's work chunks for the current configuration; false if
// some box does not fit it: an x extent that is not a whole number of 16-byte
// vectors, planes of more than 1024 lanes' vectors, more ghost items per plane
// (two ghost rows of vectors, two columns of values) or edge-column values (4
// per row) than lanes, or three plane buffers beyond one workgroup's LDS.
static bool gsrb1_plan(Plan& p) {
  std::lock_guard<std::mutex> lk(g_vc_mu);
  const int zreq = g_gsrb_zchunk.load(), want_k = g_gsrb_vpl.load();
  if (p.sweep_req_zc == zreq && p.sweep_req_k == want_k) return p.sweep_ok != 0;
  p.sweep_req_zc = zreq;
  p.sweep_req_k = want_k;
  p.sweep_ok = 0;
  const int V = 16 / p.esize;
  int pmax = 0;
  for (const Box& b : p.boxes) {
    if (b.len(0) % V) return false;
    pmax = std::max(pmax, b.len(1) * (b.len(0) / V));
  }
  if (pmax == 0) return false;
  int zc = zreq;
  if (zc == 0) {
    auto chunks = [&](int z) {
      int64_t n = 0;
      for (const Box& b : p.boxes) n += (b.len(2) + z - 1) / z;
      return n;
    };
    zc = 32;
    while (zc > 8 && chunks(zc) < 256) zc /= 2;
  }
  const int k = want_k > 0 ? want_k : (pmax <= 512 ? 1 : 2);
  if (k != 1 && k != 2) return false;
  const int block = ((pmax + k - 1) / k + 63) / 64 * 64;
  if (block > 1024) return false;
  size_t lds = 0;
  for (const Box& b : p.boxes) {
    if (2 * (b.len(0) / V) + 2 * b.len(1) > block || 4 * b.len(1) > block) return false;
    lds = std::max(lds, gsrb_sweep_lds(b.len(0), b.len(1), V, p.esize));
  }
  if (lds > mg_bottom_lds_limit()) return false;
  // chunks of zc planes; the chunks of 8 boxes at a time dealt out so that a
  // box's chunks run on one XCD (workgroups go to the XCDs in turn) and share
  // its L2 for the planes where they overlap
  std::vector<DevRedChunk> w;
  const int nb = (int)p.boxes.size();
  for (int g0 = 0; g0 < nb; g0 += 8) {
    const int g1 = std::min(nb, g0 + 8);
    int maxc = 0;
    for (int b = g0; b < g1; ++b) maxc = std::max(maxc, (p.boxes[b].len(2) + zc - 1) / zc);
    for (int j = 0; j < maxc; ++j)
      for (int b = g0; b < g1; ++b) {
        const int ez = p.boxes[b].len(2);
        if (j * zc < ez) w.push_back(DevRedChunk{b, j * zc, std::min(ez, (j + 1) * zc), 0});
      }
  }
  (void)hipFree(p.dsweep);
  p.dsweep = nullptr;
  if (upload(&p.dsweep, w, "hipMalloc/hipMemcpy(sweep chunks)") != BL_OK) return false;
  p.hsweep.swap(w);
  p.sweep_zc = zc;
  p.sweep_k = k;
  p.sweep_block = block;
  p.sweep_lds = lds;
  p.sweep_ok = 1;
  return true;
}

// nsweeps sweeps in one pass each, ping-ponging between phi and a second buffer
// of its layout (copied back after an odd count).  FillBoundary of phi once;
// per sweep the ring kernel (new red values into the face ghosts), then the
// sweep into the other buffer, which also writes both its edge copies and fills
// its face ghosts.  Norms: the black part of sweep s plus the red part of sweep
// s+1; after the last sweep, the residual norm of the result.
static bl_status gsrb_one_pass(Plan& p, bl_multifab* phi, const bl_multifab* f, double h2, int nsweeps,
                               double* resnorm_host, hipStream_t stream, bool edges_current = false,
                               bool ghosts_current = false) {
  bool fresh = false;
  if (!phi->dtwin) {
    BL_HIP(hipMalloc(&phi->dtwin, phi->bytes));
    fresh = true;
  }
  const size_t m2bytes = ((size_t)p.mir2_total * p.esize + 255) / 256 * 256;
  if (!phi->dmir2) BL_HIP(hipMalloc(&phi->dmir2, 2 * m2bytes));
  const int nw = (int)p.hsweep.size();
  double* slots = nullptr;
  double* norms = nullptr;
  if (resnorm_host) {
    bl_status st = ensure_scratch(phi, 3 * (size_t)nw + reduce_slots(p) + (size_t)nsweeps + 8, (size_t)nsweeps + 8);
    if (st != BL_OK) return st;
    slots = phi->dscratch;
    norms = phi->dscratch + 3 * (size_t)nw + reduce_slots(p);
  }
  void* buf[2] = {phi->data, phi->dtwin};
  void* m2[2] = {phi->dmir2, static_cast<char*>(phi->dmir2) + m2bytes};
  // both edge-column copies of the starting state, unless the caller knows them
  // current (the previous call on this state was a one-pass call of an even count)
  if (!edges_current) BL_HIP(launch_extract_edges2(p, phi->data, m2[0], stream));
  bl_multifab* fm = const_cast<bl_multifab*>(f);  // f's values are not changed: only its edge mirror is written
  if (!fm->mirror_current) {
    BL_HIP(launch_extract_mirror(p, fm->data, stream));
    fm->mark_mirror(true);
  }
  // ghost cells no box covers keep their values in both buffers (and a new
  // second buffer starts as a copy, so that it holds no undefined values)
  if (fresh || !p.faces_covered)
    BL_HIP(hipMemcpyAsync(phi->dtwin, phi->data, phi->bytes, hipMemcpyDeviceToDevice, stream));
  // the face ghosts of the starting state, unless the caller knows them current
  // (the previous call on this state was a one-pass call: its last sweep pushed
  // them; the sweeps read no edge or corner ghost)
  if (!ghosts_current) BL_HIP(launch_fill(p, phi->data, 0, 1, stream, true));
  for (int s = 0; s < nsweeps; ++s) {
    const int c = s & 1;
    BL_HIP(launch_gsrb_ring(p, buf[c], f->data, m2[c], h2, stream));
    double* red = slots && s > 0 ? slots + nw : nullptr;
    double* black = slots ? slots + (s & 1 ? 2 * nw : 0) : nullptr;
    BL_HIP(launch_gsrb_sweep(p, p.dsweep, nw, p.sweep_block, p.sweep_k, p.sweep_lds, buf[c], buf[c ^ 1], f->data,
                             m2[c ^ 1], h2, red, black, stream));
    if (slots && s > 0)
      BL_HIP(launch_reduce_partials(slots + ((s - 1) & 1 ? nw : 0), 2 * nw, 1, norms + s - 1, stream));
  }
  if (nsweeps & 1) BL_HIP(hipMemcpyAsync(phi->data, phi->dtwin, phi->bytes, hipMemcpyDeviceToDevice, stream));
  phi->mark_mirror(true);
  if (slots) {
    BL_HIP(residual_norm_dev(p, phi, f, h2, slots + 3 * nw, norms + nsweeps - 1, stream));
    BL_HIP(hipMemcpyAsync(phi->hres, norms, sizeof(double) * nsweeps, hipMemcpyDeviceToHost, stream));
    BL_HIP(hipStreamSynchronize(stream));
    std::memcpy(resnorm_host, phi->hres, sizeof(double) * nsweeps);
  }
  return BL_OK;
}

bl_status bl_gsrb_sweeps(bl_multifab* phi, const bl_multifab* f, double h2, int32_t nsweeps, double* resnorm_host,
                         hipStream_t stream) {
  clear_error();
  bl_status st = check_gsrb(phi, f);
  if (st != BL_OK) return st;
  if (nsweeps < 0) return fail(BL_EINVAL, "nsweeps < 0");
  if (nsweeps > 0 && g_gsrb_one_pass.load() && gsrb1_plan(*phi->plan))
    return gsrb_one_pass(*phi->plan, phi, f, h2, nsweeps, resnorm_host, stream);
  const Plan& p = *phi->plan;
  const size_t nt = p.htiles.size();
  if (gsrb_fused_ok(p, block_of(p))) {
    // fused form: no FillBoundary; each colour pass reads the neighbour boxes
    // through the face records.  The norm after sweep s is the black cells'
    // part, taken in its black pass, plus the red cells' part, taken in the
    // red pass of sweep s+1 (after the last sweep: a pass that only reads).
    const int grid = persistent_grid(tile_config().persist);
    const size_t g = (size_t)gsrb_fused_grid(p, grid);
    if (resnorm_host && (st = ensure_scratch(phi, 2 * g + (size_t)nsweeps + 8, (size_t)nsweeps + 8)) != BL_OK)
      return st;
    double* red_part = resnorm_host ? phi->dscratch : nullptr;
    double* black_part = resnorm_host ? phi->dscratch + g : nullptr;
    double* norms = resnorm_host ? phi->dscratch + 2 * g : nullptr;
    // the edge mirror of the starting state first, unless it is current: over
    // many sweeps one extraction costs less than a first pass reading the
    // neighbours' rows
    if (nsweeps > 0 && !phi->mirror_current) BL_HIP(launch_extract_mirror(p, phi->data, stream));
    if (nsweeps > 0) phi->mark_mirror(true);  // every colour pass writes it
    for (int s = 0; s < nsweeps; ++s) {
      BL_HIP(launch_gsrb_fused(p, phi->data, f->data, h2, 0, 0, s > 0 ? red_part : nullptr, grid, block_of(p),
                               stream));
      if (resnorm_host && s > 0) BL_HIP(launch_reduce_partials(phi->dscratch, (int)(2 * g), 1, norms + s - 1, stream));
      BL_HIP(launch_gsrb_fused(p, phi->data, f->data, h2, 1, 1, black_part, grid, block_of(p), stream));
    }
    if (resnorm_host && nsweeps > 0) {
      BL_HIP(launch_gsrb_fused(p, phi->data, f->data, h2, -1, 0, red_part, grid, block_of(p), stream));
      BL_HIP(launch_reduce_partials(phi->dscratch, (int)(2 * g), 1, norms + nsweeps - 1, stream));
      BL_HIP(hipMemcpyAsync(phi->hres, norms, sizeof(double) * nsweeps, hipMemcpyDeviceToHost, stream));
      BL_HIP(hipStreamSynchronize(stream));
      std::memcpy(resnorm_host, phi->hres, sizeof(double) * nsweeps);
    }
    return BL_OK;
  }
  if (resnorm_host && (st = ensure_scratch(phi, nt + (size_t)nsweeps + 8, (size_t)nsweeps + 8)) != BL_OK) return st;
  if (nsweeps > 0) phi->mark_mirror(false);  // the colour passes of this form do not write it
  for (int s = 0; s < nsweeps; ++s) {
    for (int color = 0; color < 2; ++color) {
      BL_HIP(launch_fill(p, phi->data, 0, 1, stream));
      BL_HIP(launch_gsrb(p, phi->data, f->data, h2, color, block_of(p), stream));
    }
    if (resnorm_host) {
      BL_HIP(launch_fill(p, phi->data, 0, 1, stream));
      BL_HIP(launch_residual(p, phi->data, f->data, h2, phi->dscratch, phi->dscratch + nt + s, block_of(p), stream));
    }
  }
  if (resnorm_host && nsweeps > 0) {
    BL_HIP(hipMemcpyAsync(phi->hres, phi->dscratch + nt, sizeof(double) * nsweeps, hipMemcpyDeviceToHost, stream));
    BL_HIP(hipStreamSynchronize(stream));
    std::memcpy(resnorm_host, phi->hres, sizeof(double) * nsweeps);
  }
  return BL_OK;
}

bl_status bl_set_gsrb_config(int32_t one_pass, int32_t zchunk, int32_t vectors_per_lane) {
  clear_error();
  if (zchunk < 0) return fail(BL_EINVAL, "zchunk must be >= 0 (0: chosen per level)");
  if (vectors_per_lane < 0 || vectors_per_lane > 2) return fail(BL_EINVAL, "vectors_per_lane must be 0, 1 or 2");
  g_gsrb_one_pass = one_pass ? 1 : 0;
  g_gsrb_zchunk = zchunk;
  g_gsrb_vpl = vectors_per_lane;
  return BL_OK;
}

bl_status bl_get_gsrb_config(int32_t* one_pass, int32_t* zchunk, int32_t* vectors_per_lane) {
  clear_error();
  if (!one_pass || !zchunk || !vectors_per_lane) return fail(BL_EINVAL, "NULL argument");
  *one_pass = g_gsrb_one_pass.load();
  *zchunk = g_gsrb_zchunk.load();
  *vectors_per_lane = g_gsrb_vpl.load();
  return BL_OK;
}

bl_status bl_gsrb_one_pass_applies(const bl_multifab* phi, int32_t* applies) {
  clear_error();
  if (!phi || !applies) return fail(BL_EINVAL, "NULL argument");
  *applies = (g_gsrb_one_pass.load() && phi->plan->ncomp == 1 && phi->plan->ng >= 1 && gsrb1_plan(*phi->plan)) ? 1 : 0;
  return BL_OK;
}

// ---------------------------------------------------------------- multigrid
// fine and coarse: single-component MultiFabs of one dtype, coarse on the fine
// BoxArray coarsened by 2 (box by box)
static bl_status check_transfer(const bl_multifab* fine, const bl_multifab* coarse) {
  if (!fine || !coarse) return fail(BL_EINVAL, "NULL MultiFab");
  const Plan& F = *fine->plan;
  const Plan& C = *coarse->plan;
  if (F.dtype != C.dtype) return fail(BL_EDTYPE, "fine and coarse MultiFabs differ in dtype");
  if (F.ncomp != 1 || C.ncomp != 1) return fail(BL_EINVAL, "the grid transfers act on single-component MultiFabs");
  if (F.boxes.size() != C.boxes.size()) return fail(BL_ESHAPE, "coarse BoxArray has another number of boxes");
  for (size_t b = 0; b < F.boxes.size(); ++b)
    for (int d = 0; d < 3; ++d) {
      const Box& fb = F.boxes[b];
      const Box& cb = C.boxes[b];
      if (fb.lo[d] % 2 || fb.len(d) % 2 || cb.lo[d] * 2 != fb.lo[d] || (cb.hi[d] + 1) * 2 != fb.hi[d] + 1)
        return fail(BL_ESHAPE, "box %zu of the coarse BoxArray is not box %zu of the fine one coarsened by 2", b, b);
    }
  if (F.hpairpre.empty() || C.hcellpre.empty()) return fail(BL_EINVAL, "too many cells for the grid transfers");
  return BL_OK;
}

bl_status bl_mg_restrict_residual(bl_multifab* phi, const bl_multifab* f, double h2, bl_multifab* fc,
                                  hipStream_t stream) {
  clear_error();
  bl_status st = same_shape(phi, f);
  if (st != BL_OK) return st;
  if ((st = check_transfer(phi, fc)) != BL_OK) return st;
  if (phi->plan->ng < 1) return fail(BL_EINVAL, "the residual needs nghost >= 1");
  if (fc->data == phi->data || fc->data == f->data) return fail(BL_EINVAL, "fc shares storage with phi or f");
  BL_HIP(launch_fill(*phi->plan, phi->data, 0, 1, stream, phi->mirror_current));
  fc->mark_mirror(false);
  BL_HIP(launch_restrict_residual(*phi->plan, *fc->plan, phi->data, f->data, fc->data, h2, stream));
  return BL_OK;
}

bl_status bl_mg_prolong_add(bl_multifab* phi, const bl_multifab* pc, hipStream_t stream) {
  clear_error();
  bl_status st = check_transfer(phi, pc);
  if (st != BL_OK) return st;
  if (pc->data == phi->data) return fail(BL_EINVAL, "pc shares storage with phi");
  phi->mark_mirror(false);
  BL_HIP(launch_prolong_add(*phi->plan, *pc->plan, phi->data, pc->data, stream));
  return BL_OK;
}

}  // extern "C"

struct bl_mg {
  uint64_t ba_uid = 0;
  int dtype = 0;
  int bottom = -1;     // first level of the fused bottom (levels bottom.. in one workgroup), -1: none
  bl::MgBottom mb{};   // its levels' extents, corners and LDS offsets
  std::vector<bl_boxarray*> ba;     // levels 1..: owned coarse BoxArrays (ba[0] unused)
  std::vector<bl_multifab*> phi, f; // levels 1..: in the caller's workspace (index 0 unused)
  // per level, during bl_mg_vcycles: phi's edge-column copies hold its current
  // state (its last write was a one-pass smoothing call of an even count)
  std::vector<char> edges;
  // per level, during bl_mg_vcycles: phi's covered face ghosts hold its current
  // state (its last write was a one-pass smoothing call, whose last sweep
  // pushed them)
  std::vector<char> ghosts;
  ~bl_mg() {
    for (bl_multifab* m : phi) bl_multifab_destroy(m);
    for (bl_multifab* m : f) bl_multifab_destroy(m);
    for (bl_boxarray* b : ba) bl_boxarray_destroy(b);
  }
};

namespace bl {
// The coarse levels of ba: coarsened by 2 while every box and the domain have
// even corners and extents and every periodic axis keeps an even extent, up to
// max_levels levels in all.  levels[0] is left null (the caller's BoxArray).
static bl_status mg_levels(const bl_boxarray* ba, int max_levels, std::vector<bl_boxarray*>* levels) {
  levels->assign(1, nullptr);
  const bl_boxarray* cur = ba;
  while ((int)levels->size() < max_levels) {
    bool ok = true;
    auto even = [](const Box& b) {
      for (int d = 0; d < 3; ++d)
        if (b.lo[d] % 2 || b.len(d) % 2) return false;
      return true;
    };
    ok = even(cur->domain);
    for (size_t i = 0; ok && i < cur->boxes.size(); ++i) ok = even(cur->boxes[i]);
    for (int d = 0; ok && d < 3; ++d)
      if (cur->periodic[d] && (cur->domain.len(d) / 2) % 2) ok = false;
    if (!ok) break;
    bl_boxarray* c = nullptr;
    bl_status st = bl_boxarray_coarsen(cur, 2, &c);
    if (st != BL_OK) {
      for (bl_boxarray* b : *levels) bl_boxarray_destroy(b);
      levels->clear();
      return st;
    }
    levels->push_back(c);
    cur = c;
  }
  return BL_OK;
}

static size_t mg_round(size_t n) { return (n + 255) & ~(size_t)255; }

// A level's boxes cover its whole domain, which is periodic on every axis: its
// FillBoundary is then the periodic wrap of a dense array's index.
static bool covers_periodic_domain(const bl_boxarray* ba) {
  for (int d = 0; d < 3; ++d)
    if (!ba->periodic[d]) return false;
  int64_t v = 0;
  for (const Box& b : ba->boxes) v += b.volume();
  return v == ba->domain.volume();  // the boxes are disjoint and inside the domain
}
static void mg_plan_bottom(const bl_boxarray* ba0, bl_mg* mg);
}  // namespace bl

extern "C" {

bl_status bl_mg_workspace_bytes(const bl_boxarray* ba, bl_dtype dtype, int32_t max_levels, size_t* bytes,
                                int32_t* nlevels) {
  clear_error();
  if (!ba || !bytes) return fail(BL_EINVAL, "NULL argument");
  if (max_levels < 1) return fail(BL_EINVAL, "max_levels %d < 1", max_levels);
  if (dtype != BL_F64 && dtype != BL_F32) return fail(BL_EDTYPE, "unknown dtype %d", (int)dtype);
  std::vector<bl_boxarray*> lv;
  bl_status st = mg_levels(ba, max_levels, &lv);
  if (st != BL_OK) return st;
  size_t total = 0;
  for (size_t l = 1; l < lv.size() && st == BL_OK; ++l) {
    size_t b = 0;
    st = bl_multifab_bytes(lv[l], 1, 1, dtype, &b);
    total += 2 * mg_round(b);
  }
  for (bl_boxarray* b : lv) bl_boxarray_destroy(b);
  if (st != BL_OK) return st;
  *bytes = total;
  if (nlevels) *nlevels = (int32_t)lv.size();
  return BL_OK;
}

bl_status bl_mg_create(const bl_boxarray* ba, bl_dtype dtype, int32_t max_levels, void* work_dev, size_t bytes,
                       bl_mg** out) {
  clear_error();
  if (!ba || !out) return fail(BL_EINVAL, "NULL argument");
  *out = nullptr;
  size_t need = 0;
  int32_t nl = 0;
  bl_status st = bl_mg_workspace_bytes(ba, dtype, max_levels, &need, &nl);
  if (st != BL_OK) return st;
  if (need > 0 && !work_dev) return fail(BL_EINVAL, "NULL workspace");
  if (((uintptr_t)work_dev) % 256 != 0) return fail(BL_EINVAL, "workspace is not 256-byte aligned");
  if (bytes < need) return fail(BL_ENOMEM, "workspace of %zu bytes, the hierarchy needs %zu", bytes, need);
  std::unique_ptr<bl_mg> mg(new (std::nothrow) bl_mg);
  if (!mg) return fail(BL_ENOMEM, "host allocation");
  mg->ba_uid = ba->uid;
  mg->dtype = dtype;
  if ((st = mg_levels(ba, max_levels, &mg->ba)) != BL_OK) return st;
  mg->phi.assign(1, nullptr);
  mg->f.assign(1, nullptr);
  char* w = static_cast<char*>(work_dev);
  for (size_t l = 1; l < mg->ba.size(); ++l) {
    size_t b = 0;
    if ((st = bl_multifab_bytes(mg->ba[l], 1, 1, dtype, &b)) != BL_OK) return st;
    b = mg_round(b);
    bl_multifab* p = nullptr;
    bl_multifab* q = nullptr;
    if ((st = bl_multifab_create(mg->ba[l], nullptr, 1, 1, dtype, w, b, &p)) != BL_OK) return st;
    mg->phi.push_back(p);
    if ((st = bl_multifab_create(mg->ba[l], nullptr, 1, 1, dtype, w + b, b, &q)) != BL_OK) return st;
    mg->f.push_back(q);
    w += 2 * b;
  }
  mg_plan_bottom(ba, mg.get());
  *out = mg.release();
  return BL_OK;
}

bl_status bl_mg_bottom_level(const bl_mg* mg, int32_t* level) {
  clear_error();
  if (!mg || !level) return fail(BL_EINVAL, "NULL argument");
  *level = mg->bottom;
  return BL_OK;
}

bl_status bl_mg_levels(const bl_mg* mg, int32_t* nlevels) {
  clear_error();
  if (!mg || !nlevels) return fail(BL_EINVAL, "NULL argument");
  *nlevels = (int32_t)mg->ba.size();
  return BL_OK;
}

void bl_mg_destroy(bl_mg* mg) { delete mg; }

}  // extern "C"

namespace bl {
// The fused bottom: the finest level L from which every level covers a fully
// periodic domain and all of L.. fit one workgroup's LDS (phi and f of each).
static void mg_plan_bottom(const bl_boxarray* ba0, bl_mg* mg) {
  const int nl = (int)mg->ba.size();
  const int esize = mg->dtype == BL_F64 ? 8 : 4;
  const size_t limit = mg_bottom_lds_limit();
  mg->bottom = -1;
  size_t need = 0;
  for (int l = nl - 1; l >= 0; --l) {
    const bl_boxarray* ba = l == 0 ? ba0 : mg->ba[l];
    if (!covers_periodic_domain(ba) || nl - l > kMgBottomMaxLevels) break;
    need += 2 * (size_t)ba->domain.volume() * esize;
    if (need > limit) break;
    mg->bottom = l;
  }
  if (mg->bottom < 0) return;
  MgBottom& m = mg->mb;
  m.nlev = nl - mg->bottom;
  int off = 0;
  for (int i = 0; i < m.nlev; ++i) {
    const int l = mg->bottom + i;
    const bl_boxarray* ba = l == 0 ? ba0 : mg->ba[l];
    for (int d = 0; d < 3; ++d) {
      m.n[i][d] = ba->domain.len(d);
      m.lo[i][d] = ba->domain.lo[d];
    }
    m.off[i] = off;
    off += 2 * (int)ba->domain.volume();
  }
}

// nu smoothing sweeps on level l: the one-pass form where it applies on levels
// of at least kMgOnePassCells cells and nu is even (the result then lands in phi
// itself and its edge copies stay current), else the two colour passes.
constexpr int64_t kMgOnePassCells = 4 << 20;
static bl_status mg_smooth(bl_mg* mg, size_t l, bl_multifab* phi, const bl_multifab* f, double h2, int nu,
                           hipStream_t stream) {
  Plan& p = *phi->plan;
  int64_t cells = 0;
  for (const Box& b : p.boxes) cells += b.volume();
  if (nu > 0 && nu % 2 == 0 && cells >= kMgOnePassCells && g_gsrb_one_pass.load() && gsrb1_plan(p)) {
    bl_status st = gsrb_one_pass(p, phi, f, h2, nu, nullptr, stream, mg->edges[l] != 0, mg->ghosts[l] != 0);
    mg->edges[l] = mg->ghosts[l] = st == BL_OK;
    return st;
  }
  mg->edges[l] = mg->ghosts[l] = 0;
  BL_HIP(gsrb_smooth(p, phi->data, f->data, h2, nu, stream));
  return BL_OK;
}

// One V-cycle from level l (phi, f the level's MultiFabs, h2 its spacing squared).
static bl_status vcycle(bl_mg* mg, size_t l, bl_multifab* phi, const bl_multifab* f, double h2, int nu1, int nu2,
                        int nu_bottom, hipStream_t stream) {
  const Plan& p = *phi->plan;
  if ((int)l == mg->bottom && p.dcellpre) {  // this level and every coarser one in one workgroup
    BL_HIP(launch_mg_bottom(p, phi->data, f->data, mg->mb, h2, l == 0 ? 1 : 0, nu1, nu2, nu_bottom, stream));
    return BL_OK;
  }
  if (l + 1 == mg->ba.size()) {
    BL_HIP(gsrb_smooth(p, phi->data, f->data, h2, nu_bottom, stream));
    return BL_OK;
  }
  bl_status st = mg_smooth(mg, l, phi, f, h2, nu1, stream);
  if (st != BL_OK) return st;
  bl_multifab* pc = mg->phi[l + 1];
  bl_multifab* fc = mg->f[l + 1];
  // the residual reads face ghosts only: current after a one-pass smoothing
  if (!mg->ghosts[l]) BL_HIP(launch_fill(p, phi->data, 0, 1, stream));
  BL_HIP(launch_restrict_residual(p, *fc->plan, phi->data, f->data, fc->data, h2, stream));
  fc->mark_mirror(false);
  // the coarse level starts from 0 (the fused bottom sets it itself)
  if ((int)(l + 1) != mg->bottom) BL_HIP(launch_set_val(*pc->plan, pc->data, 0.0, 0, 1, 1, 256, stream));
  mg->edges[l + 1] = mg->ghosts[l + 1] = 0;
  st = vcycle(mg, l + 1, pc, fc, 4.0 * h2, nu1, nu2, nu_bottom, stream);
  if (st != BL_OK) return st;
  BL_HIP(launch_prolong_add(p, *pc->plan, phi->data, pc->data, stream));
  mg->edges[l] = mg->ghosts[l] = 0;
  return mg_smooth(mg, l, phi, f, h2, nu2, stream);
}
}  // namespace bl

extern "C" {

bl_status bl_mg_vcycles(bl_mg* mg, bl_multifab* phi, const bl_multifab* f, double h2, int32_t ncycles, int32_t nu1,
                        int32_t nu2, int32_t nu_bottom, double* resnorm_host, hipStream_t stream) {
  clear_error();
  if (!mg) return fail(BL_EINVAL, "NULL hierarchy");
  bl_status st = check_gsrb(phi, f);
  if (st != BL_OK) return st;
  if (phi->plan->ba_uid != mg->ba_uid) return fail(BL_ESHAPE, "phi lives on another BoxArray than the hierarchy");
  if (phi->plan->dtype != mg->dtype) return fail(BL_EDTYPE, "phi's dtype differs from the hierarchy's");
  if (phi->plan->ng != 1) return fail(BL_EINVAL, "the hierarchy's levels have one ghost layer; phi needs nghost 1");
  if (ncycles < 0 || nu1 < 0 || nu2 < 0 || nu_bottom < 0) return fail(BL_EINVAL, "negative count");
  const Plan& p = *phi->plan;
  const size_t slots = reduce_slots(p) + 8;
  if (resnorm_host && (st = ensure_scratch(phi, slots + (size_t)ncycles, (size_t)ncycles + 8)) != BL_OK) return st;
  mg->edges.assign(mg->phi.size(), 0);  // nothing known of the levels' edge copies and ghosts at the start
  mg->ghosts.assign(mg->phi.size(), 0);
  for (int c = 0; c < ncycles; ++c) {
    if ((st = vcycle(mg, 0, phi, f, h2, nu1, nu2, nu_bottom, stream)) != BL_OK) return st;
    if (resnorm_host)
      BL_HIP(residual_norm_dev(p, phi->data, f->data, h2, phi->dscratch, phi->dscratch + slots + c, stream));
  }
  if (ncycles > 0) phi->mark_mirror(false);  // conservatively: prolongation writes phi without its mirror
  if (resnorm_host && ncycles > 0) {
    BL_HIP(hipMemcpyAsync(phi->hres, phi->dscratch + slots, sizeof(double) * ncycles, hipMemcpyDeviceToHost, stream));
    BL_HIP(hipStreamSynchronize(stream));
    std::memcpy(resnorm_host, phi->hres, sizeof(double) * ncycles);
  }
  return BL_OK;
}

bl_status bl_device_copy(void* dst, const void* src, size_t bytes, hipStream_t stream) {
  clear_error();
  if (bytes == 0) return BL_OK;
  if (!dst || !src) return fail(BL_EINVAL, "NULL pointer");
  if (((uintptr_t)dst | (uintptr_t)src | bytes) % 16 != 0)
    return fail(BL_EINVAL, "pointers and size must be multiples of 16 bytes");
  const uintptr_t d = (uintptr_t)dst, s0 = (uintptr_t)src;
  if (d < s0 + bytes && s0 < d + bytes) return fail(BL_EINVAL, "source and destination overlap");
  if (bytes / 16 / 256 >= (size_t)UINT32_MAX) return fail(BL_EINVAL, "copy too large for one launch");
  BL_HIP(launch_copy16(dst, src, bytes, stream));
  return BL_OK;
}

bl_status bl_set_tile_config(int32_t zchunk, int32_t waves, int32_t persist, int32_t block, int32_t zsteps) {
  clear_error();
  if (zchunk < 1 || zchunk > 16384 || waves < 1 || waves > kStencilMaxThreads / 64 || persist < 0 ||
      persist > 64 || block < 0 || block > 3 || zsteps < 1 || zsteps > 64)
    return fail(BL_EINVAL,
                "need 1 <= zchunk <= 16384, 1 <= waves <= %d, 0 <= persist <= 64, block in {0, 1, 2, 3}, "
                "1 <= zsteps <= 64",
                kStencilMaxThreads / 64);
  if (block && zchunk != 2 && zchunk != 4 && zchunk != 8)
    return fail(BL_EINVAL, "the block form needs zchunk 2, 4 or 8");
  TileConfig& c = tile_config();
  c.zchunk = zchunk;
  c.waves = waves;
  c.persist = persist;
  c.block = block;
  c.zsteps = zsteps;
  std::lock_guard<std::mutex> lk(g_plan_mu);
  g_tuned.clear();  // an explicit choice replaces earlier autotuned ones
  return BL_OK;
}

bl_status bl_autotune(const bl_boxarray* ba, bl_multifab* u0, bl_multifab* u1, double c, int32_t trial_steps,
                      int32_t max_results, int32_t* nresults, int32_t* configs, float* ms_per_step,
                      int32_t best[5], hipStream_t stream) {
  clear_error();
  if (!ba) return fail(BL_EINVAL, "NULL BoxArray");
  bl_status st = check_heat(u0, u1);
  if (st != BL_OK) return st;
  if (u0->plan->ba_uid != ba->uid) return fail(BL_ESHAPE, "the MultiFabs are not on this BoxArray");
  if (trial_steps < 1 || trial_steps > 1000) return fail(BL_EINVAL, "need 1 <= trial_steps <= 1000");
  if (max_results < 0) return fail(BL_EINVAL, "max_results < 0");
  const Plan& p0 = *u0->plan;
  const int ncomp = p0.ncomp, ng = p0.ng, dtype = p0.dtype;
  const int persist = tile_config().persist;
  std::vector<TileConfig> cands;
  for (int block : {3, 2})
    for (int z : {2, 4, 8})
      for (int w : {2, 3, 4})
        for (int zs : {1, 2, 4, 8})
          if (block == 3 || zs == 1) cands.push_back(TileConfig{z, w, persist, block, zs});
  hipEvent_t e0 = nullptr, e1 = nullptr;
  BL_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(BL_EHIP, "hipEventCreate");
  }
  struct Ev {
    hipEvent_t a, b;
    ~Ev() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  } ev{e0, e1};
  float best_ms = 0.f;
  int best_i = -1;
  std::shared_ptr<Plan> best_plan;
  int nres = 0;
  for (size_t i = 0; i < cands.size(); ++i) {
    const TileConfig& cfg = cands[i];
    std::shared_ptr<Plan> pl;
    if ((st = get_plan_cfg(ba, ncomp, ng, dtype, cfg, true, &pl)) != BL_OK) return st;
    HeatArgs a{pl->dtiles, (int)pl->htiles.size(), pl->dboxes, pl->dfacerecs, member_of(u0, u1, c), nullptr, 0,
               pl->fvec, cfg.zchunk, cfg.block, pl->rmax, pl->nvtmax,
               pl->dlin, (int)pl->hlin.size(), pl->yhmax, pl->xhmax};
    const int grid = persistent_grid(cfg.persist), block = 64 * cfg.waves;
    BL_HIP(launch_extract_mirror(*pl, u0->data, stream));
    for (int s = 0; s < 2; ++s) {  // warm-up; an even count leaves the state in u0
      a.flip = s;
      BL_HIP(launch_heat(dtype, pl->vec, true, a, grid, block, stream));
    }
    BL_HIP(hipEventRecord(e0, stream));
    for (int s = 0; s < 2 * trial_steps; ++s) {
      a.flip = s & 1;
      BL_HIP(launch_heat(dtype, pl->vec, true, a, grid, block, stream));
    }
    BL_HIP(hipEventRecord(e1, stream));
    BL_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    BL_HIP(hipEventElapsedTime(&ms, e0, e1));
    ms /= (float)(2 * trial_steps);
    if (nres < max_results) {
      if (configs) {
        configs[5 * nres + 0] = cfg.zchunk;
        configs[5 * nres + 1] = cfg.waves;
        configs[5 * nres + 2] = cfg.persist;
        configs[5 * nres + 3] = cfg.block;
        configs[5 * nres + 4] = cfg.zsteps;
      }
      if (ms_per_step) ms_per_step[nres] = ms;
      ++nres;
    }
    if (best_i < 0 || ms < best_ms) {
      best_ms = ms;
      best_i = (int)i;
      best_plan = pl;
    }
  }
  if (nresults) *nresults = nres;
  const TileConfig& bc = cands[best_i];
  {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    g_tuned[std::make_tuple(ba->uid, ncomp, ng, dtype)] = bc;
  }
  forget_graphs(u0);
  forget_graphs(u1);
  u0->mark_mirror(false);  // the trial steps overwrote both
  u1->mark_mirror(false);
  u0->plan = best_plan;
  u1->plan = best_plan;
  if (best) {
    best[0] = bc.zchunk;
    best[1] = bc.waves;
    best[2] = bc.persist;
    best[3] = bc.block;
    best[4] = bc.zsteps;
  }
  return BL_OK;
}

bl_status bl_get_tile_config(int32_t* zchunk, int32_t* waves, int32_t* persist, int32_t* block, int32_t* zsteps) {
  clear_error();
  const TileConfig& c = tile_config();
  if (zchunk) *zchunk = c.zchunk;
  if (waves) *waves = c.waves;
  if (persist) *persist = c.persist;
  if (block) *block = c.block;
  if (zsteps) *zsteps = c.zsteps;
  return BL_OK;
}

bl_status bl_fill_plan(const bl_boxarray* cba, int32_t nghost, int32_t* nrec, int32_t* rec) {
  clear_error();
  if (!cba || !nrec) return fail(BL_EINVAL, "NULL argument");
  if (nghost < 0) return fail(BL_EINVAL, "nghost < 0");
  const auto plan = fill_plan(const_cast<bl_boxarray*>(cba), nghost);
  const auto& recs = *plan;
  *nrec = (int32_t)recs.size();
  if (rec)
    for (size_t i = 0; i < recs.size(); ++i) {
      int32_t* r = rec + 11 * i;
      r[0] = recs[i].dst;
      r[1] = recs[i].src;
      for (int d = 0; d < 3; ++d) {
        r[2 + d] = recs[i].region.lo[d];
        r[5 + d] = recs[i].region.hi[d];
        r[8 + d] = recs[i].shift[d];
      }
    }
  return BL_OK;
}

bl_status bl_face_plan(const bl_boxarray* cba, int32_t* nrec, int32_t* rec) {
  clear_error();
  if (!cba || !nrec) return fail(BL_EINVAL, "NULL argument");
  const auto plan = face_plan(const_cast<bl_boxarray*>(cba), 1);
  const auto& recs = *plan;
  *nrec = (int32_t)recs.size();
  if (rec)
    for (size_t i = 0; i < recs.size(); ++i) {
      int32_t* r = rec + 12 * i;
      r[0] = recs[i].box;
      r[1] = recs[i].face;
      r[2] = recs[i].src;
      for (int d = 0; d < 3; ++d) {
        r[3 + d] = recs[i].region.lo[d];
        r[6 + d] = recs[i].region.hi[d];
        r[9 + d] = recs[i].shift[d];
      }
    }
  return BL_OK;
}

bl_status bl_tile_list(const bl_boxarray* ba, int32_t ncomp, int32_t nghost, bl_dtype dtype, int32_t* ntiles,
                       int32_t* tiles) {
  clear_error();
  if (!ba || !ntiles) return fail(BL_EINVAL, "NULL argument");
  if (ncomp < 1 || nghost < 0) return fail(BL_EINVAL, "need ncomp >= 1 and nghost >= 0");
  if (dtype != BL_F64 && dtype != BL_F32) return fail(BL_EDTYPE, "unknown dtype %d", (int)dtype);
  std::shared_ptr<Plan> plan;
  bl_status st = get_plan(ba, ncomp, nghost, dtype, false, &plan);
  if (st != BL_OK) return st;
  const auto& t = plan->htiles;
  *ntiles = (int32_t)t.size();
  if (tiles)
    for (size_t i = 0; i < t.size(); ++i) {
      int32_t* r = tiles + 9 * i;
      r[0] = t[i].box;
      r[1] = t[i].comp;
      r[2] = t[i].xv0;
      r[3] = t[i].nvt;
      r[4] = t[i].y0;
      r[5] = t[i].rows;
      r[6] = t[i].z0;
      r[7] = t[i].z1;
      r[8] = plan->vec;
    }
  return BL_OK;
}

bl_status bl_stencil_tiles(const bl_boxarray* ba, int32_t ncomp, int32_t nghost, bl_dtype dtype, int32_t* ntiles,
                           int32_t* tiles) {
  clear_error();
  if (!ba || !ntiles) return fail(BL_EINVAL, "NULL argument");
  if (ncomp < 1 || nghost < 0) return fail(BL_EINVAL, "need ncomp >= 1 and nghost >= 0");
  if (dtype != BL_F64 && dtype != BL_F32) return fail(BL_EDTYPE, "unknown dtype %d", (int)dtype);
  std::shared_ptr<Plan> plan;
  bl_status st = get_plan(ba, ncomp, nghost, dtype, false, &plan);
  if (st != BL_OK) return st;
  const auto& t = plan->hlin;
  *ntiles = (int32_t)t.size();
  if (tiles)
    for (size_t i = 0; i < t.size(); ++i) {
      int32_t* r = tiles + 11 * i;
      r[0] = t[i].box;
      r[1] = t[i].comp;
      r[2] = t[i].q0;
      r[3] = t[i].nq;
      r[4] = t[i].nzs;
      r[5] = t[i].z0;
      r[6] = t[i].z1;
      r[7] = plan->cfg.zchunk;
      r[8] = plan->vec;
      r[9] = 64 * plan->cfg.waves;
      r[10] = plan->cfg.zsteps;
    }
  return BL_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- batching
struct bl_batch {
  struct Member {
    bl_multifab* u0;
    bl_multifab* u1;
    double c;
    int64_t joined;               // tick of its first step
    int id;
    bool mirrored = false;        // its current state's edge mirror is valid
    std::vector<DevTile> tiles;   // member-local numbering (box, face record, member 0)
    std::vector<DevLinTile> lin;  // the same for the linear-tile form (block form 3)
    int yh = 1, xh = 1;
  };
  // Device table of one kind, grown on demand and refilled in stream order from
  // pinned staging memory, so a rebuild needs no device synchronisation.
  template <typename T>
  struct Table {
    T* dev = nullptr;
    T* host = nullptr;
    size_t cap = 0, n = 0;
    void release() {
      (void)hipFree(dev);
      (void)hipHostFree(host);
      dev = host = nullptr;
      cap = n = 0;
    }
  };
  struct Group {
    int dtype = 0, vec = 1, fvec = 1, rmax = 1, nvtmax = 1;
    std::vector<int> members;  // indices into mems
    Table<DevBox> boxes;
    Table<DevFaceRec> recs;
    Table<DevTile> tiles;
    Table<DevLinTile> lin;
    Table<DevMember> dmembers;
    int yhmax = 1, xhmax = 1;
    hipEvent_t staged = nullptr;  // the last upload from the staging buffers
  };
  std::vector<Member> mems;
  std::vector<Group> groups;
  int next_id = 0;
  int64_t tick = 0;
  bool dirty = true;
  TileConfig cfg;
  bool have_cfg = false;

  ~bl_batch() {
    for (auto& g : groups) {
      if (g.staged) (void)hipEventSynchronize(g.staged);
      g.boxes.release();
      g.recs.release();
      g.tiles.release();
      g.lin.release();
      g.dmembers.release();
      if (g.staged) (void)hipEventDestroy(g.staged);
    }
  }
};

namespace bl {

// Make room for n entries; a device buffer that must grow is replaced after the
// stream has drained (rare: capacities double).
template <typename T>
static bl_status table_reserve(bl_batch::Table<T>& t, size_t n, hipStream_t stream) {
  if (n <= t.cap) return BL_OK;
  size_t cap = std::max<size_t>(n, 2 * t.cap);
  BL_HIP(hipStreamSynchronize(stream));
  (void)hipFree(t.dev);
  (void)hipHostFree(t.host);
  t.dev = nullptr;
  t.host = nullptr;
  t.cap = 0;
  BL_HIP(hipMalloc((void**)&t.dev, cap * sizeof(T)));
  BL_HIP(hipHostMalloc((void**)&t.host, cap * sizeof(T), hipHostMallocDefault));
  t.cap = cap;
  return BL_OK;
}

template <typename T>
static bl_status table_upload(bl_batch::Table<T>& t, hipStream_t stream) {
  if (t.n) BL_HIP(hipMemcpyAsync(t.dev, t.host, t.n * sizeof(T), hipMemcpyHostToDevice, stream));
  return BL_OK;
}

}  // namespace bl

static bl_status batch_rebuild(bl_batch* b, hipStream_t stream) {
  const TileConfig cfg = tile_config();
  const bool cfg_changed = !b->have_cfg || cfg.zchunk != b->cfg.zchunk || cfg.waves != b->cfg.waves ||
                           cfg.block != b->cfg.block || cfg.persist != b->cfg.persist;
  b->cfg = cfg;
  b->have_cfg = true;
  for (auto& m : b->mems)
    if (cfg_changed || m.tiles.empty()) {
      m.tiles.clear();
      m.lin.clear();
      m.yh = m.xh = 1;
      build_tiles(*m.u0->plan, cfg, 0, 0, 0, m.tiles, nullptr);
      if (cfg.block == 3) build_lin_tiles(*m.u0->plan, cfg, 0, 0, 0, m.lin, &m.yh, &m.xh);
    }
  // members grouped by (dtype, vector width): one launch per group
  for (auto& g : b->groups) {
    g.members.clear();
    g.fvec = 1;
  }
  for (size_t i = 0; i < b->mems.size(); ++i) {
    const Plan& p = *b->mems[i].u0->plan;
    bl_batch::Group* g = nullptr;
    for (auto& x : b->groups)
      if (x.dtype == p.dtype && x.vec == p.vec) g = &x;
    if (!g) {
      b->groups.emplace_back();
      g = &b->groups.back();
      g->dtype = p.dtype;
      g->vec = p.vec;
    }
    g->members.push_back((int)i);
    if (!p.fvec) g->fvec = 0;
  }
  for (auto& g : b->groups) {
    size_t nb = 0, nr = 0, nt = 0, nl = 0;
    g.yhmax = g.xhmax = 1;
    bool lin_ok = cfg.block == 3;
    for (int i : g.members) {
      const bl_batch::Member& m = b->mems[i];
      const Plan& p = *m.u0->plan;
      nb += p.hboxes.size();
      nr += p.hfacerecs.size();
      nt += m.tiles.size();
      nl += m.lin.size();
      g.yhmax = std::max(g.yhmax, m.yh);
      g.xhmax = std::max(g.xhmax, m.xh);
      if (m.lin.empty()) lin_ok = false;
    }
    if (lin_ok && lin_lds_bytes(cfg, g.dtype == BL_F64 ? 8 : 4, g.vec, g.yhmax, g.xhmax) > kDmaLdsMax) lin_ok = false;
    if (!lin_ok) nl = 0;
    if (g.staged) BL_HIP(hipEventSynchronize(g.staged));  // staging buffers free again
    bl_status st;
    if ((st = table_reserve(g.boxes, nb, stream)) != BL_OK) return st;
    if ((st = table_reserve(g.recs, nr, stream)) != BL_OK) return st;
    if ((st = table_reserve(g.tiles, nt, stream)) != BL_OK) return st;
    if ((st = table_reserve(g.lin, nl, stream)) != BL_OK) return st;
    if ((st = table_reserve(g.dmembers, g.members.size(), stream)) != BL_OK) return st;
    size_t ob = 0, orr = 0, ot = 0, ol = 0;
    g.rmax = g.nvtmax = 1;
    for (size_t k = 0; k < g.members.size(); ++k) {
      const bl_batch::Member& m = b->mems[g.members[k]];
      const Plan& p = *m.u0->plan;
      const int box_base = (int)ob, rec_base = (int)orr;
      for (DevBox B : p.hboxes) {
        for (int f = 0; f < 6; ++f) B.face_start[f] += rec_base;
        g.boxes.host[ob++] = B;
      }
      for (const DevFaceRec& R : p.hfacerecs) g.recs.host[orr++] = R;
      for (DevTile t : m.tiles) {
        t.box += box_base;
        t.member = (int32_t)k;
        for (int f = 0; f < 6; ++f)
          if (t.frec[f] >= 0) t.frec[f] += rec_base;
        g.rmax = std::max<int>(g.rmax, t.rows);
        g.nvtmax = std::max<int>(g.nvtmax, t.nvt);
        g.tiles.host[ot++] = t;
      }
      if (nl)
        for (DevLinTile t : m.lin) {
          t.box += box_base;
          t.member = (int32_t)k;
          for (int f = 0; f < 6; ++f)
            if (t.frec[f] >= 0) t.frec[f] += rec_base;
          g.lin.host[ol++] = t;
        }
      DevMember dm;
      std::memset(&dm, 0, sizeof dm);
      dm.a = m.u0->data;
      dm.b = m.u1->data;
      dm.c = m.c;
      dm.flip_offset = (int32_t)(m.joined & 1);
      g.dmembers.host[k] = dm;
    }
    g.boxes.n = nb;
    g.recs.n = nr;
    g.tiles.n = nt;
    g.lin.n = nl;
    g.dmembers.n = g.members.size();
    if ((st = table_upload(g.boxes, stream)) != BL_OK) return st;
    if ((st = table_upload(g.recs, stream)) != BL_OK) return st;
    if ((st = table_upload(g.tiles, stream)) != BL_OK) return st;
    if ((st = table_upload(g.lin, stream)) != BL_OK) return st;
    if ((st = table_upload(g.dmembers, stream)) != BL_OK) return st;
    if (!g.staged) BL_HIP(hipEventCreateWithFlags(&g.staged, hipEventDisableTiming));
    BL_HIP(hipEventRecord(g.staged, stream));
  }
  // edge-column mirrors of the newly joined members' current states (the fused
  // kernel keeps every other member's mirror current)
  for (auto& m : b->mems)
    if (!m.mirrored) {
      bl_multifab* cur = ((b->tick - m.joined) & 1) ? m.u1 : m.u0;
      BL_HIP(launch_extract_mirror(*cur->plan, cur->data, stream));
      m.mirrored = true;
    }
  b->dirty = false;
  return BL_OK;
}

extern "C" {

bl_status bl_batch_create(bl_batch** out) {
  clear_error();
  if (!out) return fail(BL_EINVAL, "NULL argument");
  *out = new (std::nothrow) bl_batch;
  if (!*out) return fail(BL_ENOMEM, "host allocation");
  return BL_OK;
}

bl_status bl_batch_add(bl_batch* b, bl_multifab* u0, bl_multifab* u1, double c, int32_t* member_id) {
  clear_error();
  if (!b || !member_id) return fail(BL_EINVAL, "NULL argument");
  bl_status st = check_heat(u0, u1);
  if (st != BL_OK) return st;
  bl_batch::Member m;
  m.u0 = u0;
  m.u1 = u1;
  u0->mark_mirror(false);  // the batch keeps its own record while the pair is a member
  u1->mark_mirror(false);
  m.c = c;
  m.joined = b->tick;
  m.id = b->next_id++;
  b->mems.push_back(std::move(m));
  b->dirty = true;
  *member_id = b->mems.back().id;
  return BL_OK;
}

bl_status bl_batch_remove(bl_batch* b, int32_t member_id) {
  clear_error();
  if (!b) return fail(BL_EINVAL, "NULL batch");
  for (size_t i = 0; i < b->mems.size(); ++i)
    if (b->mems[i].id == member_id) {
      b->mems.erase(b->mems.begin() + i);
      b->dirty = true;
      return BL_OK;
    }
  return fail(BL_EINVAL, "no member %d", member_id);
}

bl_status bl_batch_parity(const bl_batch* b, int32_t member_id, int32_t* steps_done) {
  clear_error();
  if (!b || !steps_done) return fail(BL_EINVAL, "NULL argument");
  for (const auto& m : b->mems)
    if (m.id == member_id) {
      *steps_done = (int32_t)(b->tick - m.joined);
      return BL_OK;
    }
  return fail(BL_EINVAL, "no member %d", member_id);
}

bl_status bl_batch_steps(bl_batch* b, int32_t nsteps, hipStream_t stream) {
  clear_error();
  if (!b) return fail(BL_EINVAL, "NULL batch");
  if (nsteps < 0) return fail(BL_EINVAL, "nsteps < 0");
  bl_status st;
  if (nsteps > 0 && b->dirty && (st = batch_rebuild(b, stream)) != BL_OK) return st;
  for (int32_t s = 0; s < nsteps; ++s) {
    for (auto& g : b->groups) {
      if (g.members.empty()) continue;
      HeatArgs a{g.tiles.dev, (int)g.tiles.n, g.boxes.dev, g.recs.dev, DevMember{}, g.dmembers.dev,
                 (int)(b->tick & 1), g.fvec, b->cfg.block ? b->cfg.zchunk : 0, b->cfg.block, g.rmax, g.nvtmax,
                 g.lin.n ? g.lin.dev : nullptr, (int)g.lin.n, g.yhmax, g.xhmax};
      BL_HIP(launch_heat(g.dtype, g.vec, true, a, persistent_grid(b->cfg.persist), 64 * b->cfg.waves, stream));
    }
    b->tick++;
  }
  return BL_OK;
}

bl_status bl_batch_step(bl_batch* b, hipStream_t stream) { return bl_batch_steps(b, 1, stream); }

void bl_batch_destroy(bl_batch* b) { delete b; }

}  // extern "C"
