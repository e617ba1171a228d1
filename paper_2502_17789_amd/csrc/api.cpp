// C ABI of the A-term IDG library: plan creation (host partition + device
// upload), batched gridding/degridding launches and error reporting.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "aidg_internal.h"

using namespace aidg;

namespace {

thread_local std::string g_last_error;

aidg_status fail(aidg_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

aidg_status hip_fail(hipError_t e, const char* what) {
  return fail(AIDG_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// One library stream per device on which plan memory is returned to the device's
// stream-ordered pool (null if it cannot be created: memory is then freed
// synchronously).  Default priority, non-blocking.
hipStream_t release_stream(int device) {
  static std::mutex mu;
  static std::map<int, hipStream_t> streams;
  std::lock_guard<std::mutex> lock(mu);
  auto it = streams.find(device);
  if (it != streams.end()) return it->second;
  int cur = 0;
  hipStream_t s = nullptr;
  if (hipGetDevice(&cur) == hipSuccess && (cur == device || hipSetDevice(device) == hipSuccess)) {
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      (void)hipGetLastError();
      s = nullptr;
    }
    if (cur != device) (void)hipSetDevice(cur);
  }
  streams[device] = s;
  return s;
}

}  // namespace

struct aidg_plan {
  Geometry g{};
  int n_st = 0, nbl = 0, nt = 0, nc = 0, n_int = 0, W = 1, max_nv = 1, device = 0;
  int64_t n_pervis = 0, n_direct = 0;  // subgrids the degridder takes in these forms
  std::vector<aidg_subgrid> table;
  std::vector<double> w0;
  int64_t n_excluded = 0;
  // Subgrids sharing w-layer and centre are consecutive and form a group;
  // group k holds subgrids [grp_begin[k], grp_begin[k+1]).  sg_group maps a
  // subgrid to its group.  Batches are runs of whole groups: [batch_begin[b],
  // batch_begin[b+1]) in subgrids, at most `batch` groups each.
  std::vector<int64_t> grp_begin, batch_begin;
  std::vector<int32_t> sg_group;
  int64_t batch = 1;
  size_t elem = 8, aterm_bytes = 0, device_bytes = 0, scratch_bytes = 0;
  SubgridDev* d_sg = nullptr;
  double* d_uvw = nullptr;
  double* d_fc = nullptr;
  void* d_aterms = nullptr;
  void* d_taper = nullptr;
  void* d_tw = nullptr;
  void* d_scratch = nullptr;
  int64_t* d_excl = nullptr;
  int64_t* d_grp = nullptr;
  KernelArgs* d_args = nullptr;  // device copy of args()
  // image level (invert / predict): Stockham radices of N, twiddles exp(-2 pi i k / N)
  // and the reciprocal of the taper's axis at image resolution (FP64); absent when N
  // is not supported
  ImageRadices img_fr{};
  bool img_ok = false;
  void* d_img_tw = nullptr;
  double* d_img_itaper = nullptr;
  // inverse A-term mode: (A^-1)^H planes for the gridder, the distinct (A_p plane,
  // A_q plane) pairs of the table [n][2] with their visibility counts, the partial sums
  // [chunks][L^2] and the weighted-average normalisation map [L^2]
  void* d_ainvh = nullptr;
  int32_t* d_npairs = nullptr;
  double* d_ncount = nullptr;
  double* d_npartial = nullptr;
  double* d_nmap = nullptr;
  int64_t n_pairs = 0, pair_chunk = 1;
  int n_chunks = 1;
  double n_total = 0.0;
  hipEvent_t last = nullptr;
  std::atomic<bool> busy{false};
  // profiling: events around each kernel launch
  struct Timed {
    int kind;
    int64_t vp, nsg;
    hipEvent_t a, b;
  };
  bool profiling = false;
  std::vector<hipEvent_t> pool;
  size_t pool_next = 0;
  std::vector<Timed> timed;
  std::vector<int64_t> vp_prefix;  // prefix sums of n_vis * L^2 over the table

  KernelArgs args() const {
    KernelArgs a;
    a.sg = d_sg;
    a.uvw = d_uvw;
    a.fc = d_fc;
    a.aterms = d_aterms;
    a.ainvh = d_ainvh;
    a.taper = d_taper;
    a.twiddle = d_tw;
    a.grp_begin = d_grp;
    a.nt_total = nt;
    a.nc_total = nc;
    a.N = g.N;
    a.npol = g.npol;
    a.du = g.du;
    a.lstep = g.fov / g.L;
    return a;
  }

  // Device memory comes from the device's stream-ordered pool (hipMallocAsync on
  // the creation stream) where the device supports it.  It goes back on a library
  // stream after the plan's last recorded work, so destroying a plan never
  // synchronises the device: a serving loop retires plans while other jobs run.
  bool async_mem = false;

  void release() {
    void* ptrs[] = {d_sg,     d_uvw,       d_fc,    d_aterms,  d_taper,    d_tw,     d_scratch,
                    d_excl,   d_grp,       d_args,  d_img_tw,  d_img_itaper, d_ainvh, d_npairs,
                    d_ncount, d_npartial,  d_nmap};
    hipStream_t fs = async_mem ? release_stream(device) : nullptr;
    int cur = device;
    if (fs) {
      (void)hipGetDevice(&cur);
      if (cur != device) (void)hipSetDevice(device);
      if (last) (void)hipStreamWaitEvent(fs, last, 0);
    }
    for (void* p : ptrs) {
      if (!p) continue;
      if (!fs)
        (void)hipFree(p);
      else if (hipFreeAsync(p, fs) != hipSuccess)
        (void)hipGetLastError();
    }
    if (fs && cur != device) (void)hipSetDevice(cur);
    if (last) (void)hipEventDestroy(last);
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    pool.clear();
    timed.clear();
    d_sg = nullptr;
    d_uvw = d_fc = nullptr;
    d_aterms = d_taper = d_tw = d_scratch = nullptr;
    d_excl = nullptr;
    d_grp = nullptr;
    d_args = nullptr;
    d_img_tw = nullptr;
    d_img_itaper = nullptr;
    d_ainvh = nullptr;
    d_npairs = nullptr;
    d_ncount = d_npartial = d_nmap = nullptr;
    last = nullptr;
  }
};

struct aidg_executor {
  void* d_scratch = nullptr;
  int64_t bytes = 0;
  int device = 0;
  hipEvent_t last = nullptr;
  std::atomic<bool> busy{false};
};

namespace {

struct BusyGuard {
  aidg_plan* p;
  bool ok;
  explicit BusyGuard(aidg_plan* q) : p(q) {
    bool expected = false;
    ok = p->busy.compare_exchange_strong(expected, true);
  }
  ~BusyGuard() {
    if (ok) p->busy.store(false);
  }
};

bool gpu_subgrid_size(int L) { return L == 32 || L == 64 || L == 96; }

// Record a timing event pair around a launch when the plan is profiling.
struct TimedLaunch {
  aidg_plan* p;
  hipStream_t st;
  hipEvent_t ea = nullptr, eb = nullptr;
  TimedLaunch(aidg_plan* plan, hipStream_t stream) : p(plan), st(stream) {
    if (p && p->profiling && p->pool_next + 2 <= p->pool.size()) {
      ea = p->pool[p->pool_next++];
      eb = p->pool[p->pool_next++];
      (void)hipEventRecord(ea, st);
    }
  }
  void done(KernelClass k, int64_t vp, int64_t nsg) {
    if (!ea) return;
    (void)hipEventRecord(eb, st);
    p->timed.push_back({(int)k, vp, nsg, ea, eb});
  }
};

// Launch one kernel class over subgrids [b0, b0 + n) of one plan.
aidg_status run(aidg_plan* p, KernelClass k, int64_t b0, int64_t n, const void* in, void* out,
                void* stream, int adjoint = 0) {
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  TimedLaunch tl(p, st);
  int rc;
  if (k == kZeroVis) {
    rc = launch_zero_vis(p->g.precision, p->d_excl, p->n_excluded, out, stream);
  } else {
    Group g;
    std::memset(&g, 0, sizeof(g));
    g.n = 1;
    g.total_sg = n;
    g.total_grp = p->sg_group[b0 + n - 1] - p->sg_group[b0] + 1;
    g.scratch = p->d_scratch;
    g.job[0] = {p->d_args, in, out, b0, b0 + n, p->sg_group[b0], 0, 0, adjoint, 0};
    rc = launch_group(k, p->g.L, p->g.precision, g, stream, p->max_nv);
  }
  if (rc != 0) return hip_fail((hipError_t)rc, "kernel launch");
  tl.done(k, k == kZeroVis ? 0 : p->vp_prefix[b0 + n] - p->vp_prefix[b0], k == kZeroVis ? 0 : n);
  return AIDG_OK;
}

template <typename T>
aidg_status dalloc(T** p, size_t bytes, aidg_plan* plan, const char* what, hipStream_t stream) {
  void* q = nullptr;
  const size_t n = std::max<size_t>(bytes, 256);
  const hipError_t e = plan->async_mem ? hipMallocAsync(&q, n, stream) : hipMalloc(&q, n);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(AIDG_E_NOMEM, std::string("device allocation of ") + what + " failed: " +
                                  hipGetErrorString(e));
  }
  *p = reinterpret_cast<T*>(q);
  plan->device_bytes += n;
  return AIDG_OK;
}

// Inverse A-term mode: recompute the (A^-1)^H planes and the normalisation map from
// the plan's A-terms, on stream.
aidg_status refresh_inverse_aterms(aidg_plan* p, hipStream_t stream) {
  if (!p->g.amode) return AIDG_OK;
  const int64_t n = (int64_t)p->n_int * p->n_st * p->g.L * p->g.L;
  int rc = launch_aterm_inverse_h(p->g.precision, p->d_aterms, p->d_ainvh, n, stream);
  if (rc == 0)
    rc = launch_aterm_norm(p->g.precision, p->d_ainvh, p->d_npairs, p->d_ncount, p->n_pairs, p->n_chunks,
                           p->pair_chunk, p->g.L * p->g.L, p->n_total > 0 ? 1.0 / p->n_total : 0.0,
                           p->d_npartial, p->d_nmap, stream);
  return rc == 0 ? AIDG_OK : hip_fail((hipError_t)rc, "inverse A-term kernels");
}

}  // namespace

namespace {

// Shared checks of aidg_invert / aidg_predict.
aidg_status image_args(aidg_plan* plan, const void* a, const void* b, const void* ws, int64_t ws_bytes) {
  if (!plan || !a || !b || !ws) return fail(AIDG_E_INVALID, "NULL plan, grid, image or workspace");
  if (!plan->img_ok)
    return fail(AIDG_E_UNSUPPORTED, "image-level transforms need N = 2^a 3^b 5^c <= 8192 with a row of N "
                                    "complex values within 64 KB");
  const int64_t N = plan->g.N;
  if (ws_bytes < 2 * N * N * (int64_t)plan->elem)
    return fail(AIDG_E_INVALID, "workspace smaller than aidg_image_workspace_bytes");
  return AIDG_OK;
}

// Run one image-level launcher, timed as class k when the plan is profiling.
template <typename F>
aidg_status image_step(aidg_plan* p, hipStream_t st, KernelClass k, F&& launch) {
  TimedLaunch tl(p, st);
  const int rc = launch();
  if (rc != 0) return hip_fail((hipError_t)rc, "image kernel launch");
  tl.done(k, 0, 0);
  return AIDG_OK;
}

// Gridding and degridding of a whole plan, batch by batch; adjoint = 1 selects the
// exact adjoint of the other direction (differs on Stokes-I plans only).
aidg_status grid_calls(aidg_plan* plan, const void* vis, void* grid, void* hip_stream, int adjoint) {
  if (!plan || !vis || !grid) return fail(AIDG_E_INVALID, "NULL plan, vis or grid");
  BusyGuard guard(plan);
  if (!guard.ok) return fail(AIDG_E_BUSY, "plan in use by another thread");
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  hipError_t e = hipStreamWaitEvent(st, plan->last, 0);
  if (e != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
  for (size_t b = 0; b + 1 < plan->batch_begin.size(); ++b) {
    const int64_t b0 = plan->batch_begin[b], nb = plan->batch_begin[b + 1] - b0;
    aidg_status r = run(plan, kGridDft, b0, nb, vis, nullptr, hip_stream, adjoint);
    if (r == AIDG_OK) r = run(plan, kFftAdd, b0, nb, nullptr, grid, hip_stream, adjoint);
    if (r != AIDG_OK) return r;
  }
  e = hipEventRecord(plan->last, st);
  return e == hipSuccess ? AIDG_OK : hip_fail(e, "hipEventRecord");
}

aidg_status degrid_calls(aidg_plan* plan, const void* grid, void* vis_out, void* hip_stream, int adjoint) {
  if (!plan || !vis_out || !grid) return fail(AIDG_E_INVALID, "NULL plan, grid or vis");
  BusyGuard guard(plan);
  if (!guard.ok) return fail(AIDG_E_BUSY, "plan in use by another thread");
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  hipError_t e = hipStreamWaitEvent(st, plan->last, 0);
  if (e != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
  aidg_status r = AIDG_OK;
  if (plan->n_excluded > 0) r = run(plan, kZeroVis, 0, 0, nullptr, vis_out, hip_stream);
  if (r != AIDG_OK) return r;
  for (size_t b = 0; b + 1 < plan->batch_begin.size(); ++b) {
    const int64_t b0 = plan->batch_begin[b], nb = plan->batch_begin[b + 1] - b0;
    r = run(plan, kSplitIfft, b0, nb, grid, nullptr, hip_stream, adjoint);
    if (r == AIDG_OK) r = run(plan, kDegridDft, b0, nb, nullptr, vis_out, hip_stream, adjoint);
    if (r != AIDG_OK) return r;
  }
  e = hipEventRecord(plan->last, st);
  return e == hipSuccess ? AIDG_OK : hip_fail(e, "hipEventRecord");
}

// Shared body of aidg_execute and aidg_execute_static: pack the items' ranges into
// grouped launches whose group images fit in `scratch` (scratch_bytes), after the
// named plans' earlier work and, when `last` is given, after the event's; record the
// plans' events and `last` behind the launches.
aidg_status execute_items(void* scratch, int64_t scratch_bytes, hipEvent_t last, const aidg_work* items,
                          int32_t n_items, void* hip_stream) {
  if ((n_items > 0 && !items) || n_items < 0) return fail(AIDG_E_INVALID, "bad items");
  for (int32_t i = 0; i < n_items; ++i) {
    const aidg_work& w = items[i];
    if (!w.plan || !w.in || !w.out || (w.direction != AIDG_DIR_GRID && w.direction != AIDG_DIR_DEGRID) ||
        w.sg_begin < 0 || w.sg_end < w.sg_begin || w.sg_end > (int64_t)w.plan->table.size())
      return fail(AIDG_E_INVALID, "work item " + std::to_string(i) + ": bad plan, buffers, direction or range");
  }
  std::vector<aidg_plan*> plans;
  for (int32_t i = 0; i < n_items; ++i)
    if (std::find(plans.begin(), plans.end(), items[i].plan) == plans.end()) plans.push_back(items[i].plan);
  size_t held = 0;
  for (; held < plans.size(); ++held) {
    bool ex2 = false;
    if (!plans[held]->busy.compare_exchange_strong(ex2, true)) break;
  }
  auto release = [&]() {
    for (size_t k = 0; k < held; ++k) plans[k]->busy.store(false);
  };
  if (held < plans.size()) {
    release();
    return fail(AIDG_E_BUSY, "a plan is in use by another thread");
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  aidg_status r = AIDG_OK;
  hipError_t e = last ? hipStreamWaitEvent(st, last, 0) : hipSuccess;
  for (aidg_plan* p : plans)
    if (e == hipSuccess) e = hipStreamWaitEvent(st, p->last, 0);
  if (e != hipSuccess) r = hip_fail(e, "hipStreamWaitEvent");
  // degridding ranges that start the table also clear the excluded visibilities
  for (int32_t i = 0; i < n_items && r == AIDG_OK; ++i) {
    const aidg_work& w = items[i];
    if (w.direction == AIDG_DIR_DEGRID && w.sg_begin == 0 && w.plan->n_excluded > 0) {
      const int rc = launch_zero_vis(w.plan->g.precision, w.plan->d_excl, w.plan->n_excluded, w.out,
                                     hip_stream);
      if (rc != 0) r = hip_fail((hipError_t)rc, "zeroing excluded visibilities");
    }
  }
  // group by (direction, L, precision); pack ranges into launches
  std::vector<bool> done(n_items, false);
  for (int32_t i0 = 0; i0 < n_items && r == AIDG_OK; ++i0) {
    if (done[i0]) continue;
    const int dir = items[i0].direction, L = items[i0].plan->g.L, prec = items[i0].plan->g.precision;
    const int64_t per_sg = (int64_t)4 * L * L * (prec == AIDG_FP32 ? 8 : 16);
    const int64_t cap = std::min<int64_t>(scratch_bytes / per_sg, 65535);
    if (cap < 1) {
      r = fail(AIDG_E_INVALID, "workspace smaller than one subgrid image");
      break;
    }
    Group g;
    std::memset(&g, 0, sizeof(g));
    g.scratch = scratch;
    int max_nv = 1;
    auto flush = [&]() -> aidg_status {
      if (g.total_sg == 0) return AIDG_OK;
      const KernelClass k0 = dir == AIDG_DIR_GRID ? kGridDft : kSplitIfft;
      const KernelClass k1 = dir == AIDG_DIR_GRID ? kFftAdd : kDegridDft;
      int rc = launch_group(k0, L, prec, g, hip_stream, max_nv);
      if (rc == 0) rc = launch_group(k1, L, prec, g, hip_stream, max_nv);
      std::memset(&g, 0, sizeof(g));
      g.scratch = scratch;
      max_nv = 1;
      return rc == 0 ? AIDG_OK : hip_fail((hipError_t)rc, "grouped kernel launch");
    };
    for (int32_t i = i0; i < n_items && r == AIDG_OK; ++i) {
      const aidg_work& w = items[i];
      if (done[i] || w.direction != dir || w.plan->g.L != L || w.plan->g.precision != prec) continue;
      done[i] = true;
      // a launch takes whole or partial groups until `cap` group images
      const aidg_plan* p = w.plan;
      for (int64_t b = w.sg_begin; b < w.sg_end && r == AIDG_OK;) {
        if (g.n == kMaxGroup || g.total_grp == cap) r = flush();
        if (r != AIDG_OK) break;
        const int64_t g0 = p->sg_group[b], room = cap - g.total_grp;
        const int64_t gn = (int64_t)p->grp_begin.size() - 1;
        const int64_t e = g0 + room < gn ? std::min(w.sg_end, p->grp_begin[g0 + room]) : w.sg_end;
        g.job[g.n] = {p->d_args, w.in, w.out, b, e, g0, g.total_sg, g.total_grp, 0, 0};
        g.n += 1;
        g.total_sg += e - b;
        g.total_grp += p->sg_group[e - 1] - g0 + 1;
        max_nv = std::max(max_nv, p->max_nv);
        b = e;
      }
    }
    if (r == AIDG_OK) r = flush();
  }
  if (r == AIDG_OK) {
    e = last ? hipEventRecord(last, st) : hipSuccess;
    for (aidg_plan* p : plans)
      if (e == hipSuccess) e = hipEventRecord(p->last, st);
    if (e != hipSuccess) r = hip_fail(e, "hipEventRecord");
  }
  release();
  return r;
}

}  // namespace

extern "C" {

int32_t aidg_abi_version(void) { return AIDG_ABI_VERSION; }

const char* aidg_last_error(void) { return g_last_error.c_str(); }

aidg_status aidg_partition(const aidg_geometry* geo, int32_t n_stations, int32_t n_baselines,
                           int32_t n_times, int32_t n_chans, const int32_t* baselines,
                           const double* uvw_m, const double* freqs_hz, aidg_subgrid* out,
                           int64_t cap, int64_t* n_out, double* w_step_out) {
  try {
    Geometry g;
    std::string err;
    aidg_status st = validate_geometry(geo, &g, &err);
    if (st != AIDG_OK) return fail(st, err);
    PartitionResult pr;
    st = partition(g, n_stations, n_baselines, n_times, n_chans, baselines, uvw_m, freqs_hz, &pr, &err);
    if (st != AIDG_OK) return fail(st, err);
    if (n_out) *n_out = (int64_t)pr.table.size();
    if (w_step_out) *w_step_out = pr.w_step;
    if ((int64_t)pr.table.size() > cap || (pr.table.size() && !out))
      return fail(AIDG_E_INVALID, "output capacity too small for the partition");
    std::copy(pr.table.begin(), pr.table.end(), out);
    return AIDG_OK;
  } catch (const std::bad_alloc&) {
    return fail(AIDG_E_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(AIDG_E_INVALID, "unexpected host exception");
  }
}

aidg_status aidg_plan_create(const aidg_geometry* geo, int32_t n_stations, int32_t n_baselines,
                             int32_t n_times, int32_t n_chans, const int32_t* baselines,
                             const double* uvw_m, const double* freqs_hz, const void* aterms,
                             const aidg_subgrid* table, int64_t n_table, void* hip_stream,
                             aidg_plan** out) {
  if (!out) return fail(AIDG_E_INVALID, "out is NULL");
  *out = nullptr;
  aidg_plan* plan = nullptr;
  try {
    plan = new aidg_plan();
    Geometry& g = plan->g;
    std::string err;
    aidg_status st = validate_geometry(geo, &g, &err);
    if (st != AIDG_OK) {
      delete plan;
      return fail(st, err);
    }
    if (!gpu_subgrid_size(g.L)) {
      delete plan;
      return fail(AIDG_E_UNSUPPORTED, "the GPU kernels support subgrid sizes 32, 64 and 96");
    }
    if (!aterms || n_baselines < 1 || n_times < 1 || n_chans < 1 || n_stations < 1) {
      delete plan;
      return fail(AIDG_E_INVALID, "empty observation or NULL A-terms");
    }
    plan->n_st = n_stations;
    plan->nbl = n_baselines;
    plan->nt = n_times;
    plan->nc = n_chans;
    plan->n_int = (n_times + g.aterm_interval - 1) / g.aterm_interval;
    plan->elem = g.precision == AIDG_FP32 ? 8 : 16;

    PartitionResult pr;
    if (!baselines || !uvw_m || !freqs_hz) {
      st = AIDG_E_INVALID;
      err = "NULL host arrays";
    } else if (!table) {
      st = partition(g, n_stations, n_baselines, n_times, n_chans, baselines, uvw_m, freqs_hz, &pr,
                     &err);
    } else if (n_table < 0) {
      st = AIDG_E_INVALID;
      err = "negative table size";
    } else {
      st = adopt_table(g, n_stations, n_baselines, n_times, n_chans, baselines, table, n_table, &pr,
                       &err);
    }
    if (st != AIDG_OK) {
      delete plan;
      return fail(st, err);
    }
    plan->table = split_large(pr.table, g.max_sg_vis, n_times, n_chans);
    plan->n_excluded = (int64_t)pr.excluded.size();
    if (table) {
      int32_t wmax = 0;
      for (const auto& s : plan->table) wmax = std::max(wmax, s.wlayer);
      plan->W = wmax + 1;
      plan->w0.assign(plan->W, 0.0);
      for (const auto& s : plan->table) plan->w0[s.wlayer] = s.w0;
    } else {
      plan->W = (int)(pr.jmax - pr.jmin + 1);
      plan->w0.resize(plan->W);
      for (int j = 0; j < plan->W; ++j)
        plan->w0[j] = pr.w_step > 0 ? (pr.jmin + j + (g.fold ? 0.5 : 0.0)) * pr.w_step : 0.0;
    }
    // Order: subgrids with the same w-layer and centre are consecutive, so that a
    // group shares one image sum, one FFT and one grid update (gridding) or one
    // split and inverse FFT (degridding).  A group is capped at kGroupVisFactor
    // times the mean group's visibilities (larger ones become several groups with
    // the same centre) so that no gridder workgroup runs far longer than the rest.
    // Groups go longest-first (longest-processing-time-first), and inside a group
    // the largest sub-tables go first for the degridder.
    {
      auto& t = plan->table;
      auto same_centre = [](const aidg_subgrid& x, const aidg_subgrid& y) {
        return x.wlayer == y.wlayer && x.U0 == y.U0 && x.V0 == y.V0;
      };
      std::stable_sort(t.begin(), t.end(), [](const aidg_subgrid& x, const aidg_subgrid& y) {
        if (x.wlayer != y.wlayer) return x.wlayer < y.wlayer;
        if (x.V0 != y.V0) return x.V0 < y.V0;
        if (x.U0 != y.U0) return x.U0 < y.U0;
        if (x.nt * x.nc != y.nt * y.nc) return x.nt * x.nc > y.nt * y.nc;
        return x.aint != y.aint ? x.aint < y.aint : x.bl < y.bl;
      });
      struct Span {
        size_t b, e;
        int64_t nv;
      };
      std::vector<Span> spans;
      int64_t total_nv = 0, n_centres = 0;
      for (size_t i = 0; i < t.size(); ++i) {
        total_nv += (int64_t)t[i].nt * t[i].nc;
        if (i == 0 || !same_centre(t[i], t[i - 1])) ++n_centres;
      }
      const int64_t cap_nv = n_centres ? std::max<int64_t>(
          (int64_t)g.max_sg_vis, kGroupVisFactor * ((total_nv + n_centres - 1) / n_centres)) : 1;
      for (size_t i = 0; i < t.size();) {
        size_t j = i;
        int64_t nv = 0;
        while (j < t.size() && same_centre(t[j], t[i]) &&
               (j == i || nv + (int64_t)t[j].nt * t[j].nc <= cap_nv)) {
          nv += (int64_t)t[j].nt * t[j].nc;
          ++j;
        }
        spans.push_back({i, j, nv});
        i = j;
      }
      std::stable_sort(spans.begin(), spans.end(), [](const Span& x, const Span& y) { return x.nv > y.nv; });
      std::vector<aidg_subgrid> ordered;
      ordered.reserve(t.size());
      plan->grp_begin.assign(1, 0);
      plan->sg_group.clear();
      plan->sg_group.reserve(t.size());
      for (const Span& sp : spans) {
        for (size_t k = sp.b; k < sp.e; ++k) {
          ordered.push_back(t[k]);
          plan->sg_group.push_back((int32_t)(plan->grp_begin.size() - 1));
        }
        plan->grp_begin.push_back((int64_t)ordered.size());
      }
      t.swap(ordered);
    }
    plan->max_nv = 1;
    plan->vp_prefix.assign(plan->table.size() + 1, 0);
    for (size_t i = 0; i < plan->table.size(); ++i) {
      const aidg_subgrid& s = plan->table[i];
      plan->max_nv = std::max(plan->max_nv, s.nt * s.nc);
      plan->vp_prefix[i + 1] = plan->vp_prefix[i] + (int64_t)s.nt * s.nc * g.L * g.L;
    }

    // device records; folded sub-tables read their rows from a negated copy of uvw
    // and swap the stations' A-terms
    const double inv_c = 1.0 / kSpeedOfLight;
    bool any_folded = false;
    for (const auto& s : plan->table) any_folded = any_folded || s.folded;
    const size_t uvw_rows = (size_t)n_baselines * n_times;
    std::vector<double> uvw_dev(uvw_m, uvw_m + 3 * uvw_rows);
    if (any_folded) {
      uvw_dev.resize(6 * uvw_rows);
      for (size_t i = 0; i < 3 * uvw_rows; ++i) uvw_dev[3 * uvw_rows + i] = -uvw_m[i];
    }
    std::vector<SubgridDev> dev(plan->table.size());
    for (size_t i = 0; i < plan->table.size(); ++i) {
      const aidg_subgrid& s = plan->table[i];
      SubgridDev& d = dev[i];
      std::memset(&d, 0, sizeof(d));
      d.t0 = s.t0;
      d.nt = s.nt;
      d.c0 = s.c0;
      d.nc = s.nc;
      d.U0 = s.U0;
      d.V0 = s.V0;
      d.wlayer = s.wlayer;
      d.ap = s.aint * n_stations + (s.folded ? s.st2 : s.st1);
      d.aq = s.aint * n_stations + (s.folded ? s.st1 : s.st2);
      d.bl = s.bl;
      d.vis0 = s.vis_offset;
      d.uvw0 = (int64_t)s.bl * n_times + s.t0 + (s.folded ? (int64_t)uvw_rows : 0);
      d.fold = s.folded;
      d.w0 = s.w0;
      d.group = plan->sg_group[i];
      const double df = s.nc > 1 ? freqs_hz[s.c0 + 1] - freqs_hz[s.c0] : 0.0;
      bool uniform = true;
      for (int c = s.c0 + 1; c < s.c0 + s.nc; ++c)
        if (std::fabs((freqs_hz[c] - freqs_hz[c - 1]) - df) > 1e-9 * std::fabs(df)) uniform = false;
      d.dfc = df * inv_c;
      d.R = uniform ? g.R : 1;
      d.kind = degrid_form(g, s.nt, s.nc, uniform);
      plan->n_pervis += d.kind == kDegridPerVis;
      plan->n_direct += d.kind == kDegridDirect;
    }
    // inverse A-term mode: distinct (A_p plane, A_q plane) pairs with their visibility
    // counts, for the normalisation map
    std::vector<int32_t> pairs;
    std::vector<double> pair_count;
    if (g.amode) {
      std::map<std::pair<int32_t, int32_t>, double> cnt;
      for (const SubgridDev& d : dev) cnt[{d.ap, d.aq}] += (double)d.nt * d.nc;
      for (const auto& kv : cnt) {
        pairs.push_back(kv.first.first);
        pairs.push_back(kv.first.second);
        pair_count.push_back(kv.second);
        plan->n_total += kv.second;
      }
      plan->n_pairs = (int64_t)pair_count.size();
      // about 64 pairs per chunk and at most 64 chunks
      plan->n_chunks = (int)std::max<int64_t>(1, std::min<int64_t>(64, (plan->n_pairs + 63) / 64));
      plan->pair_chunk = std::max<int64_t>(1, (plan->n_pairs + plan->n_chunks - 1) / plan->n_chunks);
    }
    std::vector<double> fc(n_chans);
    for (int c = 0; c < n_chans; ++c) fc[c] = freqs_hz[c] * inv_c;
    const int L = g.L;
    std::vector<double> T;
    kaiser_bessel_taper(L, g.beta, &T);
    for (int y = 0; y < L; ++y)
      for (int x = 0; x < L; ++x)
        if ((x + y) & 1) T[(size_t)y * L + x] = -T[(size_t)y * L + x];
    std::vector<double> tw(2 * L);
    for (int k = 0; k < L; ++k) {
      const double ang = -2.0 * M_PI * k / L;
      tw[2 * k] = std::cos(ang);
      tw[2 * k + 1] = std::sin(ang);
    }
    const bool f32 = g.precision == AIDG_FP32;
    std::vector<float> Tf(T.begin(), T.end()), twf(tw.begin(), tw.end());
    // image level: twiddles exp(-2 pi i k / N) and the reciprocal 1 / t[X] of the taper
    // axis at image resolution
    std::vector<double> img_t, img_tw;
    plan->img_ok = image_radices(g.N, (int)plan->elem, &plan->img_fr);
    if (plan->img_ok) {
      kaiser_bessel_axis(g.N, g.beta, &img_t);
      for (double& v : img_t) v = 1.0 / v;
      img_tw.resize(2 * (size_t)g.N);
      for (int k = 0; k < g.N; ++k) {
        const double ang = -2.0 * M_PI * k / g.N;
        img_tw[2 * (size_t)k] = std::cos(ang);
        img_tw[2 * (size_t)k + 1] = std::sin(ang);
      }
    }
    std::vector<float> img_twf(img_tw.begin(), img_tw.end());

    plan->aterm_bytes = (size_t)plan->n_int * n_stations * L * L * 4 * plan->elem;
    const size_t per_sg = (size_t)4 * L * L * plan->elem;
    const int64_t nsg = (int64_t)plan->table.size();
    const int64_t n_groups = (int64_t)plan->grp_begin.size() - 1;
    plan->batch = std::max<int64_t>(1, std::min<int64_t>(g.workspace / (int64_t)per_sg, 65535));
    plan->batch = std::min<int64_t>(plan->batch, std::max<int64_t>(n_groups, 1));
    plan->scratch_bytes = (size_t)plan->batch * per_sg;
    plan->batch_begin.clear();
    for (int64_t k = 0; k < n_groups; k += plan->batch) plan->batch_begin.push_back(plan->grp_begin[k]);
    plan->batch_begin.push_back(nsg);

    hipStream_t stream = reinterpret_cast<hipStream_t>(hip_stream);
    hipError_t e = hipGetDevice(&plan->device);
    if (e != hipSuccess) {
      delete plan;
      return hip_fail(e, "hipGetDevice");
    }
    int pools = 0;
    plan->async_mem = hipDeviceGetAttribute(&pools, hipDeviceAttributeMemoryPoolsSupported, plan->device) ==
                          hipSuccess && pools != 0 && release_stream(plan->device) != nullptr;
    (void)hipGetLastError();
    // on failure after the first allocation: let the creation stream finish, then free
    auto abandon = [&]() {
      (void)hipStreamSynchronize(stream);
      (void)hipGetLastError();
      plan->release();
      delete plan;
    };
    if ((st = dalloc(&plan->d_sg, dev.size() * sizeof(SubgridDev), plan, "subgrid table", stream)) ||
        (st = dalloc(&plan->d_uvw, uvw_dev.size() * sizeof(double), plan, "uvw", stream)) ||
        (st = dalloc(&plan->d_fc, fc.size() * sizeof(double), plan, "frequencies", stream)) ||
        (st = dalloc(&plan->d_aterms, plan->aterm_bytes, plan, "A-terms", stream)) ||
        (st = dalloc(&plan->d_taper, (size_t)L * L * (f32 ? 4 : 8), plan, "taper", stream)) ||
        (st = dalloc(&plan->d_tw, (size_t)L * (f32 ? 8 : 16), plan, "twiddles", stream)) ||
        (st = dalloc(&plan->d_excl, pr.excluded.size() * sizeof(int64_t), plan, "excluded list", stream)) ||
        (st = dalloc(&plan->d_grp, plan->grp_begin.size() * sizeof(int64_t), plan, "group index", stream)) ||
        (st = dalloc(&plan->d_scratch, plan->scratch_bytes, plan, "subgrid workspace", stream)) ||
        (st = dalloc(&plan->d_args, sizeof(KernelArgs), plan, "launch parameters", stream)) ||
        (plan->img_ok &&
         ((st = dalloc(&plan->d_img_tw, (size_t)g.N * plan->elem, plan, "image twiddles", stream)) ||
          (st = dalloc(&plan->d_img_itaper, (size_t)g.N * sizeof(double), plan, "image taper", stream)))) ||
        (g.amode &&
         ((st = dalloc(&plan->d_ainvh, plan->aterm_bytes, plan, "inverse A-terms", stream)) ||
          (st = dalloc(&plan->d_npairs, pairs.size() * sizeof(int32_t), plan, "A-term pairs", stream)) ||
          (st = dalloc(&plan->d_ncount, pair_count.size() * sizeof(double), plan, "pair counts", stream)) ||
          (st = dalloc(&plan->d_npartial, (size_t)plan->n_chunks * L * L * sizeof(double), plan,
                       "normalisation partial sums", stream)) ||
          (st = dalloc(&plan->d_nmap, (size_t)L * L * sizeof(double), plan, "normalisation map", stream))))) {
      abandon();
      return st;
    }
    const KernelArgs host_args = plan->args();
    struct Copy {
      void* dst;
      const void* src;
      size_t n;
      hipMemcpyKind kind;
    } copies[] = {
        {plan->d_sg, dev.data(), dev.size() * sizeof(SubgridDev), hipMemcpyHostToDevice},
        {plan->d_uvw, uvw_dev.data(), uvw_dev.size() * sizeof(double), hipMemcpyHostToDevice},
        {plan->d_fc, fc.data(), fc.size() * sizeof(double), hipMemcpyHostToDevice},
        {plan->d_aterms, aterms, plan->aterm_bytes, hipMemcpyDeviceToDevice},
        {plan->d_taper, f32 ? (const void*)Tf.data() : (const void*)T.data(), (size_t)L * L * (f32 ? 4 : 8),
         hipMemcpyHostToDevice},
        {plan->d_tw, f32 ? (const void*)twf.data() : (const void*)tw.data(), (size_t)L * (f32 ? 8 : 16),
         hipMemcpyHostToDevice},
        {plan->d_excl, pr.excluded.data(), pr.excluded.size() * sizeof(int64_t), hipMemcpyHostToDevice},
        {plan->d_grp, plan->grp_begin.data(), plan->grp_begin.size() * sizeof(int64_t), hipMemcpyHostToDevice},
        {plan->d_args, &host_args, sizeof(KernelArgs), hipMemcpyHostToDevice},
        {plan->d_img_tw, f32 ? (const void*)img_twf.data() : (const void*)img_tw.data(),
         plan->img_ok ? (size_t)g.N * plan->elem : 0, hipMemcpyHostToDevice},
        {plan->d_img_itaper, img_t.data(), plan->img_ok ? (size_t)g.N * sizeof(double) : 0,
         hipMemcpyHostToDevice},
        {plan->d_npairs, pairs.data(), pairs.size() * sizeof(int32_t), hipMemcpyHostToDevice},
        {plan->d_ncount, pair_count.data(), pair_count.size() * sizeof(double), hipMemcpyHostToDevice},
    };
    for (const Copy& c : copies) {
      if (!c.n) continue;
      e = hipMemcpyAsync(c.dst, c.src, c.n, c.kind, stream);
      if (e != hipSuccess) {
        abandon();
        return hip_fail(e, "hipMemcpyAsync (plan upload)");
      }
    }
    if ((st = refresh_inverse_aterms(plan, stream)) != AIDG_OK) {
      abandon();
      return st;
    }
    if ((e = hipEventCreateWithFlags(&plan->last, hipEventDisableTiming)) != hipSuccess ||
        (e = hipEventRecord(plan->last, stream)) != hipSuccess ||
        (e = hipStreamSynchronize(stream)) != hipSuccess) {
      abandon();
      return hip_fail(e, "plan upload");
    }
    *out = plan;
    return AIDG_OK;
  } catch (const std::bad_alloc&) {
    if (plan) {
      if (plan->async_mem && plan->d_sg) (void)hipDeviceSynchronize();  // allocations in flight
      plan->release();
      delete plan;
    }
    return fail(AIDG_E_NOMEM, "host allocation failed");
  }
}

aidg_status aidg_plan_info_get(const aidg_plan* plan, aidg_plan_info* info) {
  if (!plan || !info) return fail(AIDG_E_INVALID, "NULL plan or info");
  std::memset(info, 0, sizeof(*info));
  info->n_subgrids = (int64_t)plan->table.size();
  info->n_vis = (int64_t)plan->nbl * plan->nt * plan->nc;
  info->n_excluded = plan->n_excluded;
  info->n_wlayers = plan->W;
  info->subgrid_size = plan->g.L;
  info->w_step = plan->g.w_step;
  info->device_bytes = (int64_t)plan->device_bytes;
  info->workspace_bytes = (int64_t)plan->scratch_bytes;
  info->grid_bytes = (int64_t)plan->W * plan->g.npol * plan->g.N * plan->g.N * (int64_t)plan->elem;
  info->vis_bytes = info->n_vis * 4 * (int64_t)plan->elem;
  info->n_batches = plan->batch_begin.empty() ? 0 : (int64_t)plan->batch_begin.size() - 1;
  info->n_groups = plan->grp_begin.empty() ? 0 : (int64_t)plan->grp_begin.size() - 1;
  info->max_subgrid_vis = plan->max_nv;
  info->n_subgrids_pervis = plan->n_pervis;
  info->n_subgrids_direct = plan->n_direct;
  return AIDG_OK;
}

aidg_status aidg_plan_subgrids(const aidg_plan* plan, aidg_subgrid* out, int64_t cap) {
  if (!plan || (!out && cap > 0)) return fail(AIDG_E_INVALID, "NULL plan or output");
  const int64_t n = std::min<int64_t>(cap, (int64_t)plan->table.size());
  if (n > 0) std::memcpy(out, plan->table.data(), (size_t)n * sizeof(aidg_subgrid));
  return AIDG_OK;
}

aidg_status aidg_plan_wlayers(const aidg_plan* plan, double* w0, int32_t cap) {
  if (!plan || (!w0 && cap > 0)) return fail(AIDG_E_INVALID, "NULL plan or output");
  for (int j = 0; j < std::min(cap, (int32_t)plan->W); ++j) w0[j] = plan->w0[j];
  return AIDG_OK;
}

aidg_status aidg_plan_set_aterms(aidg_plan* plan, const void* aterms, void* hip_stream) {
  if (!plan || !aterms) return fail(AIDG_E_INVALID, "NULL plan or A-terms");
  BusyGuard guard(plan);
  if (!guard.ok) return fail(AIDG_E_BUSY, "plan in use by another thread");
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  hipError_t e = hipStreamWaitEvent(st, plan->last, 0);
  if (e == hipSuccess)
    e = hipMemcpyAsync(plan->d_aterms, aterms, plan->aterm_bytes, hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return hip_fail(e, "A-term copy");
  const aidg_status r = refresh_inverse_aterms(plan, st);
  if (r != AIDG_OK) return r;
  e = hipEventRecord(plan->last, st);
  return e == hipSuccess ? AIDG_OK : hip_fail(e, "hipEventRecord");
}

aidg_status aidg_plan_aterm_norm(aidg_plan* plan, double* out, int64_t cap) {
  if (!plan || (!out && cap > 0)) return fail(AIDG_E_INVALID, "NULL plan or output");
  if (!plan->g.amode) return fail(AIDG_E_INVALID, "the plan is in the adjoint A-term mode (no normalisation)");
  BusyGuard guard(plan);
  if (!guard.ok) return fail(AIDG_E_BUSY, "plan in use by another thread");
  hipError_t e = hipEventSynchronize(plan->last);
  const int64_t n = std::min<int64_t>(cap, (int64_t)plan->g.L * plan->g.L);
  if (e == hipSuccess && n > 0) e = hipMemcpy(out, plan->d_nmap, (size_t)n * sizeof(double), hipMemcpyDeviceToHost);
  return e == hipSuccess ? AIDG_OK : hip_fail(e, "normalisation map copy");
}

aidg_status aidg_grid(aidg_plan* plan, const void* vis, void* grid, void* hip_stream) {
  return grid_calls(plan, vis, grid, hip_stream, 0);
}

aidg_status aidg_grid_adjoint(aidg_plan* plan, const void* vis, void* grid, void* hip_stream) {
  if (plan && plan->g.amode) return fail(AIDG_E_INVALID, "inverse A-term mode: gridding has no adjoint pair");
  return grid_calls(plan, vis, grid, hip_stream, 1);
}

aidg_status aidg_degrid(aidg_plan* plan, const void* grid, void* vis_out, void* hip_stream) {
  return degrid_calls(plan, grid, vis_out, hip_stream, 0);
}

aidg_status aidg_degrid_adjoint(aidg_plan* plan, const void* grid, void* vis_out, void* hip_stream) {
  if (plan && plan->g.amode) return fail(AIDG_E_INVALID, "inverse A-term mode: gridding has no adjoint pair");
  return degrid_calls(plan, grid, vis_out, hip_stream, 1);
}

aidg_status aidg_footprint_estimate(const aidg_geometry* geo, int32_t n_stations, int32_t n_baselines,
                                    int32_t n_times, int32_t n_chans, const double* uvw_m,
                                    const double* freqs_hz, aidg_footprint* out) {
  if (!out) return fail(AIDG_E_INVALID, "out is NULL");
  std::memset(out, 0, sizeof(*out));
  try {
    Geometry g;
    std::string err;
    aidg_status st = validate_geometry(geo, &g, &err);
    if (st != AIDG_OK) return fail(st, err);
    if (n_stations < 1 || n_baselines < 0 || n_times < 0 || n_chans < 0 ||
        (n_baselines && n_times && !uvw_m) || (n_chans && !freqs_hz))
      return fail(AIDG_E_INVALID, "bad observation sizes or NULL host arrays");
    for (int c = 1; c < n_chans; ++c)
      if (!(freqs_hz[c] > freqs_hz[c - 1])) return fail(AIDG_E_INVALID, "frequencies must be strictly increasing");
    ShapeEstimate se;
    estimate_shape(g, n_baselines, n_times, n_chans, uvw_m, freqs_hz, &se);
    const int64_t elem = g.precision == AIDG_FP32 ? 8 : 16;
    const int64_t L = g.L, N = g.N;
    const int64_t n_vis = (int64_t)n_baselines * n_times * n_chans;
    const int64_t n_int = n_times ? (n_times + g.aterm_interval - 1) / g.aterm_interval : 0;
    const int64_t n_sg = se.n_subgrids;
    out->n_wlayers = (int32_t)(se.jmax - se.jmin + 1);
    out->n_pol = g.npol;
    out->w_step = g.w_step > 0 ? g.w_step : 0.0;
    out->n_subgrids = n_sg;
    out->n_groups = se.n_groups;
    out->n_excluded = se.n_excluded;
    out->grid_bytes = (int64_t)out->n_wlayers * g.npol * N * N * elem;
    out->vis_bytes = n_vis * 4 * elem;
    out->aterm_bytes = n_int * n_stations * L * L * 4 * elem * (g.amode ? 2 : 1);
    // what aidg_plan_create allocates, each allocation at least 256 bytes
    auto al = [](int64_t b) { return std::max<int64_t>(b, 256); };
    const int64_t per_image = 4 * L * L * elem;
    const int64_t batch = std::max<int64_t>(1, std::min<int64_t>({g.workspace / per_image, 65535, se.n_groups}));
    int64_t b = al(n_sg * (int64_t)sizeof(SubgridDev)) + al((int64_t)n_baselines * n_times * 24 * (g.fold ? 2 : 1)) +
                al((int64_t)n_chans * 8) + out->aterm_bytes + al(L * L * elem / 2) + al(L * elem) +
                al(se.n_excluded * 8) + al((n_sg + 1) * 8) + al(batch * per_image) + al(sizeof(KernelArgs));
    if (N <= kMaxImageN) b += al(N * elem) + al(N * 8);
    if (g.amode) {
      const int64_t pairs = std::min<int64_t>(n_sg, (int64_t)n_int * n_baselines);
      // the normalisation map's partial sums: one chunk per about 64 pairs, at most 64
      const int64_t chunks = std::max<int64_t>(1, std::min<int64_t>(64, (pairs + 63) / 64));
      b += al(pairs * 8) + al(pairs * 8) + al(chunks * L * L * 8) + al(L * L * 8);
    }
    out->plan_bytes = b;
    return AIDG_OK;
  } catch (const std::bad_alloc&) {
    return fail(AIDG_E_NOMEM, "host allocation failed");
  }
}

aidg_status aidg_image_workspace_bytes(const aidg_plan* plan, int64_t* bytes) {
  if (!plan || !bytes) return fail(AIDG_E_INVALID, "NULL plan or output");
  if (!plan->img_ok)
    return fail(AIDG_E_UNSUPPORTED, "image-level transforms need N = 2^a 3^b 5^c <= 8192 with a row of N "
                                    "complex values within 64 KB");
  *bytes = 2 * (int64_t)plan->g.N * plan->g.N * (int64_t)plan->elem;
  return AIDG_OK;
}

aidg_status aidg_invert(aidg_plan* plan, const void* grid, void* image, void* workspace,
                        int64_t workspace_bytes, void* hip_stream) {
  aidg_status r = image_args(plan, grid, image, workspace, workspace_bytes);
  if (r != AIDG_OK) return r;
  BusyGuard guard(plan);
  if (!guard.ok) return fail(AIDG_E_BUSY, "plan in use by another thread");
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  hipError_t e = hipStreamWaitEvent(st, plan->last, 0);
  if (e != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
  const int N = plan->g.N, prec = plan->g.precision;
  const size_t plane = (size_t)N * N * plan->elem;
  char* A = static_cast<char*>(workspace);
  char* B = A + plane;
  const double dl = plan->g.dl, inv_l2 = 1.0 / ((double)plan->g.L * plan->g.L);
  for (int pol = 0; pol < plan->g.npol && r == AIDG_OK; ++pol) {
    char* img = static_cast<char*>(image) + pol * plane;
    for (int w = 0; w < plan->W && r == AIDG_OK; ++w) {
      const char* G = static_cast<const char*>(grid) + ((size_t)w * plan->g.npol + pol) * plane;
      // rows: G[gv][gu] -> A[gv][X]; transpose -> B[X][gv]; rows -> B[X][Y]; add into img[Y][X]
      r = image_step(plan, st, kImageFft, [&] {
        return launch_image_fft_rows(prec, +1, false, G, A, N, plan->img_fr, plan->d_img_tw,
                                     plan->d_img_itaper, dl, 0.0, inv_l2, st);
      });
      if (r == AIDG_OK)
        r = image_step(plan, st, kImageWstack, [&] { return launch_image_transpose(prec, A, B, N, st); });
      if (r == AIDG_OK)
        r = image_step(plan, st, kImageFft, [&] {
          return launch_image_fft_rows(prec, +1, false, B, B, N, plan->img_fr, plan->d_img_tw,
                                       plan->d_img_itaper, dl, 0.0, inv_l2, st);
        });
      if (r == AIDG_OK)
        r = image_step(plan, st, kImageWstack, [&] {
          return launch_image_wstack(prec, B, img, N, plan->d_img_itaper, dl, plan->w0[w], inv_l2, w == 0,
                                     w == plan->W - 1 ? plan->d_nmap : nullptr, plan->g.L, st);
        });
    }
  }
  if (r != AIDG_OK) return r;
  e = hipEventRecord(plan->last, st);
  return e == hipSuccess ? AIDG_OK : hip_fail(e, "hipEventRecord");
}

aidg_status aidg_predict(aidg_plan* plan, const void* image, void* grid, void* workspace,
                         int64_t workspace_bytes, void* hip_stream) {
  aidg_status r = image_args(plan, image, grid, workspace, workspace_bytes);
  if (r != AIDG_OK) return r;
  BusyGuard guard(plan);
  if (!guard.ok) return fail(AIDG_E_BUSY, "plan in use by another thread");
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  hipError_t e = hipStreamWaitEvent(st, plan->last, 0);
  if (e != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
  const int N = plan->g.N, prec = plan->g.precision;
  const size_t plane = (size_t)N * N * plan->elem;
  char* A = static_cast<char*>(workspace);
  char* B = A + plane;
  const double dl = plan->g.dl, inv_l2 = 1.0 / ((double)plan->g.L * plan->g.L);
  for (int w = 0; w < plan->W && r == AIDG_OK; ++w) {
    for (int pol = 0; pol < plan->g.npol && r == AIDG_OK; ++pol) {
      const char* img = static_cast<const char*>(image) + pol * plane;
      char* G = static_cast<char*>(grid) + ((size_t)w * plan->g.npol + pol) * plane;
      // rows of img[Y][X] times the w-term -> A[Y][gu]; transpose -> B[gu][Y];
      // rows -> B[gu][gv]; transpose -> G[gv][gu]
      r = image_step(plan, st, kImageFft, [&] {
        return launch_image_fft_rows(prec, -1, true, img, A, N, plan->img_fr, plan->d_img_tw,
                                     plan->d_img_itaper, dl, plan->w0[w], inv_l2, st);
      });
      if (r == AIDG_OK)
        r = image_step(plan, st, kImageWstack, [&] { return launch_image_transpose(prec, A, B, N, st); });
      if (r == AIDG_OK)
        r = image_step(plan, st, kImageFft, [&] {
          return launch_image_fft_rows(prec, -1, false, B, B, N, plan->img_fr, plan->d_img_tw,
                                       plan->d_img_itaper, dl, 0.0, inv_l2, st);
        });
      if (r == AIDG_OK)
        r = image_step(plan, st, kImageWstack, [&] { return launch_image_transpose(prec, B, G, N, st); });
    }
  }
  if (r != AIDG_OK) return r;
  e = hipEventRecord(plan->last, st);
  return e == hipSuccess ? AIDG_OK : hip_fail(e, "hipEventRecord");
}

aidg_status aidg_plan_set_profiling(aidg_plan* plan, int32_t enable) {
  if (!plan) return fail(AIDG_E_INVALID, "NULL plan");
  BusyGuard guard(plan);
  if (!guard.ok) return fail(AIDG_E_BUSY, "plan in use by another thread");
  if (enable && plan->pool.empty()) {
    const size_t n = 2 * 4096;
    plan->pool.reserve(n);
    for (size_t i = 0; i < n; ++i) {
      hipEvent_t e;
      const hipError_t err = hipEventCreate(&e);
      if (err != hipSuccess) return hip_fail(err, "hipEventCreate");
      plan->pool.push_back(e);
    }
  }
  plan->profiling = enable != 0;
  return AIDG_OK;
}

aidg_status aidg_plan_kernel_times(aidg_plan* plan, aidg_kernel_times* out) {
  if (!plan || !out) return fail(AIDG_E_INVALID, "NULL plan or output");
  BusyGuard guard(plan);
  if (!guard.ok) return fail(AIDG_E_BUSY, "plan in use by another thread");
  std::memset(out, 0, sizeof(*out));
  for (const auto& t : plan->timed) {
    hipError_t e = hipEventSynchronize(t.b);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, t.a, t.b);
    if (e != hipSuccess) return hip_fail(e, "reading kernel timers");
    out->ms[t.kind] += ms;
    out->launches[t.kind] += 1;
    out->vis_pixels[t.kind] += t.vp;
    out->subgrids[t.kind] += t.nsg;
  }
  plan->timed.clear();
  plan->pool_next = 0;
  return AIDG_OK;
}

aidg_status aidg_executor_create(int64_t workspace_bytes, aidg_executor** out) {
  if (!out || workspace_bytes < 0) return fail(AIDG_E_INVALID, "NULL output or negative size");
  *out = nullptr;
  aidg_executor* ex = new (std::nothrow) aidg_executor();
  if (!ex) return fail(AIDG_E_NOMEM, "host allocation failed");
  ex->bytes = workspace_bytes ? workspace_bytes : kWorkspaceDefault;
  hipError_t e = hipGetDevice(&ex->device);
  if (e == hipSuccess) e = hipMalloc(&ex->d_scratch, (size_t)ex->bytes);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&ex->last, hipEventDisableTiming);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    if (ex->d_scratch) (void)hipFree(ex->d_scratch);
    delete ex;
    return fail(e == hipErrorOutOfMemory ? AIDG_E_NOMEM : AIDG_E_DEVICE,
                std::string("executor workspace: ") + hipGetErrorString(e));
  }
  *out = ex;
  return AIDG_OK;
}

aidg_status aidg_execute(aidg_executor* ex, const aidg_work* items, int32_t n_items, void* hip_stream) {
  if (!ex) return fail(AIDG_E_INVALID, "NULL executor");
  bool expected = false;
  if (!ex->busy.compare_exchange_strong(expected, true)) return fail(AIDG_E_BUSY, "executor in use");
  const aidg_status r = execute_items(ex->d_scratch, ex->bytes, ex->last, items, n_items, hip_stream);
  ex->busy.store(false);
  return r;
}

aidg_status aidg_execute_static(const aidg_work* items, int32_t n_items, int64_t workspace_bytes,
                                void* hip_stream) {
  if (workspace_bytes < 0 || workspace_bytes > kStaticWorkspaceBytes)
    return fail(AIDG_E_INVALID, "workspace_bytes " + std::to_string(workspace_bytes) +
                                    " outside 0.." + std::to_string(kStaticWorkspaceBytes) +
                                    " (the static workspace's size, AIDG_STATIC_WORKSPACE_BYTES)");
  if ((n_items > 0 && !items) || n_items < 0) return fail(AIDG_E_INVALID, "bad items");
  if (n_items == 0) return AIDG_OK;
  int device = 0;
  const hipError_t e = hipGetDevice(&device);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::string err;
  void* ws = static_workspace(device, &err);
  if (!ws) return fail(AIDG_E_DEVICE, err);
  return execute_items(ws, workspace_bytes ? workspace_bytes : kStaticWorkspaceBytes, nullptr, items, n_items,
                       hip_stream);
}

void aidg_executor_destroy(aidg_executor* ex) {
  if (!ex) return;
  if (ex->last) {
    (void)hipEventSynchronize(ex->last);
    (void)hipEventDestroy(ex->last);
  }
  if (ex->d_scratch) (void)hipFree(ex->d_scratch);
  delete ex;
}

void aidg_plan_destroy(aidg_plan* plan) {
  if (!plan) return;
  if (plan->last) (void)hipEventSynchronize(plan->last);
  plan->release();
  delete plan;
}

}  // extern "C"
