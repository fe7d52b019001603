// dwt2_fwd_batched (and the inverse and adjoint): a ragged list of images.
//
// Plan (cached per shape set and workspace, at most 16): every (step, image)
// becomes one descriptor, and the work items of a step are numbered over all
// images (largest first).  Three schedules: one persistent job whose queue
// holds level 1 of all images, then level 2, and so on, so an image's next
// level starts as soon as the rows it reads exist while other images are
// still at the previous level; one table-driven launch per level; or one per
// step with levels 1 and 2 in the pair kernels.  The schedule and segment
// heights come from a small autotuner that times the policies on the first
// call.  Each call refreshes the step descriptors (image pointers) in pinned
// staging and replays a HIP graph:
//   copy staging -> workspace tables, then the persistent job (after clearing
//   its sync words) or the per-step launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "plan.h"

using namespace dwt2;

namespace {

constexpr int kBatchCh = 2;     // prefetch chunk of the batched job kernel
constexpr int kMinSeg = 2 * kBatchCh;
// Schedules: one cooperative persistent launch whose items wait for the rows
// of the previous level of the same image (kChained); one launch per level
// over every image's items (kLevelSync; levels meet at kernel boundaries,
// nothing waits); or the same with levels 1 and 2 of every image in one
// launch of the pair kernels (kPairSync; when every image's level-1 input is
// at least kPairMinEdge on each side).  A policy is a schedule plus the
// level-1 segment height, coded as kind * kPolicyKind + base.
constexpr int kChained = 0, kLevelSync = 1, kPairSync = 2, kPolicyKind = 10000;
constexpr int kPairMinEdge = 8;

// `pointers`: also check pointers, strides and aliasing (a size query reads
// only the geometry).
int validate_images(const dwt2_image_t* images, int32_t n, int32_t levels, int32_t mode, std::vector<Geo>& geos,
                    bool pointers = true) {
  if (!images || n < 1) return fail(DWT2_ERR_ARG, "need a host array of at least one image");
  if (mode != DWT2_F32 && mode != DWT2_I32_REV) return fail(DWT2_ERR_MODE, "unknown mode %d", mode);
  geos.resize(n);
  for (int i = 0; i < n; ++i) {
    const dwt2_image_t& im = images[i];
    if (pointers && (!im.src || !im.dst)) return fail(DWT2_ERR_ARG, "image %d: null src or dst", i);
    if (pointers && (((uintptr_t)im.src | (uintptr_t)im.dst) & 3))
      return fail(DWT2_ERR_ARG, "image %d: src and dst must be 4-byte aligned", i);
    if (pointers && im.width >= 2 && (im.src_stride < im.width || im.dst_stride < im.width))
      return fail(DWT2_ERR_ARG, "image %d: stride < width", i);
    const int st = check_geometry(im.width, im.height, levels, geos[i]);
    if (st) {
      const std::string why = dwt2_last_error();
      return fail(st, "image %d: %s", i, why.c_str());
    }
  }
  return DWT2_OK;
}

// Every output range must be disjoint from every other output, every input
// and the workspace (inputs may overlap each other: they are only read).
int check_aliasing(const dwt2_image_t* images, int32_t n, const void* workspace, size_t ws_bytes) {
  struct Out {
    Span s;
    int img;  // -1: the workspace
  };
  std::vector<Out> outs;
  outs.reserve(n + 1);
  for (int i = 0; i < n; ++i) {
    const dwt2_image_t& im = images[i];
    outs.push_back({image_span(im.dst, im.dst_stride, 0, im.width, im.height, 1), i});
  }
  const uintptr_t w0 = reinterpret_cast<uintptr_t>(workspace);
  outs.push_back({Span{w0, w0 + ws_bytes}, -1});
  std::sort(outs.begin(), outs.end(), [](const Out& a, const Out& b) { return a.s.lo < b.s.lo; });
  auto name = [](int i, char* buf, size_t len) {
    if (i < 0) snprintf(buf, len, "the workspace");
    else snprintf(buf, len, "image %d's dst", i);
  };
  char b1[48], b2[48];
  for (size_t k = 1; k < outs.size(); ++k)
    if (overlap(outs[k - 1].s, outs[k].s)) {
      name(outs[k - 1].img, b1, sizeof b1);
      name(outs[k].img, b2, sizeof b2);
      return fail(DWT2_ERR_ALIAS, "%s overlaps %s", b1, b2);
    }
  // the outputs are disjoint and sorted, so their ends are sorted too: the
  // first output ending past an input's start is the only candidate
  for (int i = 0; i < n; ++i) {
    const dwt2_image_t& im = images[i];
    const Span in = image_span(im.src, im.src_stride, 0, im.width, im.height, 1);
    auto it = std::upper_bound(outs.begin(), outs.end(), in.lo, [](uintptr_t v, const Out& o) { return v < o.s.hi; });
    if (it != outs.end() && overlap(it->s, in)) {
      name(it->img, b1, sizeof b1);
      return fail(DWT2_ERR_ALIAS, "image %d's src overlaps %s", i, b1);
    }
  }
  return DWT2_OK;
}

struct Layout {
  size_t sync, descs, items, ll;  // byte offsets
  size_t total;
  std::vector<size_t> ll_off;     // per image, relative to ll
  int64_t max_items, max_counters;
};

// Workspace layout; the bounds assume the smallest segment height.
Layout layout(const std::vector<Geo>& geos) {
  Layout L;
  const int n = (int)geos.size();
  int64_t counters = 0, items = 0;
  L.ll_off.resize(n);
  size_t ll = 0;
  for (int i = 0; i < n; ++i) {
    const Geo& g = geos[i];
    for (int k = 1; k <= g.L; ++k) {
      const int64_t segs = (ceil_half(g.h[k - 1]) + kMinSeg - 1) / kMinSeg;
      counters += segs;
      items += segs * num_strips(g.w[k - 1]);
    }
    L.ll_off[i] = ll;
    ll += ws_per_image(g);
  }
  // a pair-schedule plan: levels 1-2 in the pair kernels' strips, level-2
  // rows per item at least kMinSeg; then the single levels 3..L
  int64_t pair_items = 0;
  for (int i = 0; i < n; ++i) {
    const Geo& g = geos[i];
    if (g.L < 2) continue;
    const int q = pair_strip_q(kFwd);
    pair_items += (int64_t)((ceil_half(g.w[0]) + q - 1) / q) * ((ceil_half(ceil_half(g.h[0])) + kMinSeg - 1) / kMinSeg);
    for (int k = 3; k <= g.L; ++k)
      pair_items += (int64_t)num_strips(g.w[k - 1]) * ((ceil_half(g.h[k - 1]) + kMinSeg - 1) / kMinSeg);
  }
  if (pair_items > items) items = pair_items;
  L.max_items = items;
  L.max_counters = counters;
  L.sync = 0;
  L.descs = round256((size_t)(kSyncCounters + kCounterStride * counters) * 4);
  L.items = L.descs + round256((size_t)n * geos[0].L * sizeof(JobDesc));
  L.ll = L.items + round256((size_t)items * 4);
  L.total = L.ll + ll;
  return L;
}

// Segment height of level k (quadruple rows of its input) under policy
// `base`: the level-1 height, halved per level, never below kMinSeg.
int seg_for(int base, int k, int ns_h) {
  int s = base >> (k - 1);
  if (s < kMinSeg) s = kMinSeg;
  s = (s + kMinSeg - 1) / kMinSeg * kMinSeg;
  const int cap = (ns_h + kMinSeg - 1) / kMinSeg * kMinSeg;
  return s < cap ? s : cap;
}

struct Plan {
  int n = 0, levels = 0, mode = 0;
  int dir = kFwd;               // kFwd, kInv or kBwd
  int kind = 0;                 // kChained, kLevelSync or kPairSync
  int base_seg = 32;
  std::vector<Geo> geos;
  std::vector<int> order;       // images by decreasing pixel count
  Layout lay;
  int32_t ndesc = 0, total_items = 0, counters = 0;
  std::vector<uint32_t> item_desc;
  std::vector<int> desc_seg;    // segment height per desc
  int nsteps = 0;               // launches (level-synchronous kinds) or levels (chained)
  std::vector<int> step_level;  // per step: its (finer) level
  std::vector<char> step_pair;  // per step: levels k and k+1 in the pair kernels
  std::vector<int32_t> step_begin;   // first item of each step, plus the total
  std::vector<int64_t> step_ll_bytes;  // LL output bytes of each step over all images
  // device side
  char* ws = nullptr;
  void* staging = nullptr;      // pinned: descs then items
  size_t staging_bytes = 0;
  hipEvent_t done = nullptr;
  bool pending = false;
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  int blocks = 0;
  ~Plan() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (done) (void)hipEventDestroy(done);
    if (staging) (void)hipHostFree(staging);
  }
};

// The plan cache and the tuning results live for the whole process and are
// never destroyed at exit (no HIP calls from static destructors, which
// would run after the runtime has gone); dwt2_clear_plan_cache and the LRU
// eviction below release plans explicitly.  At most kMaxPlans plans are
// kept: a plan holds a graph and pinned staging, and callers that pass a new
// workspace each time would otherwise add one per call.
constexpr size_t kMaxPlans = 16;
struct CachedPlan {
  std::unique_ptr<Plan> plan;
  uint64_t last_use = 0;
};
std::mutex g_mu;
std::map<std::string, CachedPlan>& g_plans = *new std::map<std::string, CachedPlan>;
std::map<std::string, int>& g_tuned = *new std::map<std::string, int>;  // shape set -> policy code
uint64_t g_use_clock = 0;
bool g_tune_loaded = false;

// A policy is usable if its schedule is one of the two and its level-1
// segment height lies in [kMinSeg, kMaxSeg]; anything else (a stale or
// edited tuning file, an out-of-range environment override) is ignored.
constexpr int kMaxSeg = 4096;
bool valid_policy(int policy) {
  if (policy < 0) return false;
  const int kind = policy / kPolicyKind, base = policy % kPolicyKind;
  return (kind == kChained || kind == kLevelSync || kind == kPairSync) && base >= kMinSeg && base <= kMaxSeg;
}

std::string shape_key(int dir, const dwt2_image_t* images, int n, int levels, int mode) {
  std::string k;
  char buf[96];
  snprintf(buf, sizeof buf, "d%d:%d:%d:%d|", dir, n, levels, mode);
  k += buf;
  for (int i = 0; i < n; ++i) {
    snprintf(buf, sizeof buf, "%d,%d;", images[i].width, images[i].height);
    k += buf;
  }
  return k;
}

std::string hash_key(const std::string& s) {  // FNV-1a, for the tune-cache file
  uint64_t h = 1469598103934665603ull;
  for (unsigned char c : s) h = (h ^ c) * 1099511628211ull;
  char buf[32];
  snprintf(buf, sizeof buf, "%016llx", (unsigned long long)h);
  return buf;
}

void load_tune_cache() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = getenv("DWT2_TUNE_CACHE");
  if (!path) return;
  FILE* f = fopen(path, "r");
  if (!f) return;
  char key[64];
  int base;
  while (fscanf(f, "%63s %d", key, &base) == 2)
    if (valid_policy(base)) g_tuned[key] = base;
  fclose(f);
}

void save_tune(const std::string& hk, int base) {
  const char* path = getenv("DWT2_TUNE_CACHE");
  if (!path) return;
  FILE* f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "%s %d\n", hk.c_str(), base);
  fclose(f);
}

// Item table and segment heights for a policy.
// Whether every image can run levels 1 and 2 in the pair kernels.
bool pairs_apply(const Plan& p) {
  if (p.levels < 2) return false;
  for (const Geo& g : p.geos)
    if (g.w[0] < kPairMinEdge || g.h[0] < kPairMinEdge) return false;
  return true;
}

void build_schedule(Plan& p, int policy) {
  const int base = policy % kPolicyKind;
  p.kind = policy / kPolicyKind;
  p.base_seg = base;
  // steps in execution order: the forward runs finest first, the inverse
  // and adjoint coarsest first; kPairSync joins levels 1 and 2
  p.step_level.clear();
  p.step_pair.clear();
  const bool pair = p.kind == kPairSync;
  for (int t = 0; t < p.levels; ++t) {
    const int k = p.dir == kFwd ? t + 1 : p.levels - t;
    if (pair && k == 2) continue;  // inside the pair step of level 1
    p.step_level.push_back(k);
    p.step_pair.push_back(pair && k == 1);
  }
  p.nsteps = (int)p.step_level.size();
  p.ndesc = p.n * p.nsteps;
  p.desc_seg.assign(p.ndesc, 0);
  p.step_begin.assign(p.nsteps + 1, 0);
  p.step_ll_bytes.assign(p.nsteps, 0);
  p.item_desc.clear();
  p.counters = 0;
  for (int t = 0; t < p.nsteps; ++t) {
    p.step_begin[t] = (int32_t)p.item_desc.size();
    const int k = p.step_level[t];
    for (int oi = 0; oi < p.n; ++oi) {
      const int i = p.order[oi];
      const Geo& g = p.geos[i];
      const int j = t * p.n + oi;
      int seg, nsegs, items;
      if (p.step_pair[t]) {  // segments of level-2 quadruple rows
        const int ns_h1 = ceil_half(ceil_half(g.h[0]));
        seg = seg_for(base, 2, ns_h1);
        nsegs = (ns_h1 + seg - 1) / seg;
        const int q = pair_strip_q(p.dir);
        items = nsegs * ((ceil_half(g.w[0]) + q - 1) / q);
        // LL_2 (forward) or the image (inverse, adjoint)
        p.step_ll_bytes[t] += p.dir == kFwd ? (int64_t)g.w[2] * g.h[2] * 4 : (int64_t)g.w[0] * g.h[0] * 4;
      } else {
        const int ns_h = ceil_half(g.h[k - 1]);
        seg = seg_for(base, k, ns_h);
        nsegs = (ns_h + seg - 1) / seg;
        items = nsegs * num_strips(g.w[k - 1]);
        const int ko = p.dir == kFwd ? k : k - 1;  // the step's LL output
        p.step_ll_bytes[t] += (int64_t)g.w[ko] * g.h[ko] * 4;
      }
      p.desc_seg[j] = seg;
      p.item_desc.insert(p.item_desc.end(), items, (uint32_t)j);
      p.counters += nsegs;
    }
  }
  p.total_items = (int32_t)p.item_desc.size();
  p.step_begin[p.nsteps] = p.total_items;
}

// Step descriptors for the current pointers, written to the staging buffer.
void fill_descs(Plan& p, const dwt2_image_t* images, JobDesc* out) {
  int32_t start = 0, cbase = 0;
  for (int t = 0; t < p.nsteps; ++t) {
    const int k = p.step_level[t];
    for (int oi = 0; oi < p.n; ++oi) {
      const int i = p.order[oi];
      const Geo& g = p.geos[i];
      const int j = t * p.n + oi;
      const dwt2_image_t& im = images[i];
      Call c{static_cast<const char*>(im.src), im.src_stride, 0, static_cast<char*>(im.dst), im.dst_stride, 0, 1,
             p.mode, p.ws, p.lay.ll + p.lay.ll_off[i]};
      JobDesc& jd = out[j];
      memset(&jd, 0, sizeof jd);
      LevelDesc& d = jd.d;
      if (p.step_pair[t]) {
        LevelLaunch la;
        int ch;
        pair_launch(p.dir, c, g, 1, la, ch, p.desc_seg[j], false);
        d = la.d;
        jd.pix_bstride = la.pix_bstride;
        jd.ll_bstride = la.ll_bstride;
        jd.band_bstride = la.band_bstride;
      } else {
        fill_level(d, g.w[k - 1], g.h[k - 1], p.desc_seg[j]);
        level_pointers(p.dir, c, g, k, d, jd.pix_bstride, jd.ll_bstride, jd.band_bstride);
      }
      jd.nimg = 1;
      jd.item_start = start;
      jd.items = d.nsegs * d.nstrips;
      jd.cbase = cbase;
      jd.prev = t > 0 ? (t - 1) * p.n + oi : -1;
      jd.coh = p.kind == kChained ? ((t > 0 ? 1 : 0) | (t + 1 < p.nsteps ? 2 : 0)) : 0;
      d.keep_out = p.kind != kChained && t + 1 < p.nsteps && p.step_ll_bytes[t] <= kKeepBytes;
      start += jd.items;
      cbase += d.nsegs;
    }
  }
}

JobArgs job_args(const Plan& p) {
  JobArgs a;
  memset(&a, 0, sizeof a);
  a.descs = reinterpret_cast<const JobDesc*>(p.ws + p.lay.descs);
  a.item_desc = reinterpret_cast<const uint32_t*>(p.ws + p.lay.items);
  a.sync = reinterpret_cast<uint32_t*>(p.ws + p.lay.sync);
  a.ndesc = p.ndesc;
  a.total_items = p.total_items;
  a.host_err = host_error_word();
  job_wait_settings(a.max_polls, a.unreachable);
  return a;
}

// Copy the tables, then run the schedule (on `s`): chained = clear the sync
// words and launch the persistent job; level-synchronous = one launch per
// level over that level's item range.
hipError_t enqueue(const Plan& p, hipStream_t s) {
  const size_t dbytes = (size_t)p.ndesc * sizeof(JobDesc);
  hipError_t e = hipMemcpyAsync(p.ws + p.lay.descs, p.staging, dbytes, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(p.ws + p.lay.items, static_cast<char*>(p.staging) + round256(dbytes),
                     (size_t)p.total_items * 4, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return e;
  if (p.kind != kChained) {
    for (int t = 0; t < p.nsteps; ++t) {
      TableArgs a;
      a.descs = reinterpret_cast<const JobDesc*>(p.ws + p.lay.descs);
      a.item_desc = reinterpret_cast<const uint32_t*>(p.ws + p.lay.items);
      a.item_begin = p.step_begin[t];
      a.items = p.step_begin[t + 1] - p.step_begin[t];
      const int err = p.step_pair[t] ? launch_pair_table(p.dir, p.mode, a, s) : launch_table(p.dir, p.mode, a, s);
      if (err != hipSuccess) return (hipError_t)err;
    }
    return hipSuccess;
  }
  int err = launch_zero(reinterpret_cast<uint32_t*>(p.ws + p.lay.sync), kSyncCounters + (int64_t)kCounterStride * p.counters, s);
  if (err != hipSuccess) return (hipError_t)err;
  return (hipError_t)launch_job(p.dir, p.mode, job_args(p), p.blocks, s);
}

void write_staging(Plan& p, const dwt2_image_t* images) {
  const size_t dbytes = (size_t)p.ndesc * sizeof(JobDesc);
  fill_descs(p, images, static_cast<JobDesc*>(p.staging));
  memcpy(static_cast<char*>(p.staging) + round256(dbytes), p.item_desc.data(), (size_t)p.total_items * 4);
}

int ensure_staging(Plan& p) {
  const size_t need = round256((size_t)p.ndesc * sizeof(JobDesc)) + round256((size_t)p.total_items * 4);
  if (p.staging && p.staging_bytes >= need) return DWT2_OK;
  if (p.staging) (void)hipHostFree(p.staging);
  p.staging = nullptr;
  if (hipHostMalloc(&p.staging, need, hipHostMallocDefault) != hipSuccess || !p.staging)
    return fail(DWT2_ERR_NOMEM, "pinned staging of %zu bytes", need);
  p.staging_bytes = need;
  return DWT2_OK;
}

// Times the candidate policies once (outside any capture) and keeps the
// best.  DWT2_BATCH_SCHEDULE (0 chained, 1 level-synchronous) and
// DWT2_BATCH_SEG (level-1 segment height) force a policy.
int autotune(Plan& p, const dwt2_image_t* images, hipStream_t s, const std::string& hk) {
  static const int candidates[] = {kChained * kPolicyKind + 8,    kChained * kPolicyKind + 16,
                                   kChained * kPolicyKind + 32,   kChained * kPolicyKind + 64,
                                   kLevelSync * kPolicyKind + 8,  kLevelSync * kPolicyKind + 16,
                                   kLevelSync * kPolicyKind + 32, kLevelSync * kPolicyKind + 64,
                                   kLevelSync * kPolicyKind + 128, kPairSync * kPolicyKind + 8,
                                   kPairSync * kPolicyKind + 16,  kPairSync * kPolicyKind + 32,
                                   kPairSync * kPolicyKind + 64};
  const char* fk = getenv("DWT2_BATCH_SCHEDULE");
  const char* fs = getenv("DWT2_BATCH_SEG");
  const int forced_kind = fk ? atoi(fk) : -1;
  const int forced_seg = fs ? atoi(fs) : 0;
  if (forced_kind == kChained || forced_kind == kLevelSync || forced_kind == kPairSync) {
    const int policy = forced_kind * kPolicyKind + (forced_seg > 0 ? forced_seg : 32);
    if (!valid_policy(policy))
      return fail(DWT2_ERR_ARG, "DWT2_BATCH_SEG must lie in [%d, %d] (got %d)", kMinSeg, kMaxSeg, forced_seg);
    if (forced_kind == kPairSync && !pairs_apply(p))
      return fail(DWT2_ERR_ARG, "the pair schedule needs two levels and images of at least %d x %d", kPairMinEdge,
                  kPairMinEdge);
    build_schedule(p, policy);
    return DWT2_OK;
  }
  auto it = g_tuned.find(hk);
  if (it != g_tuned.end() && (it->second / kPolicyKind != kPairSync || pairs_apply(p))) {
    build_schedule(p, it->second);
    return DWT2_OK;
  }
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(DWT2_ERR_HIP, "event creation failed");
  float best = 1e30f;
  int best_policy = kLevelSync * kPolicyKind + 32;
  for (int policy : candidates) {
    if (policy / kPolicyKind == kPairSync && !pairs_apply(p)) continue;
    build_schedule(p, policy);
    if (p.total_items > p.lay.max_items || p.counters > p.lay.max_counters) continue;
    int st = ensure_staging(p);
    if (st) return st;
    write_staging(p, images);
    float t = 0.f;
    for (int rep = 0; rep < 2; ++rep) {
      hipError_t e = hipEventRecord(e0, s);
      const char* what = "event record";
      if (e == hipSuccess) {
        e = enqueue(p, s);
        what = "launch";
      }
      if (e == hipSuccess) e = hipEventRecord(e1, s);
      if (e == hipSuccess) {
        e = hipEventSynchronize(e1);
        what = "run";
      }
      if (e != hipSuccess) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return fail(DWT2_ERR_HIP, "autotune %s of %s schedule, segment %d failed: %s", what,
                    p.kind == kChained ? "chained" : (p.kind == kLevelSync ? "level-synchronous" : "pair"),
                    p.base_seg, hipGetErrorString(e));
      }
      (void)hipEventElapsedTime(&t, e0, e1);
    }
    if (t < best) {
      best = t;
      best_policy = policy;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  // a persistent candidate that gave up a wait invalidates the tuning run
  if (int e = report_async_error()) return e;
  build_schedule(p, best_policy);
  g_tuned[hk] = best_policy;
  save_tune(hk, best_policy);
  return DWT2_OK;
}

int build_plan(Plan& p, int dir, const dwt2_image_t* images, int n, int levels, int mode, std::vector<Geo>&& geos,
               char* ws, hipStream_t s, const std::string& key) {
  p.dir = dir;
  p.n = n;
  p.levels = levels;
  p.mode = mode;
  p.geos = std::move(geos);
  p.ws = ws;
  p.lay = layout(p.geos);
  p.order.resize(n);
  for (int i = 0; i < n; ++i) p.order[i] = i;
  std::stable_sort(p.order.begin(), p.order.end(), [&](int a, int b) {
    return (int64_t)images[a].width * images[a].height > (int64_t)images[b].width * images[b].height;
  });
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  int bpc = job_blocks_per_cu(dir, mode, true);
  p.blocks = (bpc > 0 ? bpc : 1) * (cus > 0 ? cus : 256);
  load_tune_cache();
  int st = autotune(p, images, s, hash_key(key));
  if (st) return st;
  st = ensure_staging(p);
  if (st) return st;
  if (hipEventCreateWithFlags(&p.done, hipEventDisableTiming) != hipSuccess)
    return fail(DWT2_ERR_HIP, "event creation failed");
  static const int use_graph = [] {
    const char* e = getenv("DWT2_BATCH_GRAPH");
    return e ? atoi(e) : 1;
  }();
  if (use_graph) {
    hipStream_t cap;
    if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess)
      return fail(DWT2_ERR_HIP, "capture stream creation failed");
    bool ok = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) == hipSuccess;
    ok = ok && enqueue(p, cap) == hipSuccess;
    hipGraph_t graph = nullptr;
    ok = (hipStreamEndCapture(cap, &graph) == hipSuccess) && ok && graph;
    (void)hipStreamDestroy(cap);
    // a runtime that cannot capture or instantiate the cooperative launch
    // keeps the plan on direct launches
    if (ok) {
      p.graph = graph;
      if (hipGraphInstantiate(&p.exec, graph, nullptr, nullptr, 0) != hipSuccess) p.exec = nullptr;
    } else if (graph) {
      (void)hipGraphDestroy(graph);
    }
    (void)hipGetLastError();
  }
  const char* verbose = getenv("DWT2_VERBOSE");
  if (verbose && atoi(verbose) > 0)
    fprintf(stderr, "dwt2 batched %s plan: %d images, %d levels, %s schedule, level-1 segment %d, %d items, %s\n",
            dir == kFwd ? "forward" : (dir == kInv ? "inverse" : "adjoint"), n, levels,
            p.kind == kChained ? "chained persistent" : (p.kind == kLevelSync ? "level-synchronous" : "pair"),
            p.base_seg, p.total_items,
            p.exec ? "graph replay" : "direct launches");
  return DWT2_OK;
}

static int batched(int dir, const dwt2_image_t* images, int32_t n, int32_t levels, int32_t mode, int32_t boundary,
                   void* workspace, size_t workspace_bytes, void* stream) {
  clear_error();
  if (int e = report_async_error()) return e;
  if (boundary != DWT2_EXT_SYMMETRIC) return fail(DWT2_ERR_ARG, "unknown boundary %d", boundary);
  std::vector<Geo> geos;
  int st = validate_images(images, n, levels, mode, geos);
  if (st) return st;
  if (dir == kBwd && mode != DWT2_F32) return fail(DWT2_ERR_MODE, "the adjoint exists for DWT2_F32 only");
  const size_t total = layout(geos).total;
  if (!workspace || workspace_bytes < total)
    return fail(DWT2_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", total, workspace ? workspace_bytes : 0);
  st = check_aliasing(images, n, workspace, total);
  if (st) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(DWT2_ERR_HIP, "no current device");
  std::string key = shape_key(dir, images, n, levels, mode);
  char wsbuf[64];
  snprintf(wsbuf, sizeof wsbuf, "|ws%p|dev%d", workspace, dev);
  const std::string plan_key = key + wsbuf;

  std::lock_guard<std::mutex> lock(g_mu);
  auto it = g_plans.find(plan_key);
  if (it == g_plans.end()) {
    if (g_plans.size() >= kMaxPlans) {  // evict the least recently used plan
      auto lru = g_plans.begin();
      for (auto j = g_plans.begin(); j != g_plans.end(); ++j)
        if (j->second.last_use < lru->second.last_use) lru = j;
      if (lru->second.plan->pending) (void)hipEventSynchronize(lru->second.plan->done);
      g_plans.erase(lru);
    }
    std::unique_ptr<Plan> p(new Plan);
    st = build_plan(*p, dir, images, n, levels, mode, std::move(geos), static_cast<char*>(workspace), s, key);
    if (st) return st;
    it = g_plans.emplace(plan_key, CachedPlan{std::move(p), 0}).first;
  }
  it->second.last_use = ++g_use_clock;
  Plan& p = *it->second.plan;
  // the previous call of this plan must have consumed the staging buffer
  if (p.pending && hipEventSynchronize(p.done) != hipSuccess) return fail(DWT2_ERR_HIP, "event wait failed");
  write_staging(p, images);
  hipError_t e = p.exec ? hipGraphLaunch(p.exec, s) : enqueue(p, s);
  if (e == hipSuccess) e = hipEventRecord(p.done, s);
  if (e != hipSuccess) return fail(DWT2_ERR_HIP, "batched launch failed: %s", hipGetErrorString(e));
  p.pending = true;
  return DWT2_OK;
}

}  // namespace

extern "C" {

size_t dwt2_batched_workspace_size(const dwt2_image_t* images, int32_t n, int32_t levels, int32_t mode) {
  std::vector<Geo> geos;
  if (validate_images(images, n, levels, mode, geos, false) != DWT2_OK) return 0;
  return layout(geos).total;
}

int dwt2_fwd_batched(const dwt2_image_t* images, int32_t n, int32_t levels, int32_t mode, int32_t boundary,
                     void* workspace, size_t workspace_bytes, void* stream) {
  return batched(kFwd, images, n, levels, mode, boundary, workspace, workspace_bytes, stream);
}

int dwt2_inv_batched(const dwt2_image_t* images, int32_t n, int32_t levels, int32_t mode, int32_t boundary,
                     void* workspace, size_t workspace_bytes, void* stream) {
  return batched(kInv, images, n, levels, mode, boundary, workspace, workspace_bytes, stream);
}

int dwt2_bwd_batched(const dwt2_image_t* images, int32_t n, int32_t levels, int32_t mode, int32_t boundary,
                     void* workspace, size_t workspace_bytes, void* stream) {
  return batched(kBwd, images, n, levels, mode, boundary, workspace, workspace_bytes, stream);
}

int32_t dwt2_plan_cache_size(void) {
  std::lock_guard<std::mutex> lock(g_mu);
  return (int32_t)g_plans.size();
}

void dwt2_clear_plan_cache(void) {
  std::lock_guard<std::mutex> lock(g_mu);
  for (auto& kv : g_plans)
    if (kv.second.plan->pending) (void)hipEventSynchronize(kv.second.plan->done);
  g_plans.clear();
}

}  // extern "C"
