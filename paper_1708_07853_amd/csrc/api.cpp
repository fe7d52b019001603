// C-ABI entry points of libdwt2: argument validation, level geometry,
// workspace layout and the per-level launch sequence.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "dwt2_internal.h"
#include "plan.h"

namespace dwt2 {

namespace {
thread_local std::string g_last_error;
}

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

void clear_error() { g_last_error.clear(); }

int check_geometry(int32_t width, int32_t height, int32_t levels, Geo& g) {
  if (width < 2 || height < 2) return fail(DWT2_ERR_ARG, "width and height must be >= 2 (got %d x %d)", width, height);
  if (width > DWT2_MAX_DIM || height > DWT2_MAX_DIM)
    return fail(DWT2_ERR_SIZE, "dimension above %d", DWT2_MAX_DIM);
  if (levels < 1 || levels > DWT2_MAX_LEVELS) return fail(DWT2_ERR_SIZE, "levels must be in [1, %d] (got %d)", DWT2_MAX_LEVELS, levels);
  g.L = levels;
  g.w[0] = width;
  g.h[0] = height;
  for (int k = 1; k <= levels; ++k) {
    if (g.w[k - 1] < 2 || g.h[k - 1] < 2)
      return fail(DWT2_ERR_SIZE, "level %d input is %d x %d, below 2 x 2", k, g.w[k - 1], g.h[k - 1]);
    g.w[k] = ceil_half(g.w[k - 1]);
    g.h[k] = ceil_half(g.h[k - 1]);
  }
  return DWT2_OK;
}

size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

// Per-image workspace: one LL buffer per intermediate level (LL_1 ..
// LL_{L-1}), each with a row pitch padded to 64 elements.  Levels of a
// persistent job overlap in time, so no buffer is reused within a call.
size_t ll_offset(const Geo& g, int m) {
  size_t off = 0;
  for (int k = 1; k < m; ++k) off += round256((size_t)ll_pitch(g.w[k]) * g.h[k] * 4);
  return off;
}

size_t ws_per_image(const Geo& g) { return ll_offset(g, g.L); }

// Synchronisation words of a persistent job: the queue head, the error word
// and one completion counter per (image, level, segment); a segment holds at
// least one quadruple row, so sum_k h_k counters per image always suffice.
size_t sync_bytes(const Geo& g, int64_t batch) {
  int64_t rows = 0;
  for (int k = 1; k <= g.L; ++k) rows += g.h[k];
  return round256((size_t)(kSyncCounters + kCounterStride * batch * rows) * 4);
}

static int env_int(const char* name) {
  const char* e = getenv(name);
  return e ? atoi(e) : 0;
}

// Compute units of the current device (cached per device).
static int device_cus() {
  static std::mutex mu;
  static int cache[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  std::lock_guard<std::mutex> lock(mu);
  if (!cache[dev]) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
    cache[dev] = n;
  }
  return cache[dev];
}

// Segment height (quadruple rows per work item) and chunk size.
// Per-level launches: about kLevelWavesPerCU waves per compute unit, each
// walking a power-of-two number of quadruple rows.  Measured on MI355X
// (float32 and int32, levels from 16384^2 down to 2048^2), this beats
// filling every resident wave slot: longer walks re-read fewer halo rows at
// segment starts, and power-of-two heights avoided slow address patterns
// that other heights hit (8192^2 level 1: 91 us at 64 rows, 105-117 us at
// 24 or 48).  Among the power-of-two heights that give at least that many
// waves, the choice is the one whose busiest compute unit walks the fewest
// rows: ceil(waves / CUs) items of height + 1 rows (the +1 is the halo row
// an item re-reads); ties go to the longer walk.  Rounding a height up
// instead can leave most CUs with half their waves, and a wave count just
// above a multiple of the CU count gives some CUs one wave more than the
// rest (8192 x 4100, level 1: 53 us at 16 rows, 61 us at 32 with 2080
// waves, 69 us at 64).  Below ~1024^2 a level costs the launch latency
// whatever the tiling.  The persistent job passes its resident capacity as
// `slots_hint` and keeps one round of items for it, each a whole number of
// chunk pairs.
static std::atomic<int> g_forced_seg{-1}, g_forced_ch{-1}, g_persistent{-1};

// Wait settings of the persistent job (dwt2_set_job_wait).
static std::atomic<uint32_t> g_max_polls{0}, g_unreachable{0};
void job_wait_settings(uint32_t& max_polls, uint32_t& unreachable) {
  max_polls = g_max_polls.load();
  unreachable = g_unreachable.load();
}

// One pinned host word per device that a persistent launch sets when one of
// its waits gives up.  It is allocated on first use and kept for the
// process's lifetime (no exit-time HIP calls); the host reads it with plain
// loads, because the kernel's store to it is a system-scope store.
static std::mutex g_err_mu;
static uint32_t* g_err_host[64];
static uint32_t* g_err_dev[64];

uint32_t* host_error_word() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> lock(g_err_mu);
  if (!g_err_host[dev]) {
    void* h = nullptr;
    void* d = nullptr;
    if (hipHostMalloc(&h, 256, hipHostMallocDefault) != hipSuccess || !h) return nullptr;
    if (hipHostGetDevicePointer(&d, h, 0) != hipSuccess || !d) {
      (void)hipHostFree(h);
      return nullptr;
    }
    *static_cast<volatile uint32_t*>(h) = 0;
    g_err_host[dev] = static_cast<uint32_t*>(h);
    g_err_dev[dev] = static_cast<uint32_t*>(d);
  }
  return g_err_dev[dev];
}

// Reports (once) a give-up that a persistent launch on the current device
// recorded since the last report.
static int take_async_error() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return DWT2_OK;
  uint32_t* h;
  {
    std::lock_guard<std::mutex> lock(g_err_mu);
    h = g_err_host[dev];
  }
  if (!h || *static_cast<volatile uint32_t*>(h) == 0) return DWT2_OK;
  *static_cast<volatile uint32_t*>(h) = 0;
  return fail(DWT2_ERR_HIP,
              "a persistent launch on device %d gave up waiting for rows it depends on; the results of that "
              "call are invalid", dev);
}
int report_async_error() { return take_async_error(); }
constexpr int kLevelWavesPerCU = 8;

static int pow2_ceil(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

Tiling choose_tiling(int ns_h, int64_t strips_times_batch, int64_t slots_hint) {
  if (g_forced_seg.load() < 0) g_forced_seg.store(env_int("DWT2_SEG") > 0 ? env_int("DWT2_SEG") : 0);
  if (g_forced_ch.load() < 0) g_forced_ch.store(env_int("DWT2_CH") > 0 ? env_int("DWT2_CH") : 0);
  const int forced_seg = g_forced_seg.load(), forced_ch = g_forced_ch.load();
  Tiling t;
  t.ch = forced_ch > 0 ? (forced_ch >= 4 ? 4 : (forced_ch >= 2 ? 2 : 1)) : 2;
  int seg;
  if (slots_hint > 0) {
    const int64_t per_strip = slots_hint / strips_times_batch > 1 ? slots_hint / strips_times_batch : 1;
    seg = (int)((ns_h + per_strip - 1) / per_strip);
    if (forced_ch <= 0 && seg < 2 * t.ch) t.ch = 1;
    seg = (seg + 2 * t.ch - 1) / (2 * t.ch) * (2 * t.ch);
  } else {
    const int64_t cus = device_cus();
    const int64_t min_waves = (int64_t)kLevelWavesPerCU * cus;
    const int top = pow2_ceil(ns_h > 2 ? ns_h : 2);
    seg = 0;
    int64_t best = 0;
    for (int s = 2; s <= top; s <<= 1) {
      const int64_t waves = strips_times_batch * ((ns_h + s - 1) / s);
      if (waves < min_waves) continue;
      const int64_t cost = (waves + cus - 1) / cus * (s + 1);
      if (seg == 0 || cost < best || (cost == best && s > seg)) {
        seg = s;
        best = cost;
      }
    }
    if (seg == 0) seg = 2;  // no height reaches the wave target: the most waves
    if (forced_ch <= 0 && seg < 2 * t.ch) t.ch = 1;
  }
  t.seg = forced_seg > 0 ? forced_seg : seg;
  return t;
}

// Segment heights picked by dwt2_tune, per launch shape (launch kind,
// direction, mode, level-k input size, batch), each with the prefetch chunk
// it was timed with (value seg | ch << 16; ch 0: choose_tiling's rule for
// that height).  While dwt2_tune times one launch, g_trial holds the height
// and chunk under test for that shape.  The table is never destroyed, so
// process exit runs no teardown code for it.
struct TuneKey {
  int kind, dir, mode, w, h, batch;
  bool operator<(const TuneKey& o) const {
    return std::tie(kind, dir, mode, w, h, batch) < std::tie(o.kind, o.dir, o.mode, o.w, o.h, o.batch);
  }
  bool operator==(const TuneKey& o) const { return !(*this < o) && !(o < *this); }
};
struct Trial {
  bool on = false;
  TuneKey key{};
  int seg = 0, ch = 0;
};
std::mutex g_tune_mu;
std::map<TuneKey, int>& g_tuned_seg = *new std::map<TuneKey, int>;
Trial g_trial;

// The tiling of a per-level-path launch: the model's (choose_tiling), or
// the tuned height for its shape; a forced tiling (dwt2_set_tiling) wins.
static Tiling tuned_tiling(Tiling t, int kind, int dir, int mode, const Geo& g, int k, int batch) {
  if (g_forced_seg.load() > 0) return t;
  const TuneKey key{kind, dir, mode, g.w[k - 1], g.h[k - 1], batch};
  int seg = 0, ch = 0;
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    if (g_trial.on && g_trial.key == key) {
      seg = g_trial.seg;
      ch = g_trial.ch;
    } else {
      auto it = g_tuned_seg.find(key);
      if (it != g_tuned_seg.end()) {
        seg = it->second & 0xffff;
        ch = it->second >> 16;
      }
    }
  }
  if (seg > 0) {
    t.seg = seg;
    if (g_forced_ch.load() <= 0) t.ch = ch > 0 ? ch : (seg < 4 ? 1 : 2);  // else choose_tiling's chunk rule
  }
  return t;
}

void fill_level(LevelDesc& d, int W, int H, int seg) {
  d.W = W;
  d.H = H;
  d.seg = seg;
  d.nstrips = num_strips(W);
  d.nsegs = (ceil_half(H) + seg - 1) / seg;
}

// LL_m of each image's workspace slice (the slices follow the sync area).
static char* ll_buf(const Call& c, const Geo& g, int m) { return c.ws + c.ll_base + ll_offset(g, m); }

// Geometry, pointers and tiling of level k for a call.
// Buffers of level k in direction `dir` (element strides between images in
// *_bs): the level input / output pixels are the image (k = 1) or LL_{k-1};
// LL_k is the packed array's corner at the last level, else a workspace
// buffer; the H bands live in the packed array.
void level_pointers(int dir, const Call& c, const Geo& g, int k, LevelDesc& d, int64_t& pix_bs, int64_t& ll_bs,
                    int64_t& band_bs) {
  const int64_t ws_bs = (int64_t)(ws_per_image(g) / 4);
  const bool px_is_image = (k == 1);
  char* px = px_is_image ? (dir == kFwd ? const_cast<char*>(c.src) : c.dst) : ll_buf(c, g, k - 1);
  d.pix_stride = px_is_image ? (dir == kFwd ? c.src_stride : c.dst_stride) : ll_pitch(g.w[k - 1]);
  pix_bs = px_is_image ? (dir == kFwd ? c.src_bs : c.dst_bs) : ws_bs;
  const bool ll_is_packed = (k == g.L);
  char* ll = ll_is_packed ? (dir == kFwd ? c.dst : const_cast<char*>(c.src)) : ll_buf(c, g, k);
  d.ll_stride = ll_is_packed ? (dir == kFwd ? c.dst_stride : c.src_stride) : ll_pitch(g.w[k]);
  ll_bs = ll_is_packed ? (dir == kFwd ? c.dst_bs : c.src_bs) : ws_bs;
  if (dir == kFwd) {
    d.pix_in = px;
    d.ll_out = ll;
    d.band_out = c.dst;
    d.band_stride = c.dst_stride;
    band_bs = c.dst_bs;
  } else {
    d.pix_out = px;
    d.ll_in = ll;
    d.band_in = c.src;
    d.band_stride = c.src_stride;
    band_bs = c.src_bs;
  }
}

static void level_launch(int dir, const Call& c, const Geo& g, int k, int64_t slots_hint, LevelLaunch& a, int& ch) {
  memset(&a, 0, sizeof a);
  const int W = g.w[k - 1], H = g.h[k - 1];
  const int64_t strips_batch = (int64_t)num_strips(W) * c.batch;
  Tiling t = choose_tiling(ceil_half(H), strips_batch, slots_hint);
  if (slots_hint == 0) t = tuned_tiling(t, kLaunchLevel, dir, c.mode, g, k, c.batch);
  ch = t.ch;
  fill_level(a.d, W, H, t.seg);
  level_pointers(dir, c, g, k, a.d, a.pix_bstride, a.ll_bstride, a.band_bstride);
  // the LL output feeds the next level's launch (forward: LL_k, k < L;
  // inverse / adjoint: LL_{k-1}, k > 1) and fits the caches
  const int ko = dir == kFwd ? k : k - 1;
  const bool feeds = dir == kFwd ? (k < g.L) : (k > 1);
  a.d.keep_out = feeds && (int64_t)g.w[ko] * g.h[ko] * 4 * c.batch <= kKeepBytes;
  a.items_per_image = a.d.nstrips * a.d.nsegs;
  a.items = (int64_t)a.items_per_image * c.batch;
}

// Levels k and k+1 in one pair launch: level k's pixels (input of the
// forward, output of the inverse and adjoint), LL_{k+1} (output of the
// forward, input of the others), and the packed array's bands of both.
constexpr int kPairStageStrips = 24;
void pair_launch(int dir, const Call& c, const Geo& g, int k, LevelLaunch& a, int& ch, int seg_override,
                 bool allow_stage) {
  memset(&a, 0, sizeof a);
  const int W = g.w[k - 1], H = g.h[k - 1];
  const int ns_w = ceil_half(W), ns_h1 = ceil_half(ceil_half(H));
  const int strips = (ns_w + pair_strip_q(dir) - 1) / pair_strip_q(dir);
  Tiling t = tuned_tiling(choose_tiling(ns_h1, (int64_t)strips * c.batch), kLaunchPair, dir, c.mode, g, k, c.batch);
  if (seg_override > 0) t.seg = seg_override;
  ch = t.ch;
  a.d.W = W;
  a.d.H = H;
  a.d.seg = t.seg;
  // the forward pair stages its stores through LDS per workgroup of four
  // adjacent strips (whole 128-byte lines instead of runs that split lines
  // at strip edges) when the image has at least kPairStageStrips strips:
  // then the strips are padded to a multiple of four (the extra strips lie
  // past the image and store nothing), which costs more than it saves on
  // narrower images.  Measured on MI355X, forward, default path: 8192^2
  // six levels 129.8 staged vs 133.1 us, 16384^2 483 vs 508, 6144^2 83.0
  // vs 86.7, 12000^2 287 vs 293; 4096^2 45.5 vs 44.0, 3000^2 five levels
  // 33.2 vs 29.0, 32 x 3 x 1024^2 four levels 246 vs 204 (5 strips -> 8).
  // DWT2_PAIR_STAGE=1 / 0 forces either form (read per call: tests switch it).
  const char* stage_env = getenv("DWT2_PAIR_STAGE");
  const bool staged = allow_stage && (stage_env && *stage_env ? atoi(stage_env) != 0 : strips >= kPairStageStrips);
  a.d.stage = dir == kFwd && staged;
  a.d.nstrips = a.d.stage ? (strips + kWavesPerBlock - 1) / kWavesPerBlock * kWavesPerBlock : strips;
  a.d.nsegs = (ns_h1 + t.seg - 1) / t.seg;
  LevelDesc dk, dk1;
  int64_t pix_bs, ll_bs, band_bs, u0, u1, u2;
  memset(&dk, 0, sizeof dk);
  memset(&dk1, 0, sizeof dk1);
  level_pointers(dir, c, g, k, dk, pix_bs, u0, band_bs);
  level_pointers(dir, c, g, k + 1, dk1, u1, ll_bs, u2);
  a.d.pix_in = dk.pix_in;
  a.d.pix_out = dk.pix_out;
  a.d.pix_stride = dk.pix_stride;
  a.d.band_in = dk.band_in;
  a.d.band_out = dk.band_out;
  a.d.band_stride = dk.band_stride;
  a.d.ll_in = dk1.ll_in;
  a.d.ll_out = dk1.ll_out;
  a.d.ll_stride = dk1.ll_stride;
  a.pix_bstride = pix_bs;
  a.ll_bstride = ll_bs;
  a.band_bstride = band_bs;
  // the output a later launch reads: LL_{k+1} (forward, k+1 < L), LL_{k-1}
  // (inverse / adjoint, k > 1)
  const int ko = dir == kFwd ? k + 1 : k - 1;
  const bool feeds = dir == kFwd ? (k + 1 < g.L) : (k > 1);
  a.d.keep_out = feeds && (int64_t)g.w[ko] * g.h[ko] * 4 * c.batch <= kKeepBytes;
  a.items_per_image = a.d.nstrips * a.d.nsegs;
  a.items = (int64_t)a.items_per_image * c.batch;
}

// One kernel launch per level (levels meet at kernel boundaries).
// Timing probe (dwt2_set_probe): events recorded around one level's launch.
struct Probe {
  int dir = -1, level = 0;
  hipEvent_t begin = nullptr, end = nullptr;
};
std::mutex g_probe_mu;
Probe g_probe;

// First level of the fused tail (0: none): the last 2..kTailMaxLevels
// levels whose inputs hold at most kTailArea pixels over the whole batch
// (inverse: at most two levels).  Larger levels are bandwidth-bound and run
// faster in the strip kernels than with the tail's recomputed halos; the
// tail wins only where launch latency dominates.  The inverse tail's
// coarse-to-fine walk leaves half its lanes idle, so a pair launch takes
// its finest level: 8192^2 float at six levels inside the benchmark step,
// tail 5-6 + pair 3-4 + pair 1-2 129.0 us against tail 4-6 + level 3 +
// pair 1-2 132.0 us (forward and adjoint measured no faster that way).
static int tail_first_level(int dir, const Geo& g, int batch) {
  int k = g.L, n = 0;
  const int nmax = dir == kInv ? 2 : kTailMaxLevels;
  while (k >= 1 && n < nmax && (int64_t)g.w[k - 1] * g.h[k - 1] * batch <= kTailArea) {
    --k;
    ++n;
  }
  // the inverse tail reads at most two quadruples past an edge through a
  // division-free fold, exact for levels of at least 4 x 4
  if (dir == kInv && (g.w[g.L - 1] < 4 || g.h[g.L - 1] < 4)) return 0;
  return n >= 2 ? k + 1 : 0;
}

static int launch_tail_levels(int dir, const Call& c, const Geo& g, int k0, void* stream) {
  TailArgs t;
  memset(&t, 0, sizeof t);
  const int64_t ws_bs = (int64_t)(ws_per_image(g) / 4);
  t.n = g.L - k0 + 1;
  t.batch = c.batch;
  for (int m = 0; m <= t.n; ++m) {
    t.W[m] = g.w[k0 - 1 + m];
    t.H[m] = g.h[k0 - 1 + m];
  }
  t.tiles_x = (t.W[0] + kTailS - 1) / kTailS;
  t.tiles_y = (t.H[0] + kTailS - 1) / kTailS;
  // the finest tail level's pixels: the image (k0 = 1) or LL_{k0-1}
  const void* px = k0 == 1 ? (dir == kFwd ? static_cast<const void*>(c.src) : static_cast<const void*>(c.dst))
                           : static_cast<const void*>(ll_buf(c, g, k0 - 1));
  const int64_t px_stride = k0 == 1 ? (dir == kFwd ? c.src_stride : c.dst_stride) : ll_pitch(g.w[k0 - 1]);
  const int64_t px_bs = k0 == 1 ? (dir == kFwd ? c.src_bs : c.dst_bs) : ws_bs;
  if (dir == kFwd) {  // pixels in, packed coefficients out
    t.in = px;
    t.in_stride = px_stride;
    t.in_bstride = px_bs;
    t.out = c.dst;
    t.out_stride = c.dst_stride;
    t.out_bstride = c.dst_bs;
  } else {  // packed coefficients in, pixels out
    t.in = c.src;
    t.in_stride = c.src_stride;
    t.in_bstride = c.src_bs;
    t.out = const_cast<void*>(px);
    t.out_stride = px_stride;
    t.out_bstride = px_bs;
  }
  return launch_tail(dir, c.mode, t, stream);
}

// Which pairs the default path uses, from measurements on MI355X (whole
// calls, default path against single levels, same tail):
//   inverse, adjoint: faster everywhere (8192^2 float six levels 127 vs 144
//     us and 132 vs 147 us; 16384^2 int32 inverse 472 vs 554 us;
//     32 x 3 x 1024^2 at four levels 186 vs 219 and 192 vs 219 us; 96 x 512^2
//     at four levels 51 vs 71 and 60 vs 69 us);
//   forward: faster unless most of the strips' owned lanes are idle.  With
//     tuned heights: 8192^2 131.5 vs 140.9 us, 16384^2 int32 486 vs 552 us,
//     24 x 2048^2 at five levels 206 vs 229 us; 96 x 512^2 at four levels
//     49 vs 66 us (256 quadruple columns in 3 strips: 76 % of the owned
//     lanes), 24 x 700^2 30 vs 44 us (78 %), 96 x 300^2 at three levels 30
//     vs 42 us (67 %); but 96 x 256^2 at three levels 28.2 vs 26.5 us (128
//     columns in 2 strips: 57 %).  So the forward pairs a level when at
//     least 60 % of its strips' owned lanes hold quadruples, or when the
//     level is small (at most kPairSmallArea input pixels over the batch),
//     where launch latency, not lane use, decides: levels 2-3 of 96 x 256^2
//     (1.6 Mpx) 21.4 vs 26.1 us, levels 3-4 of 96 x 512^2 49.2 vs 56.3 us
//     for the whole call; but levels 3-4 of 32 x 3 x 1024^2 (6.3 Mpx) 193.1
//     vs 190.4 us.
constexpr int kPairMin = 8;
constexpr int64_t kPairSmallArea = 2 * kTailArea;
static bool default_pair(int dir, const Geo& g, int k, int batch) {
  if (dir != kFwd) return true;
  const int ns_w = ceil_half(g.w[k - 1]), q = pair_strip_q(dir);
  const int strips = (ns_w + q - 1) / q;
  return 5 * ns_w >= 3 * strips * q || (int64_t)g.w[k - 1] * g.h[k - 1] * batch <= kPairSmallArea;
}

// The launches of levels 1..L before the fused tail at level k0 (0: none),
// in pairs where `pairs` asks for them and they apply, finest first.
static int plan_levels(int dir, const Geo& g, int batch, int k0, int pairs, Launch* out) {
  const int last_single = k0 ? k0 - 1 : g.L;  // levels 1 .. last_single precede the tail
  int n = 0;
  for (int k = 1; k <= last_single;) {
    const bool want = pairs == kPairsAll || (pairs == kPairsDefault && default_pair(dir, g, k, batch));
    if (want && k + 1 <= last_single && g.w[k - 1] >= kPairMin && g.h[k - 1] >= kPairMin) {
      out[n++] = Launch{k, k + 1, kLaunchPair};
      k += 2;
    } else {
      out[n++] = Launch{k, k, kLaunchLevel};
      k += 1;
    }
  }
  if (k0) out[n++] = Launch{k0, g.L, kLaunchTail};
  return n;
}

// The launches of a plain call on the per-level path, in execution order:
// each covers levels [first, last] -- one level, a pair of levels, or the
// fused tail.  Levels before the tail go in pairs from the finest one where
// the pair kernels apply (a level-k input of at least kPairMin x kPairMin,
// see fused.h), else one by one.  The default path keeps the fused tail
// only where it saves a launch: a pair launch now runs small levels faster
// than the tail (8192^2 float six levels, pairs 1-2, 3-4, 5-6 against pairs
// 1-2, level 3, tail 4-6: forward 124.9 vs 128.8 us, inverse 124.5 vs 127.5,
// adjoint 132.7 vs 133.3; 2048^2: 26.4 / 25.3 / 32.1 vs 26.8 / 29.1 / 34.1
// us), while a tail that replaces two launches with one still wins on tiny
// images (256^2 at five levels: forward 19.3 vs 21.4 us).
int plan_launches(int dir, const Geo& g, int batch, bool tail, int pairs, Launch* out) {
  Launch a[DWT2_MAX_LEVELS + 1], b[DWT2_MAX_LEVELS + 1];
  const int k0 = tail ? tail_first_level(dir, g, batch) : 0;
  int n = plan_levels(dir, g, batch, k0, pairs, a);
  const Launch* p = a;
  if (pairs == kPairsDefault && k0) {
    const int nb = plan_levels(dir, g, batch, 0, pairs, b);
    if (nb <= n) {
      n = nb;
      p = b;
    }
  }
  for (int i = 0; i < n; ++i) out[i] = dir == kFwd ? p[i] : p[n - 1 - i];  // the inverses run coarsest first
  return n;
}


int run_levels(int dir, const Call& c, const Geo& g, void* stream, bool tail, int pairs) {
  Launch plan[DWT2_MAX_LEVELS];
  const int nl = plan_launches(dir, g, c.batch, tail, pairs, plan);
  Probe pr;
  {
    std::lock_guard<std::mutex> lock(g_probe_mu);
    pr = g_probe;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  for (int i = 0; i < nl; ++i) {
    const Launch& l = plan[i];
    // a probe on any level of a launch times that launch
    const bool probed = pr.dir == dir && pr.level >= l.first && pr.level <= l.last;
    if (probed && hipEventRecord(pr.begin, s) != hipSuccess) return fail(DWT2_ERR_HIP, "probe event record failed");
    int err;
    if (l.kind == kLaunchLevel) {
      LevelLaunch a;
      int ch;
      level_launch(dir, c, g, l.first, 0, a, ch);
      err = launch_level(dir, c.mode, ch, a, stream);
    } else if (l.kind == kLaunchPair) {
      LevelLaunch a;
      int ch;
      pair_launch(dir, c, g, l.first, a, ch);
      err = launch_pair(dir, c.mode, ch >= 4 ? 2 : 1, a, stream);
    } else {
      err = launch_tail_levels(dir, c, g, l.first, stream);
    }
    if (err != hipSuccess)
      return fail(DWT2_ERR_HIP, "levels %d..%d launch failed: %s", l.first, l.last, hipGetErrorString((hipError_t)err));
    if (probed && hipEventRecord(pr.end, s) != hipSuccess) return fail(DWT2_ERR_HIP, "probe event record failed");
  }
  return DWT2_OK;
}

int64_t job_slots(int dir, int mode) {
  static std::mutex mu;
  static int cache[3][2] = {};
  int blocks;
  {
    std::lock_guard<std::mutex> lock(mu);
    int& c = cache[dir][mode];
    if (!c) {
      c = job_blocks_per_cu(dir, mode, false);
      if (c <= 0) c = 1;
    }
    blocks = c;
  }
  return (int64_t)blocks;
}

// All levels in one persistent launch (after a small kernel that clears the
// synchronisation words).
int run_job(int dir, const Call& c, const Geo& g, void* stream) {
  const int64_t blocks_per_cu = job_slots(dir, c.mode);
  const int64_t slots = blocks_per_cu * kWavesPerBlock * device_cus();
  static JobArgs args;  // large; filled per call under the lock below
  static std::mutex mu;
  std::lock_guard<std::mutex> lock(mu);
  memset(&args, 0, sizeof args);
  int32_t items = 0, counters = 0;
  for (int t = 0; t < g.L; ++t) {
    const int k = dir == kFwd ? t + 1 : g.L - t;
    LevelLaunch a;
    int ch_unused;
    level_launch(dir, c, g, k, slots, a, ch_unused);
    JobDesc& jd = args.inl[t];
    jd.d = a.d;
    jd.pix_bstride = a.pix_bstride;
    jd.ll_bstride = a.ll_bstride;
    jd.band_bstride = a.band_bstride;
    jd.nimg = c.batch;
    jd.item_start = items;
    jd.items = (int32_t)a.items;
    jd.cbase = counters;
    jd.prev = t - 1;
    jd.coh = (t > 0 ? 1 : 0) | (t + 1 < g.L ? 2 : 0);
    items += (int32_t)a.items;
    counters += c.batch * a.d.nsegs;
  }
  args.ndesc = g.L;
  args.total_items = items;
  args.sync = reinterpret_cast<uint32_t*>(c.ws);
  args.host_err = host_error_word();
  job_wait_settings(args.max_polls, args.unreachable);
  int err = launch_zero(args.sync, kSyncCounters + (int64_t)kCounterStride * counters, stream);
  if (err == hipSuccess) {
    const int64_t want = (items + kWavesPerBlock - 1) / kWavesPerBlock;
    const int64_t cap = blocks_per_cu * device_cus();
    const int blocks = (int)(want < cap ? want : cap);
    err = launch_job(dir, c.mode, args, blocks, stream);
  }
  if (err != hipSuccess) return fail(DWT2_ERR_HIP, "persistent launch failed: %s", hipGetErrorString((hipError_t)err));
  return DWT2_OK;
}

// Separable baseline: the plain workspace followed by one work array per
// image (the level-1 input's size, rows padded like the LL buffers).
static size_t sep_work_per_image(const Geo& g) { return round256((size_t)ll_pitch(g.w[0]) * g.h[0] * 4); }

static int run_separable(const Call& c, const Geo& g, void* stream) {
  const size_t work_base = c.ll_base + ws_per_image(g) * (size_t)c.batch;
  const int64_t ws_bs = (int64_t)(ws_per_image(g) / 4);
  for (int k = 1; k <= g.L; ++k) {
    SepLevel a;
    memset(&a, 0, sizeof a);
    a.W = g.w[k - 1];
    a.H = g.h[k - 1];
    a.batch = c.batch;
    if (k == 1) {
      a.src = c.src;
      a.src_stride = c.src_stride;
      a.src_bstride = c.src_bs;
    } else {
      a.src = ll_buf(c, g, k - 1);
      a.src_stride = ll_pitch(g.w[k - 1]);
      a.src_bstride = ws_bs;
    }
    a.work = c.ws + work_base;
    a.work_pitch = ll_pitch(g.w[0]);
    a.work_bstride = (int64_t)(sep_work_per_image(g) / 4);
    if (k == g.L) {
      a.ll = c.dst;
      a.ll_stride = c.dst_stride;
      a.ll_bstride = c.dst_bs;
    } else {
      a.ll = ll_buf(c, g, k);
      a.ll_stride = ll_pitch(g.w[k]);
      a.ll_bstride = ws_bs;
    }
    a.band = c.dst;
    a.band_stride = c.dst_stride;
    a.band_bstride = c.dst_bs;
    const int err = launch_separable_level(c.mode, a, stream);
    if (err != hipSuccess)
      return fail(DWT2_ERR_HIP, "separable level %d launch failed: %s", k, hipGetErrorString((hipError_t)err));
  }
  return DWT2_OK;
}

// LDS-tiled comparison kernels: one launch per level, LL through the plain
// workspace's buffers.
static int run_lds(int scheme, const Call& c, const Geo& g, void* stream) {
  const int64_t ws_bs = (int64_t)(ws_per_image(g) / 4);
  for (int k = 1; k <= g.L; ++k) {
    SepLevel a;
    memset(&a, 0, sizeof a);
    a.W = g.w[k - 1];
    a.H = g.h[k - 1];
    a.batch = c.batch;
    int tx, ty;
    if (!lds_tiles(a.W, a.H, tx, ty)) return fail(DWT2_ERR_SIZE, "level %d needs more tiles than a launch holds", k);
    if (k == 1) {
      a.src = c.src;
      a.src_stride = c.src_stride;
      a.src_bstride = c.src_bs;
    } else {
      a.src = ll_buf(c, g, k - 1);
      a.src_stride = ll_pitch(g.w[k - 1]);
      a.src_bstride = ws_bs;
    }
    if (k == g.L) {
      a.ll = c.dst;
      a.ll_stride = c.dst_stride;
      a.ll_bstride = c.dst_bs;
    } else {
      a.ll = ll_buf(c, g, k);
      a.ll_stride = ll_pitch(g.w[k]);
      a.ll_bstride = ws_bs;
    }
    a.band = c.dst;
    a.band_stride = c.dst_stride;
    a.band_bstride = c.dst_bs;
    const int err = launch_lds_level(scheme, c.mode, a, stream);
    if (err != hipSuccess)
      return fail(DWT2_ERR_HIP, "LDS-tiled level %d launch failed: %s", k, hipGetErrorString((hipError_t)err));
  }
  return DWT2_OK;
}

// CDF 9/7: one launch per level, LL through the plain workspace's buffers.
constexpr int64_t kTiled97Area = 512 * 512;
constexpr int kTiled97Strips = 10;
constexpr int kTile97Px = 128;  // a tiled-kernel tile's width in pixels (64 quadruples)

// Whether a CDF 9/7 level with input W x H runs in a strip kernel (else the
// tiled one); nstrips: the strips per image.  Levels of at least 16 x 16 run
// in the strip kernels, bit-identical to the tiled ones, except the
// forward's levels of at most kTiled97Strips strips per image (at least a
// fifth of them edge strips, whose folded single-element loads are slow),
// whose width is a whole number of tiles (kTile97Px) and that hold more
// than kTiled97Area pixels over the batch (below that, launch latency
// decides).  Forward, whole calls, strips only against this choice:
// 16 x 1024^2 four levels 58.6 vs 53.4 us, 96 x 256^2 three levels 44.8 vs
// 30.3, 4 x 2048^2 five levels 61.5 vs 58.8, 8192^2 six levels 167.3 vs
// 165.1.  The tiled kernel lost on 1500-pixel-wide levels (1500^2 at four
// levels 26.0 against 28.2 us; 3000^2 at five, whose level 2 is 1500 wide,
// 44.0 against 46.0) and on a level of 14 strips (3000^2 with level 1 tiled
// too: 44.5 against 47.7).  The inverse's strip kernels were faster
// everywhere.  DWT2_CDF97_TILED=1 / 0, read per call, forces the tiled /
// strip kernels for tests and comparisons.
static bool cdf97_strip_level(int dir, bool separable, int W, int H, int batch, int& nstrips) {
  nstrips = 0;
  const char* tiled_env = getenv("DWT2_CDF97_TILED");
  const int force = tiled_env && *tiled_env ? atoi(tiled_env) : -1;
  bool strip = !separable && cdf97_strip_geometry(W, H, nstrips) && force != 1;
  if (strip && force != 0 && dir == kFwd && nstrips <= kTiled97Strips && W % kTile97Px == 0 &&
      (int64_t)W * H * batch > kTiled97Area)
    strip = false;
  return strip;
}
// First level of the 9/7 forward's fused tail (0: none): the last
// 2..kTailMaxLevels levels whose inputs hold at most kTailArea pixels over
// the batch, each at least kTail97Min on a side.  Off unless
// DWT2_CDF97_TAIL=1 (read per call; either DWT2_CDF97_TILED setting turns
// it off again): measured on MI355X it is slower than the per-level
// launches it replaces, whose strip kernels keep their state in registers,
// while the tail runs a dozen barrier-separated LDS phases in one
// workgroup per CU (96 KiB of LDS each).  Whole forward calls, tail
// against per-level: 8192^2 six levels 169 vs 165 us, 16 x 1024^2 four
// levels 56.9 vs 53.2, 1500^2 four levels 30.9 vs 26.4; with at most two
// tail levels 169.5 vs 164.4 and 57 vs 53; with 32-pixel tiles and 512
// threads 184 vs 165 and 67 vs 54 (only a lone 1024^2 image at four
// levels gained, 24.0 vs 26.6).
constexpr int kTail97Min = 8;
static int cdf97_tail_first(const Call& c, const Geo& g) {
  const char* tail_env = getenv("DWT2_CDF97_TAIL");
  const char* tiled_env = getenv("DWT2_CDF97_TILED");
  if (!(tail_env && *tail_env && atoi(tail_env) == 1) || (tiled_env && *tiled_env)) return 0;
  int k = g.L, n = 0;
  while (k >= 1 && n < kTailMaxLevels && (int64_t)g.w[k - 1] * g.h[k - 1] * c.batch <= kTailArea &&
         g.w[k - 1] >= kTail97Min && g.h[k - 1] >= kTail97Min) {
    --k;
    ++n;
  }
  return n >= 2 ? k + 1 : 0;
}

// dwt2_tune's direction codes for the CDF 9/7 forward and inverse (the
// probe of a 9/7 level carries them, so that it never matches a 5/3 call).
constexpr int kTune97 = 3;

static int run_cdf97(int dir, bool separable, const Call& c, const Geo& g, void* stream) {
  const int64_t ws_bs = (int64_t)(ws_per_image(g) / 4);
  const int k0 = dir == kFwd && !separable ? cdf97_tail_first(c, g) : 0;
  Probe pr;
  {
    std::lock_guard<std::mutex> lock(g_probe_mu);
    pr = g_probe;
  }
  hipStream_t hs = static_cast<hipStream_t>(stream);
  for (int s = 0; s < g.L; ++s) {
    const int k = dir == kFwd ? s + 1 : g.L - s;  // the inverse runs coarsest first
    if (k0 && k >= k0) break;  // the forward's last levels: the fused tail below
    Level97 a;
    memset(&a, 0, sizeof a);
    a.W = g.w[k - 1];
    a.H = g.h[k - 1];
    a.batch = c.batch;
    a.final_out = dir == kFwd ? k == g.L : k == 1;  // no later level reads them
    int tx, ty;
    if (!cdf97_tiles(a.W, a.H, tx, ty)) return fail(DWT2_ERR_SIZE, "level %d needs more tiles than a launch holds", k);
    if (dir == kFwd) {
      if (k == 1) {
        a.in = c.src;
        a.in_stride = c.src_stride;
        a.in_bstride = c.src_bs;
      } else {
        a.in = ll_buf(c, g, k - 1);
        a.in_stride = ll_pitch(g.w[k - 1]);
        a.in_bstride = ws_bs;
      }
      if (k == g.L) {
        a.ll = c.dst;
        a.ll_stride = c.dst_stride;
        a.ll_bstride = c.dst_bs;
      } else {
        a.ll = ll_buf(c, g, k);
        a.ll_stride = ll_pitch(g.w[k]);
        a.ll_bstride = ws_bs;
      }
      a.out = c.dst;
      a.out_stride = c.dst_stride;
      a.out_bstride = c.dst_bs;
    } else {
      if (k == g.L) {
        a.in = c.src;
        a.in_stride = c.src_stride;
        a.in_bstride = c.src_bs;
      } else {
        a.in = ll_buf(c, g, k);
        a.in_stride = ll_pitch(g.w[k]);
        a.in_bstride = ws_bs;
      }
      a.bands = c.src;
      a.bands_stride = c.src_stride;
      a.bands_bstride = c.src_bs;
      if (k == 1) {
        a.out = c.dst;
        a.out_stride = c.dst_stride;
        a.out_bstride = c.dst_bs;
      } else {
        a.out = ll_buf(c, g, k - 1);
        a.out_stride = ll_pitch(g.w[k - 1]);
        a.out_bstride = ws_bs;
      }
    }
    // Levels of at least 16 x 16 run in the strip kernels (cdf97_strip_level).
    int nstrips = 0;
    const bool strip = cdf97_strip_level(dir, separable, a.W, a.H, c.batch, nstrips);
    // a probe on this level (dwt2_tune) times its launch
    const bool probed = !separable && pr.dir == kTune97 + dir && pr.level == k;
    if (probed && hipEventRecord(pr.begin, hs) != hipSuccess) return fail(DWT2_ERR_HIP, "probe event record failed");
    int err;
    if (strip) {
      // the model's segment height, or the one dwt2_tune recorded for the shape
      const Tiling t = tuned_tiling(choose_tiling(ceil_half(a.H), (int64_t)nstrips * c.batch), kLaunch97, dir, c.mode,
                                    g, k, c.batch);
      // the forward stages its stores from kPairStageStrips strips, as the pairs
      // do (DWT2_PAIR_STAGE=1 / 0 forces either form, read per call)
      const char* stage_env = getenv("DWT2_PAIR_STAGE");
      const bool staged = stage_env && *stage_env ? atoi(stage_env) != 0 : nstrips >= kPairStageStrips;
      err = launch_cdf97_strip(dir, a, t.seg, t.ch, staged, stream);
    } else {
      err = launch_cdf97_level(dir, separable, a, stream);
    }
    if (err != hipSuccess)
      return fail(DWT2_ERR_HIP, "CDF 9/7 level %d launch failed: %s", k, hipGetErrorString((hipError_t)err));
    if (probed && hipEventRecord(pr.end, hs) != hipSuccess) return fail(DWT2_ERR_HIP, "probe event record failed");
  }
  if (k0) {
    TailArgs t;
    memset(&t, 0, sizeof t);
    t.n = g.L - k0 + 1;
    t.batch = c.batch;
    for (int m = 0; m <= t.n; ++m) {
      t.W[m] = g.w[k0 - 1 + m];
      t.H[m] = g.h[k0 - 1 + m];
    }
    if (k0 == 1) {
      t.in = c.src;
      t.in_stride = c.src_stride;
      t.in_bstride = c.src_bs;
    } else {
      t.in = ll_buf(c, g, k0 - 1);
      t.in_stride = ll_pitch(g.w[k0 - 1]);
      t.in_bstride = ws_bs;
    }
    t.out = c.dst;
    t.out_stride = c.dst_stride;
    t.out_bstride = c.dst_bs;
    cdf97_tail_tiles(t.W[0], t.H[0], t.tiles_x, t.tiles_y);
    const int err = launch_cdf97_tail(t, stream);
    if (err != hipSuccess)
      return fail(DWT2_ERR_HIP, "CDF 9/7 levels %d..%d launch failed: %s", k0, g.L, hipGetErrorString((hipError_t)err));
  }
  return DWT2_OK;
}

// Which kernels compute a call: the product path, one of the comparison
// baselines (separable passes, LDS-tiled separable, LDS-tiled non-separable),
// or the CDF 9/7 kernels.
enum { kProduct = 0, kSepPasses = 1, kLdsSep = 2, kLdsNonSep = 3, kCdf97 = 4, kLdsAdapted = 5, kCdf97Sep = 6,
       kProductLevels = 7 };

static int transform(int dir, const void* src, int64_t src_stride, int64_t src_bs, void* dst, int64_t dst_stride,
                     int64_t dst_bs, int32_t width, int32_t height, int32_t batch, int32_t levels, int32_t mode,
                     int32_t boundary, void* workspace, size_t workspace_bytes, void* stream,
                     int variant = kProduct) {
  const bool separable = variant == kSepPasses;
  clear_error();
  if (int st = take_async_error()) return st;
  if (!src || !dst) return fail(DWT2_ERR_ARG, "null src or dst");
  if (((uintptr_t)src | (uintptr_t)dst | (uintptr_t)workspace) & 3)
    return fail(DWT2_ERR_ARG, "src, dst and workspace must be 4-byte aligned");
  if (boundary != DWT2_EXT_SYMMETRIC) return fail(DWT2_ERR_ARG, "unknown boundary %d", boundary);
  if (batch < 1) return fail(DWT2_ERR_ARG, "batch must be >= 1 (got %d)", batch);
  if (width >= 2 && (src_stride < width || dst_stride < width))
    return fail(DWT2_ERR_ARG, "row stride below width (src %lld, dst %lld, width %d)", (long long)src_stride,
                (long long)dst_stride, width);
  Geo g;
  int st = check_geometry(width, height, levels, g);
  if (st) return st;
  if (batch > 1 && (src_bs < src_stride * height || dst_bs < dst_stride * height))
    return fail(DWT2_ERR_ARG, "batch stride below stride * height");
  if (mode != DWT2_F32 && mode != DWT2_I32_REV) return fail(DWT2_ERR_MODE, "unknown mode %d", mode);
  if (dir == kBwd && mode != DWT2_F32) return fail(DWT2_ERR_MODE, "the adjoint exists for DWT2_F32 only");
  if ((variant == kCdf97 || variant == kCdf97Sep) && mode != DWT2_F32)
    return fail(DWT2_ERR_MODE, "the CDF 9/7 transform exists for DWT2_F32 only");
  if (variant == kLdsAdapted && mode != DWT2_F32)
    return fail(DWT2_ERR_MODE, "the adapted scheme exists for DWT2_F32 only");
  const size_t need =
      sync_bytes(g, batch) + (ws_per_image(g) + (separable ? sep_work_per_image(g) : 0)) * (size_t)batch;
  const Span ss = image_span(src, src_stride, src_bs, width, height, batch);
  const Span ds = image_span(dst, dst_stride, dst_bs, width, height, batch);
  if (overlap(ss, ds)) return fail(DWT2_ERR_ALIAS, "src and dst overlap; the transform is out of place");
  if (!workspace || workspace_bytes < need)
    return fail(DWT2_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", need, workspace ? workspace_bytes : 0);
  const Span ws{reinterpret_cast<uintptr_t>(workspace), reinterpret_cast<uintptr_t>(workspace) + need};
  if (overlap(ws, ss) || overlap(ws, ds)) return fail(DWT2_ERR_ALIAS, "the workspace overlaps src or dst");
  Call c{static_cast<const char*>(src), src_stride, src_bs, static_cast<char*>(dst), dst_stride, dst_bs, batch, mode,
         static_cast<char*>(workspace), sync_bytes(g, batch)};
  if (separable) return run_separable(c, g, stream);
  if (variant == kLdsSep) return run_lds(DWT2_SCHEME_SEPARABLE, c, g, stream);
  if (variant == kLdsNonSep) return run_lds(DWT2_SCHEME_NONSEPARABLE, c, g, stream);
  if (variant == kLdsAdapted) return run_lds(DWT2_SCHEME_ADAPTED, c, g, stream);
  if (variant == kCdf97 || variant == kCdf97Sep) return run_cdf97(dir, variant == kCdf97Sep, c, g, stream);
  // the default per-level path (path 0) whatever the process-wide setting
  // (the entry point without a workspace: it must not reach the persistent
  // path, whose host-visible error word is allocated on first use)
  if (variant == kProductLevels) return run_levels(dir, c, g, stream, true, kPairsDefault);
  if (g_persistent.load() < 0) g_persistent.store(env_int("DWT2_PERSISTENT") == 1 ? 1 : 0);
  const int path = g_persistent.load();
  if (path == 1 && g.L <= kInlineDescs) return run_job(dir, c, g, stream);
  if (path == 2) return run_levels(dir, c, g, stream, false, kPairsNone);
  if (path == 4) return run_levels(dir, c, g, stream, false, kPairsAll);
  return run_levels(dir, c, g, stream, true, path == 3 ? kPairsAll : (path == 5 ? kPairsNone : kPairsDefault));
}

int fwd_levels_path(const void* src, int64_t src_stride, int64_t src_bs, void* dst, int64_t dst_stride,
                    int64_t dst_bs, int32_t width, int32_t height, int32_t batch, int32_t levels, int32_t mode,
                    int32_t boundary, void* workspace, size_t workspace_bytes, void* stream) {
  return transform(kFwd, src, src_stride, src_bs, dst, dst_stride, dst_bs, width, height, batch, levels, mode,
                   boundary, workspace, workspace_bytes, stream, kProductLevels);
}

// The launches a plain call runs on the current per-level path setting
// (0 when the persistent path takes the call).
static int current_plan(int dir, const Geo& g, int batch, Launch* plan) {
  if (g_persistent.load() < 0) g_persistent.store(env_int("DWT2_PERSISTENT") == 1 ? 1 : 0);
  const int path = g_persistent.load();
  if (path == 1 && g.L <= kInlineDescs) return 0;
  const int pairs = path == 3 || path == 4 ? kPairsAll : (path == 0 ? kPairsDefault : kPairsNone);
  return plan_launches(dir, g, batch, path != 2 && path != 4, pairs, plan);
}

// dwt2_tune: for each single-level or pair launch of the call (dir 0..2),
// or each strip-kernel level of a CDF 9/7 call (dir kTune97 + 0 / 1), in
// execution order, times the whole call once per candidate segment height
// with events around that launch (the median of kTuneReps calls after two
// untimed ones) and keeps the fastest height if it beats the model's by
// more than kTuneGain; later calls of the same shapes use it.
constexpr int kTuneReps = 5;
constexpr float kTuneGain = 0.02f;
static int tune(int dir, const void* src, int64_t src_stride, int64_t src_bs, void* dst, int64_t dst_stride,
                int64_t dst_bs, int32_t width, int32_t height, int32_t batch, int32_t levels, int32_t mode,
                int32_t boundary, void* workspace, size_t workspace_bytes, void* stream) {
  const bool is97 = dir >= kTune97;
  const int tdir = is97 ? dir - kTune97 : dir;  // the transform's direction
  auto call = [&]() {
    return transform(tdir, src, src_stride, src_bs, dst, dst_stride, dst_bs, width, height, batch, levels, mode,
                     boundary, workspace, workspace_bytes, stream, is97 ? kCdf97 : kProduct);
  };
  if (int st = call()) return st;  // validates every argument
  Geo g;
  check_geometry(width, height, levels, g);
  Launch plan[DWT2_MAX_LEVELS];
  int n = 0;
  if (g_forced_seg.load() > 0) {
    n = 0;  // a forced tiling: nothing to tune
  } else if (is97) {
    Call cc{};
    cc.batch = batch;
    const int k0 = tdir == kFwd ? cdf97_tail_first(cc, g) : 0;
    for (int s = 0; s < g.L; ++s) {
      const int k = tdir == kFwd ? s + 1 : g.L - s;
      int ns;
      if (k0 && k >= k0) break;
      if (cdf97_strip_level(tdir, false, g.w[k - 1], g.h[k - 1], batch, ns)) plan[n++] = Launch{k, k, kLaunch97};
    }
  } else {
    n = current_plan(dir, g, batch, plan);
  }
  if (n == 0) return DWT2_OK;  // a forced tiling or the persistent path: nothing to tune
  hipEvent_t ev[2 * kTuneReps] = {};
  for (hipEvent_t& e : ev)
    if (hipEventCreate(&e) != hipSuccess) {
      for (hipEvent_t& f : ev)
        if (f) (void)hipEventDestroy(f);
      return fail(DWT2_ERR_HIP, "tuning event creation failed");
    }
  Probe saved;
  {
    std::lock_guard<std::mutex> lock(g_probe_mu);
    saved = g_probe;
  }
  static const int kPairSegs[] = {0, 1, 2, 3, 4, 6, 8, 10, 12, 16, 20, 24, 32};
  static const int kLevelSegs[] = {0, 1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64};
  int st = DWT2_OK;
  for (int i = 0; i < n && st == DWT2_OK; ++i) {
    const Launch& l = plan[i];
    if (l.kind == kLaunchTail) continue;
    const int k = l.first;
    const bool pair = l.kind == kLaunchPair;
    const int rows = pair ? ceil_half(ceil_half(g.h[k - 1])) : ceil_half(g.h[k - 1]);
    const TuneKey key{l.kind, tdir, mode, g.w[k - 1], g.h[k - 1], batch};
    {
      std::lock_guard<std::mutex> lock(g_tune_mu);
      g_tuned_seg.erase(key);  // candidate 0 is the model's height
    }
    // candidates: (height, chunk), chunk 0 taking the rule's; the 9/7 strip
    // levels also try the other chunk at the heights where the rule switches
    // (forced on every level, 3 rows with a two-row chunk took level 2 of
    // the 8192^2 forward from 33.7 to 24.4 us)
    int cseg[32], cch[32], ncand = 0;
    const int* base = pair ? kPairSegs : kLevelSegs;
    const int nbase = pair ? (int)(sizeof kPairSegs / sizeof *kPairSegs) : (int)(sizeof kLevelSegs / sizeof *kLevelSegs);
    for (int j = 0; j < nbase; ++j) {
      cseg[ncand] = base[j];
      cch[ncand++] = 0;
    }
    if (l.kind == kLaunch97) {
      static const int kExtra97[][2] = {{2, 2}, {3, 2}, {4, 1}, {6, 1}};
      for (const auto& e : kExtra97) {
        cseg[ncand] = e[0];
        cch[ncand++] = e[1];
      }
    }
    float model_ms = 0.f, best_ms = 0.f;
    int best = 0;
    for (int j = 0; j < ncand && st == DWT2_OK; ++j) {
      const int seg = cseg[j];
      if (seg > rows) continue;
      {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        g_trial.on = seg > 0;
        g_trial.key = key;
        g_trial.seg = seg;
        g_trial.ch = cch[j];
      }
      float t[kTuneReps];
      for (int r = -2; r < kTuneReps && st == DWT2_OK; ++r) {
        {
          std::lock_guard<std::mutex> lock(g_probe_mu);
          g_probe = Probe();
          if (r >= 0) {
            g_probe.dir = dir;
            g_probe.level = k;
            g_probe.begin = ev[2 * r];
            g_probe.end = ev[2 * r + 1];
          }
        }
        st = call();
      }
      if (st) break;
      if (hipEventSynchronize(ev[2 * kTuneReps - 1]) != hipSuccess) {
        st = fail(DWT2_ERR_HIP, "tuning event wait failed");
        break;
      }
      for (int r = 0; r < kTuneReps && st == DWT2_OK; ++r)
        if (hipEventElapsedTime(&t[r], ev[2 * r], ev[2 * r + 1]) != hipSuccess)
          st = fail(DWT2_ERR_HIP, "tuning event time failed");
      if (st) break;
      std::sort(t, t + kTuneReps);
      const float med = t[kTuneReps / 2];
      if (seg == 0) model_ms = med;
      if (j == 0 || med < best_ms) {
        best_ms = med;
        best = seg | cch[j] << 16;
      }
    }
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_trial = Trial();
    if (st == DWT2_OK && best > 0 && best_ms < (1.f - kTuneGain) * model_ms) g_tuned_seg[key] = best;
  }
  {
    std::lock_guard<std::mutex> lock(g_probe_mu);
    g_probe = saved;
  }
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_trial = Trial();
  }
  for (hipEvent_t& e : ev) (void)hipEventDestroy(e);
  return st;
}

}  // namespace dwt2

using namespace dwt2;

extern "C" {

size_t dwt2_workspace_size(int32_t width, int32_t height, int32_t batch, int32_t levels, int32_t mode) {
  Geo g;
  if (batch < 1 || (mode != DWT2_F32 && mode != DWT2_I32_REV)) return 0;
  if (check_geometry(width, height, levels, g) != DWT2_OK) return 0;
  return sync_bytes(g, batch) + ws_per_image(g) * (size_t)batch;
}

size_t dwt2_separable_workspace_size(int32_t width, int32_t height, int32_t batch, int32_t levels, int32_t mode) {
  Geo g;
  if (batch < 1 || (mode != DWT2_F32 && mode != DWT2_I32_REV)) return 0;
  if (check_geometry(width, height, levels, g) != DWT2_OK) return 0;
  return sync_bytes(g, batch) + (ws_per_image(g) + sep_work_per_image(g)) * (size_t)batch;
}

int dwt2_fwd_separable(const void* src, int64_t src_stride, int64_t src_batch_stride, void* dst, int64_t dst_stride,
                       int64_t dst_batch_stride, int32_t width, int32_t height, int32_t batch, int32_t levels,
                       int32_t mode, int32_t boundary, void* workspace, size_t workspace_bytes, void* stream) {
  return transform(kFwd, src, src_stride, src_batch_stride, dst, dst_stride, dst_batch_stride, width, height, batch,
                   levels, mode, boundary, workspace, workspace_bytes, stream, kSepPasses);
}

int dwt2_fwd_cdf97(const void* src, int64_t src_stride, int64_t src_batch_stride, void* dst, int64_t dst_stride,
                   int64_t dst_batch_stride, int32_t width, int32_t height, int32_t batch, int32_t levels, int32_t mode,
                   int32_t boundary, void* workspace, size_t workspace_bytes, void* stream) {
  return transform(kFwd, src, src_stride, src_batch_stride, dst, dst_stride, dst_batch_stride, width, height, batch,
                   levels, mode, boundary, workspace, workspace_bytes, stream, kCdf97);
}

int dwt2_fwd_cdf97_separable(const void* src, int64_t src_stride, int64_t src_batch_stride, void* dst,
                             int64_t dst_stride, int64_t dst_batch_stride, int32_t width, int32_t height,
                             int32_t batch, int32_t levels, int32_t mode, int32_t boundary, void* workspace,
                             size_t workspace_bytes, void* stream) {
  return transform(kFwd, src, src_stride, src_batch_stride, dst, dst_stride, dst_batch_stride, width, height, batch,
                   levels, mode, boundary, workspace, workspace_bytes, stream, kCdf97Sep);
}

int dwt2_inv_cdf97(const void* src, int64_t src_stride, int64_t src_batch_stride, void* dst, int64_t dst_stride,
                   int64_t dst_batch_stride, int32_t width, int32_t height, int32_t batch, int32_t levels, int32_t mode,
                   int32_t boundary, void* workspace, size_t workspace_bytes, void* stream) {
  return transform(kInv, src, src_stride, src_batch_stride, dst, dst_stride, dst_batch_stride, width, height, batch,
                   levels, mode, boundary, workspace, workspace_bytes, stream, kCdf97);
}

int dwt2_fwd_lds(const void* src, int64_t src_stride, int64_t src_batch_stride, void* dst, int64_t dst_stride,
                 int64_t dst_batch_stride, int32_t width, int32_t height, int32_t batch, int32_t levels, int32_t mode,
                 int32_t boundary, int32_t scheme, void* workspace, size_t workspace_bytes, void* stream) {
  if (scheme != DWT2_SCHEME_SEPARABLE && scheme != DWT2_SCHEME_NONSEPARABLE && scheme != DWT2_SCHEME_ADAPTED) {
    clear_error();
    return fail(DWT2_ERR_ARG, "unknown scheme %d", scheme);
  }
  return transform(kFwd, src, src_stride, src_batch_stride, dst, dst_stride, dst_batch_stride, width, height, batch,
                   levels, mode, boundary, workspace, workspace_bytes, stream,
                   scheme == DWT2_SCHEME_SEPARABLE ? kLdsSep
                                                   : (scheme == DWT2_SCHEME_NONSEPARABLE ? kLdsNonSep : kLdsAdapted));
}

int dwt2_fwd(const void* src, int64_t src_stride, int64_t src_batch_stride, void* dst, int64_t dst_stride,
             int64_t dst_batch_stride, int32_t width, int32_t height, int32_t batch, int32_t levels, int32_t mode,
             int32_t boundary, void* workspace, size_t workspace_bytes, void* stream) {
  return transform(kFwd, src, src_stride, src_batch_stride, dst, dst_stride, dst_batch_stride, width, height, batch,
                   levels, mode, boundary, workspace, workspace_bytes, stream);
}

int dwt2_inv(const void* src, int64_t src_stride, int64_t src_batch_stride, void* dst, int64_t dst_stride,
             int64_t dst_batch_stride, int32_t width, int32_t height, int32_t batch, int32_t levels, int32_t mode,
             int32_t boundary, void* workspace, size_t workspace_bytes, void* stream) {
  return transform(kInv, src, src_stride, src_batch_stride, dst, dst_stride, dst_batch_stride, width, height, batch,
                   levels, mode, boundary, workspace, workspace_bytes, stream);
}

int dwt2_bwd(const void* src, int64_t src_stride, int64_t src_batch_stride, void* dst, int64_t dst_stride,
             int64_t dst_batch_stride, int32_t width, int32_t height, int32_t batch, int32_t levels, int32_t mode,
             int32_t boundary, void* workspace, size_t workspace_bytes, void* stream) {
  return transform(kBwd, src, src_stride, src_batch_stride, dst, dst_stride, dst_batch_stride, width, height, batch,
                   levels, mode, boundary, workspace, workspace_bytes, stream);
}

const char* dwt2_status_string(int status) {
  switch (status) {
    case DWT2_OK: return "ok";
    case DWT2_ERR_ARG: return "invalid argument";
    case DWT2_ERR_SIZE: return "unsupported size or level count";
    case DWT2_ERR_MODE: return "unsupported mode";
    case DWT2_ERR_WORKSPACE: return "workspace too small";
    case DWT2_ERR_ALIAS: return "source and destination alias";
    case DWT2_ERR_HIP: return "HIP runtime error";
    case DWT2_ERR_NOMEM: return "out of memory";
    default: return "unknown status";
  }
}

const char* dwt2_last_error(void) { return g_last_error.c_str(); }

int dwt2_set_probe(int32_t dir, int32_t level, void* ev_begin, void* ev_end) {
  clear_error();
  std::lock_guard<std::mutex> lock(g_probe_mu);
  if (dir < 0) {
    g_probe = Probe();
    return DWT2_OK;
  }
  if (dir > 2 || level < 1 || level > DWT2_MAX_LEVELS || !ev_begin || !ev_end)
    return fail(DWT2_ERR_ARG, "probe needs dir 0..2, level 1..%d and two events", DWT2_MAX_LEVELS);
  g_probe.dir = dir;
  g_probe.level = level;
  g_probe.begin = static_cast<hipEvent_t>(ev_begin);
  g_probe.end = static_cast<hipEvent_t>(ev_end);
  return DWT2_OK;
}

int dwt2_set_path(int32_t path) {
  clear_error();
  if (path < 0 || path > 5) return fail(DWT2_ERR_ARG, "path must be 0 .. 5");
  g_persistent.store(path);
  return DWT2_OK;
}

int dwt2_tune(int32_t dir, const void* src, int64_t src_stride, int64_t src_batch_stride, void* dst,
              int64_t dst_stride, int64_t dst_batch_stride, int32_t width, int32_t height, int32_t batch,
              int32_t levels, int32_t mode, int32_t boundary, void* workspace, size_t workspace_bytes, void* stream) {
  clear_error();
  if (dir < 0 || dir > kTune97 + 1)
    return fail(DWT2_ERR_ARG, "dir must be 0 (forward), 1 (inverse), 2 (adjoint), 3 (CDF 9/7 forward) or 4 (CDF 9/7 inverse)");
  return tune(dir, src, src_stride, src_batch_stride, dst, dst_stride, dst_batch_stride, width, height, batch, levels,
              mode, boundary, workspace, workspace_bytes, stream);
}

int32_t dwt2_tune_entries(void) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  return (int32_t)g_tuned_seg.size();
}

int dwt2_tune_clear(void) {
  clear_error();
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tuned_seg.clear();
  return DWT2_OK;
}

int32_t dwt2_launch_levels(int32_t width, int32_t height, int32_t batch, int32_t levels, int32_t dir,
                           int32_t* first, int32_t* last, int32_t cap) {
  clear_error();
  Geo g;
  if (batch < 1 || dir < 0 || dir > 2) return fail(DWT2_ERR_ARG, "batch must be >= 1 and dir 0..2");
  if (int st = check_geometry(width, height, levels, g)) return st;
  if (g_persistent.load() < 0) g_persistent.store(env_int("DWT2_PERSISTENT") == 1 ? 1 : 0);
  const int path = g_persistent.load();
  if (path == 1 && g.L <= kInlineDescs) {  // one cooperative launch covers every level
    if (cap >= 1 && first && last) {
      first[0] = 1;
      last[0] = g.L;
    }
    return 1;
  }
  Launch plan[DWT2_MAX_LEVELS];
  const int pairs = path == 3 || path == 4 ? kPairsAll : (path == 0 ? kPairsDefault : kPairsNone);
  const int n = plan_launches(dir, g, batch, path != 2 && path != 4, pairs, plan);
  for (int i = 0; i < n && i < cap && first && last; ++i) {
    first[i] = plan[i].first;
    last[i] = plan[i].last;
  }
  return n;
}

int dwt2_set_job_wait(int32_t max_polls, int32_t unreachable) {
  clear_error();
  if (max_polls < 0 || (unreachable != 0 && unreachable != 1))
    return fail(DWT2_ERR_ARG, "max_polls must be >= 0 and unreachable 0 or 1");
  g_max_polls.store((uint32_t)max_polls);
  g_unreachable.store((uint32_t)unreachable);
  return DWT2_OK;
}

int dwt2_synchronize(void* stream) {
  clear_error();
  const hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(DWT2_ERR_HIP, "stream synchronisation failed: %s", hipGetErrorString(e));
  return take_async_error();
}

int dwt2_set_tiling(int32_t seg, int32_t chunk) {
  clear_error();
  if (seg < 0 || seg > (1 << 20) || !(chunk == 0 || chunk == 1 || chunk == 2 || chunk == 4))
    return fail(DWT2_ERR_ARG, "seg must be >= 0 and chunk one of 0, 1, 2, 4");
  g_forced_seg.store(seg);
  g_forced_ch.store(chunk);
  return DWT2_OK;
}

}  // extern "C"
