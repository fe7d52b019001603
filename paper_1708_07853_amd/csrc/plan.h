// Host-side helpers shared by the plain entry points (api.cpp) and the
// batched entry point (batched.cpp).
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "dwt2_internal.h"

namespace dwt2 {

struct Geo {
  int L;
  int w[DWT2_MAX_LEVELS + 1];
  int h[DWT2_MAX_LEVELS + 1];
};

// One uniform-geometry call (a batch of equally sized images).
struct Call {
  const char* src;
  int64_t src_stride, src_bs;
  char* dst;
  int64_t dst_stride, dst_bs;
  int32_t batch;
  int32_t mode;
  char* ws;
  size_t ll_base;  // byte offset of the first image's LL buffers in ws
};

int fail(int code, const char* fmt, ...);
// Byte range [lo, hi) from the first to one past the last element of a
// (batch of) w x h images of 4-byte samples; the alias checks compare these.
struct Span {
  uintptr_t lo, hi;
};
inline Span image_span(const void* p, int64_t stride, int64_t bstride, int w, int h, int batch) {
  const uintptr_t lo = reinterpret_cast<uintptr_t>(p);
  const int64_t last = (int64_t)(batch - 1) * bstride + (int64_t)(h - 1) * stride + w;
  return Span{lo, lo + (uintptr_t)last * 4u};
}
inline bool overlap(const Span& a, const Span& b) { return a.lo < b.hi && b.lo < a.hi; }
void clear_error();
int check_geometry(int32_t width, int32_t height, int32_t levels, Geo& g);
size_t round256(size_t b);
size_t ll_offset(const Geo& g, int m);
size_t ws_per_image(const Geo& g);
size_t sync_bytes(const Geo& g, int64_t batch);
struct Tiling {
  int seg;  // quadruple rows per work item
  int ch;   // rows per prefetch chunk (kernel template)
};
Tiling choose_tiling(int ns_h, int64_t strips_times_batch, int64_t slots_hint = 0);
void fill_level(LevelDesc& d, int W, int H, int seg);
void level_pointers(int dir, const Call& c, const Geo& g, int k, LevelDesc& d, int64_t& pix_bs, int64_t& ll_bs,
                    int64_t& band_bs);
// One launch of a plain call: levels [first, last], by the single-level,
// pair or fused-tail kernels (kLaunch97: a CDF 9/7 strip-kernel level, for
// the tuning table).
enum { kLaunchLevel = 0, kLaunchPair = 1, kLaunchTail = 2, kLaunch97 = 3 };
struct Launch {
  int first, last, kind;
};
// Which levels go in pairs: none, every pair that applies, or the pairs the
// default path picks (see default_pair in api.cpp).
enum { kPairsNone = 0, kPairsAll = 1, kPairsDefault = 2 };
int plan_launches(int dir, const Geo& g, int batch, bool tail, int pairs, Launch* out);
// The launch of levels k and k+1 by the pair kernels for a call: geometry,
// pointers, tiling (seg_override > 0: that segment height in level-(k+1)
// quadruple rows) and whether the forward stages its stores (only if
// allow_stage: staging needs four adjacent strips of one image and segment
// per workgroup).
void pair_launch(int dir, const Call& c, const Geo& g, int k, LevelLaunch& a, int& ch, int seg_override = 0,
                 bool allow_stage = true);
int run_levels(int dir, const Call& c, const Geo& g, void* stream, bool tail, int pairs);
int run_job(int dir, const Call& c, const Geo& g, void* stream);
// dwt2_fwd on the per-level path whatever the process-wide path setting
// (validation, errors and results as dwt2_fwd).
int fwd_levels_path(const void* src, int64_t src_stride, int64_t src_bs, void* dst, int64_t dst_stride,
                    int64_t dst_bs, int32_t width, int32_t height, int32_t batch, int32_t levels, int32_t mode,
                    int32_t boundary, void* workspace, size_t workspace_bytes, void* stream);
// DWT2_ERR_HIP (once) if a persistent launch gave up a wait since the last report.
int report_async_error();

}  // namespace dwt2
