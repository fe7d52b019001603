// C-ABI entry points of libdwt2: argument validation, level geometry,
// workspace layout and the per-level launch sequence.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

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

static size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

// Per-image workspace: LL buffers A (odd levels) and B (even levels).
void ws_layout(const Geo& g, size_t& a_bytes, size_t& b_bytes) {
  a_bytes = g.L >= 2 ? round256((size_t)ll_pitch(g.w[1]) * g.h[1] * 4) : 0;
  b_bytes = g.L >= 3 ? round256((size_t)ll_pitch(g.w[2]) * g.h[2] * 4) : 0;
}

size_t ws_per_image(const Geo& g) {
  size_t a, b;
  ws_layout(g, a, b);
  return a + b;
}

int choose_seg(int ns_h, int64_t strips_times_batch) {
  static const int forced = [] {
    const char* e = getenv("DWT2_SEG");
    return e ? atoi(e) : 0;
  }();
  if (forced > 0) return forced;
  int seg = 64;
  while (seg > 1 && strips_times_batch * ((ns_h + seg - 1) / seg) < 4096) seg >>= 1;
  return seg;
}

void fill_level(LevelDesc& d, int W, int H, int seg) {
  d.W = W;
  d.H = H;
  d.seg = seg;
  d.nstrips = num_strips(W);
  d.nsegs = (ceil_half(H) + seg - 1) / seg;
}

// LL_m lives in buffer A (m odd) or B (m even) of each image's workspace slice.
static char* ll_buf(const Call& c, const Geo& g, int m) {
  size_t a, b;
  ws_layout(g, a, b);
  return c.ws + ((m & 1) ? 0 : a);
}

int run_levels(int dir, const Call& c, const Geo& g, void* stream) {
  const int64_t ws_bs = (int64_t)(ws_per_image(g) / 4);
  const int order_begin = dir == kFwd ? 1 : g.L, order_end = dir == kFwd ? g.L + 1 : 0;
  const int step = dir == kFwd ? 1 : -1;
  for (int k = order_begin; k != order_end; k += step) {
    LevelLaunch a;
    memset(&a, 0, sizeof a);
    const int W = g.w[k - 1], H = g.h[k - 1];
    const int64_t strips_batch = (int64_t)num_strips(W) * c.batch;
    fill_level(a.d, W, H, choose_seg(ceil_half(H), strips_batch));
    // pixels of the level input: the image (k = 1) or LL_{k-1}
    const bool px_is_image = (k == 1);
    char* px = px_is_image ? (dir == kFwd ? const_cast<char*>(c.src) : c.dst) : ll_buf(c, g, k - 1);
    a.d.pix_stride = px_is_image ? (dir == kFwd ? c.src_stride : c.dst_stride) : ll_pitch(g.w[k - 1]);
    a.pix_bstride = px_is_image ? (dir == kFwd ? c.src_bs : c.dst_bs) : ws_bs;
    // LL_k: the packed array's corner at the last level, else a workspace buffer
    const bool ll_is_packed = (k == g.L);
    char* ll = ll_is_packed ? (dir == kFwd ? c.dst : const_cast<char*>(c.src)) : ll_buf(c, g, k);
    a.d.ll_stride = ll_is_packed ? (dir == kFwd ? c.dst_stride : c.src_stride) : ll_pitch(g.w[k]);
    a.ll_bstride = ll_is_packed ? (dir == kFwd ? c.dst_bs : c.src_bs) : ws_bs;
    if (dir == kFwd) {
      a.d.pix_in = px;
      a.d.ll_out = ll;
      a.d.band_out = c.dst;
      a.d.band_stride = c.dst_stride;
      a.band_bstride = c.dst_bs;
    } else {
      a.d.pix_out = px;
      a.d.ll_in = ll;
      a.d.band_in = c.src;
      a.d.band_stride = c.src_stride;
      a.band_bstride = c.src_bs;
    }
    a.items_per_image = a.d.nstrips * a.d.nsegs;
    a.items = (int64_t)a.items_per_image * c.batch;
    const int err = launch_level(dir, c.mode, 4, a, stream);
    if (err != hipSuccess)
      return fail(DWT2_ERR_HIP, "level %d launch failed: %s", k, hipGetErrorString((hipError_t)err));
  }
  return DWT2_OK;
}

static int transform(int dir, const void* src, int64_t src_stride, int64_t src_bs, void* dst, int64_t dst_stride,
                     int64_t dst_bs, int32_t width, int32_t height, int32_t batch, int32_t levels, int32_t mode,
                     int32_t boundary, void* workspace, size_t workspace_bytes, void* stream) {
  clear_error();
  if (!src || !dst) return fail(DWT2_ERR_ARG, "null src or dst");
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
  if (src == dst) return fail(DWT2_ERR_ALIAS, "src and dst are the same buffer; the transform is out of place");
  const size_t need = ws_per_image(g) * (size_t)batch;
  if (need > 0 && (!workspace || workspace_bytes < need))
    return fail(DWT2_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", need, workspace ? workspace_bytes : 0);
  Call c{static_cast<const char*>(src), src_stride, src_bs, static_cast<char*>(dst), dst_stride, dst_bs, batch, mode,
         static_cast<char*>(workspace)};
  return run_levels(dir, c, g, stream);
}

}  // namespace dwt2

using namespace dwt2;

extern "C" {

size_t dwt2_workspace_size(int32_t width, int32_t height, int32_t batch, int32_t levels, int32_t mode) {
  Geo g;
  if (batch < 1 || (mode != DWT2_F32 && mode != DWT2_I32_REV)) return 0;
  if (check_geometry(width, height, levels, g) != DWT2_OK) return 0;
  return ws_per_image(g) * (size_t)batch;
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

}  // extern "C"
