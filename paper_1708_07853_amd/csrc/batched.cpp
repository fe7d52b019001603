// dwt2_fwd_batched: a ragged list of images.
#include <hip/hip_runtime.h>

#include <vector>

#include "plan.h"

using namespace dwt2;

namespace {

int validate_images(const dwt2_image_t* images, int32_t n, int32_t levels, int32_t mode, std::vector<Geo>& geos,
                    size_t& total_ws) {
  if (!images || n < 1) return fail(DWT2_ERR_ARG, "need a host array of at least one image");
  if (mode != DWT2_F32 && mode != DWT2_I32_REV) return fail(DWT2_ERR_MODE, "unknown mode %d", mode);
  geos.resize(n);
  total_ws = 0;
  for (int i = 0; i < n; ++i) {
    const dwt2_image_t& im = images[i];
    if (!im.src || !im.dst) return fail(DWT2_ERR_ARG, "image %d: null src or dst", i);
    if (im.width >= 2 && (im.src_stride < im.width || im.dst_stride < im.width))
      return fail(DWT2_ERR_ARG, "image %d: stride < width", i);
    const int st = check_geometry(im.width, im.height, levels, geos[i]);
    if (st) return fail(st, "image %d: %s", i, dwt2_last_error());
    if (im.src == im.dst) return fail(DWT2_ERR_ALIAS, "image %d: src == dst", i);
    total_ws += ws_per_image(geos[i]);
  }
  return DWT2_OK;
}

}  // namespace

extern "C" {

size_t dwt2_batched_workspace_size(const dwt2_image_t* images, int32_t n, int32_t levels, int32_t mode) {
  std::vector<Geo> geos;
  size_t total = 0;
  if (validate_images(images, n, levels, mode, geos, total) != DWT2_OK) return 0;
  return total;
}

int dwt2_fwd_batched(const dwt2_image_t* images, int32_t n, int32_t levels, int32_t mode, int32_t boundary,
                     void* workspace, size_t workspace_bytes, void* stream) {
  clear_error();
  if (boundary != DWT2_EXT_SYMMETRIC) return fail(DWT2_ERR_ARG, "unknown boundary %d", boundary);
  std::vector<Geo> geos;
  size_t total = 0;
  int st = validate_images(images, n, levels, mode, geos, total);
  if (st) return st;
  if (total > 0 && (!workspace || workspace_bytes < total))
    return fail(DWT2_ERR_WORKSPACE, "workspace of %zu bytes needed, %zu given", total, workspace ? workspace_bytes : 0);
  size_t off = 0;
  for (int i = 0; i < n; ++i) {
    const dwt2_image_t& im = images[i];
    Call c{static_cast<const char*>(im.src), im.src_stride, 0, static_cast<char*>(im.dst), im.dst_stride, 0, 1, mode,
           static_cast<char*>(workspace) + off};
    st = run_levels(0, c, geos[i], stream);
    if (st) return st;
    off += ws_per_image(geos[i]);
  }
  return DWT2_OK;
}

void dwt2_clear_plan_cache(void) {}

}  // extern "C"
