// Separable lifting baseline (§2, eq. (3)): the comparison point of the
// non-separable scheme.  Every lifting step of a level is its own kernel
// launch, i.e. its own pass over the level in HBM:
//   HP  copy the level input into a work array, odd columns  -= P(even columns)
//   VP  odd rows    -= P(even rows)        (in place)
//   HU  even columns += U(odd columns)     (in place)
//   VU  even rows    += U(odd rows), and the whole array is written to its
//       Mallat places (LL to the next level's input, H bands to dst).
// Each step reads only values it does not write, so in-place passes have no
// hazards.  Boundaries use whole-sample symmetric extension; float steps
// round once per step (the separable order of eq. (3)), integer steps use
// the reversible floors, so integer results equal the fused kernels' bit for
// bit and float results agree up to rounding.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "dwt2_internal.h"

namespace dwt2 {
namespace {

__device__ __forceinline__ int sfold(int p, int n) {
  if ((unsigned)p < (unsigned)n) return p;
  const int m = 2 * (n - 1);
  p %= m;
  if (p < 0) p += m;
  return p >= n ? m - p : p;
}

// predict: x - 1/2 (l + r); update: x + 1/4 (l + r)  (float)
// predict: x - floor((l + r) / 2); update: x + floor((l + r + 2) / 4)  (int)
__device__ __forceinline__ float s_pred(float x, float l, float r) { return __fmaf_rn(-0.5f, l + r, x); }
__device__ __forceinline__ float s_upd(float x, float l, float r) { return __fmaf_rn(0.25f, l + r, x); }
__device__ __forceinline__ int s_pred(int x, int l, int r) { return x - ((l + r) >> 1); }
__device__ __forceinline__ int s_upd(int x, int l, int r) { return x + ((l + r + 2) >> 2); }

constexpr int kSepBlock = 256;

// Grids: x over columns (or column pairs), y and z over rows and images
// with grid-stride loops (a grid's y and z extents are limited to 65535).
constexpr unsigned kMaxGridYZ = 65535;

// HP: one thread per (column pair n, row r) of the level input.
template <typename T>
__global__ __launch_bounds__(kSepBlock) void sep_hp(const T* __restrict__ src, int64_t ss, int64_t sbs,
                                                    T* __restrict__ X, int64_t xp, int64_t xbs, int W, int H,
                                                    int batch) {
  const int c = 2 * (int)(blockIdx.x * kSepBlock + threadIdx.x);
  if (c >= W) return;
  for (int z = blockIdx.z; z < batch; z += gridDim.z)
    for (int r = blockIdx.y; r < H; r += gridDim.y) {
      const T* s = src + z * sbs + (int64_t)r * ss;
      T* x = X + z * xbs + (int64_t)r * xp;
      const T a = s[c];
      x[c] = a;
      if (c + 1 < W) x[c + 1] = s_pred(s[c + 1], a, s[sfold(c + 2, W)]);
    }
}

// VP: one thread per (column c, odd row 2m + 1).
template <typename T>
__global__ __launch_bounds__(kSepBlock) void sep_vp(T* __restrict__ X, int64_t xp, int64_t xbs, int W, int H,
                                                    int batch) {
  const int c = blockIdx.x * kSepBlock + threadIdx.x;
  if (c >= W) return;
  for (int z = blockIdx.z; z < batch; z += gridDim.z)
    for (int m = blockIdx.y; m < (H >> 1); m += gridDim.y) {
      T* x = X + z * xbs + c;
      const int r = 2 * m + 1;
      x[(int64_t)r * xp] = s_pred(x[(int64_t)r * xp], x[(int64_t)(r - 1) * xp], x[(int64_t)sfold(r + 1, H) * xp]);
    }
}

// HU: one thread per (even column 2n, row r).
template <typename T>
__global__ __launch_bounds__(kSepBlock) void sep_hu(T* __restrict__ X, int64_t xp, int64_t xbs, int W, int H,
                                                    int batch) {
  const int c = 2 * (int)(blockIdx.x * kSepBlock + threadIdx.x);
  if (c >= W) return;
  for (int z = blockIdx.z; z < batch; z += gridDim.z)
    for (int r = blockIdx.y; r < H; r += gridDim.y) {
      T* x = X + z * xbs + (int64_t)r * xp;
      x[c] = s_upd(x[c], x[sfold(c - 1, W)], x[sfold(c + 1, W)]);
    }
}

// VU + Mallat packing: one thread per (column c, even row 2m).
template <typename T>
__global__ __launch_bounds__(kSepBlock) void sep_vu(const T* __restrict__ X, int64_t xp, int64_t xbs, int W, int H,
                                                    int batch, T* __restrict__ ll, int64_t ls, int64_t lbs,
                                                    T* __restrict__ band, int64_t bs, int64_t bbs) {
  const int c = blockIdx.x * kSepBlock + threadIdx.x;
  if (c >= W) return;
  const int ns_w = (W + 1) >> 1, ns_h = (H + 1) >> 1;
  for (int z = blockIdx.z; z < batch; z += gridDim.z)
    for (int m = blockIdx.y; m < ns_h; m += gridDim.y) {
      const T* x = X + z * xbs + c;
      const int r = 2 * m;
      const T e = s_upd(x[(int64_t)r * xp], x[(int64_t)sfold(r - 1, H) * xp], x[(int64_t)sfold(r + 1, H) * xp]);
      T* b = band + z * bbs;
      if (c & 1) b[(int64_t)m * bs + ns_w + (c >> 1)] = e;                    // HL
      else ll[z * lbs + (int64_t)m * ls + (c >> 1)] = e;                      // LL
      if (r + 1 < H) {
        const T o = x[(int64_t)(r + 1) * xp];
        b[(int64_t)(ns_h + m) * bs + ((c & 1) ? ns_w : 0) + (c >> 1)] = o;   // HH / LH
      }
    }
}

unsigned yz(int64_t n) { return (unsigned)(n < 1 ? 1 : (n > kMaxGridYZ ? kMaxGridYZ : n)); }

template <typename T>
hipError_t sep_level_t(const SepLevel& a, hipStream_t s) {
  const int W = a.W, H = a.H, B = a.batch;
  const unsigned gx_pair = (unsigned)((((W + 1) >> 1) + kSepBlock - 1) / kSepBlock);
  const unsigned gx_col = (unsigned)((W + kSepBlock - 1) / kSepBlock);
  T* X = static_cast<T*>(a.work);
  hipLaunchKernelGGL(sep_hp<T>, dim3(gx_pair, yz(H), yz(B)), dim3(kSepBlock), 0, s, static_cast<const T*>(a.src),
                     a.src_stride, a.src_bstride, X, a.work_pitch, a.work_bstride, W, H, B);
  if (H >> 1)
    hipLaunchKernelGGL(sep_vp<T>, dim3(gx_col, yz(H >> 1), yz(B)), dim3(kSepBlock), 0, s, X, a.work_pitch,
                       a.work_bstride, W, H, B);
  hipLaunchKernelGGL(sep_hu<T>, dim3(gx_pair, yz(H), yz(B)), dim3(kSepBlock), 0, s, X, a.work_pitch, a.work_bstride,
                     W, H, B);
  hipLaunchKernelGGL(sep_vu<T>, dim3(gx_col, yz((H + 1) >> 1), yz(B)), dim3(kSepBlock), 0, s,
                     static_cast<const T*>(X), a.work_pitch, a.work_bstride, W, H, B, static_cast<T*>(a.ll),
                     a.ll_stride, a.ll_bstride, static_cast<T*>(a.band), a.band_stride, a.band_bstride);
  return hipGetLastError();
}

}  // namespace

int launch_separable_level(int mode, const SepLevel& a, void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  return mode == DWT2_F32 ? sep_level_t<float>(a, s) : sep_level_t<int>(a, s);
}

}  // namespace dwt2
