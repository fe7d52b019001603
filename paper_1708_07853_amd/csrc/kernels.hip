// HIP kernels for gfx950: one level of the 2-D CDF 5/3 transform with the
// non-separable lifting scheme (§3, eq. (5)) -- forward, inverse, adjoint.
//
// Mapping.  A wave owns a vertical strip of 128 quadruple columns (lane l
// holds quadruple columns 2l and 2l+1, i.e. one 16-byte vector of each pixel
// row) and walks down a segment of quadruple rows.  Vertical neighbours stay
// in registers from one row to the next; horizontal neighbours cross lanes
// with one shuffle per exchanged value.  Each level therefore reads its input
// once and writes its output once; the only synchronisation points of the
// lifting (the "|" of eq. (5)) become lane shuffles: one exchange of the
// right neighbour's L samples for the spatial predict and one of the left
// neighbour's predicted values for the spatial update.
//
// Boundaries.  Forward and inverse read the whole-sample symmetric extension
// of their input (the interleaved coefficient array for the inverse), so the
// interior formulas hold everywhere.  The adjoint transposes that extension
// with explicit boundary weights instead (zero outside, doubled where the
// mirror folds two taps onto one sample).
#include <hip/hip_runtime.h>

#include <type_traits>

#include "dwt2_internal.h"

namespace dwt2 {
namespace {

template <typename T>
struct V4 {
  T x, y, z, w;
};
template <typename T>
using Ext2 = T __attribute__((ext_vector_type(2)));
template <typename T>
using Ext4 = T __attribute__((ext_vector_type(4)));

// Whole-sample symmetric fold of index p onto [0, n), n >= 2.
__device__ __forceinline__ int fold_idx(int p, int n) {
  if ((unsigned)p < (unsigned)n) return p;
  const int m = 2 * (n - 1);
  p %= m;
  if (p < 0) p += m;
  return p >= n ? m - p : p;
}

// Row of band coefficients for interleaved index p of parity `par` (0: L, 1: H)
// of an axis of length n, following the symmetric extension.
__device__ __forceinline__ int band_idx(int q, int n, int par) {
  return (fold_idx(2 * q + par, n) - par) >> 1;
}

__device__ __forceinline__ bool aligned(const void* p, unsigned bytes) {
  return ((uintptr_t)p & (bytes - 1)) == 0;
}

template <typename T>
__device__ __forceinline__ T shfl_dn(T v) {
  return __shfl_down(v, 1, kWave);
}
template <typename T>
__device__ __forceinline__ T shfl_up(T v) {
  return __shfl_up(v, 1, kWave);
}

// Four consecutive pixels c0..c0+3 of (folded) row r.
template <typename T>
__device__ __forceinline__ V4<T> load_px4(const T* base, int64_t stride, int r, int H, int c0, int W) {
  const T* row = base + (int64_t)fold_idx(r, H) * stride;
  V4<T> v;
  if (c0 >= 0 && c0 + 3 < W && aligned(row + c0, 16)) {
    const Ext4<T> t = *reinterpret_cast<const Ext4<T>*>(row + c0);
    v.x = t.x; v.y = t.y; v.z = t.z; v.w = t.w;
  } else {
    v.x = row[fold_idx(c0, W)];
    v.y = row[fold_idx(c0 + 1, W)];
    v.z = row[fold_idx(c0 + 2, W)];
    v.w = row[fold_idx(c0 + 3, W)];
  }
  return v;
}

// Two consecutive band coefficients q, q+1 of a band row with n entries
// (n = count of that parity on an axis of length Wl), mirrored outside.
template <typename T>
__device__ __forceinline__ void load_band2(const T* row, int q, int n, int Wl, int par, T& vL, T& vR) {
  if (q >= 0 && q + 1 < n && aligned(row + q, 8)) {
    const Ext2<T> t = *reinterpret_cast<const Ext2<T>*>(row + q);
    vL = t.x; vR = t.y;
  } else {
    vL = row[band_idx(q, Wl, par)];
    vR = row[band_idx(q + 1, Wl, par)];
  }
}

// Same, but zero outside [0, n) (adjoint: no extension).
template <typename T>
__device__ __forceinline__ void load_band2_zero(const T* row, int q, int n, T& vL, T& vR) {
  if (q >= 0 && q + 1 < n && aligned(row + q, 8)) {
    const Ext2<T> t = *reinterpret_cast<const Ext2<T>*>(row + q);
    vL = t.x; vR = t.y;
  } else {
    vL = (q >= 0 && q < n) ? row[q] : T(0);
    vR = (q + 1 >= 0 && q + 1 < n) ? row[q + 1] : T(0);
  }
}

template <typename T>
__device__ __forceinline__ void store2(T* row, int q, T vL, T vR, bool okL, bool okR) {
  if (okL && okR && aligned(row + q, 8)) {
    Ext2<T> t;
    t.x = vL; t.y = vR;
    *reinterpret_cast<Ext2<T>*>(row + q) = t;
  } else {
    if (okL) row[q] = vL;
    if (okR) row[q + 1] = vR;
  }
}

// Pixels c0..c0+3 of one output row; quadruple L covers c0, c0+1 and R covers
// c0+2, c0+3.
template <typename T>
__device__ __forceinline__ void store_px4(T* row, int c0, int W, V4<T> v, bool okL, bool okR) {
  if (okL && okR && c0 >= 0 && c0 + 3 < W && aligned(row + c0, 16)) {
    Ext4<T> t;
    t.x = v.x; t.y = v.y; t.z = v.z; t.w = v.w;
    *reinterpret_cast<Ext4<T>*>(row + c0) = t;
  } else {
    if (okL) {
      if (c0 >= 0 && c0 < W) row[c0] = v.x;
      if (c0 + 1 >= 0 && c0 + 1 < W) row[c0 + 1] = v.y;
    }
    if (okR) {
      if (c0 + 2 >= 0 && c0 + 2 < W) row[c0 + 2] = v.z;
      if (c0 + 3 >= 0 && c0 + 3 < W) row[c0 + 3] = v.w;
    }
  }
}

// ---------------------------------------------------------------------------
// Per-quadruple arithmetic.  Every kernel variant evaluates exactly these
// expressions, so results do not depend on tiling or scheduling.
// Neighbour suffixes: R = next column, D = next row, L = previous column,
// U = previous row.
// ---------------------------------------------------------------------------

// Spatial predict, eq. (5) right matrix: b' = b + P a, c' = c + P* a,
// d' = d + P c + P* b + P P* a.
__device__ __forceinline__ void f32_predict(float a, float aR, float aD, float aDR, float b, float bD,
                                            float c, float cR, float d, float& bp, float& cp, float& dp) {
  const float sh = a + aR;
  bp = __fmaf_rn(-0.5f, sh, b);
  cp = __fmaf_rn(-0.5f, a + aD, c);
  dp = __fmaf_rn(0.25f, sh + (aD + aDR), __fmaf_rn(-0.5f, b + bD, __fmaf_rn(-0.5f, c + cR, d)));
}

// Spatial update, eq. (5) left matrix: LL = a + U b' + U* c' + U U* d',
// HL = b' + U* d', LH = c' + U d' (HH = d').
__device__ __forceinline__ void f32_update(float a, float bpL, float bp, float cpU, float cp, float dpUL,
                                           float dpU, float dpL, float dp, float& ll, float& hl, float& lh) {
  hl = __fmaf_rn(0.25f, dpU + dp, bp);
  lh = __fmaf_rn(0.25f, dpL + dp, cp);
  ll = __fmaf_rn(0.0625f, (dpUL + dpU) + (dpL + dp), __fmaf_rn(0.25f, cpU + cp, __fmaf_rn(0.25f, bpL + bp, a)));
}

// Integer spatial predict: horizontal then vertical rounded predict composed
// (eq. (3) order).  Outputs b1 (HL after HP), c1 (LH after VP), d2 (final HH).
__device__ __forceinline__ void i32_predict(int a, int aR, int aD, int aDR, int b, int bD, int c, int cR,
                                            int d, int& b1, int& c1, int& d2) {
  b1 = b - ((a + aR) >> 1);
  const int d1 = d - ((c + cR) >> 1);
  c1 = c - ((a + aD) >> 1);
  const int b1D = bD - ((aD + aDR) >> 1);
  d2 = d1 - ((b1 + b1D) >> 1);
}

// The horizontal rounded update of LH: c2 = c1 + floor((d2L + d2 + 2) / 4).
__device__ __forceinline__ int i32_c2(int c1, int d2L, int d2) { return c1 + ((d2L + d2 + 2) >> 2); }

// Integer spatial update: horizontal then vertical rounded update composed.
__device__ __forceinline__ void i32_update(int a, int b1L, int b1, int c2U, int c2, int d2U, int d2, int& ll,
                                           int& hl) {
  const int a1 = a + ((b1L + b1 + 2) >> 2);
  ll = a1 + ((c2U + c2 + 2) >> 2);
  hl = b1 + ((d2U + d2 + 2) >> 2);
}

// Inverse of the spatial update (matrix inverse of eq. (5) left).
__device__ __forceinline__ void f32_inv_update(float ll, float hlL, float hl, float lhU, float lh, float hhUL,
                                               float hhU, float hhL, float hh, float& a, float& bp, float& cp) {
  bp = __fmaf_rn(-0.25f, hhU + hh, hl);
  cp = __fmaf_rn(-0.25f, hhL + hh, lh);
  a = __fmaf_rn(0.0625f, (hhUL + hhU) + (hhL + hh), __fmaf_rn(-0.25f, lhU + lh, __fmaf_rn(-0.25f, hlL + hl, ll)));
}

// Inverse of the spatial predict (matrix inverse of eq. (5) right).
__device__ __forceinline__ void f32_inv_predict(float a, float aR, float aD, float aDR, float bp, float bpD,
                                                float cp, float cpR, float dp, float& b, float& c, float& d) {
  const float sh = a + aR;
  b = __fmaf_rn(0.5f, sh, bp);
  c = __fmaf_rn(0.5f, a + aD, cp);
  d = __fmaf_rn(0.25f, sh + (aD + aDR), __fmaf_rn(0.5f, bp + bpD, __fmaf_rn(0.5f, cp + cpR, dp)));
}

// Integer inverse, first half (undo vertical then horizontal update):
// a1 = a2 - floor((c2U + c2 + 2)/4), b1 = b2 - floor((d2U + d2 + 2)/4),
// a = a1 - floor((b1L + b1 + 2)/4), c1 = c2 - floor((d2L + d2 + 2)/4).
__device__ __forceinline__ int i32_inv_b1(int b2, int d2U, int d2) { return b2 - ((d2U + d2 + 2) >> 2); }
__device__ __forceinline__ void i32_inv_update(int a2, int c2U, int c2, int b1L, int b1, int d2L, int d2, int& a,
                                               int& c1) {
  const int a1 = a2 - ((c2U + c2 + 2) >> 2);
  a = a1 - ((b1L + b1 + 2) >> 2);
  c1 = c2 - ((d2L + d2 + 2) >> 2);
}
// Second half (undo vertical then horizontal predict).
__device__ __forceinline__ int i32_inv_c(int c1, int a, int aD) { return c1 + ((a + aD) >> 1); }
__device__ __forceinline__ void i32_inv_predict(int a, int aR, int b1, int b1D, int c, int cR, int d2, int& b,
                                                int& d) {
  const int d1 = d2 + ((b1 + b1D) >> 1);
  b = b1 + ((a + aR) >> 1);
  d = d1 + ((c + cR) >> 1);
}

// Boundary weights of the transposed steps on an axis of length n
// (ns = ceil(n/2) L and nd = floor(n/2) H coefficients).
//   U^T at H index m:  alpha (own L sample m), beta (L sample m + 1)
//   P^T at L index m:  gamma (H sample m - 1), delta (H sample m)
struct AxisW {
  float alpha, beta, gamma, delta;
};
__device__ __forceinline__ AxisW axis_weights(int m, int n) {
  const int ns = (n + 1) >> 1, nd = n >> 1;
  const bool odd = n & 1;
  AxisW w;
  w.alpha = (m == 0) ? 2.f : 1.f;
  if (m < 0) w.beta = 1.f;
  else if (!odd && m + 1 >= ns) w.beta = 0.f;
  else if (odd && m == nd - 1) w.beta = 2.f;
  else if (m >= nd) w.beta = 0.f;
  else w.beta = 1.f;
  w.gamma = (m == 0) ? 0.f : 1.f;
  if (m < 0) w.delta = 1.f;
  else if (odd && m == nd) w.delta = 0.f;
  else if (!odd && m == nd - 1) w.delta = 2.f;
  else if (m >= ns) w.delta = 0.f;
  else w.delta = 1.f;
  return w;
}

// Transposed spatial update (M_U^T, predict-shaped).
__device__ __forceinline__ void f32_adj_a(float ga, float gaR, float gaD, float gaDR, float gb, float gbD,
                                          float gc, float gcR, float gd, AxisW h, AxisW v, float& gb1, float& gc1,
                                          float& gd1) {
  const float th = h.alpha * ga + h.beta * gaR;      // U^T_h ga (x4)
  const float thD = h.alpha * gaD + h.beta * gaDR;
  gb1 = __fmaf_rn(0.25f, th, gb);
  gc1 = __fmaf_rn(0.25f, v.alpha * ga + v.beta * gaD, gc);
  gd1 = __fmaf_rn(0.0625f, v.alpha * th + v.beta * thD,
                  __fmaf_rn(0.25f, h.alpha * gc + h.beta * gcR, __fmaf_rn(0.25f, v.alpha * gb + v.beta * gbD, gd)));
}

// Transposed spatial predict (M_P^T, update-shaped).
__device__ __forceinline__ void f32_adj_b(float ga, float gb1L, float gb1, float gc1U, float gc1, float gd1UL,
                                          float gd1U, float gd1L, float gd1, AxisW h, AxisW v, float& ga2,
                                          float& gb2, float& gc2) {
  gb2 = __fmaf_rn(-0.5f, v.gamma * gd1U + v.delta * gd1, gb1);
  gc2 = __fmaf_rn(-0.5f, h.gamma * gd1L + h.delta * gd1, gc1);
  const float tU = h.gamma * gd1UL + h.delta * gd1U;
  const float t0 = h.gamma * gd1L + h.delta * gd1;
  ga2 = __fmaf_rn(0.25f, v.gamma * tU + v.delta * t0,
                  __fmaf_rn(-0.5f, v.gamma * gc1U + v.delta * gc1, __fmaf_rn(-0.5f, h.gamma * gb1L + h.delta * gb1, ga)));
}

// ---------------------------------------------------------------------------
// Work item = (image, segment of quadruple rows, strip); one wave each.
// ---------------------------------------------------------------------------
struct Item {
  int W, H, ns_w, nd_w, ns_h, nd_h;
  int qL;        // global quadruple column of this lane's first quadruple
  int I0, I1;    // quadruple rows written
  bool outL, outR;
};

__device__ __forceinline__ Item make_item(const LevelDesc& d, int strip, int seg, int lane) {
  Item it;
  it.W = d.W; it.H = d.H;
  it.ns_w = (d.W + 1) >> 1; it.nd_w = d.W >> 1;
  it.ns_h = (d.H + 1) >> 1; it.nd_h = d.H >> 1;
  it.qL = kStripOut * strip - 2 + 2 * lane;
  it.I0 = seg * d.seg;
  it.I1 = min(it.I0 + d.seg, it.ns_h);
  it.outL = lane != 0;
  it.outR = lane != kWave - 1 && it.qL + 1 >= 0;
  return it;
}

// ----------------------------------------------------------------- forward
template <int CH>
__device__ void fwd_f32(const LevelDesc& d, const float* __restrict__ px, float* __restrict__ ll,
                        float* __restrict__ band, const Item& it) {
  const int W = it.W, H = it.H, c0 = 2 * it.qL;
  const int64_t ps = d.pix_stride, ls = d.ll_stride, bs = d.band_stride;
  const int qL = it.qL, qR = qL + 1;
  const bool llL = it.outL && qL < it.ns_w, llR = it.outR && qR < it.ns_w;
  const bool hlL = it.outL && qL < it.nd_w, hlR = it.outR && qR < it.nd_w;

  // prologue: predicted values of quadruple row I0 - 1
  V4<float> E = load_px4(px, ps, 2 * it.I0 - 2, H, c0, W);
  V4<float> O = load_px4(px, ps, 2 * it.I0 - 1, H, c0, W);
  V4<float> E1 = load_px4(px, ps, 2 * it.I0, H, c0, W);
  float aN = shfl_dn(E.x), aDN = shfl_dn(E1.x), cN = shfl_dn(O.x);
  float cpU_L, cpU_R, dpU_L, dpU_R, dpUL_L;
  {
    float bpL, bpR;
    f32_predict(E.x, E.z, E1.x, E1.z, E.y, E1.y, O.x, O.z, O.y, bpL, cpU_L, dpU_L);
    f32_predict(E.z, aN, E1.z, aDN, E.w, E1.w, O.z, cN, O.w, bpR, cpU_R, dpU_R);
    dpUL_L = shfl_up(dpU_R);
  }
  E = E1;
  aN = aDN;

  for (int i0 = it.I0; i0 < it.I1; i0 += CH) {
    V4<float> Ob[CH], Eb[CH];
#pragma unroll
    for (int m = 0; m < CH; ++m) {
      Ob[m] = load_px4(px, ps, 2 * (i0 + m) + 1, H, c0, W);
      Eb[m] = load_px4(px, ps, 2 * (i0 + m) + 2, H, c0, W);
    }
#pragma unroll
    for (int m = 0; m < CH; ++m) {
      const int i = i0 + m;
      if (i < it.I1) {
        const V4<float> o = Ob[m], e1 = Eb[m];
        const float aDN1 = shfl_dn(e1.x), cN1 = shfl_dn(o.x);
        float bpL, cpL, dpL, bpR, cpR, dpR;
        f32_predict(E.x, E.z, e1.x, e1.z, E.y, e1.y, o.x, o.z, o.y, bpL, cpL, dpL);
        f32_predict(E.z, aN, e1.z, aDN1, E.w, e1.w, o.z, cN1, o.w, bpR, cpR, dpR);
        const float bpP = shfl_up(bpR), dpP = shfl_up(dpR);
        float llv_L, hlv_L, lhv_L, llv_R, hlv_R, lhv_R;
        f32_update(E.x, bpP, bpL, cpU_L, cpL, dpUL_L, dpU_L, dpP, dpL, llv_L, hlv_L, lhv_L);
        f32_update(E.z, bpL, bpR, cpU_R, cpR, dpU_L, dpU_R, dpL, dpR, llv_R, hlv_R, lhv_R);
        store2(ll + (int64_t)i * ls, qL, llv_L, llv_R, llL, llR);
        store2(band + (int64_t)i * bs + it.ns_w, qL, hlv_L, hlv_R, hlL, hlR);
        if (i < it.nd_h) {
          float* r = band + (int64_t)(it.ns_h + i) * bs;
          store2(r, qL, lhv_L, lhv_R, llL, llR);
          store2(r + it.ns_w, qL, dpL, dpR, hlL, hlR);
        }
        cpU_L = cpL; cpU_R = cpR; dpU_L = dpL; dpU_R = dpR; dpUL_L = dpP;
        E = e1;
        aN = aDN1;
      }
    }
  }
}

template <int CH>
__device__ void fwd_i32(const LevelDesc& d, const int* __restrict__ px, int* __restrict__ ll,
                        int* __restrict__ band, const Item& it) {
  const int W = it.W, H = it.H, c0 = 2 * it.qL;
  const int64_t ps = d.pix_stride, ls = d.ll_stride, bs = d.band_stride;
  const int qL = it.qL, qR = qL + 1;
  const bool llL = it.outL && qL < it.ns_w, llR = it.outR && qR < it.ns_w;
  const bool hlL = it.outL && qL < it.nd_w, hlR = it.outR && qR < it.nd_w;

  V4<int> E = load_px4(px, ps, 2 * it.I0 - 2, H, c0, W);
  V4<int> O = load_px4(px, ps, 2 * it.I0 - 1, H, c0, W);
  V4<int> E1 = load_px4(px, ps, 2 * it.I0, H, c0, W);
  int aN = shfl_dn(E.x), aDN = shfl_dn(E1.x), cN = shfl_dn(O.x);
  int c2U_L, c2U_R, d2U_L, d2U_R;
  {
    int b1L, c1L, b1R, c1R;
    i32_predict(E.x, E.z, E1.x, E1.z, E.y, E1.y, O.x, O.z, O.y, b1L, c1L, d2U_L);
    i32_predict(E.z, aN, E1.z, aDN, E.w, E1.w, O.z, cN, O.w, b1R, c1R, d2U_R);
    const int d2P = shfl_up(d2U_R);
    c2U_L = i32_c2(c1L, d2P, d2U_L);
    c2U_R = i32_c2(c1R, d2U_L, d2U_R);
  }
  E = E1;
  aN = aDN;

  for (int i0 = it.I0; i0 < it.I1; i0 += CH) {
    V4<int> Ob[CH], Eb[CH];
#pragma unroll
    for (int m = 0; m < CH; ++m) {
      Ob[m] = load_px4(px, ps, 2 * (i0 + m) + 1, H, c0, W);
      Eb[m] = load_px4(px, ps, 2 * (i0 + m) + 2, H, c0, W);
    }
#pragma unroll
    for (int m = 0; m < CH; ++m) {
      const int i = i0 + m;
      if (i < it.I1) {
        const V4<int> o = Ob[m], e1 = Eb[m];
        const int aDN1 = shfl_dn(e1.x), cN1 = shfl_dn(o.x);
        int b1L, c1L, d2L, b1R, c1R, d2R;
        i32_predict(E.x, E.z, e1.x, e1.z, E.y, e1.y, o.x, o.z, o.y, b1L, c1L, d2L);
        i32_predict(E.z, aN, e1.z, aDN1, E.w, e1.w, o.z, cN1, o.w, b1R, c1R, d2R);
        const int b1P = shfl_up(b1R), d2P = shfl_up(d2R);
        const int c2L = i32_c2(c1L, d2P, d2L), c2R = i32_c2(c1R, d2L, d2R);
        int llv_L, hlv_L, llv_R, hlv_R;
        i32_update(E.x, b1P, b1L, c2U_L, c2L, d2U_L, d2L, llv_L, hlv_L);
        i32_update(E.z, b1L, b1R, c2U_R, c2R, d2U_R, d2R, llv_R, hlv_R);
        store2(ll + (int64_t)i * ls, qL, llv_L, llv_R, llL, llR);
        store2(band + (int64_t)i * bs + it.ns_w, qL, hlv_L, hlv_R, hlL, hlR);
        if (i < it.nd_h) {
          int* r = band + (int64_t)(it.ns_h + i) * bs;
          store2(r, qL, c2L, c2R, llL, llR);
          store2(r + it.ns_w, qL, d2L, d2R, hlL, hlR);
        }
        c2U_L = c2L; c2U_R = c2R; d2U_L = d2L; d2U_R = d2R;
        E = e1;
        aN = aDN1;
      }
    }
  }
}

// ----------------------------------------------------------------- inverse
// Coefficient row r of the four bands for this lane's two quadruples,
// mirrored through the interleaved symmetric extension.
template <typename T>
struct Quad2 {
  T llL, llR, hlL, hlR, lhL, lhR, hhL, hhR;
};

template <typename T>
__device__ __forceinline__ void load_even(const T* ll, int64_t ls, const T* band, int64_t bs, const Item& it, int r,
                                          Quad2<T>& q) {
  const int re = fold_idx(2 * r, it.H) >> 1;
  load_band2(ll + (int64_t)re * ls, it.qL, it.ns_w, it.W, 0, q.llL, q.llR);
  load_band2(band + (int64_t)re * bs + it.ns_w, it.qL, it.nd_w, it.W, 1, q.hlL, q.hlR);
}
template <typename T>
__device__ __forceinline__ void load_odd(const T* band, int64_t bs, const Item& it, int r, Quad2<T>& q) {
  const int ro = (fold_idx(2 * r + 1, it.H) - 1) >> 1;
  const T* row = band + (int64_t)(it.ns_h + ro) * bs;
  load_band2(row, it.qL, it.ns_w, it.W, 0, q.lhL, q.lhR);
  load_band2(row + it.ns_w, it.qL, it.nd_w, it.W, 1, q.hhL, q.hhR);
}

template <int CH>
__device__ void inv_f32(const LevelDesc& d, const float* __restrict__ ll, const float* __restrict__ band,
                        float* __restrict__ px, const Item& it) {
  const int W = it.W, c0 = 2 * it.qL;
  const int64_t ps = d.pix_stride, ls = d.ll_stride, bs = d.band_stride;

  // prologue: odd part of row I0 - 1, full row I0, undo-update of row I0
  Quad2<float> q0, q1;
  load_odd(band, bs, it, it.I0 - 1, q0);
  load_even(ll, ls, band, bs, it, it.I0, q1);
  load_odd(band, bs, it, it.I0, q1);
  float hhUL_L = shfl_up(q0.hhR);
  float a_L, a_R, bp_L, bp_R, cp_L, cp_R;
  float lhU_L = q0.lhL, lhU_R = q0.lhR, hhU_L = q0.hhL, hhU_R = q0.hhR;
  {
    const float hlP = shfl_up(q1.hlR), hhP = shfl_up(q1.hhR);
    f32_inv_update(q1.llL, hlP, q1.hlL, lhU_L, q1.lhL, hhUL_L, hhU_L, hhP, q1.hhL, a_L, bp_L, cp_L);
    f32_inv_update(q1.llR, q1.hlL, q1.hlR, lhU_R, q1.lhR, hhU_L, hhU_R, q1.hhL, q1.hhR, a_R, bp_R, cp_R);
    hhUL_L = hhP;
  }
  float hh_L = q1.hhL, hh_R = q1.hhR;
  lhU_L = q1.lhL; lhU_R = q1.lhR; hhU_L = q1.hhL; hhU_R = q1.hhR;
  float aN = shfl_dn(a_L), cpN = shfl_dn(cp_L);

  for (int i0 = it.I0; i0 < it.I1; i0 += CH) {
    Quad2<float> qb[CH];
#pragma unroll
    for (int m = 0; m < CH; ++m) {
      load_even(ll, ls, band, bs, it, i0 + m + 1, qb[m]);
      load_odd(band, bs, it, i0 + m + 1, qb[m]);
    }
#pragma unroll
    for (int m = 0; m < CH; ++m) {
      const int i = i0 + m;
      if (i < it.I1) {
        const Quad2<float> n = qb[m];
        // undo the update for row i + 1
        const float hlP = shfl_up(n.hlR), hhP = shfl_up(n.hhR);
        float a1_L, a1_R, bp1_L, bp1_R, cp1_L, cp1_R;
        f32_inv_update(n.llL, hlP, n.hlL, lhU_L, n.lhL, hhUL_L, hhU_L, hhP, n.hhL, a1_L, bp1_L, cp1_L);
        f32_inv_update(n.llR, n.hlL, n.hlR, lhU_R, n.lhR, hhU_L, hhU_R, n.hhL, n.hhR, a1_R, bp1_R, cp1_R);
        const float aN1 = shfl_dn(a1_L), cpN1 = shfl_dn(cp1_L);
        // undo the predict for row i
        V4<float> e, o;
        e.x = a_L; e.z = a_R;
        f32_inv_predict(a_L, a_R, a1_L, a1_R, bp_L, bp1_L, cp_L, cp_R, hh_L, e.y, o.x, o.y);
        f32_inv_predict(a_R, aN, a1_R, aN1, bp_R, bp1_R, cp_R, cpN, hh_R, e.w, o.z, o.w);
        store_px4(px + (int64_t)(2 * i) * ps, c0, W, e, it.outL, it.outR);
        if (2 * i + 1 < it.H) store_px4(px + (int64_t)(2 * i + 1) * ps, c0, W, o, it.outL, it.outR);
        // advance
        a_L = a1_L; a_R = a1_R; bp_L = bp1_L; bp_R = bp1_R; cp_L = cp1_L; cp_R = cp1_R;
        hh_L = n.hhL; hh_R = n.hhR;
        lhU_L = n.lhL; lhU_R = n.lhR; hhU_L = n.hhL; hhU_R = n.hhR; hhUL_L = hhP;
        aN = aN1; cpN = cpN1;
      }
    }
  }
}

template <int CH>
__device__ void inv_i32(const LevelDesc& d, const int* __restrict__ ll, const int* __restrict__ band,
                        int* __restrict__ px, const Item& it) {
  const int W = it.W, c0 = 2 * it.qL;
  const int64_t ps = d.pix_stride, ls = d.ll_stride, bs = d.band_stride;

  Quad2<int> q0, q1;
  load_odd(band, bs, it, it.I0 - 1, q0);
  load_even(ll, ls, band, bs, it, it.I0, q1);
  load_odd(band, bs, it, it.I0, q1);
  // row I0: b1 (needs HH of row I0-1), then a and c1
  int b1_L = i32_inv_b1(q1.hlL, q0.hhL, q1.hhL), b1_R = i32_inv_b1(q1.hlR, q0.hhR, q1.hhR);
  int a_L, a_R, c1_L, c1_R;
  {
    const int b1P = shfl_up(b1_R), hhP = shfl_up(q1.hhR);
    i32_inv_update(q1.llL, q0.lhL, q1.lhL, b1P, b1_L, hhP, q1.hhL, a_L, c1_L);
    i32_inv_update(q1.llR, q0.lhR, q1.lhR, b1_L, b1_R, q1.hhL, q1.hhR, a_R, c1_R);
  }
  int hh_L = q1.hhL, hh_R = q1.hhR, lh_L = q1.lhL, lh_R = q1.lhR;
  int aN = shfl_dn(a_L);

  for (int i0 = it.I0; i0 < it.I1; i0 += CH) {
    Quad2<int> qb[CH];
#pragma unroll
    for (int m = 0; m < CH; ++m) {
      load_even(ll, ls, band, bs, it, i0 + m + 1, qb[m]);
      load_odd(band, bs, it, i0 + m + 1, qb[m]);
    }
#pragma unroll
    for (int m = 0; m < CH; ++m) {
      const int i = i0 + m;
      if (i < it.I1) {
        const Quad2<int> n = qb[m];
        // first half for row i + 1
        const int b1n_L = i32_inv_b1(n.hlL, hh_L, n.hhL), b1n_R = i32_inv_b1(n.hlR, hh_R, n.hhR);
        const int b1P = shfl_up(b1n_R), hhP = shfl_up(n.hhR);
        int an_L, an_R, c1n_L, c1n_R;
        i32_inv_update(n.llL, lh_L, n.lhL, b1P, b1n_L, hhP, n.hhL, an_L, c1n_L);
        i32_inv_update(n.llR, lh_R, n.lhR, b1n_L, b1n_R, n.hhL, n.hhR, an_R, c1n_R);
        const int aN1 = shfl_dn(an_L);
        // second half for row i
        const int c_L = i32_inv_c(c1_L, a_L, an_L), c_R = i32_inv_c(c1_R, a_R, an_R);
        const int cN = shfl_dn(c_L);
        V4<int> e, o;
        e.x = a_L; e.z = a_R;
        o.x = c_L; o.z = c_R;
        i32_inv_predict(a_L, a_R, b1_L, b1n_L, c_L, c_R, hh_L, e.y, o.y);
        i32_inv_predict(a_R, aN, b1_R, b1n_R, c_R, cN, hh_R, e.w, o.w);
        store_px4(px + (int64_t)(2 * i) * ps, c0, W, e, it.outL, it.outR);
        if (2 * i + 1 < it.H) store_px4(px + (int64_t)(2 * i + 1) * ps, c0, W, o, it.outL, it.outR);
        a_L = an_L; a_R = an_R; b1_L = b1n_L; b1_R = b1n_R; c1_L = c1n_L; c1_R = c1n_R;
        hh_L = n.hhL; hh_R = n.hhR; lh_L = n.lhL; lh_R = n.lhR;
        aN = aN1;
      }
    }
  }
}

// ----------------------------------------------------------------- adjoint
__device__ __forceinline__ void load_adj(const float* ll, int64_t ls, const float* band, int64_t bs, const Item& it,
                                         int r, Quad2<float>& q) {
  if (r >= 0 && r < it.ns_h) {
    load_band2_zero(ll + (int64_t)r * ls, it.qL, it.ns_w, q.llL, q.llR);
    load_band2_zero(band + (int64_t)r * bs + it.ns_w, it.qL, it.nd_w, q.hlL, q.hlR);
  } else {
    q.llL = q.llR = q.hlL = q.hlR = 0.f;
  }
  if (r >= 0 && r < it.nd_h) {
    const float* row = band + (int64_t)(it.ns_h + r) * bs;
    load_band2_zero(row, it.qL, it.ns_w, q.lhL, q.lhR);
    load_band2_zero(row + it.ns_w, it.qL, it.nd_w, q.hhL, q.hhR);
  } else {
    q.lhL = q.lhR = q.hhL = q.hhR = 0.f;
  }
}

template <int CH>
__device__ void bwd_f32(const LevelDesc& d, const float* __restrict__ ll, const float* __restrict__ band,
                        float* __restrict__ px, const Item& it) {
  const int W = it.W, c0 = 2 * it.qL;
  const int64_t ps = d.pix_stride, ls = d.ll_stride, bs = d.band_stride;
  const AxisW hL = axis_weights(it.qL, W), hR = axis_weights(it.qL + 1, W);

  // prologue: step A (transposed update) of row I0 - 1
  Quad2<float> p, c;
  load_adj(ll, ls, band, bs, it, it.I0 - 1, p);
  load_adj(ll, ls, band, bs, it, it.I0, c);
  float gc1U_L, gc1U_R, gd1U_L, gd1U_R, gd1UL_L;
  {
    const AxisW v = axis_weights(it.I0 - 1, it.H);
    const float gaN = shfl_dn(p.llL), gaDN = shfl_dn(c.llL), gcN = shfl_dn(p.lhL);
    float gb1L, gb1R;
    f32_adj_a(p.llL, p.llR, c.llL, c.llR, p.hlL, c.hlL, p.lhL, p.lhR, p.hhL, hL, v, gb1L, gc1U_L, gd1U_L);
    f32_adj_a(p.llR, gaN, c.llR, gaDN, p.hlR, c.hlR, p.lhR, gcN, p.hhR, hR, v, gb1R, gc1U_R, gd1U_R);
    gd1UL_L = shfl_up(gd1U_R);
  }
  float gaN = shfl_dn(c.llL);

  for (int i0 = it.I0; i0 < it.I1; i0 += CH) {
    Quad2<float> qb[CH];
#pragma unroll
    for (int m = 0; m < CH; ++m) load_adj(ll, ls, band, bs, it, i0 + m + 1, qb[m]);
#pragma unroll
    for (int m = 0; m < CH; ++m) {
      const int i = i0 + m;
      if (i < it.I1) {
        const Quad2<float> n = qb[m];
        const AxisW v = axis_weights(i, it.H);
        const float gaDN = shfl_dn(n.llL), gcN = shfl_dn(c.lhL);
        float gb1_L, gc1_L, gd1_L, gb1_R, gc1_R, gd1_R;
        f32_adj_a(c.llL, c.llR, n.llL, n.llR, c.hlL, n.hlL, c.lhL, c.lhR, c.hhL, hL, v, gb1_L, gc1_L, gd1_L);
        f32_adj_a(c.llR, gaN, n.llR, gaDN, c.hlR, n.hlR, c.lhR, gcN, c.hhR, hR, v, gb1_R, gc1_R, gd1_R);
        const float gb1P = shfl_up(gb1_R), gd1P = shfl_up(gd1_R);
        V4<float> e, o;
        f32_adj_b(c.llL, gb1P, gb1_L, gc1U_L, gc1_L, gd1UL_L, gd1U_L, gd1P, gd1_L, hL, v, e.x, e.y, o.x);
        f32_adj_b(c.llR, gb1_L, gb1_R, gc1U_R, gc1_R, gd1U_L, gd1U_R, gd1_L, gd1_R, hR, v, e.z, e.w, o.z);
        o.y = gd1_L;
        o.w = gd1_R;
        store_px4(px + (int64_t)(2 * i) * ps, c0, W, e, it.outL, it.outR);
        if (2 * i + 1 < it.H) store_px4(px + (int64_t)(2 * i + 1) * ps, c0, W, o, it.outL, it.outR);
        gc1U_L = gc1_L; gc1U_R = gc1_R; gd1U_L = gd1_L; gd1U_R = gd1_R; gd1UL_L = gd1P;
        c = n;
        gaN = gaDN;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

// Consecutive logical blocks land on the same XCD (the hardware deals
// workgroups round-robin over the 8 XCDs), so halo rows shared by vertically
// adjacent items are served from one L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  const int q = nb >> 3, r = nb & 7, x = b & 7, s = b >> 3;
  return (x < r) ? x * (q + 1) + s : r * (q + 1) + (x - r) * q + s;
}

template <int DIR, typename T, int CH>
__global__ __launch_bounds__(kBlock) void level_kernel(LevelLaunch a) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const int64_t item = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * kWavesPerBlock + wave;
  if (item >= a.items) return;
  const int img = (int)(item / a.items_per_image);
  const int rem = (int)(item - (int64_t)img * a.items_per_image);
  const int seg = rem / a.d.nstrips;
  const int strip = rem - seg * a.d.nstrips;
  const Item it = make_item(a.d, strip, seg, lane);
  if (DIR == kFwd) {
    const T* px = static_cast<const T*>(a.d.pix_in) + img * a.pix_bstride;
    T* ll = static_cast<T*>(a.d.ll_out) + img * a.ll_bstride;
    T* band = static_cast<T*>(a.d.band_out) + img * a.band_bstride;
    if constexpr (std::is_same<T, float>::value) fwd_f32<CH>(a.d, (const float*)px, (float*)ll, (float*)band, it);
    else fwd_i32<CH>(a.d, (const int*)px, (int*)ll, (int*)band, it);
  } else {
    const T* ll = static_cast<const T*>(a.d.ll_in) + img * a.ll_bstride;
    const T* band = static_cast<const T*>(a.d.band_in) + img * a.band_bstride;
    T* px = static_cast<T*>(a.d.pix_out) + img * a.pix_bstride;
    if constexpr (DIR == kInv) {
      if constexpr (std::is_same<T, float>::value) inv_f32<CH>(a.d, (const float*)ll, (const float*)band, (float*)px, it);
      else inv_i32<CH>(a.d, (const int*)ll, (const int*)band, (int*)px, it);
    } else {
      bwd_f32<CH>(a.d, (const float*)ll, (const float*)band, (float*)px, it);
    }
  }
}

template <int DIR, typename T, int CH>
hipError_t launch_t(const LevelLaunch& a, hipStream_t s) {
  const int64_t blocks = (a.items + kWavesPerBlock - 1) / kWavesPerBlock;
  hipLaunchKernelGGL((level_kernel<DIR, T, CH>), dim3((unsigned)blocks), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

}  // namespace

int launch_level(int dir, int mode, int chunk, const LevelLaunch& a, void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  (void)chunk;
  if (dir == kFwd) return mode == DWT2_F32 ? launch_t<kFwd, float, 4>(a, s) : launch_t<kFwd, int, 4>(a, s);
  if (dir == kInv) return mode == DWT2_F32 ? launch_t<kInv, float, 4>(a, s) : launch_t<kInv, int, 4>(a, s);
  return launch_t<kBwd, float, 4>(a, s);
}

}  // namespace dwt2
