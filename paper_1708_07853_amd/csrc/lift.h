// Device code shared by the HIP kernels for gfx950: the per-quadruple
// arithmetic of the 2-D CDF 5/3 transform with the non-separable lifting
// scheme (§3, eq. (5)) -- forward, inverse, adjoint -- and the strip work
// items that one level's kernels run.
//
// Mapping.  A wave owns a strip of 128 quadruple columns (lane l holds the
// quadruples 2l and 2l+1, i.e. one 16-byte vector of each pixel row) and walks
// down a segment of quadruple rows.  Vertical neighbours stay in registers
// from one row to the next; horizontal neighbours cross lanes with full-wave
// DPP shifts.  The first and last lanes also load the few samples just
// outside the strip (per-lane halo loads), so every lane writes its two
// quadruples and the strip's output rows are whole, aligned 512-byte runs.
// Each level therefore reads its input once and writes its output once; the
// synchronisation points of the lifting (the "|" of eq. (5)) become one
// exchange of the right neighbour's L samples for the spatial predict and one
// exchange of the left neighbour's predicted values for the spatial update.
//
// Memory pipeline.  Rows are fetched in chunks of CH quadruple rows; while
// one chunk is computed the next one is already in flight (two register
// buffers).  Interior work items (all columns inside the image, aligned, a
// whole number of chunk pairs) run a branch-free loop so the compiler's
// wait counts stay exact; items at the image edges take a general path with
// folded gathers, masked stores and row guards.
//
// Boundaries.  Forward and inverse read the whole-sample symmetric extension
// of their input (the interleaved coefficient array for the inverse), so the
// interior formulas hold everywhere.  The adjoint transposes that extension
// with explicit boundary weights instead (zero outside, doubled where the
// mirror folds two taps onto one sample).
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "dwt2_internal.h"

namespace dwt2 {
namespace {

constexpr int kStripQ = 128;  // quadruple columns per wave

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

// Band column of quadruple column q for parity `par` (0: L, 1: H) on an axis
// of length n, following the symmetric extension of the interleaved array.
__device__ __forceinline__ int band_idx(int q, int n, int par) { return (fold_idx(2 * q + par, n) - par) >> 1; }


// Lane exchange by full-wave DPP shifts: from_next gives lane i the value of
// lane i+1 (wave_shl:1), from_prev the value of lane i-1 (wave_shr:1); the
// lane without a source receives 0.  A lane reads its neighbour's register
// only if the neighbour is active, so every exchange runs in wave-uniform
// control flow (nxt / prv below), and lanes 0 and 63 substitute their halo
// values afterwards with a select.
__device__ __forceinline__ int dpp_next(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xf, 0xf, false); }
__device__ __forceinline__ int dpp_prev(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xf, 0xf, false); }
__device__ __forceinline__ int from_next(int v) { return dpp_next(v); }
__device__ __forceinline__ int from_prev(int v) { return dpp_prev(v); }
__device__ __forceinline__ float from_next(float v) { return __int_as_float(dpp_next(__float_as_int(v))); }
__device__ __forceinline__ float from_prev(float v) { return __int_as_float(dpp_prev(__float_as_int(v))); }
// sel ? alt : neighbour value, with the exchange done by every lane
template <typename T>
__device__ __forceinline__ T nxt(bool sel, T alt, T v) {
  const T n = from_next(v);
  return sel ? alt : n;
}
template <typename T>
__device__ __forceinline__ T prv(bool sel, T alt, T v) {
  const T p = from_prev(v);
  return sel ? alt : p;
}

template <typename T>
__device__ __forceinline__ void st2(T* p, T a, T b) {
  Ext2<T> t;
  t.x = a;
  t.y = b;
  *reinterpret_cast<Ext2<T>*>(p) = t;
}
template <typename T>
__device__ __forceinline__ void st4(T* p, const V4<T>& v) {
  Ext4<T> t;
  t.x = v.x; t.y = v.y; t.z = v.z; t.w = v.w;
  *reinterpret_cast<Ext4<T>*>(p) = t;
}

// Buffer resources: CDNA buffer instructions check every access against the
// resource's byte size in hardware -- a store outside it is dropped and a
// load outside it returns 0.  One resource per row (base = row start) masks
// whole rows (size 0) and columns past the row's end without branches.
using Rsrc = __amdgpu_buffer_rsrc_t;
__device__ __forceinline__ Rsrc row_rsrc(const void* base, int64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)bytes, 0x00020000);
}
template <typename T>
__device__ __forceinline__ unsigned ubits(T v) {
  return __builtin_bit_cast(unsigned, v);
}
template <typename T>
__device__ __forceinline__ T from_bits(unsigned u) {
  return __builtin_bit_cast(T, u);
}
// Element offsets are converted to byte offsets; a negative element offset
// wraps to a huge byte offset and is therefore out of range.  The main data
// streams are touched once per level, so they use the non-temporal cache
// policy (kNT); halo values, which neighbouring lanes and strips read again,
// use the default policy.
constexpr int kNT = 2;
// Cache-policy bits: sc0 = 1, nt = 2, sc1 = 16.  Inside a persistent job
// the LL rows one item writes are read by items on other XCDs, whose L2s are
// not coherent with the writer's; those accesses carry sc1 (stores write
// through, loads miss stale L2 lines) and sc0 (loads skip the CU's L1), so no
// whole-cache writeback or invalidation is needed between items.
constexpr int kSC0 = 1, kSC1 = 16;
#ifndef DWT2_COH_LD
#define DWT2_COH_LD (kNT | kSC0 | kSC1)
#endif
#ifndef DWT2_COH_HALO
#define DWT2_COH_HALO (kSC0 | kSC1)
#endif
#ifndef DWT2_COH_ST
#define DWT2_COH_ST (kNT | kSC1)
#endif
// Access modes of the LL rows a level reads or writes:
//   kStream: final results and job inputs (non-temporal: they are touched
//            once, and keeping them would evict data still to be read);
//   kKeep:   an intermediate LL the next level's launch reads (default
//            policy, so that it can be served from the caches);
//   kCoh:    an LL shared between items of one persistent job (above).
// Measured on MI355X, keeping only the intermediate LL rows beats both
// streaming everything and keeping every output.
constexpr int kStream = 0, kKeep = 1, kCoh = 2;
template <int M>
struct Pol {
  static constexpr int ld = M == kCoh ? (DWT2_COH_LD) : kNT;    // main streams
  static constexpr int halo = M == kCoh ? (DWT2_COH_HALO) : 0;  // re-read halo values
  static constexpr int st = M == kCoh ? (DWT2_COH_ST) : (M == kKeep ? 0 : kNT);
};
template <int POL, typename T>
__device__ __forceinline__ void bst2(T a, T b, Rsrc r, int e) {
  typedef unsigned U2 __attribute__((ext_vector_type(2)));
  U2 u;
  u.x = ubits(a);
  u.y = ubits(b);
  __builtin_amdgcn_raw_buffer_store_b64(u, r, (unsigned)e * 4u, 0, POL);
}
template <int POL, typename T>
__device__ __forceinline__ void bst4(const V4<T>& v, Rsrc r, int e) {
  typedef unsigned U4 __attribute__((ext_vector_type(4)));
  U4 u;
  u.x = ubits(v.x); u.y = ubits(v.y); u.z = ubits(v.z); u.w = ubits(v.w);
  __builtin_amdgcn_raw_buffer_store_b128(u, r, (unsigned)e * 4u, 0, POL);
}
template <typename T, int POL>
__device__ __forceinline__ T bld1(Rsrc r, int e) {
  return from_bits<T>(__builtin_amdgcn_raw_buffer_load_b32(r, (unsigned)e * 4u, 0, POL));
}
template <int POL, typename T>
__device__ __forceinline__ void bld2(Rsrc r, int e, T& a, T& b) {
  const auto u = __builtin_amdgcn_raw_buffer_load_b64(r, (unsigned)e * 4u, 0, POL);
  a = from_bits<T>(u[0]);
  b = from_bits<T>(u[1]);
}
template <int POL, typename T>
__device__ __forceinline__ void bld4(Rsrc r, int e, V4<T>& v) {
  const auto u = __builtin_amdgcn_raw_buffer_load_b128(r, (unsigned)e * 4u, 0, POL);
  v.x = from_bits<T>(u[0]); v.y = from_bits<T>(u[1]); v.z = from_bits<T>(u[2]); v.w = from_bits<T>(u[3]);
}

// ---------------------------------------------------------------------------
// Per-quadruple arithmetic.  Every kernel variant evaluates exactly these
// expressions, so results do not depend on tiling, paths or scheduling.
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

// Integer inverse, first half (undo the vertical then the horizontal update):
// b1 = b2 - floor((d2U + d2 + 2)/4); a1 = a2 - floor((c2U + c2 + 2)/4),
// a = a1 - floor((b1L + b1 + 2)/4), c1 = c2 - floor((d2L + d2 + 2)/4).
__device__ __forceinline__ int i32_inv_b1(int b2, int d2U, int d2) { return b2 - ((d2U + d2 + 2) >> 2); }
__device__ __forceinline__ void i32_inv_update(int a2, int c2U, int c2, int b1L, int b1, int d2L, int d2, int& a,
                                               int& c1) {
  const int a1 = a2 - ((c2U + c2 + 2) >> 2);
  a = a1 - ((b1L + b1 + 2) >> 2);
  c1 = c2 - ((d2L + d2 + 2) >> 2);
}
// Second half (undo the vertical then the horizontal predict).
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

// Weighted pair sum wa a + wb b.  UNIT: every weight is 1 (a quadruple away
// from the borders); the plain sum then rounds exactly as the weighted one
// (products by 1 are exact and nothing is contracted), so both forms give
// the same bits.
template <bool UNIT>
__device__ __forceinline__ float wsum(float wa, float a, float wb, float b) {
  if constexpr (UNIT) return a + b;
  else return wa * a + wb * b;
}
__device__ __forceinline__ bool unit_weights(const AxisW& w) {
  return w.alpha == 1.f && w.beta == 1.f && w.gamma == 1.f && w.delta == 1.f;
}

// Transposed spatial update (M_U^T, predict-shaped).
template <bool UNIT = false>
__device__ __forceinline__ void f32_adj_a(float ga, float gaR, float gaD, float gaDR, float gb, float gbD,
                                          float gc, float gcR, float gd, AxisW h, AxisW v, float& gb1, float& gc1,
                                          float& gd1) {
  const float th = wsum<UNIT>(h.alpha, ga, h.beta, gaR);  // U^T_h ga (x4)
  const float thD = wsum<UNIT>(h.alpha, gaD, h.beta, gaDR);
  gb1 = __fmaf_rn(0.25f, th, gb);
  gc1 = __fmaf_rn(0.25f, wsum<UNIT>(v.alpha, ga, v.beta, gaD), gc);
  gd1 = __fmaf_rn(0.0625f, wsum<UNIT>(v.alpha, th, v.beta, thD),
                  __fmaf_rn(0.25f, wsum<UNIT>(h.alpha, gc, h.beta, gcR),
                            __fmaf_rn(0.25f, wsum<UNIT>(v.alpha, gb, v.beta, gbD), gd)));
}

// Transposed spatial predict (M_P^T, update-shaped).
template <bool UNIT = false>
__device__ __forceinline__ void f32_adj_b(float ga, float gb1L, float gb1, float gc1U, float gc1, float gd1UL,
                                          float gd1U, float gd1L, float gd1, AxisW h, AxisW v, float& ga2,
                                          float& gb2, float& gc2) {
  gb2 = __fmaf_rn(-0.5f, wsum<UNIT>(v.gamma, gd1U, v.delta, gd1), gb1);
  gc2 = __fmaf_rn(-0.5f, wsum<UNIT>(h.gamma, gd1L, h.delta, gd1), gc1);
  const float tU = wsum<UNIT>(h.gamma, gd1UL, h.delta, gd1U);
  const float t0 = wsum<UNIT>(h.gamma, gd1L, h.delta, gd1);
  ga2 = __fmaf_rn(0.25f, wsum<UNIT>(v.gamma, tU, v.delta, t0),
                  __fmaf_rn(-0.5f, wsum<UNIT>(v.gamma, gc1U, v.delta, gc1),
                            __fmaf_rn(-0.5f, wsum<UNIT>(h.gamma, gb1L, h.delta, gb1), ga)));
}

// ---------------------------------------------------------------------------
// Work items
// ---------------------------------------------------------------------------
struct Item {
  int W, H, ns_w, nd_w, ns_h, nd_h;
  int lane;
  int qL;       // global quadruple column of this lane's first quadruple
  int I0, I1;   // quadruple rows written
  bool first, last;
};

__device__ __forceinline__ Item make_item(const LevelDesc& d, int strip, int seg, int lane) {
  Item it;
  it.W = d.W; it.H = d.H;
  it.ns_w = (d.W + 1) >> 1; it.nd_w = d.W >> 1;
  it.ns_h = (d.H + 1) >> 1; it.nd_h = d.H >> 1;
  it.lane = lane;
  it.qL = kStripQ * strip + 2 * lane;
  it.I0 = seg * d.seg;
  it.I1 = min(it.I0 + d.seg, it.ns_h);
  it.first = lane == 0;
  it.last = lane == kWave - 1;
  return it;
}

// Double-buffered row pipeline over ceil((I1 - I0) / (2 CH)) chunk pairs.
// The caller has issued the loads of chunk A (rows I0 .. I0+CH-1) before its
// prologue.  Rows past I1 ("phantom" rows of the last pair) are computed on
// folded or zero inputs and their stores are dropped by the buffer bounds, so
// the loop has no branches and the compiler's wait counts stay exact.
template <int CH, typename Buf, typename LoadF, typename RowF>
__device__ __forceinline__ void run_rows(int I0, int I1, Buf& A, Buf& B, LoadF&& load_chunk, RowF&& row) {
  int i0 = I0;
  const int npairs = (I1 - I0 + 2 * CH - 1) / (2 * CH);
  for (int p = 1; p < npairs; ++p) {
    load_chunk(B, i0 + CH);
#pragma unroll
    for (int m = 0; m < CH; ++m) row(A, m, i0 + m);
    load_chunk(A, i0 + 2 * CH);
#pragma unroll
    for (int m = 0; m < CH; ++m) row(B, m, i0 + CH + m);
    i0 += 2 * CH;
  }
  load_chunk(B, i0 + CH);
#pragma unroll
  for (int m = 0; m < CH; ++m) row(A, m, i0 + m);
#pragma unroll
  for (int m = 0; m < CH; ++m) row(B, m, i0 + CH + m);
}

// ---------------------------------------------------------------- forward
// Pixel rows: four pixels per lane plus two halo pixels (lane 0: the two
// columns left of the strip; lane 63: the column right of it).  Each lane
// reads its four pixels with one 16-byte load at any 4-byte alignment (the
// hardware splits accesses that cross a cache line).  EDGE: the strip
// reaches the image's right edge; lanes whose pixels lie past it take the
// mirrored columns from single-element loads (the other lanes pass an
// out-of-range offset, which issues no request) and a select.
template <typename T, bool EDGE, int COH>  // COH: access mode of the rows (kStream or kCoh)
struct PxLoader {
  const T* base;
  int64_t stride;
  int W, H;
  int c0;
  int pcol[4];  // EDGE: mirrored column of pixel c0 + k past the edge, else -1
  int hc0, hc1;
  // Loads row r: the vector `m`, the EDGE patch values `pm` (applied later
  // by fix(), when the row is consumed, so that prefetched loads stay in
  // flight) and the halo pair.
  __device__ __forceinline__ void load(int r, V4<T>& m, V4<T>& pm, T& h0, T& h1) const {
    const Rsrc rs = row_rsrc(base + (int64_t)fold_idx(r, H) * stride, (int64_t)W * 4);
    bld4<Pol<COH>::ld>(rs, c0, m);
    if constexpr (EDGE) {
      pm.x = bld1<T, Pol<COH>::halo>(rs, pcol[0]);
      pm.y = bld1<T, Pol<COH>::halo>(rs, pcol[1]);
      pm.z = bld1<T, Pol<COH>::halo>(rs, pcol[2]);
      pm.w = bld1<T, Pol<COH>::halo>(rs, pcol[3]);
    }
    h0 = bld1<T, Pol<COH>::halo>(rs, hc0);
    h1 = bld1<T, Pol<COH>::halo>(rs, hc1);
  }
  __device__ __forceinline__ void fix(V4<T>& m, const V4<T>& pm) const {
    if constexpr (EDGE) {
      m.x = pcol[0] >= 0 ? pm.x : m.x;
      m.y = pcol[1] >= 0 ? pm.y : m.y;
      m.z = pcol[2] >= 0 ? pm.z : m.z;
      m.w = pcol[3] >= 0 ? pm.w : m.w;
    }
  }
};

template <typename T, bool EDGE, int COH>
__device__ __forceinline__ PxLoader<T, EDGE, COH> px_loader(const T* base, int64_t stride, const Item& it) {
  PxLoader<T, EDGE, COH> L;
  L.base = base; L.stride = stride; L.W = it.W; L.H = it.H;
  L.c0 = 2 * it.qL;
  for (int k = 0; k < 4; ++k) L.pcol[k] = (L.c0 + k < it.W) ? -1 : fold_idx(L.c0 + k, it.W);
  if (it.first) {
    L.hc0 = fold_idx(L.c0 - 2, it.W);
    L.hc1 = fold_idx(L.c0 - 1, it.W);
  } else if (it.last) {
    L.hc0 = L.hc1 = fold_idx(L.c0 + 4, it.W);
  } else {
    // interior lanes take their neighbours' values over DPP and never use
    // the halo: an out-of-range offset makes the hardware drop their request
    L.hc0 = L.hc1 = -1;
  }
  return L;
}

template <typename T, int CH>
struct PxBuf {
  V4<T> o[CH], e[CH];
  V4<T> po[CH], pe[CH];  // edge patches (EDGE items only)
  T ho0[CH], ho1[CH], he0[CH], he1[CH];
};

// Stores of one row of the four bands (forward): one buffer resource per band
// row; rows past I1 (and LH / HH rows past nd_h) have size 0.  Each lane
// writes its two quadruples with one 8-byte store at any 4-byte alignment;
// the range check drops every dword past the band's width on its own.
template <typename T, bool EDGE, int COH>  // COH: mode of the LL rows
struct BandStore {
  T* ll;
  int64_t ls;
  T* band;
  int64_t bs;
  int ns_w, nd_w, ns_h, nd_h, qL, I1;
  __device__ __forceinline__ void put(int i, T llL, T llR, T hlL, T hlR, T lhL, T lhR, T hhL, T hhR) const {
    const bool real = i < I1, real2 = real && i < nd_h;
    const Rsrc rl = row_rsrc(ll + (int64_t)i * ls, real ? ns_w * 4 : 0);
    const Rsrc rh = row_rsrc(band + (int64_t)i * bs + ns_w, real ? nd_w * 4 : 0);
    T* row2 = band + (int64_t)(ns_h + i) * bs;
    const Rsrc rlh = row_rsrc(row2, real2 ? ns_w * 4 : 0);
    const Rsrc rhh = row_rsrc(row2 + ns_w, real2 ? nd_w * 4 : 0);
    // only LL rows are read again inside a job; the bands are final
    constexpr int P = Pol<COH>::st, PB = kNT;
    bst2<P>(llL, llR, rl, qL);
    bst2<PB>(hlL, hlR, rh, qL);
    bst2<PB>(lhL, lhR, rlh, qL);
    bst2<PB>(hhL, hhR, rhh, qL);
  }
};

template <typename T, bool EDGE, int COH>
__device__ __forceinline__ BandStore<T, EDGE, COH> band_store(T* ll, int64_t ls, T* band, int64_t bs, const Item& it) {
  BandStore<T, EDGE, COH> S;
  S.ll = ll; S.ls = ls; S.band = band; S.bs = bs;
  S.ns_w = it.ns_w; S.nd_w = it.nd_w; S.ns_h = it.ns_h; S.nd_h = it.nd_h; S.qL = it.qL; S.I1 = it.I1;
  return S;
}

template <int CH, bool EDGE, int CI, int CO>
__device__ void fwd_f32(const LevelDesc& d, const float* __restrict__ px, float* __restrict__ ll,
                        float* __restrict__ band, const Item& it) {
  const PxLoader<float, EDGE, CI> L = px_loader<float, EDGE, CI>(px, d.pix_stride, it);
  const BandStore<float, EDGE, CO> S = band_store<float, EDGE, CO>(ll, d.ll_stride, band, d.band_stride, it);
  const bool first = it.first, last = it.last;
  using Buf = PxBuf<float, CH>;
  auto load_chunk = [&](Buf& b, int i0) {
#pragma unroll
    for (int m = 0; m < CH; ++m) {
      L.load(2 * (i0 + m) + 1, b.o[m], b.po[m], b.ho0[m], b.ho1[m]);
      L.load(2 * (i0 + m) + 2, b.e[m], b.pe[m], b.he0[m], b.he1[m]);
    }
  };
  V4<float> E, O, E1, pE, pO, pE1;
  float hE0, hE1, hO0, hO1, hN0, hN1;
  L.load(2 * it.I0 - 2, E, pE, hE0, hE1);
  L.load(2 * it.I0 - 1, O, pO, hO0, hO1);
  L.load(2 * it.I0, E1, pE1, hN0, hN1);
  L.fix(E, pE);
  L.fix(O, pO);
  L.fix(E1, pE1);
  Buf A, B;
  load_chunk(A, it.I0);

  // prologue: predicted values of quadruple row I0 - 1
  float cpU_L, cpU_R, dpU_L, dpU_R, dpUL_L;
  {
    const float aN = nxt(last, hE0, E.x), aDN = nxt(last, hN0, E1.x);
    const float cN = nxt(last, hO0, O.x);
    float bpL, bpR, bpH, cpH, dpH;
    f32_predict(E.x, E.z, E1.x, E1.z, E.y, E1.y, O.x, O.z, O.y, bpL, cpU_L, dpU_L);
    f32_predict(E.z, aN, E1.z, aDN, E.w, E1.w, O.z, cN, O.w, bpR, cpU_R, dpU_R);
    f32_predict(hE0, E.x, hN0, E1.x, hE1, hN1, hO0, O.x, hO1, bpH, cpH, dpH);
    dpUL_L = prv(first, dpH, dpU_R);
  }
  E = E1;
  hE0 = hN0;
  hE1 = hN1;
  float aN = nxt(last, hE0, E.x);

  auto row = [&](const Buf& b, int m, int i) {
    V4<float> o = b.o[m], e1 = b.e[m];
    L.fix(o, b.po[m]);
    L.fix(e1, b.pe[m]);
    const float aDN = nxt(last, b.he0[m], e1.x);
    const float cN = nxt(last, b.ho0[m], o.x);
    float bpL, cpL, dpL, bpR, cpR, dpR, bpH, cpH, dpH;
    f32_predict(E.x, E.z, e1.x, e1.z, E.y, e1.y, o.x, o.z, o.y, bpL, cpL, dpL);
    f32_predict(E.z, aN, e1.z, aDN, E.w, e1.w, o.z, cN, o.w, bpR, cpR, dpR);
    f32_predict(hE0, E.x, b.he0[m], e1.x, hE1, b.he1[m], b.ho0[m], o.x, b.ho1[m], bpH, cpH, dpH);
    const float bpP = prv(first, bpH, bpR);
    const float dpP = prv(first, dpH, dpR);
    float llL, hlL, lhL, llR, hlR, lhR;
    f32_update(E.x, bpP, bpL, cpU_L, cpL, dpUL_L, dpU_L, dpP, dpL, llL, hlL, lhL);
    f32_update(E.z, bpL, bpR, cpU_R, cpR, dpU_L, dpU_R, dpL, dpR, llR, hlR, lhR);
    S.put(i, llL, llR, hlL, hlR, lhL, lhR, dpL, dpR);
    cpU_L = cpL; cpU_R = cpR; dpU_L = dpL; dpU_R = dpR; dpUL_L = dpP;
    E = e1;
    hE0 = b.he0[m];
    hE1 = b.he1[m];
    aN = aDN;
  };
  run_rows<CH>(it.I0, it.I1, A, B, load_chunk, row);
}

template <int CH, bool EDGE, int CI, int CO>
__device__ void fwd_i32(const LevelDesc& d, const int* __restrict__ px, int* __restrict__ ll,
                        int* __restrict__ band, const Item& it) {
  const PxLoader<int, EDGE, CI> L = px_loader<int, EDGE, CI>(px, d.pix_stride, it);
  const BandStore<int, EDGE, CO> S = band_store<int, EDGE, CO>(ll, d.ll_stride, band, d.band_stride, it);
  const bool first = it.first, last = it.last;
  using Buf = PxBuf<int, CH>;
  auto load_chunk = [&](Buf& b, int i0) {
#pragma unroll
    for (int m = 0; m < CH; ++m) {
      L.load(2 * (i0 + m) + 1, b.o[m], b.po[m], b.ho0[m], b.ho1[m]);
      L.load(2 * (i0 + m) + 2, b.e[m], b.pe[m], b.he0[m], b.he1[m]);
    }
  };
  V4<int> E, O, E1, pE, pO, pE1;
  int hE0, hE1, hO0, hO1, hN0, hN1;
  L.load(2 * it.I0 - 2, E, pE, hE0, hE1);
  L.load(2 * it.I0 - 1, O, pO, hO0, hO1);
  L.load(2 * it.I0, E1, pE1, hN0, hN1);
  L.fix(E, pE);
  L.fix(O, pO);
  L.fix(E1, pE1);
  Buf A, B;
  load_chunk(A, it.I0);

  int c2U_L, c2U_R, d2U_L, d2U_R;
  {
    const int aN = nxt(last, hE0, E.x), aDN = nxt(last, hN0, E1.x);
    const int cN = nxt(last, hO0, O.x);
    int b1L, c1L, b1R, c1R, b1H, c1H, d2H;
    i32_predict(E.x, E.z, E1.x, E1.z, E.y, E1.y, O.x, O.z, O.y, b1L, c1L, d2U_L);
    i32_predict(E.z, aN, E1.z, aDN, E.w, E1.w, O.z, cN, O.w, b1R, c1R, d2U_R);
    i32_predict(hE0, E.x, hN0, E1.x, hE1, hN1, hO0, O.x, hO1, b1H, c1H, d2H);
    const int d2P = prv(first, d2H, d2U_R);
    c2U_L = i32_c2(c1L, d2P, d2U_L);
    c2U_R = i32_c2(c1R, d2U_L, d2U_R);
  }
  E = E1;
  hE0 = hN0;
  hE1 = hN1;
  int aN = nxt(last, hE0, E.x);

  auto row = [&](const Buf& b, int m, int i) {
    V4<int> o = b.o[m], e1 = b.e[m];
    L.fix(o, b.po[m]);
    L.fix(e1, b.pe[m]);
    const int aDN = nxt(last, b.he0[m], e1.x);
    const int cN = nxt(last, b.ho0[m], o.x);
    int b1L, c1L, d2L, b1R, c1R, d2R, b1H, c1H, d2H;
    i32_predict(E.x, E.z, e1.x, e1.z, E.y, e1.y, o.x, o.z, o.y, b1L, c1L, d2L);
    i32_predict(E.z, aN, e1.z, aDN, E.w, e1.w, o.z, cN, o.w, b1R, c1R, d2R);
    i32_predict(hE0, E.x, b.he0[m], e1.x, hE1, b.he1[m], b.ho0[m], o.x, b.ho1[m], b1H, c1H, d2H);
    const int b1P = prv(first, b1H, b1R);
    const int d2P = prv(first, d2H, d2R);
    const int c2L = i32_c2(c1L, d2P, d2L), c2R = i32_c2(c1R, d2L, d2R);
    int llL, hlL, llR, hlR;
    i32_update(E.x, b1P, b1L, c2U_L, c2L, d2U_L, d2L, llL, hlL);
    i32_update(E.z, b1L, b1R, c2U_R, c2R, d2U_R, d2R, llR, hlR);
    S.put(i, llL, llR, hlL, hlR, c2L, c2R, d2L, d2R);
    c2U_L = c2L; c2U_R = c2R; d2U_L = d2L; d2U_R = d2R;
    E = e1;
    hE0 = b.he0[m];
    hE1 = b.he1[m];
    aN = aDN;
  };
  run_rows<CH>(it.I0, it.I1, A, B, load_chunk, row);
}

// ------------------------------------------------------- inverse / adjoint
// Band rows for this lane's two quadruples plus two halo values per part
// (even part: LL and HL rows; odd part: LH and HH rows).  MIRROR reads the
// symmetric extension of the interleaved coefficients (inverse: folded
// indices, always in range); otherwise values outside the bands are zero
// (adjoint: bounds-checked buffer loads, rows outside get a size-0 resource).
// Patch offset that marks "keep the vector load's value"; it is out of any
// buffer's range, so its single-element load issues no request.
constexpr int kNoPatch = -1;

template <typename T, bool EDGE, bool MIRROR, int COH>  // COH: mode of the LL rows
struct BandLoader {
  const T* ll;
  int64_t ls;
  const T* band;
  int64_t bs;
  int H, ns_h, nd_h, ns_w, nd_w, qL;
  int pl0, pl1, ph0, ph1;  // EDGE: columns re-read for quads qL, qL+1 of L / H rows, or kNoPatch
  int hp0, hp1;            // halo band parity
  int hc0, hc1;            // halo columns (MIRROR: folded; else raw, may be outside)

  // `ll_row`: rl is an LL row (written earlier in the same job when COH);
  // H-band rows are job inputs and take the plain policies.  Each lane reads
  // its two quadruples of a band row with one 8-byte load; EDGE lanes whose
  // quadruples reach the band's end re-read them one by one at the folded
  // (MIRROR) or raw (else: past the end reads 0) columns.
  // The patch values go to `pt` and are applied by fix() when the row is
  // consumed, so that prefetched loads stay in flight.  Without MIRROR the
  // per-dword range check already yields the zeros past a band's end.
  __device__ __forceinline__ void part(const T* rl, const T* rh, bool valid, bool ll_row, T& lL, T& lR, T& hL, T& hR,
                                       V4<T>& pt, T& h0, T& h1) const {
    // LL rows outside a persistent job take the caching policy: the two
    // halo values of the strip's edge lanes usually come from LL rows, and
    // with the rows streamed they missed in L2 (8192^2 float, one level:
    // inverse 97.6 -> 94.0 us, adjoint 99.8 -> 96.4 us; caching the H-band
    // rows as well measured slower than either).
    constexpr int P = COH == kCoh ? Pol<COH>::ld : 0, PH = Pol<COH>::halo, PB = kNT;
    const Rsrc bl = row_rsrc(rl, (MIRROR || valid) ? ns_w * 4 : 0);
    const Rsrc bh = row_rsrc(rh, (MIRROR || valid) ? nd_w * 4 : 0);
    if (ll_row) bld2<P>(bl, qL, lL, lR);
    else bld2<PB>(bl, qL, lL, lR);
    bld2<PB>(bh, qL, hL, hR);
    if constexpr (EDGE && MIRROR) {
      pt.x = bld1<T, PH>(bl, pl0);
      pt.y = bld1<T, PH>(bl, pl1);
      pt.z = bld1<T, PH>(bh, ph0);
      pt.w = bld1<T, PH>(bh, ph1);
    }
    h0 = bld1<T, PH>(hp0 ? bh : bl, hc0);
    h1 = bld1<T, PH>(hp1 ? bh : bl, hc1);
  }
  __device__ __forceinline__ void fix(const V4<T>& pt, T& lL, T& lR, T& hL, T& hR) const {
    if constexpr (EDGE && MIRROR) {
      lL = pl0 != kNoPatch ? pt.x : lL;
      lR = pl1 != kNoPatch ? pt.y : lR;
      hL = ph0 != kNoPatch ? pt.z : hL;
      hR = ph1 != kNoPatch ? pt.w : hR;
    }
  }
  // row r of LL and HL
  __device__ __forceinline__ void even(int r, T& lL, T& lR, T& hL, T& hR, V4<T>& pt, T& h0, T& h1) const {
    const int re = MIRROR ? (fold_idx(2 * r, H) >> 1) : r;
    const T* rl = ll + (int64_t)re * ls;
    const T* rh = band + (int64_t)re * bs + ns_w;
    part(rl, rh, r >= 0 && r < ns_h, true, lL, lR, hL, hR, pt, h0, h1);
  }
  // row r of LH and HH
  __device__ __forceinline__ void odd(int r, T& lL, T& lR, T& hL, T& hR, V4<T>& pt, T& h0, T& h1) const {
    const int ro = MIRROR ? ((fold_idx(2 * r + 1, H) - 1) >> 1) : r;
    const T* rl = band + (int64_t)(ns_h + ro) * bs;
    const T* rh = rl + ns_w;
    part(rl, rh, r >= 0 && r < nd_h, false, lL, lR, hL, hR, pt, h0, h1);
  }
};

// Halo assignment: (parity, quadruple column) of the two halo values of
// lanes 0 and 63; the other lanes issue out-of-range loads (no memory request).
template <typename T, bool EDGE, bool MIRROR, int COH>
__device__ __forceinline__ BandLoader<T, EDGE, MIRROR, COH> band_loader(const T* ll, int64_t ls, const T* band,
                                                                        int64_t bs, const Item& it, int p0_first,
                                                                        int p1_first, int p0_last, int p1_last) {
  BandLoader<T, EDGE, MIRROR, COH> L;
  L.ll = ll; L.ls = ls; L.band = band; L.bs = bs;
  L.H = it.H; L.ns_h = it.ns_h; L.nd_h = it.nd_h; L.ns_w = it.ns_w; L.nd_w = it.nd_w; L.qL = it.qL;
  const int W = it.W, q = it.qL;
  auto col = [&](int qq, int par) { return MIRROR ? band_idx(qq, W, par) : qq; };
  // a lane whose pair of quadruples reaches a band's end re-reads both
  const bool lpatch = q + 1 >= it.ns_w, hpatch = q + 1 >= it.nd_w;
  L.pl0 = lpatch ? col(q, 0) : kNoPatch;
  L.pl1 = lpatch ? col(q + 1, 0) : kNoPatch;
  L.ph0 = hpatch ? col(q, 1) : kNoPatch;
  L.ph1 = hpatch ? col(q + 1, 1) : kNoPatch;
  int qq = q;
  L.hp0 = 0; L.hp1 = 0;
  if (it.first) {
    qq = q - 1; L.hp0 = p0_first; L.hp1 = p1_first;
  } else if (it.last) {
    qq = q + 2; L.hp0 = p0_last; L.hp1 = p1_last;
  }
  L.hc0 = col(qq, L.hp0);
  L.hc1 = col(qq, L.hp1);
  if (!it.first && !it.last) L.hc0 = L.hc1 = -1;  // unused: out of range, no memory request
  return L;
}

template <typename T, int CH>
struct QBuf {
  T llL[CH], llR[CH], hlL[CH], hlR[CH], he0[CH], he1[CH];
  T lhL[CH], lhR[CH], hhL[CH], hhR[CH], ho0[CH], ho1[CH];
  V4<T> pe[CH], po[CH];  // edge patches (EDGE items of the inverse only)
};

// Stores of pixel rows (inverse / adjoint): four pixels per lane, one buffer
// resource per row (size 0 for rows past I1's last pixel row or past H).
template <typename T, bool EDGE, int COH>  // COH: mode of the pixel rows
struct PxStore {
  T* base;
  int64_t stride;
  int W, H, c0, rows_end;  // rows_end: first pixel row not to write (min(2 I1, H))
  // one 16-byte store per lane at any 4-byte alignment; dwords past the
  // row's end are dropped one by one by the range check
  __device__ __forceinline__ void row(int r, const V4<T>& v) const {
    const Rsrc rs = row_rsrc(base + (int64_t)r * stride, r < rows_end ? W * 4 : 0);
    bst4<Pol<COH>::st>(v, rs, c0);
  }
};

template <int CH, bool EDGE, int CI, int CO>
__device__ void inv_f32(const LevelDesc& d, const float* __restrict__ ll, const float* __restrict__ band,
                        float* __restrict__ px, const Item& it) {
  // halos: lane 0 -> HL / HH of quad qL-1 (parity 1); lane 63 -> quad qL+2:
  // h0 = LL / LH (parity 0), h1 = HL / HH (parity 1)
  const BandLoader<float, EDGE, true, CI> L =
      band_loader<float, EDGE, true, CI>(ll, d.ll_stride, band, d.band_stride, it, 1, 1, 0, 1);
  const PxStore<float, EDGE, CO> S{px, d.pix_stride, it.W, it.H, 2 * it.qL, min(2 * it.I1, it.H)};
  const bool first = it.first, last = it.last;
  using Buf = QBuf<float, CH>;
  auto load_chunk = [&](Buf& b, int i0) {
#pragma unroll
    for (int m = 0; m < CH; ++m) {
      L.even(i0 + m + 1, b.llL[m], b.llR[m], b.hlL[m], b.hlR[m], b.pe[m], b.he0[m], b.he1[m]);
      L.odd(i0 + m + 1, b.lhL[m], b.lhR[m], b.hhL[m], b.hhR[m], b.po[m], b.ho0[m], b.ho1[m]);
    }
  };
  float lhU_L, lhU_R, hhU_L, hhU_R, hoU0, hoU1;
  {
    V4<float> pt_;
    L.odd(it.I0 - 1, lhU_L, lhU_R, hhU_L, hhU_R, pt_, hoU0, hoU1);
    L.fix(pt_, lhU_L, lhU_R, hhU_L, hhU_R);
  }
  float q_llL, q_llR, q_hlL, q_hlR, q_he0, q_he1, q_lhL, q_lhR, q_hhL, q_hhR, q_ho0, q_ho1;
  {
    V4<float> pt_;
    L.even(it.I0, q_llL, q_llR, q_hlL, q_hlR, pt_, q_he0, q_he1);
    L.fix(pt_, q_llL, q_llR, q_hlL, q_hlR);
  }
  {
    V4<float> pt_;
    L.odd(it.I0, q_lhL, q_lhR, q_hhL, q_hhR, pt_, q_ho0, q_ho1);
    L.fix(pt_, q_lhL, q_lhR, q_hhL, q_hhR);
  }
  Buf A, B;
  load_chunk(A, it.I0);

  float hhUL_L = prv(first, hoU0, hhU_R);
  float a_L, a_R, bp_L, bp_R, cp_L, cp_R, aN, cpN, hh_L, hh_R;
  // undo the update of one coefficient row (L, R and the right halo quad X)
  auto undo_update = [&](float llL, float llR, float hlL, float hlR, float he0, float he1, float lhL, float lhR,
                         float hhL, float hhR, float ho0, float ho1, float& oaL, float& oaR, float& obL,
                         float& obR, float& ocL, float& ocR, float& oaN, float& ocN) {
    const float hlP = prv(first, he0, hlR);
    const float hhP = prv(first, ho0, hhR);
    f32_inv_update(llL, hlP, hlL, lhU_L, lhL, hhUL_L, hhU_L, hhP, hhL, oaL, obL, ocL);
    f32_inv_update(llR, hlL, hlR, lhU_R, lhR, hhU_L, hhU_R, hhL, hhR, oaR, obR, ocR);
    float aX, bX, cX;
    f32_inv_update(he0, hlR, he1, hoU0, ho0, hhU_R, hoU1, hhR, ho1, aX, bX, cX);
    oaN = nxt(last, aX, oaL);
    ocN = nxt(last, cX, ocL);
    lhU_L = lhL; lhU_R = lhR; hhU_L = hhL; hhU_R = hhR; hhUL_L = hhP; hoU0 = ho0; hoU1 = ho1;
  };
  undo_update(q_llL, q_llR, q_hlL, q_hlR, q_he0, q_he1, q_lhL, q_lhR, q_hhL, q_hhR, q_ho0, q_ho1, a_L, a_R, bp_L,
              bp_R, cp_L, cp_R, aN, cpN);
  hh_L = q_hhL;
  hh_R = q_hhR;

  auto row = [&](const Buf& b, int m, int i) {
    float r_llL = b.llL[m], r_llR = b.llR[m], r_hlL = b.hlL[m], r_hlR = b.hlR[m];
    float r_lhL = b.lhL[m], r_lhR = b.lhR[m], r_hhL = b.hhL[m], r_hhR = b.hhR[m];
    L.fix(b.pe[m], r_llL, r_llR, r_hlL, r_hlR);
    L.fix(b.po[m], r_lhL, r_lhR, r_hhL, r_hhR);
    float a1_L, a1_R, bp1_L, bp1_R, cp1_L, cp1_R, aN1, cpN1;
    undo_update(r_llL, r_llR, r_hlL, r_hlR, b.he0[m], b.he1[m], r_lhL, r_lhR, r_hhL,
                r_hhR, b.ho0[m], b.ho1[m], a1_L, a1_R, bp1_L, bp1_R, cp1_L, cp1_R, aN1, cpN1);
    V4<float> e, o;
    e.x = a_L;
    e.z = a_R;
    f32_inv_predict(a_L, a_R, a1_L, a1_R, bp_L, bp1_L, cp_L, cp_R, hh_L, e.y, o.x, o.y);
    f32_inv_predict(a_R, aN, a1_R, aN1, bp_R, bp1_R, cp_R, cpN, hh_R, e.w, o.z, o.w);
    S.row(2 * i, e);
    S.row(2 * i + 1, o);
    a_L = a1_L; a_R = a1_R; bp_L = bp1_L; bp_R = bp1_R; cp_L = cp1_L; cp_R = cp1_R;
    aN = aN1; cpN = cpN1;
    hh_L = r_hhL;
    hh_R = r_hhR;
  };
  run_rows<CH>(it.I0, it.I1, A, B, load_chunk, row);
}

template <int CH, bool EDGE, int CI, int CO>
__device__ void inv_i32(const LevelDesc& d, const int* __restrict__ ll, const int* __restrict__ band,
                        int* __restrict__ px, const Item& it) {
  const BandLoader<int, EDGE, true, CI> L =
      band_loader<int, EDGE, true, CI>(ll, d.ll_stride, band, d.band_stride, it, 1, 1, 0, 1);
  const PxStore<int, EDGE, CO> S{px, d.pix_stride, it.W, it.H, 2 * it.qL, min(2 * it.I1, it.H)};
  const bool first = it.first, last = it.last;
  using Buf = QBuf<int, CH>;
  auto load_chunk = [&](Buf& b, int i0) {
#pragma unroll
    for (int m = 0; m < CH; ++m) {
      L.even(i0 + m + 1, b.llL[m], b.llR[m], b.hlL[m], b.hlR[m], b.pe[m], b.he0[m], b.he1[m]);
      L.odd(i0 + m + 1, b.lhL[m], b.lhR[m], b.hhL[m], b.hhR[m], b.po[m], b.ho0[m], b.ho1[m]);
    }
  };
  // state of the previous coefficient row: LH (c2U) and HH (d2U) of L, R;
  // odd halos (lane 0: HH of quad qL-1; lane 63: LH / HH of quad qL+2)
  int lhU_L, lhU_R, hhU_L, hhU_R, hoU0, hoU1;
  {
    V4<int> pt_;
    L.odd(it.I0 - 1, lhU_L, lhU_R, hhU_L, hhU_R, pt_, hoU0, hoU1);
    L.fix(pt_, lhU_L, lhU_R, hhU_L, hhU_R);
  }
  int q_llL, q_llR, q_hlL, q_hlR, q_he0, q_he1, q_lhL, q_lhR, q_hhL, q_hhR, q_ho0, q_ho1;
  {
    V4<int> pt_;
    L.even(it.I0, q_llL, q_llR, q_hlL, q_hlR, pt_, q_he0, q_he1);
    L.fix(pt_, q_llL, q_llR, q_hlL, q_hlR);
  }
  {
    V4<int> pt_;
    L.odd(it.I0, q_lhL, q_lhR, q_hhL, q_hhR, pt_, q_ho0, q_ho1);
    L.fix(pt_, q_lhL, q_lhR, q_hhL, q_hhR);
  }
  Buf A, B;
  load_chunk(A, it.I0);

  // first half of one coefficient row: b1, a, c1 for L, R and the right halo
  // quad X; lane 0 forms b1 of quad qL-1 from its halo.
  auto first_half = [&](int llL, int llR, int hlL, int hlR, int he0, int he1, int lhL, int lhR, int hhL, int hhR,
                        int ho0, int ho1, int& b1L, int& b1R, int& aL, int& aR, int& aX, int& c1L, int& c1R,
                        int& c1X) {
    b1L = i32_inv_b1(hlL, hhU_L, hhL);
    b1R = i32_inv_b1(hlR, hhU_R, hhR);
    const int b1X = i32_inv_b1(he1, hoU1, ho1);
    const int b1H = i32_inv_b1(he0, hoU0, ho0);
    const int b1P = prv(first, b1H, b1R);
    const int hhP = prv(first, ho0, hhR);
    i32_inv_update(llL, lhU_L, lhL, b1P, b1L, hhP, hhL, aL, c1L);
    i32_inv_update(llR, lhU_R, lhR, b1L, b1R, hhL, hhR, aR, c1R);
    i32_inv_update(he0, hoU0, ho0, b1R, b1X, hhR, ho1, aX, c1X);
    lhU_L = lhL; lhU_R = lhR; hhU_L = hhL; hhU_R = hhR; hoU0 = ho0; hoU1 = ho1;
  };
  int b1_L, b1_R, a_L, a_R, a_X, c1_L, c1_R, c1_X;
  const int hh0_L = q_hhL, hh0_R = q_hhR;
  first_half(q_llL, q_llR, q_hlL, q_hlR, q_he0, q_he1, q_lhL, q_lhR, q_hhL, q_hhR, q_ho0, q_ho1, b1_L, b1_R, a_L,
             a_R, a_X, c1_L, c1_R, c1_X);
  int hh_L = hh0_L, hh_R = hh0_R;

  auto row = [&](const Buf& b, int m, int i) {
    int r_llL = b.llL[m], r_llR = b.llR[m], r_hlL = b.hlL[m], r_hlR = b.hlR[m];
    int r_lhL = b.lhL[m], r_lhR = b.lhR[m], r_hhL = b.hhL[m], r_hhR = b.hhR[m];
    L.fix(b.pe[m], r_llL, r_llR, r_hlL, r_hlR);
    L.fix(b.po[m], r_lhL, r_lhR, r_hhL, r_hhR);
    int b1n_L, b1n_R, an_L, an_R, an_X, c1n_L, c1n_R, c1n_X;
    first_half(r_llL, r_llR, r_hlL, r_hlR, b.he0[m], b.he1[m], r_lhL, r_lhR, r_hhL,
               r_hhR, b.ho0[m], b.ho1[m], b1n_L, b1n_R, an_L, an_R, an_X, c1n_L, c1n_R, c1n_X);
    const int c_L = i32_inv_c(c1_L, a_L, an_L), c_R = i32_inv_c(c1_R, a_R, an_R);
    const int c_X = i32_inv_c(c1_X, a_X, an_X);
    const int aN = nxt(last, a_X, a_L);
    const int cN = nxt(last, c_X, c_L);
    V4<int> e, o;
    e.x = a_L;
    e.z = a_R;
    o.x = c_L;
    o.z = c_R;
    i32_inv_predict(a_L, a_R, b1_L, b1n_L, c_L, c_R, hh_L, e.y, o.y);
    i32_inv_predict(a_R, aN, b1_R, b1n_R, c_R, cN, hh_R, e.w, o.w);
    S.row(2 * i, e);
    S.row(2 * i + 1, o);
    a_L = an_L; a_R = an_R; a_X = an_X; b1_L = b1n_L; b1_R = b1n_R; c1_L = c1n_L; c1_R = c1n_R; c1_X = c1n_X;
    hh_L = r_hhL;
    hh_R = r_hhR;
  };
  run_rows<CH>(it.I0, it.I1, A, B, load_chunk, row);
}

template <int CH, bool EDGE, int CI, int CO>
__device__ void bwd_f32(const LevelDesc& d, const float* __restrict__ ll, const float* __restrict__ band,
                        float* __restrict__ px, const Item& it) {
  // halos: lane 0 -> quad qL-1: h0 = LL / LH (parity 0), h1 = HL / HH (parity 1);
  // lane 63 -> quad qL+2: h0 = LL / LH (parity 0)
  const BandLoader<float, EDGE, false, CI> L =
      band_loader<float, EDGE, false, CI>(ll, d.ll_stride, band, d.band_stride, it, 0, 1, 0, 0);
  const PxStore<float, EDGE, CO> S{px, d.pix_stride, it.W, it.H, 2 * it.qL, min(2 * it.I1, it.H)};
  const bool first = it.first, last = it.last;
  const AxisW hL = axis_weights(it.qL, it.W), hR = axis_weights(it.qL + 1, it.W), hH = axis_weights(it.qL - 1, it.W);
  // whole item away from the left and right borders: the horizontal weights
  // are all 1 (then rows away from the top and bottom take the plain sums)
  const bool unit_h = __all(unit_weights(hL) && unit_weights(hR) && unit_weights(hH));
  using Buf = QBuf<float, CH>;
  auto load_chunk = [&](Buf& b, int i0) {
#pragma unroll
    for (int m = 0; m < CH; ++m) {
      L.even(i0 + m + 1, b.llL[m], b.llR[m], b.hlL[m], b.hlR[m], b.pe[m], b.he0[m], b.he1[m]);
      L.odd(i0 + m + 1, b.lhL[m], b.lhR[m], b.hhL[m], b.hhR[m], b.po[m], b.ho0[m], b.ho1[m]);
    }
  };
  // current coefficient row (starts as row I0 - 1)
  float ga_L, ga_R, gb_L, gb_R, ge0, ge1, gc_L, gc_R, gd_L, gd_R, go0, go1;
  {
    V4<float> pt_;
    L.even(it.I0 - 1, ga_L, ga_R, gb_L, gb_R, pt_, ge0, ge1);
    L.fix(pt_, ga_L, ga_R, gb_L, gb_R);
  }
  {
    V4<float> pt_;
    L.odd(it.I0 - 1, gc_L, gc_R, gd_L, gd_R, pt_, go0, go1);
    L.fix(pt_, gc_L, gc_R, gd_L, gd_R);
  }
  float n_llL, n_llR, n_hlL, n_hlR, n_he0, n_he1, n_lhL, n_lhR, n_hhL, n_hhR, n_ho0, n_ho1;
  {
    V4<float> pt_;
    L.even(it.I0, n_llL, n_llR, n_hlL, n_hlR, pt_, n_he0, n_he1);
    L.fix(pt_, n_llL, n_llR, n_hlL, n_hlR);
  }
  {
    V4<float> pt_;
    L.odd(it.I0, n_lhL, n_lhR, n_hhL, n_hhR, pt_, n_ho0, n_ho1);
    L.fix(pt_, n_lhL, n_lhR, n_hhL, n_hhR);
  }
  Buf A, B;
  load_chunk(A, it.I0);

  // step A (transposed update) of the current row given the next row's even part
  auto step_a = [&](int i, float nL, float nR, float nbL, float nbR, float ne0, float ne1, float& gb1L, float& gb1R,
                    float& gc1L, float& gc1R, float& gd1L, float& gd1R, float& gb1H, float& gd1H) {
    const AxisW v = axis_weights(i, it.H);
    const float gaN = nxt(last, ge0, ga_L), gaDN = nxt(last, ne0, nL);
    const float gcN = nxt(last, go0, gc_L);
    float gc1H;
    if (unit_h && unit_weights(v)) {
      f32_adj_a<true>(ga_L, ga_R, nL, nR, gb_L, nbL, gc_L, gc_R, gd_L, hL, v, gb1L, gc1L, gd1L);
      f32_adj_a<true>(ga_R, gaN, nR, gaDN, gb_R, nbR, gc_R, gcN, gd_R, hR, v, gb1R, gc1R, gd1R);
      f32_adj_a<true>(ge0, ga_L, ne0, nL, ge1, ne1, go0, gc_L, go1, hH, v, gb1H, gc1H, gd1H);
    } else {
      f32_adj_a(ga_L, ga_R, nL, nR, gb_L, nbL, gc_L, gc_R, gd_L, hL, v, gb1L, gc1L, gd1L);
      f32_adj_a(ga_R, gaN, nR, gaDN, gb_R, nbR, gc_R, gcN, gd_R, hR, v, gb1R, gc1R, gd1R);
      f32_adj_a(ge0, ga_L, ne0, nL, ge1, ne1, go0, gc_L, go1, hH, v, gb1H, gc1H, gd1H);
    }
  };
  float gc1U_L, gc1U_R, gd1U_L, gd1U_R, gd1UL_L;
  {
    float gb1L, gb1R, gb1H, gd1H;
    step_a(it.I0 - 1, n_llL, n_llR, n_hlL, n_hlR, n_he0, n_he1, gb1L, gb1R, gc1U_L, gc1U_R, gd1U_L, gd1U_R, gb1H,
           gd1H);
    gd1UL_L = prv(first, gd1H, gd1U_R);
  }
  ga_L = n_llL; ga_R = n_llR; gb_L = n_hlL; gb_R = n_hlR; ge0 = n_he0; ge1 = n_he1;
  gc_L = n_lhL; gc_R = n_lhR; gd_L = n_hhL; gd_R = n_hhR; go0 = n_ho0; go1 = n_ho1;

  auto row = [&](const Buf& b, int m, int i) {
    float r_llL = b.llL[m], r_llR = b.llR[m], r_hlL = b.hlL[m], r_hlR = b.hlR[m];
    float r_lhL = b.lhL[m], r_lhR = b.lhR[m], r_hhL = b.hhL[m], r_hhR = b.hhR[m];
    L.fix(b.pe[m], r_llL, r_llR, r_hlL, r_hlR);
    L.fix(b.po[m], r_lhL, r_lhR, r_hhL, r_hhR);
    float gb1_L, gb1_R, gc1_L, gc1_R, gd1_L, gd1_R, gb1H, gd1H;
    step_a(i, r_llL, r_llR, r_hlL, r_hlR, b.he0[m], b.he1[m], gb1_L, gb1_R, gc1_L, gc1_R, gd1_L, gd1_R,
           gb1H, gd1H);
    const float gb1P = prv(first, gb1H, gb1_R);
    const float gd1P = prv(first, gd1H, gd1_R);
    const AxisW v = axis_weights(i, it.H);
    V4<float> e, o;
    if (unit_h && unit_weights(v)) {
      f32_adj_b<true>(ga_L, gb1P, gb1_L, gc1U_L, gc1_L, gd1UL_L, gd1U_L, gd1P, gd1_L, hL, v, e.x, e.y, o.x);
      f32_adj_b<true>(ga_R, gb1_L, gb1_R, gc1U_R, gc1_R, gd1U_L, gd1U_R, gd1_L, gd1_R, hR, v, e.z, e.w, o.z);
    } else {
      f32_adj_b(ga_L, gb1P, gb1_L, gc1U_L, gc1_L, gd1UL_L, gd1U_L, gd1P, gd1_L, hL, v, e.x, e.y, o.x);
      f32_adj_b(ga_R, gb1_L, gb1_R, gc1U_R, gc1_R, gd1U_L, gd1U_R, gd1_L, gd1_R, hR, v, e.z, e.w, o.z);
    }
    o.y = gd1_L;
    o.w = gd1_R;
    S.row(2 * i, e);
    S.row(2 * i + 1, o);
    gc1U_L = gc1_L; gc1U_R = gc1_R; gd1U_L = gd1_L; gd1U_R = gd1_R; gd1UL_L = gd1P;
    ga_L = r_llL; ga_R = r_llR; gb_L = r_hlL; gb_R = r_hlR; ge0 = b.he0[m]; ge1 = b.he1[m];
    gc_L = r_lhL; gc_R = r_lhR; gd_L = r_hhL; gd_R = r_hhR; go0 = b.ho0[m]; go1 = b.ho1[m];
  };
  run_rows<CH>(it.I0, it.I1, A, B, load_chunk, row);
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

// Whether an item's strip reaches the right edge of the image or of a band:
// then lanes past the edge patch their vector loads with mirrored (inverse
// / forward) or zero (adjoint) single elements.
__device__ __forceinline__ bool edge_item(const Item& it, int strip) { return kStripQ * (strip + 1) > it.nd_w; }

// One work item: (image pointers already offset, strip, segment), with the
// LL input rows coherent (CI: written earlier in the same job) and the LL
// output rows coherent (CO: read later in the same job).
template <int DIR, typename T, int CH, int CI, int CO>
__device__ __forceinline__ void run_item_p(const LevelDesc& d, int64_t pix_off, int64_t ll_off, int64_t band_off,
                                           int strip, int seg, int lane) {
  const Item it = make_item(d, strip, seg, lane);
  const bool edge = edge_item(it, strip);
  if constexpr (DIR == kFwd) {
    const T* px = static_cast<const T*>(d.pix_in) + pix_off;
    T* ll = static_cast<T*>(d.ll_out) + ll_off;
    T* band = static_cast<T*>(d.band_out) + band_off;
    if constexpr (std::is_same<T, float>::value) {
      if (edge) fwd_f32<CH, true, CI, CO>(d, px, ll, band, it);
      else fwd_f32<CH, false, CI, CO>(d, px, ll, band, it);
    } else {
      if (edge) fwd_i32<CH, true, CI, CO>(d, px, ll, band, it);
      else fwd_i32<CH, false, CI, CO>(d, px, ll, band, it);
    }
  } else {
    const T* ll = static_cast<const T*>(d.ll_in) + ll_off;
    const T* band = static_cast<const T*>(d.band_in) + band_off;
    T* px = static_cast<T*>(d.pix_out) + pix_off;
    if constexpr (DIR == kInv) {
      if constexpr (std::is_same<T, float>::value) {
        if (edge) inv_f32<CH, true, CI, CO>(d, ll, band, px, it);
        else inv_f32<CH, false, CI, CO>(d, ll, band, px, it);
      } else {
        if (edge) inv_i32<CH, true, CI, CO>(d, ll, band, px, it);
        else inv_i32<CH, false, CI, CO>(d, ll, band, px, it);
      }
    } else {
      if (edge) bwd_f32<CH, true, CI, CO>(d, ll, band, px, it);
      else bwd_f32<CH, false, CI, CO>(d, ll, band, px, it);
    }
  }
}

// Level launches: the level's LL output is kept (kKeep) when a later launch
// reads it (d.keep_out), else streamed.  Persistent job steps: `coh` bit 0
// marks LL input rows written earlier in the job, bit 1 LL output rows read
// later in it (both kCoh).
template <int DIR, typename T, int CH, bool JOB>
__device__ __forceinline__ void run_item(const LevelDesc& d, int coh, int64_t pix_off, int64_t ll_off,
                                         int64_t band_off, int strip, int seg, int lane) {
  if constexpr (!JOB) {
    if (d.keep_out) run_item_p<DIR, T, CH, kStream, kKeep>(d, pix_off, ll_off, band_off, strip, seg, lane);
    else run_item_p<DIR, T, CH, kStream, kStream>(d, pix_off, ll_off, band_off, strip, seg, lane);
  } else {
    switch (coh & 3) {
      case 0: run_item_p<DIR, T, CH, kStream, kStream>(d, pix_off, ll_off, band_off, strip, seg, lane); break;
      case 1: run_item_p<DIR, T, CH, kCoh, kStream>(d, pix_off, ll_off, band_off, strip, seg, lane); break;
      case 2: run_item_p<DIR, T, CH, kStream, kCoh>(d, pix_off, ll_off, band_off, strip, seg, lane); break;
      default: run_item_p<DIR, T, CH, kCoh, kCoh>(d, pix_off, ll_off, band_off, strip, seg, lane); break;
    }
  }
}

}  // namespace
}  // namespace dwt2
