// HIP kernels for gfx950: one level of the 2-D CDF 5/3 transform with the
// non-separable lifting scheme (§3, eq. (5)) -- forward, inverse, adjoint.
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
    constexpr int P = Pol<COH>::ld, PH = Pol<COH>::halo, PB = kNT;
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

// One launch per level: one wave per work item.
template <int DIR, typename T, int CH>
__global__ __launch_bounds__(kBlock) void level_kernel(LevelLaunch a) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // wave-uniform
  const int64_t item = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * kWavesPerBlock + wave;
  if (item >= a.items) return;
  const int img = (int)(item / a.items_per_image);
  const int rem = (int)(item - (int64_t)img * a.items_per_image);
  const int seg = rem / a.d.nstrips;
  const int strip = rem - seg * a.d.nstrips;
  run_item<DIR, T, CH, false>(a.d, 0, img * a.pix_bstride, img * a.ll_bstride, img * a.band_bstride, strip, seg, lane);
}

// ---------------------------------------------------------------------------
// Persistent job: all levels of a transform (of one or many images) in one
// cooperative launch.  Work items are numbered step by step (a step is one
// level of one image, or of a batch of images); wave w takes items w,
// w + N, w + 2N, ... (N waves, all co-resident by the cooperative launch).
// An item of step t first waits until the items of step t-1 that produced
// the rows it reads have finished (per-segment completion counters), so
// levels overlap instead of meeting at a grid-wide barrier.  An item waits
// only for items with smaller numbers, each owned by a running wave that
// reaches it after finishing its own smaller items, so the schedule cannot
// deadlock; a wait that exceeds a fixed poll budget sets the error word and
// gives up rather than hang.
// ---------------------------------------------------------------------------
// s_sleep(16) pauses about 16 * 64 clocks (~0.43 us at 2.4 GHz); a poll
// backs off to at most kNapCap of them (~1.7 us), so a waiter sees a finished
// producer within about that time, and gives up after kSpinLimit polls (~2 s).
constexpr uint32_t kNapCap = 4;
constexpr uint32_t kSpinLimit = 1u << 20;

// Wait until rows [r_lo, r_hi] of the output of step p (image img) exist.
// `pixels`: the rows are pixel rows of p's output (inverse / adjoint, two per
// quadruple row); otherwise they are p's LL rows (forward, one per row).
__device__ __forceinline__ void wait_rows(const JobDesc& p, uint32_t* sync, int img, int r_lo, int r_hi,
                                          bool pixels) {
  const int ns_h = (p.d.H + 1) >> 1;
  int q_lo = pixels ? (r_lo >> 1) : r_lo, q_hi = pixels ? (r_hi >> 1) : r_hi;
  q_lo = q_lo < 0 ? 0 : q_lo;
  q_hi = q_hi > ns_h - 1 ? ns_h - 1 : q_hi;
  const int g_lo = q_lo / p.d.seg, g_hi = q_hi / p.d.seg;
  uint32_t* ctr = sync + kSyncCounters + (int64_t)kCounterStride * (p.cbase + img * p.d.nsegs);
  for (int g = g_lo; g <= g_hi; ++g) {
    uint32_t spins = 0, nap = 1;
    // every lane reads the same word; readfirstlane makes the loop wave-uniform
    while (__builtin_amdgcn_readfirstlane(__hip_atomic_load(ctr + (int64_t)kCounterStride * g, __ATOMIC_RELAXED,
                                                            __HIP_MEMORY_SCOPE_AGENT)) < (uint32_t)p.d.nstrips) {
      if (++spins > kSpinLimit) {
        __hip_atomic_store(sync + kSyncError, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      for (uint32_t k = 0; k < nap; ++k) __builtin_amdgcn_s_sleep(16);
      nap = nap < kNapCap ? 2 * nap : kNapCap;
    }
  }
  // the item's loads of the producers' rows are coherent (sc0 sc1) and are
  // issued only after the counters were seen; the fence keeps the compiler
  // from moving them above the wait
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// TABLE: descriptors and the slot -> descriptor map live in device memory
// (ragged batches); otherwise the descriptors are kernel arguments and the
// descriptor of a slot is found by a scan (at most kInlineDescs steps).
// Either way they are wave-uniform and stay in scalar registers.
template <int DIR, typename T, int CH, bool TABLE>
__global__ __launch_bounds__(kBlock) void job_kernel(JobArgs a) {
  const int lane = threadIdx.x & (kWave - 1);
  const JobDesc* __restrict__ D = TABLE ? a.descs : a.inl;
  uint32_t* sync = a.sync;
  const uint32_t one = lane == 0 ? 1u : 0u;  // wave-uniform atomic: lane 0 adds 1, the rest add 0
  const uint32_t wave = (uint32_t)xcd_remap(blockIdx.x, gridDim.x) * kWavesPerBlock +
                        __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const uint32_t nwaves = gridDim.x * kWavesPerBlock;
  int j = 0;
  for (uint32_t q = wave; q < (uint32_t)a.total_items; q += nwaves) {
    if constexpr (TABLE) {
      j = __builtin_amdgcn_readfirstlane(((const uint32_t* __restrict__)a.item_desc)[q]);
    } else {
      while (j + 1 < a.ndesc && a.inl[j + 1].item_start <= (int)q) ++j;  // items only move forward
    }
    const JobDesc jd = D[j];
    const int item = (int)q - jd.item_start;
    const int per_img = jd.d.nsegs * jd.d.nstrips;
    const int img = item / per_img;
    const int rem = item - img * per_img;
    const int seg = rem / jd.d.nstrips;
    const int strip = rem - seg * jd.d.nstrips;
    if (jd.prev >= 0) {
      const JobDesc p = D[jd.prev];
      const int I0 = seg * jd.d.seg;
      const int I1 = min(I0 + jd.d.seg, (jd.d.H + 1) >> 1);
      // rows this item reads from p's output, with a margin that covers the
      // symmetric folds at the image edges
      if (DIR == kFwd) wait_rows(p, sync, img, 2 * I0 - 4, 2 * I1 + 2, false);
      else wait_rows(p, sync, img, I0 - 3, I1 + 2, true);
    }
    run_item<DIR, T, CH, true>(jd.d, jd.coh, img * jd.pix_bstride, img * jd.ll_bstride, img * jd.band_bstride, strip,
                               seg, lane);
    // publish: the item's stores write through (sc1); once they have
    // completed (s_waitcnt 0) the count makes them visible to every XCD
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __hip_atomic_fetch_add(sync + kSyncCounters + (int64_t)kCounterStride * (jd.cbase + img * jd.d.nsegs + seg), one,
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// One step range of a ragged batch per launch (level-synchronous schedule,
// any direction):
// one wave per work item, the item's step found through the device
// item -> step table.  Steps of one launch never depend on each other.
template <int DIR, typename T, int CH>
__global__ __launch_bounds__(kBlock) void table_kernel(TableArgs a) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int64_t w = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * kWavesPerBlock + wave;
  if (w >= a.items) return;
  const int q = a.item_begin + (int)w;
  const int j = __builtin_amdgcn_readfirstlane(((const uint32_t* __restrict__)a.item_desc)[q]);
  const JobDesc jd = ((const JobDesc* __restrict__)a.descs)[j];
  const int item = q - jd.item_start;
  const int per_img = jd.d.nsegs * jd.d.nstrips;
  const int img = item / per_img;
  const int rem = item - img * per_img;
  const int seg = rem / jd.d.nstrips;
  const int strip = rem - seg * jd.d.nstrips;
  run_item<DIR, T, CH, false>(jd.d, 0, img * jd.pix_bstride, img * jd.ll_bstride, img * jd.band_bstride, strip, seg,
                              lane);
}

// ---------------------------------------------------------------------------
// Tail kernel: the last n (2 or 3) levels of a transform, whose inputs are
// small, in one launch.  Each workgroup owns a kTailS x kTailS tile of the
// first tail level's input and runs every remaining level in LDS on that
// tile plus a recompute halo of 2^(n+1) - 2 pixels (a 5/3 level reads two
// pixels on each side of a quadruple, so each coarser level doubles the
// halo and adds two), then writes the coefficients of its own tile.  Every
// read goes through the symmetric fold of its level, so values past an
// edge are the ones the strip kernels see, and the per-quadruple arithmetic
// is the strip kernels' own: results are bit-identical.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int tail_halo(int n, int m) { return (2 << (n - m)) - 2; }

// The symmetric fold for positions in [-2, n + 1] (all that the tail reads,
// n >= 2), without the division of the general fold: one reflection at 0,
// one at n - 1, and a last one at 0 for n = 2.
__device__ __forceinline__ int fold_near(int p, int n) {
  int q = p < 0 ? -p : p;
  q = q > n - 1 ? 2 * (n - 1) - q : q;
  return q < 0 ? -q : q;
}

// Threads walk 2-D ranges in rows of 64 (one wave per row), so that no
// division is needed and a wave touches consecutive columns.
constexpr int kTailRowT = 64, kTailRows = kTailBlock / kTailRowT;
// loads per thread that cover the largest level-0 region (n = 3)
constexpr int kTailLoads = ((kTailS + 2 * 14) * (kTailS + 2 * 14) + kTailBlock - 1) / kTailBlock;

template <typename T>
__global__ __launch_bounds__(kTailBlock) void tail_fwd(TailArgs a) {
  __shared__ T lds[kTailLds];
  const int lx = threadIdx.x & (kTailRowT - 1), ly = threadIdx.x / kTailRowT;
  const int tx = blockIdx.x % a.tiles_x, ty = blockIdx.x / a.tiles_x;
  const int n = a.n;
  // region arrays, one per level, then the three predict arrays
  int base[kTailMaxLevels];
  int acc = 0;
  for (int m = 0; m < n; ++m) {
    base[m] = acc;
    const int N = (kTailS >> m) + 2 * tail_halo(n, m);
    acc += N * N;
  }
  const int NP = (kTailS >> 1) + 2 * tail_halo(n, 1) + 1;
  T* P0 = lds + acc;
  T* P1 = P0 + NP * NP;
  T* P2 = P1 + NP * NP;
  for (int img = blockIdx.y; img < a.batch; img += gridDim.y) {
    const T* in = static_cast<const T*>(a.in) + img * a.in_bstride;
    T* dst = static_cast<T*>(a.out) + img * a.out_bstride;
    // level 0 input: the in-image part of the region.  Every thread issues
    // all its loads before the first LDS store, so they are in flight
    // together; surplus lanes load a valid element and discard it.
    {
      const int r = tail_halo(n, 0), N = kTailS + 2 * r;
      const int ox = tx * kTailS - r, oy = ty * kTailS - r;
      const int x0 = max(ox, 0), x1 = min(ox + N, a.W[0]), y0 = max(oy, 0), y1 = min(oy + N, a.H[0]);
      const int w = x1 - x0, cnt = w * (y1 - y0);
      // element e = threadIdx.x + k * kTailBlock sits at (y0 + e / w, x0 + e % w);
      // one division, then steps of kTailBlock elements
      const int dq = kTailBlock / w, dr = kTailBlock - dq * w;
      int ey = (int)threadIdx.x / w, ex = (int)threadIdx.x - ey * w;
      T v[kTailLoads];
      int slot[kTailLoads];
#pragma unroll
      for (int k = 0; k < kTailLoads; ++k) {
        const bool ok = (int)threadIdx.x + k * kTailBlock < cnt;
        const int gy = ok ? y0 + ey : y0, gx = ok ? x0 + ex : x0;  // surplus lanes reload a valid element
        v[k] = in[(int64_t)gy * a.in_stride + gx];
        slot[k] = ok ? base[0] + (gy - oy) * N + (gx - ox) : -1;
        ex += dr;
        ey += dq;
        if (ex >= w) {
          ex -= w;
          ++ey;
        }
      }
#pragma unroll
      for (int k = 0; k < kTailLoads; ++k)
        if (slot[k] >= 0) lds[slot[k]] = v[k];
    }
    __syncthreads();
    for (int m = 0; m < n; ++m) {
      const int Wm = a.W[m], Hm = a.H[m];
      const int r = tail_halo(n, m);
      const int N = (kTailS >> m) + 2 * r, ox = tx * (kTailS >> m) - r, oy = ty * (kTailS >> m) - r;
      const T* A = lds + base[m];
      // quadruples this level produces: the next region (or, at the last
      // level, the core), inside the image
      const int rn = m + 1 < n ? tail_halo(n, m + 1) : 0;
      const int S1 = kTailS >> (m + 1), cx = tx * S1, cy = ty * S1;
      const int ns_w = (Wm + 1) >> 1, ns_h = (Hm + 1) >> 1, nd_w = Wm >> 1, nd_h = Hm >> 1;
      const int ux0 = max(cx - rn, 0), ux1 = min(cx + S1 + rn, ns_w);
      const int uy0 = max(cy - rn, 0), uy1 = min(cy + S1 + rn, ns_h);
      // predict over the produced quadruples and one more on the left and top
      const int px0 = ux0 - 1, py0 = uy0 - 1;
      // the ranges are at most NP <= kTailRowT quadruples wide, so each
      // thread owns one column: its folded LDS columns are fixed per level
      const int qx = px0 + lx;
      const int c0 = fold_near(2 * qx, Wm) - ox, c1 = fold_near(2 * qx + 1, Wm) - ox;
      const int c2 = fold_near(2 * qx + 2, Wm) - ox;
      for (int qy = py0 + ly; qy < uy1; qy += kTailRows) {
        // folded rows 2qy .. 2qy+2 as LDS offsets
        const int r0 = (fold_near(2 * qy, Hm) - oy) * N, r1 = (fold_near(2 * qy + 1, Hm) - oy) * N;
        const int r2 = (fold_near(2 * qy + 2, Hm) - oy) * N;
        if (qx < ux1) {
          const int o = (qy - py0) * NP + (qx - px0);
          if constexpr (std::is_same<T, float>::value)
            f32_predict(A[r0 + c0], A[r0 + c2], A[r2 + c0], A[r2 + c2], A[r0 + c1], A[r2 + c1], A[r1 + c0],
                        A[r1 + c2], A[r1 + c1], P0[o], P1[o], P2[o]);
          else
            i32_predict(A[r0 + c0], A[r0 + c2], A[r2 + c0], A[r2 + c2], A[r0 + c1], A[r2 + c1], A[r1 + c0],
                        A[r1 + c2], A[r1 + c1], P0[o], P1[o], P2[o]);
        }
      }
      __syncthreads();
      const bool last = m + 1 == n;
      const int rn_base = last ? 0 : base[m + 1];
      const int Nn = S1 + 2 * rn, oxn = cx - rn, oyn = cy - rn;
      const int ux = ux0 + lx;
      const int cu = fold_near(2 * ux, Wm) - ox;
      const bool own_col = ux >= cx && ux < cx + S1;
      for (int qy = uy0 + ly; qy < uy1; qy += kTailRows) {
        const int r0 = (fold_near(2 * qy, Hm) - oy) * N;
        const bool own_row = qy >= cy && qy < cy + S1;
        if (ux < ux1) {
          const int qx = ux;
          const int o = (qy - py0) * NP + (qx - px0);
          const T va = A[r0 + cu];
          T ll, hl, lh, hh;
          if constexpr (std::is_same<T, float>::value) {
            f32_update(va, P0[o - 1], P0[o], P1[o - NP], P1[o], P2[o - NP - 1], P2[o - NP], P2[o - 1], P2[o], ll, hl,
                       lh);
            hh = P2[o];
          } else {
            const int c2 = i32_c2(P1[o], P2[o - 1], P2[o]);
            const int c2U = i32_c2(P1[o - NP], P2[o - NP - 1], P2[o - NP]);
            i32_update(va, P0[o - 1], P0[o], c2U, c2, P2[o - NP], P2[o], ll, hl);
            lh = c2;
            hh = P2[o];
          }
          if (!last) lds[rn_base + (qy - oyn) * Nn + (qx - oxn)] = ll;
          if (own_row && own_col) {  // this tile's own quadruples
            if (last) dst[(int64_t)qy * a.out_stride + qx] = ll;
            if (qx < nd_w) dst[(int64_t)qy * a.out_stride + ns_w + qx] = hl;
            if (qy < nd_h) {
              dst[(int64_t)(ns_h + qy) * a.out_stride + qx] = lh;
              if (qx < nd_w) dst[(int64_t)(ns_h + qy) * a.out_stride + ns_w + qx] = hh;
            }
          }
        }
      }
      __syncthreads();
    }
  }
}

// Inverse tail: the last n levels of an inverse (coarsest first) in one
// launch.  Each workgroup owns a kTailS x kTailS tile of the finest tail
// output and works back through the coarser levels: output pixels [d0, d1)
// of a level need its quadruples q0..q1, their coefficients one quadruple
// around (read through the symmetric extension of the interleaved array, as
// the strip kernels read them), and the LL pixels the update at q0..q1+1
// reads, which the coarser level produces (the coarsest reads them from the
// packed array).  Every array is kTailInvE wide; the index facts are walked
// on the CPU for many sizes.
constexpr int kTailInvE = kTailS / 2 + 2;
constexpr int kTailInvPasses = (kTailInvE + kTailRows - 1) / kTailRows;

__device__ __forceinline__ int band_near(int q, int n, int par) { return (fold_near(2 * q + par, n) - par) >> 1; }

template <typename T>
__global__ __launch_bounds__(kTailBlock) void tail_inv(TailArgs a) {
  __shared__ T lds[8 * kTailInvE * kTailInvE];
  constexpr int E = kTailInvE, EE = E * E;
  T* CHL = lds;           // coefficients over quadruples [q0 - 1, q1 + 1]
  T* CLH = CHL + EE;
  T* CHH = CLH + EE;
  T* U0 = CHH + EE;       // undone update (float: a, b', c'; int: b1, a, c1)
  T* U1 = U0 + EE;
  T* U2 = U1 + EE;
  T* XB[2] = {U2 + EE, U2 + 2 * EE};  // LL input of a level / its output
  const int lx = threadIdx.x & (kTailRowT - 1), ly = threadIdx.x / kTailRowT;
  const int tx = blockIdx.x % a.tiles_x, ty = blockIdx.x / a.tiles_x;
  const int n = a.n;
  // ranges per level (x, y): output pixels [d0, d1), quadruples [q0, q1]
  int d0x[kTailMaxLevels + 1], d1x[kTailMaxLevels + 1], d0y[kTailMaxLevels + 1], d1y[kTailMaxLevels + 1];
  d0x[0] = tx * kTailS;
  d1x[0] = min(tx * kTailS + kTailS, a.W[0]);
  d0y[0] = ty * kTailS;
  d1y[0] = min(ty * kTailS + kTailS, a.H[0]);
  for (int m = 0; m < n; ++m) {
    const int q0x = d0x[m] >> 1, q1x = (d1x[m] - 1) >> 1, q0y = d0y[m] >> 1, q1y = (d1y[m] - 1) >> 1;
    d0x[m + 1] = min(q0x, band_near(q1x + 1, a.W[m], 0));
    d1x[m + 1] = min(q1x + 2, a.W[m + 1]);
    d0y[m + 1] = min(q0y, band_near(q1y + 1, a.H[m], 0));
    d1y[m + 1] = min(q1y + 2, a.H[m + 1]);
  }
  for (int img = blockIdx.y; img < a.batch; img += gridDim.y) {
    const T* src = static_cast<const T*>(a.in) + img * a.in_bstride;
    T* out = static_cast<T*>(a.out) + img * a.out_bstride;
    int cur = 0;  // XB[cur]: LL input of the level being inverted
    // the coarsest level's LL from the packed array
    {
      const int x0 = d0x[n], y0 = d0y[n], w = d1x[n] - x0, h = d1y[n] - y0;
      T v[kTailInvPasses];
#pragma unroll
      for (int k = 0; k < kTailInvPasses; ++k) {
        const int y = min(ly + k * kTailRows, h - 1), x = min(lx, w - 1);
        v[k] = src[(int64_t)(y0 + y) * a.in_stride + x0 + x];
      }
#pragma unroll
      for (int k = 0; k < kTailInvPasses; ++k)
        if (lx < w && ly + k * kTailRows < h) XB[cur][(ly + k * kTailRows) * E + lx] = v[k];
    }
    for (int m = n - 1; m >= 0; --m) {
      const int Wm = a.W[m], Hm = a.H[m];
      const int ns_w = (Wm + 1) >> 1, ns_h = (Hm + 1) >> 1;
      const int q0x = d0x[m] >> 1, q1x = (d1x[m] - 1) >> 1, q0y = d0y[m] >> 1, q1y = (d1y[m] - 1) >> 1;
      const int bx = q0x - 1, by = q0y - 1;  // array origin (quadruples)
      // this thread's column: quadruple bx + lx, with its folded band columns
      const int qx = bx + lx;
      const bool col_c = qx <= q1x + 1;  // inside the coefficient range
      const int cl = band_near(qx, Wm, 0), ch = ns_w + band_near(qx, Wm, 1);
      // coefficients HL, LH, HH over [q0 - 1, q1 + 1]
      {
        const int h = q1y - q0y + 3;
        T vhl[kTailInvPasses], vlh[kTailInvPasses], vhh[kTailInvPasses];
#pragma unroll
        for (int k = 0; k < kTailInvPasses; ++k) {
          const int qy = by + min(ly + k * kTailRows, h - 1);
          const int re = band_near(qy, Hm, 0), ro = ns_h + band_near(qy, Hm, 1);
          const int c0 = col_c ? cl : 0, c1 = col_c ? ch : 0;
          vhl[k] = src[(int64_t)re * a.in_stride + c1];
          vlh[k] = src[(int64_t)ro * a.in_stride + c0];
          vhh[k] = src[(int64_t)ro * a.in_stride + c1];
        }
#pragma unroll
        for (int k = 0; k < kTailInvPasses; ++k) {
          const int row = ly + k * kTailRows;
          if (col_c && row < h) {
            CHL[row * E + lx] = vhl[k];
            CLH[row * E + lx] = vlh[k];
            CHH[row * E + lx] = vhh[k];
          }
        }
      }
      __syncthreads();
      const T* LL = XB[cur];
      const int lx0 = d0x[m + 1], ly0 = d0y[m + 1];
      const int llc = band_near(qx, Wm, 0) - lx0;  // this column's LL position in XB[cur]
      if constexpr (std::is_same<T, float>::value) {
        // undo the update at [q0, q1 + 1]
        for (int qy = q0y + ly; qy <= q1y + 1; qy += kTailRows) {
          if (qx < q0x || qx > q1x + 1) continue;
          const int o = (qy - by) * E + lx;
          const T ll = LL[(band_near(qy, Hm, 0) - ly0) * E + llc];
          f32_inv_update(ll, CHL[o - 1], CHL[o], CLH[o - E], CLH[o], CHH[o - E - 1], CHH[o - E], CHH[o - 1], CHH[o],
                         U0[o], U1[o], U2[o]);
        }
      } else {
        // b1 over columns [q0 - 1, q1 + 1], rows [q0, q1 + 1]
        for (int qy = q0y + ly; qy <= q1y + 1; qy += kTailRows) {
          if (!col_c) continue;
          const int o = (qy - by) * E + lx;
          U0[o] = i32_inv_b1(CHL[o], CHH[o - E], CHH[o]);
        }
        __syncthreads();
        for (int qy = q0y + ly; qy <= q1y + 1; qy += kTailRows) {
          if (qx < q0x || qx > q1x + 1) continue;
          const int o = (qy - by) * E + lx;
          const T ll = LL[(band_near(qy, Hm, 0) - ly0) * E + llc];
          i32_inv_update(ll, CLH[o - E], CLH[o], U0[o - 1], U0[o], CHH[o - 1], CHH[o], U1[o], U2[o]);
        }
      }
      __syncthreads();
      // undo the predict at [q0, q1]: pixels of quadruple (qx, qy)
      T* X = m > 0 ? XB[cur ^ 1] : nullptr;
      const int ox = d0x[m], oy = d0y[m];
      for (int qy = q0y + ly; qy <= q1y; qy += kTailRows) {
        if (qx < q0x || qx > q1x) continue;
        const int o = (qy - by) * E + lx;
        T va, vb, vc, vd;
        if constexpr (std::is_same<T, float>::value) {
          va = U0[o];
          f32_inv_predict(U0[o], U0[o + 1], U0[o + E], U0[o + E + 1], U1[o], U1[o + E], U2[o], U2[o + 1], CHH[o], vb,
                          vc, vd);
        } else {
          va = U1[o];
          vc = i32_inv_c(U2[o], U1[o], U1[o + E]);
          const int cR = i32_inv_c(U2[o + 1], U1[o + 1], U1[o + E + 1]);
          i32_inv_predict(U1[o], U1[o + 1], U0[o], U0[o + E], vc, cR, CHH[o], vb, vd);
        }
        const int px = 2 * qx, py = 2 * qy;
        const T vals[4] = {va, vb, vc, vd};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int x = px + (k & 1), y = py + (k >> 1);
          if (x < d0x[m] || x >= d1x[m] || y < d0y[m] || y >= d1y[m]) continue;
          if (m > 0) X[(y - oy) * E + (x - ox)] = vals[k];
          else out[(int64_t)y * a.out_stride + x] = vals[k];
        }
      }
      __syncthreads();
      cur ^= 1;
    }
  }
}

// Adjoint tail: the last n levels of W^T (coarsest first) in one launch, on
// the inverse tail's tiles.  The adjoint reads no symmetric extension:
// coefficients outside their bands are zero and the transposed boundary
// weights of the axis carry the edges, exactly as in the strip kernel.
// Output pixels [d0, d1) of a level need its quadruples q0..q1, the
// transposed update at q0-1..q1, coefficients at q0-1..q1+1, and LL pixels
// [max(q0 - 1, 0), min(q1 + 2, size)) from the coarser level.
__global__ __launch_bounds__(kTailBlock) void tail_bwd(TailArgs a) {
  __shared__ float lds[8 * kTailInvE * kTailInvE];
  constexpr int E = kTailInvE, EE = E * E;
  float* CLL = lds;          // coefficients over quadruples [q0 - 1, q1 + 1]
  float* CHL = CLL + EE;
  float* CLH = CHL + EE;
  float* CHH = CLH + EE;
  float* GB = CHH + EE;      // transposed update over [q0 - 1, q1]
  float* GC = GB + EE;
  float* GD = GC + EE;
  float* XO = GD + EE;       // a level's output pixels (the finer level's LL)
  const int lx = threadIdx.x & (kTailRowT - 1), ly = threadIdx.x / kTailRowT;
  const int tx = blockIdx.x % a.tiles_x, ty = blockIdx.x / a.tiles_x;
  const int n = a.n;
  int d0x[kTailMaxLevels + 1], d1x[kTailMaxLevels + 1], d0y[kTailMaxLevels + 1], d1y[kTailMaxLevels + 1];
  d0x[0] = tx * kTailS;
  d1x[0] = min(tx * kTailS + kTailS, a.W[0]);
  d0y[0] = ty * kTailS;
  d1y[0] = min(ty * kTailS + kTailS, a.H[0]);
  for (int m = 0; m < n; ++m) {
    const int q0x = d0x[m] >> 1, q1x = (d1x[m] - 1) >> 1, q0y = d0y[m] >> 1, q1y = (d1y[m] - 1) >> 1;
    d0x[m + 1] = max(q0x - 1, 0);
    d1x[m + 1] = min(q1x + 2, a.W[m + 1]);
    d0y[m + 1] = max(q0y - 1, 0);
    d1y[m + 1] = min(q1y + 2, a.H[m + 1]);
  }
  for (int img = blockIdx.y; img < a.batch; img += gridDim.y) {
    const float* src = static_cast<const float*>(a.in) + img * a.in_bstride;
    float* out = static_cast<float*>(a.out) + img * a.out_bstride;
    for (int m = n - 1; m >= 0; --m) {
      const int Wm = a.W[m], Hm = a.H[m];
      const int ns_w = (Wm + 1) >> 1, ns_h = (Hm + 1) >> 1, nd_w = Wm >> 1, nd_h = Hm >> 1;
      const int q0x = d0x[m] >> 1, q1x = (d1x[m] - 1) >> 1, q0y = d0y[m] >> 1, q1y = (d1y[m] - 1) >> 1;
      const int bx = q0x - 1, by = q0y - 1;
      const int qx = bx + lx;
      const bool col_c = qx <= q1x + 1;
      // coefficients over [q0 - 1, q1 + 1]; zero outside their bands.  LL
      // comes from the packed array at the coarsest level, else from the
      // coarser level's output in XO (LDS).
      {
        const int h = q1y - q0y + 3;
        const int lxo = d0x[m + 1], lyo = d0y[m + 1];
        float vll[kTailInvPasses], vhl[kTailInvPasses], vlh[kTailInvPasses], vhh[kTailInvPasses];
#pragma unroll
        for (int k = 0; k < kTailInvPasses; ++k) {
          const int qy = by + min(ly + k * kTailRows, h - 1);
          const bool rl = qy >= 0 && qy < ns_h, rh = qy >= 0 && qy < nd_h;
          const bool cl = qx >= 0 && qx < ns_w, chh = qx >= 0 && qx < nd_w;
          const int ry = rl ? qy : 0, ryo = ns_h + (rh ? qy : 0), cx = cl ? qx : 0, cxh = ns_w + (chh ? qx : 0);
          const bool ok = col_c;
          vhl[k] = (ok && rl && chh) ? src[(int64_t)ry * a.in_stride + cxh] : 0.f;
          vlh[k] = (ok && rh && cl) ? src[(int64_t)ryo * a.in_stride + cx] : 0.f;
          vhh[k] = (ok && rh && chh) ? src[(int64_t)ryo * a.in_stride + cxh] : 0.f;
          if (m == n - 1) vll[k] = (ok && rl && cl) ? src[(int64_t)ry * a.in_stride + cx] : 0.f;
          else vll[k] = (ok && rl && cl) ? XO[(ry - lyo) * E + (cx - lxo)] : 0.f;
        }
#pragma unroll
        for (int k = 0; k < kTailInvPasses; ++k) {
          const int row = ly + k * kTailRows;
          if (col_c && row < h) {
            CLL[row * E + lx] = vll[k];
            CHL[row * E + lx] = vhl[k];
            CLH[row * E + lx] = vlh[k];
            CHH[row * E + lx] = vhh[k];
          }
        }
      }
      __syncthreads();
      // transposed update at [q0 - 1, q1]
      const AxisW h0 = axis_weights(qx, Wm);
      for (int qy = by + ly; qy <= q1y; qy += kTailRows) {
        if (qx > q1x) continue;
        const int o = (qy - by) * E + lx;
        f32_adj_a(CLL[o], CLL[o + 1], CLL[o + E], CLL[o + E + 1], CHL[o], CHL[o + E], CLH[o], CLH[o + 1], CHH[o], h0,
                  axis_weights(qy, Hm), GB[o], GC[o], GD[o]);
      }
      __syncthreads();
      // transposed predict at [q0, q1]: pixels of quadruple (qx, qy)
      const int ox = d0x[m], oy = d0y[m];
      for (int qy = q0y + ly; qy <= q1y; qy += kTailRows) {
        if (qx < q0x || qx > q1x) continue;
        const int o = (qy - by) * E + lx;
        float ga2, gb2, gc2;
        f32_adj_b(CLL[o], GB[o - 1], GB[o], GC[o - E], GC[o], GD[o - E - 1], GD[o - E], GD[o - 1], GD[o], h0,
                  axis_weights(qy, Hm), ga2, gb2, gc2);
        const float vals[4] = {ga2, gb2, gc2, GD[o]};
        const int px = 2 * qx, py = 2 * qy;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int x = px + (k & 1), y = py + (k >> 1);
          if (x < d0x[m] || x >= d1x[m] || y < d0y[m] || y >= d1y[m]) continue;
          if (m > 0) XO[(y - oy) * E + (x - ox)] = vals[k];
          else out[(int64_t)y * a.out_stride + x] = vals[k];
        }
      }
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// LDS-tiled level kernels: the two schemes compared with their data movement
// held equal (the comparison of §4).  Each workgroup copies a tile of the
// level input plus a two-pixel halo on every side (through the symmetric
// fold) into LDS, runs the lifting steps with a workgroup barrier between
// consecutive steps, and stores its quadruples' four coefficients.
//   separable (eq. (3)):      HP | VP | HU | VU      four barriers
//   non-separable (eq. (5)):  spatial predict | spatial update   two barriers
// Since the fold commutes with lifting (whole-sample symmetry keeps every
// index's parity), computing on folded halo pixels gives exactly the values
// the boundary rules give, so each step runs on a fixed local range.
// ---------------------------------------------------------------------------
constexpr int kLdsQX = 64, kLdsQY = 16;                              // output quadruples per tile
constexpr int kLdsPX = 2 * kLdsQX + 4, kLdsPY = 2 * kLdsQY + 4;      // pixel tile incl. halo
constexpr int kLdsBlock = 256, kLdsWaves = kLdsBlock / kWave;
constexpr int kLdsQ1 = kLdsQX + 1, kLdsPQ = kLdsQ1 * (kLdsQY + 1);   // predicted quadruples

// Separable 1-D steps: predict x - 1/2 (l + r), update x + 1/4 (l + r);
// integer: x - floor((l + r) / 2), x + floor((l + r + 2) / 4).
__device__ __forceinline__ float lp(float x, float l, float r) { return __fmaf_rn(-0.5f, l + r, x); }
__device__ __forceinline__ float lu(float x, float l, float r) { return __fmaf_rn(0.25f, l + r, x); }
__device__ __forceinline__ int lp(int x, int l, int r) { return x - ((l + r) >> 1); }
__device__ __forceinline__ int lu(int x, int l, int r) { return x + ((l + r + 2) >> 2); }

// Runs f(row, q) over quadruple columns q in [0, kLdsQX] and rows
// [0, nrows): a wave per row for q < kLdsQX, then the last column of every
// row in one pass of the block.
template <typename F>
__device__ __forceinline__ void lds_walk65(int nrows, int lane, int wv, F&& f) {
  for (int r = wv; r < nrows; r += kLdsWaves) f(r, lane);
  if ((int)threadIdx.x < nrows) f((int)threadIdx.x, kLdsQX);
}

template <typename T, bool SEP>
__global__ __launch_bounds__(kLdsBlock) void lds_level(SepLevel a, int tiles_x) {
  __shared__ T X[kLdsPX * kLdsPY];
  __shared__ T PB[SEP ? 1 : 3 * kLdsPQ];
  // the wave index is uniform: as a scalar, row folds and row pointers are
  // scalar code, not per-lane branches
  const int lane = threadIdx.x & (kWave - 1), wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int ty = tile / tiles_x, tx = tile - ty * tiles_x;
  const int W = a.W, H = a.H;
  const int ns_w = (W + 1) >> 1, ns_h = (H + 1) >> 1, nd_w = W >> 1, nd_h = H >> 1;
  const int ox = 2 * kLdsQX * tx - 2, oy = 2 * kLdsQY * ty - 2;  // image position of X[0]
  // this lane's folded source columns: lane, lane + 64, and 128 + lane % 4
  // (stored by lanes 0..3 only; the others reload one of those four)
  const int gc0 = fold_idx(ox + lane, W), gc1 = fold_idx(ox + kWave + lane, W);
  const int gc2 = fold_idx(ox + 2 * kWave + (lane & 3), W);
  constexpr int kRowsPerWave = kLdsPY / kLdsWaves;
  static_assert(kLdsPY % kLdsWaves == 0 && kLdsPX == 2 * kWave + 4, "tile shape");
  const int gqx = tx * kLdsQX + lane;  // image quadruple column of local column lane + 1
  for (int img = blockIdx.y; img < a.batch; img += gridDim.y) {
    const T* src = static_cast<const T*>(a.src) + img * a.src_bstride;
    T* ll = static_cast<T*>(a.ll) + img * a.ll_bstride;
    T* band = static_cast<T*>(a.band) + img * a.band_bstride;
    {
      T v0[kRowsPerWave], v1[kRowsPerWave], v2[kRowsPerWave];
#pragma unroll
      for (int k = 0; k < kRowsPerWave; ++k) {
        const T* row = src + (int64_t)fold_idx(oy + wv + k * kLdsWaves, H) * a.src_stride;
        v0[k] = row[gc0];
        v1[k] = row[gc1];
        v2[k] = row[gc2];
      }
#pragma unroll
      for (int k = 0; k < kRowsPerWave; ++k) {
        T* x = X + (wv + k * kLdsWaves) * kLdsPX;
        x[lane] = v0[k];
        x[kWave + lane] = v1[k];
        if (lane < 4) x[2 * kWave + lane] = v2[k];
      }
    }
    __syncthreads();
    // every step below leaves the quadruples (i, q), i in [1, kLdsQY],
    // q in [1, kLdsQX], final: LL at X[2i][2q], HL at X[2i][2q+1] (sep.)
    T ll_v[kLdsQY / kLdsWaves], hl_v[kLdsQY / kLdsWaves], lh_v[kLdsQY / kLdsWaves], hh_v[kLdsQY / kLdsWaves];
    if constexpr (SEP) {
      // HP: odd columns, every row
      lds_walk65(kLdsPY, lane, wv, [&](int r, int q) {
        T* x = X + r * kLdsPX + 2 * q;
        x[1] = lp(x[1], x[0], x[2]);
      });
      __syncthreads();
      // VP: odd rows 2i + 1, i in [0, kLdsQY], both columns of quadruple q
      lds_walk65(kLdsQY + 1, lane, wv, [&](int i, int q) {
        T* x = X + (2 * i + 1) * kLdsPX + 2 * q;
        x[0] = lp(x[0], x[-kLdsPX], x[kLdsPX]);
        x[1] = lp(x[1], x[1 - kLdsPX], x[1 + kLdsPX]);
      });
      __syncthreads();
      // HU: even columns 2q, q in [1, kLdsQX], rows [1, 2 kLdsQY + 1]
      for (int r = 1 + wv; r <= 2 * kLdsQY + 1; r += kLdsWaves) {
        T* x = X + r * kLdsPX + 2 * (lane + 1);
        x[0] = lu(x[0], x[-1], x[1]);
      }
      __syncthreads();
      // VU: even rows 2i, i in [1, kLdsQY]; the odd rows are final
#pragma unroll
      for (int k = 0; k < kLdsQY / kLdsWaves; ++k) {
        const int i = 1 + wv + k * kLdsWaves;
        const T* x = X + 2 * i * kLdsPX + 2 * (lane + 1);
        ll_v[k] = lu(x[0], x[-kLdsPX], x[kLdsPX]);
        hl_v[k] = lu(x[1], x[1 - kLdsPX], x[1 + kLdsPX]);
        lh_v[k] = x[kLdsPX];
        hh_v[k] = x[kLdsPX + 1];
      }
    } else {
      // spatial predict over quadruples [0, kLdsQY] x [0, kLdsQX] into PB
      lds_walk65(kLdsQY + 1, lane, wv, [&](int i, int q) {
        const T* x0 = X + 2 * i * kLdsPX + 2 * q;
        const T* x1 = x0 + kLdsPX;
        const T* x2 = x1 + kLdsPX;
        const int o = i * kLdsQ1 + q;
        if constexpr (std::is_same<T, float>::value)
          f32_predict(x0[0], x0[2], x2[0], x2[2], x0[1], x2[1], x1[0], x1[2], x1[1], PB[o], PB[kLdsPQ + o],
                      PB[2 * kLdsPQ + o]);
        else
          i32_predict(x0[0], x0[2], x2[0], x2[2], x0[1], x2[1], x1[0], x1[2], x1[1], PB[o], PB[kLdsPQ + o],
                      PB[2 * kLdsPQ + o]);
      });
      __syncthreads();
      // spatial update over [1, kLdsQY] x [1, kLdsQX]
      const T* P0 = PB;
      const T* P1 = PB + kLdsPQ;
      const T* P2 = PB + 2 * kLdsPQ;
#pragma unroll
      for (int k = 0; k < kLdsQY / kLdsWaves; ++k) {
        const int i = 1 + wv + k * kLdsWaves, q = lane + 1;
        const int o = i * kLdsQ1 + q;
        const T va = X[2 * i * kLdsPX + 2 * q];
        if constexpr (std::is_same<T, float>::value) {
          f32_update(va, P0[o - 1], P0[o], P1[o - kLdsQ1], P1[o], P2[o - kLdsQ1 - 1], P2[o - kLdsQ1], P2[o - 1],
                     P2[o], ll_v[k], hl_v[k], lh_v[k]);
        } else {
          const int c2 = i32_c2(P1[o], P2[o - 1], P2[o]);
          const int c2U = i32_c2(P1[o - kLdsQ1], P2[o - kLdsQ1 - 1], P2[o - kLdsQ1]);
          i32_update(va, P0[o - 1], P0[o], c2U, c2, P2[o - kLdsQ1], P2[o], ll_v[k], hl_v[k]);
          lh_v[k] = c2;
        }
        hh_v[k] = P2[o];
      }
    }
    // store this tile's quadruples (rows and columns inside the level)
#pragma unroll
    for (int k = 0; k < kLdsQY / kLdsWaves; ++k) {
      const int gqy = ty * kLdsQY + wv + k * kLdsWaves;
      if (gqx < ns_w && gqy < ns_h) {
        ll[(int64_t)gqy * a.ll_stride + gqx] = ll_v[k];
        if (gqx < nd_w) band[(int64_t)gqy * a.band_stride + ns_w + gqx] = hl_v[k];
        if (gqy < nd_h) {
          band[(int64_t)(ns_h + gqy) * a.band_stride + gqx] = lh_v[k];
          if (gqx < nd_w) band[(int64_t)(ns_h + gqy) * a.band_stride + ns_w + gqx] = hh_v[k];
        }
      }
    }
    if (img + (int)gridDim.y < a.batch) __syncthreads();  // X and PB are reused for the next image
  }
}

// The adapted non-separable scheme (§3) on the same tiles, float only.  Each
// filter splits into its constant term and the rest, P = P0 + P1 and
// U = U0 + U1 (for the 5/3: P0 = -1/2, P1 = -1/2 z, U0 = 1/4, U1 = 1/4 z^-1).
// The constant terms touch only a quadruple's own samples, so they run
// separably without an exchange: P0 as each thread loads its quadruples, U0
// right after the one-sided predict P1, before the barrier.  The scheme keeps
// the two barriers of eq. (5) but needs 18 multiply-adds per quadruple
// instead of 23 operations.  The constant and one-sided parts commute
// (polynomials commute), so the result equals eq. (5)'s up to rounding.
constexpr int kLdsQW = kLdsPX / 2, kLdsQH = kLdsPY / 2;  // quadruples of the tile incl. halo

__global__ __launch_bounds__(kLdsBlock) void lds_adapted(SepLevel a, int tiles_x) {
  constexpr int NQ = kLdsQW * kLdsQH;
  __shared__ float Q[4 * NQ];        // a, b, c, d after P0
  __shared__ float R[4 * kLdsPQ];    // a, b', c', d' after P1 and U0
  const float* Qa = Q;
  const float* Qb = Q + NQ;
  const float* Qc = Q + 2 * NQ;
  const float* Qd = Q + 3 * NQ;
  float* Ra = R;
  float* Rb = R + kLdsPQ;
  float* Rc = R + 2 * kLdsPQ;
  float* Rd = R + 3 * kLdsPQ;
  // the wave index is uniform: as a scalar, row folds and row pointers are
  // scalar code, not per-lane branches
  const int lane = threadIdx.x & (kWave - 1), wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const int ty = tile / tiles_x, tx = tile - ty * tiles_x;
  const int W = a.W, H = a.H;
  const int ns_w = (W + 1) >> 1, ns_h = (H + 1) >> 1, nd_w = W >> 1, nd_h = H >> 1;
  const int ox = 2 * kLdsQX * tx - 2, oy = 2 * kLdsQY * ty - 2;  // image position of the tile's pixel (0, 0)
  const int cx0 = fold_idx(ox + 2 * lane, W), cx1 = fold_idx(ox + 2 * lane + 1, W);
  constexpr int kExtraQ = kLdsQW - kWave;                        // quadruple columns past the waves' 64
  constexpr int kR = (kLdsQH + kLdsWaves - 1) / kLdsWaves;       // quadruple rows per wave
  static_assert(kExtraQ * kLdsQH <= kLdsBlock, "adapted load mapping");
  const int gqx = tx * kLdsQX + lane;
  // rows (and images) start 8-byte aligned: a quadruple row's two pixels
  // load as one float2
  const bool pairs = ((reinterpret_cast<uintptr_t>(a.src) | (uintptr_t)(a.src_stride << 2) |
                       (uintptr_t)(a.src_bstride << 2)) & 7) == 0;
  const bool interior = pairs && ox >= 0 && ox + kLdsPX <= W;  // ox is even
  for (int img = blockIdx.y; img < a.batch; img += gridDim.y) {
    const float* src = static_cast<const float*>(a.src) + img * a.src_bstride;
    float* ll = static_cast<float*>(a.ll) + img * a.ll_bstride;
    float* band = static_cast<float*>(a.band) + img * a.band_bstride;
    {
      // every quadruple of the tile once: wave rows for columns 0..63, then
      // the last columns in one pass; all loads before the first LDS store
      float va[kR + 1], vb[kR + 1], vc[kR + 1], vd[kR + 1];
      int slot[kR + 1];
      // VEC: the tile's columns lie inside the image and rows are 8-byte
      // aligned, so a quadruple row's two pixels load as one float2; the
      // choice is uniform over the block, so every load is issued at once
      auto load_all = [&](auto vec_tag) {
        constexpr bool VEC = decltype(vec_tag)::value;
#pragma unroll
        for (int k = 0; k <= kR; ++k) {
          const bool extra = k == kR;
          const int t = threadIdx.x;
          const int row = wv + k * kLdsWaves;
          const bool live = extra ? t < kExtraQ * kLdsQH : row < kLdsQH;
          const int i = live ? (extra ? t / kExtraQ : row) : 0;
          const int q = extra ? kWave + t % kExtraQ : lane;
          const float* r0 = src + (int64_t)fold_idx(oy + 2 * i, H) * a.src_stride;
          const float* r1 = src + (int64_t)fold_idx(oy + 2 * i + 1, H) * a.src_stride;
          if constexpr (VEC) {
            const int x0 = ox + 2 * q;
            const float2 p0 = *reinterpret_cast<const float2*>(r0 + x0);
            const float2 p1 = *reinterpret_cast<const float2*>(r1 + x0);
            va[k] = p0.x;
            vb[k] = p0.y;
            vc[k] = p1.x;
            vd[k] = p1.y;
          } else {
            const int x0 = extra ? fold_idx(ox + 2 * q, W) : cx0, x1 = extra ? fold_idx(ox + 2 * q + 1, W) : cx1;
            va[k] = r0[x0];
            vb[k] = r0[x1];
            vc[k] = r1[x0];
            vd[k] = r1[x1];
          }
          slot[k] = live ? i * kLdsQW + q : -1;
        }
      };
      if (interior) load_all(std::true_type{});
      else load_all(std::false_type{});
#pragma unroll
      for (int k = 0; k <= kR; ++k) {
        const int o = slot[k];
        if (o >= 0) {
          // constant predict parts: horizontal, then vertical
          const float b = __fmaf_rn(-0.5f, va[k], vb[k]);
          float d = __fmaf_rn(-0.5f, vc[k], vd[k]);
          const float c = __fmaf_rn(-0.5f, va[k], vc[k]);
          d = __fmaf_rn(-0.5f, b, d);
          Q[o] = va[k];
          Q[NQ + o] = b;
          Q[2 * NQ + o] = c;
          Q[3 * NQ + o] = d;
        }
      }
    }
    __syncthreads();
    // step 1 over quadruples [0, kLdsQY] x [0, kLdsQX]: the one-sided predict
    // (neighbours after P0), then the constant update parts
    lds_walk65(kLdsQY + 1, lane, wv, [&](int i, int q) {
      const int o = i * kLdsQW + q;
      float bp = __fmaf_rn(-0.5f, Qa[o + 1], Qb[o]);
      float cp = __fmaf_rn(-0.5f, Qa[o + kLdsQW], Qc[o]);
      const float dp = __fmaf_rn(0.25f, Qa[o + kLdsQW + 1],
                                 __fmaf_rn(-0.5f, Qb[o + kLdsQW], __fmaf_rn(-0.5f, Qc[o + 1], Qd[o])));
      float an = __fmaf_rn(0.25f, bp, Qa[o]);
      cp = __fmaf_rn(0.25f, dp, cp);
      an = __fmaf_rn(0.25f, cp, an);
      bp = __fmaf_rn(0.25f, dp, bp);
      const int p = i * kLdsQ1 + q;
      Ra[p] = an;
      Rb[p] = bp;
      Rc[p] = cp;
      Rd[p] = dp;
    });
    __syncthreads();
    // step 2 over [1, kLdsQY] x [1, kLdsQX]: the one-sided update
#pragma unroll
    for (int k = 0; k < kLdsQY / kLdsWaves; ++k) {
      const int i = 1 + wv + k * kLdsWaves;
      const int p = i * kLdsQ1 + lane + 1;
      const float vll = __fmaf_rn(0.0625f, Rd[p - kLdsQ1 - 1], __fmaf_rn(0.25f, Rc[p - kLdsQ1], __fmaf_rn(0.25f, Rb[p - 1], Ra[p])));
      const float vhl = __fmaf_rn(0.25f, Rd[p - kLdsQ1], Rb[p]);
      const float vlh = __fmaf_rn(0.25f, Rd[p - 1], Rc[p]);
      const float vhh = Rd[p];
      const int gqy = ty * kLdsQY + wv + k * kLdsWaves;
      if (gqx < ns_w && gqy < ns_h) {
        ll[(int64_t)gqy * a.ll_stride + gqx] = vll;
        if (gqx < nd_w) band[(int64_t)gqy * a.band_stride + ns_w + gqx] = vhl;
        if (gqy < nd_h) {
          band[(int64_t)(ns_h + gqy) * a.band_stride + gqx] = vlh;
          if (gqx < nd_w) band[(int64_t)(ns_h + gqy) * a.band_stride + ns_w + gqx] = vhh;
        }
      }
    }
    if (img + (int)gridDim.y < a.batch) __syncthreads();
  }
}

__global__ void zero_kernel(uint32_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

template <int DIR, typename T, int CH>
hipError_t launch_t(const LevelLaunch& a, hipStream_t s) {
  const int64_t blocks = (a.items + kWavesPerBlock - 1) / kWavesPerBlock;
  hipLaunchKernelGGL((level_kernel<DIR, T, CH>), dim3((unsigned)blocks), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

template <int DIR, typename T>
hipError_t launch_ch(int chunk, const LevelLaunch& a, hipStream_t s) {
  if (chunk >= 4) return launch_t<DIR, T, 4>(a, s);
  if (chunk >= 2) return launch_t<DIR, T, 2>(a, s);
  return launch_t<DIR, T, 1>(a, s);
}


// Cooperative launch: the runtime places every block at once or fails.
template <int DIR, typename T, int CH>
hipError_t launch_job_t(const JobArgs& a, int blocks, hipStream_t s) {
  void* args[] = {const_cast<JobArgs*>(&a)};
  const void* f = a.descs ? reinterpret_cast<const void*>(&job_kernel<DIR, T, CH, true>)
                          : reinterpret_cast<const void*>(&job_kernel<DIR, T, CH, false>);
  return hipLaunchCooperativeKernel(f, dim3((unsigned)blocks), dim3(kBlock), args, 0, s);
}

template <int DIR, typename T>
hipError_t launch_job_ch(int chunk, const JobArgs& a, int blocks, hipStream_t s) {
  if (chunk >= 4) return launch_job_t<DIR, T, 4>(a, blocks, s);
  if (chunk >= 2) return launch_job_t<DIR, T, 2>(a, blocks, s);
  return launch_job_t<DIR, T, 1>(a, blocks, s);
}

// Resident blocks per CU of the job kernel variant that a launch uses
// (TABLE: descriptors in device memory); the cooperative launch fails if
// the grid exceeds what this variant can hold at once.
template <int DIR, typename T, int CH>
int occ_job(bool table) {
  int n = 0;
  const void* f = table ? reinterpret_cast<const void*>(&job_kernel<DIR, T, CH, true>)
                        : reinterpret_cast<const void*>(&job_kernel<DIR, T, CH, false>);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, kBlock, 0) != hipSuccess) n = 0;
  return n;
}

template <int CH>
int occ_job_dir(int dir, int mode, bool table) {
  if (dir == kFwd) return mode == DWT2_F32 ? occ_job<kFwd, float, CH>(table) : occ_job<kFwd, int, CH>(table);
  if (dir == kInv) return mode == DWT2_F32 ? occ_job<kInv, float, CH>(table) : occ_job<kInv, int, CH>(table);
  return occ_job<kBwd, float, CH>(table);
}

}  // namespace

int launch_job(int dir, int mode, int chunk, const JobArgs& a, int blocks, void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (dir == kFwd)
    return mode == DWT2_F32 ? launch_job_ch<kFwd, float>(chunk, a, blocks, s) : launch_job_ch<kFwd, int>(chunk, a, blocks, s);
  if (dir == kInv)
    return mode == DWT2_F32 ? launch_job_ch<kInv, float>(chunk, a, blocks, s) : launch_job_ch<kInv, int>(chunk, a, blocks, s);
  return launch_job_ch<kBwd, float>(chunk, a, blocks, s);
}

int job_blocks_per_cu(int dir, int mode, int chunk, bool table) {
  if (chunk >= 4) return occ_job_dir<4>(dir, mode, table);
  if (chunk >= 2) return occ_job_dir<2>(dir, mode, table);
  return occ_job_dir<1>(dir, mode, table);
}

template <int DIR, typename T>
hipError_t launch_table_t(int chunk, const TableArgs& a, hipStream_t s) {
  const dim3 grid((unsigned)((a.items + kWavesPerBlock - 1) / kWavesPerBlock));
  if (chunk >= 2) hipLaunchKernelGGL((table_kernel<DIR, T, 2>), grid, dim3(kBlock), 0, s, a);
  else hipLaunchKernelGGL((table_kernel<DIR, T, 1>), grid, dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

int launch_table(int dir, int mode, int chunk, const TableArgs& a, void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (a.items <= 0) return hipSuccess;
  if (dir == kFwd)
    return mode == DWT2_F32 ? launch_table_t<kFwd, float>(chunk, a, s) : launch_table_t<kFwd, int>(chunk, a, s);
  if (dir == kInv)
    return mode == DWT2_F32 ? launch_table_t<kInv, float>(chunk, a, s) : launch_table_t<kInv, int>(chunk, a, s);
  return launch_table_t<kBwd, float>(chunk, a, s);
}

int launch_tail(int dir, int mode, const TailArgs& a, void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  const dim3 grid((unsigned)(a.tiles_x * a.tiles_y), (unsigned)(a.batch < 65535 ? a.batch : 65535));
  if (dir == kFwd) {
    if (mode == DWT2_F32) hipLaunchKernelGGL(tail_fwd<float>, grid, dim3(kTailBlock), 0, s, a);
    else hipLaunchKernelGGL(tail_fwd<int>, grid, dim3(kTailBlock), 0, s, a);
  } else if (dir == kInv) {
    if (mode == DWT2_F32) hipLaunchKernelGGL(tail_inv<float>, grid, dim3(kTailBlock), 0, s, a);
    else hipLaunchKernelGGL(tail_inv<int>, grid, dim3(kTailBlock), 0, s, a);
  } else {
    if (mode != DWT2_F32) return hipErrorInvalidValue;
    hipLaunchKernelGGL(tail_bwd, grid, dim3(kTailBlock), 0, s, a);
  }
  return hipGetLastError();
}

int lds_tiles(int W, int H, int& tiles_x, int& tiles_y) {
  tiles_x = (((W + 1) >> 1) + kLdsQX - 1) / kLdsQX;
  tiles_y = (((H + 1) >> 1) + kLdsQY - 1) / kLdsQY;
  return (int64_t)tiles_x * tiles_y <= 0x7fffffff;
}

int launch_lds_level(int scheme, int mode, const SepLevel& a, void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  int tx, ty;
  if (!lds_tiles(a.W, a.H, tx, ty)) return hipErrorInvalidValue;
  const dim3 grid((unsigned)(tx * ty), (unsigned)(a.batch < 65535 ? a.batch : 65535));
  if (scheme == DWT2_SCHEME_ADAPTED) {
    if (mode != DWT2_F32) return hipErrorInvalidValue;
    hipLaunchKernelGGL(lds_adapted, grid, dim3(kLdsBlock), 0, s, a, tx);
  } else if (scheme == DWT2_SCHEME_SEPARABLE) {
    if (mode == DWT2_F32) hipLaunchKernelGGL((lds_level<float, true>), grid, dim3(kLdsBlock), 0, s, a, tx);
    else hipLaunchKernelGGL((lds_level<int, true>), grid, dim3(kLdsBlock), 0, s, a, tx);
  } else {
    if (mode == DWT2_F32) hipLaunchKernelGGL((lds_level<float, false>), grid, dim3(kLdsBlock), 0, s, a, tx);
    else hipLaunchKernelGGL((lds_level<int, false>), grid, dim3(kLdsBlock), 0, s, a, tx);
  }
  return hipGetLastError();
}

int launch_zero(uint32_t* p, int64_t n, void* stream) {
  const int64_t blocks = n < 256 * 256 ? (n + 255) / 256 : 256;
  hipLaunchKernelGGL(zero_kernel, dim3((unsigned)(blocks > 0 ? blocks : 1)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), p, n);
  return hipGetLastError();
}

int launch_level(int dir, int mode, int chunk, const LevelLaunch& a, void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (dir == kFwd) return mode == DWT2_F32 ? launch_ch<kFwd, float>(chunk, a, s) : launch_ch<kFwd, int>(chunk, a, s);
  if (dir == kInv) return mode == DWT2_F32 ? launch_ch<kInv, float>(chunk, a, s) : launch_ch<kInv, int>(chunk, a, s);
  return launch_ch<kBwd, float>(chunk, a, s);
}

}  // namespace dwt2
