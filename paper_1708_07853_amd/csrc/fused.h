// Two levels of the transform in one pass over HBM ("pair" kernels): a wave
// computes level k of a strip and, on chip, level k+1 of the LL_k values it
// has just produced (forward; the inverse and adjoint run the pair coarsest
// first).  LL_k never goes to memory: a pair reads the level-k input once
// and writes the two levels' H bands and LL_{k+1} (forward), so its HBM
// bytes are those of one level plus a quarter.
//
// Mapping.  A wave covers 128 level-k quadruple columns, lane l holding two
// adjacent quadruples (one 16-byte vector per pixel row, as in the
// single-level strip kernels) and, at level k+1, the quadruple they form
// (LL_k columns 2Q, 2Q+1 sit in the same lane).  Strips overlap: a strip
// owns 56 lanes' columns and its edge lanes recompute the neighbouring
// strips' columns, so every neighbour value a level needs crosses lanes by
// DPP and no lane loads or lifts a halo of its own (which lanes are owned:
// PairLanes).
//
// Rows.  A work item walks level-(k+1) quadruple rows [J0, J1), i.e. level-k
// quadruple rows [2 J0, 2 J1), with level k+1 lagging level k by one pair of
// rows; the few rows above the segment that the two levels' vertical
// neighbours need are recomputed (not stored).
//
// Boundaries.  Level k reads the symmetric extension of its input exactly as
// the single-level kernels do.  The extension level k+1 needs is that of
// LL_k, which at the bottom and right edges differs from what level k would
// produce past the edge for even sizes (level k mirrors about the last pixel,
// level k+1 about the last LL_k sample), so LL_k values past its edges are
// replaced explicitly: rows by uniform selects of rows already held,
// columns by DPP from the lanes to the left.  At the top and left edges (a
// mirror about index 0) both extensions agree for level-k inputs of at
// least 5 x 5, which the host guarantees.  The adjoint reads zeros outside
// the bands instead and needs only masks.
//
// Results are bit-identical to the single-level kernels: every coefficient
// is computed by the same per-quadruple functions from the same values.
#pragma once

#include "lift.h"

namespace dwt2 {
namespace {

// ---------------------------------------------------------------------------
// The per-quadruple arithmetic behind one interface for float and int32.
// Spatial predict: (p0, p1, p2) = (b', c', d') (float) or (b1, c1, d2) (int).
// Spatial update: LL, HL, LH from a and the predicted values (int: the
// rounded horizontal update of LH needs the left neighbour's d2, recomputed
// here for the row above).  Inverse update: (u0, u1, u2) = (a, b', c')
// (float) or (a, b1, c1) (int).  Inverse predict: (b, c, d).
// ---------------------------------------------------------------------------
template <typename T>
struct Ops;

template <>
struct Ops<float> {
  static __device__ __forceinline__ void predict(float a, float aR, float aD, float aDR, float b, float bD, float c,
                                                 float cR, float d, float& p0, float& p1, float& p2) {
    f32_predict(a, aR, aD, aDR, b, bD, c, cR, d, p0, p1, p2);
  }
  static __device__ __forceinline__ void update(float a, float p0L, float p0, float p1U, float p1, float p2UL,
                                                float p2U, float p2L, float p2, float& ll, float& hl, float& lh) {
    f32_update(a, p0L, p0, p1U, p1, p2UL, p2U, p2L, p2, ll, hl, lh);
  }
  static __device__ __forceinline__ void inv_update(float ll, float hlL, float hl, float lhU, float lh, float hhUL,
                                                    float hhU, float hhL, float hh, float& u0, float& u1,
                                                    float& u2) {
    f32_inv_update(ll, hlL, hl, lhU, lh, hhUL, hhU, hhL, hh, u0, u1, u2);
  }
  static __device__ __forceinline__ void inv_predict(float a, float aR, float aD, float aDR, float u1, float u1D,
                                                     float u2, float u2R, float hh, float& b, float& c, float& d) {
    f32_inv_predict(a, aR, aD, aDR, u1, u1D, u2, u2R, hh, b, c, d);
  }
};

template <>
struct Ops<int> {
  static __device__ __forceinline__ void predict(int a, int aR, int aD, int aDR, int b, int bD, int c, int cR, int d,
                                                 int& p0, int& p1, int& p2) {
    i32_predict(a, aR, aD, aDR, b, bD, c, cR, d, p0, p1, p2);
  }
  static __device__ __forceinline__ void update(int a, int p0L, int p0, int p1U, int p1, int p2UL, int p2U, int p2L,
                                                int p2, int& ll, int& hl, int& lh) {
    const int c2 = i32_c2(p1, p2L, p2), c2U = i32_c2(p1U, p2UL, p2U);
    i32_update(a, p0L, p0, c2U, c2, p2U, p2, ll, hl);
    lh = c2;
  }
  static __device__ __forceinline__ void inv_update(int ll, int hlL, int hl, int lhU, int lh, int hhUL, int hhU,
                                                    int hhL, int hh, int& u0, int& u1, int& u2) {
    u1 = i32_inv_b1(hl, hhU, hh);
    const int b1L = i32_inv_b1(hlL, hhUL, hhL);
    i32_inv_update(ll, lhU, lh, b1L, u1, hhL, hh, u0, u2);
  }
  static __device__ __forceinline__ void inv_predict(int a, int aR, int aD, int aDR, int u1, int u1D, int u2, int u2R,
                                                     int hh, int& b, int& c, int& d) {
    c = i32_inv_c(u2, a, aD);
    const int cR = i32_inv_c(u2R, aR, aDR);
    i32_inv_predict(a, aR, u1, u1D, c, cR, hh, b, d);
  }
};

// Lanes a strip owns: 4..59.  Validity shrinks from the wave's edges as
// values cross lanes: the forward's first level-k step reads the right
// neighbour (valid up to lane 62, and lane 63's first LL_k column is still
// valid), its second the left one (from lane 1), and level k+1 repeats that
// on LL_k, so lanes 2..62 are whole; the inverse (left neighbour first) is
// whole in lanes 1..61, the adjoint in 2..61.  Owning 56 lanes (112
// level-k quadruple columns) instead of the most each direction allows
// makes every strip's stores start on a 64-byte boundary -- a level-k band
// row run is 448 bytes, a pixel row run 896 -- which measured 14-20 % faster
// than owning 61 lanes with stores that straddle the boundaries.
template <int DIR>
struct PairLanes {
  static constexpr int base = 4;
  static constexpr int count = 56;
};

static_assert(pair_strip_q(kFwd) == 2 * PairLanes<kFwd>::count && pair_strip_q(kInv) == 2 * PairLanes<kInv>::count &&
                  pair_strip_q(kBwd) == 2 * PairLanes<kBwd>::count,
              "the host's strip pitch must match the owned lanes");

// One work item of a pair launch.
struct PairItem {
  int W, H;                        // level-k input
  int ns_w, nd_w, ns_h, nd_h;      // level-k bands; LL_k is ns_w x ns_h
  int ns_w1, nd_w1, ns_h1, nd_h1;  // level-(k+1) bands
  int qL;                          // level-k quadruple of the lane's first column (may be negative)
  int Q;                           // level-(k+1) quadruple of the lane (qL / 2)
  int J0, J1;                      // level-(k+1) quadruple rows written
  bool own;                        // the lane's columns are the strip's own
};

template <int DIR>
__device__ __forceinline__ PairItem make_pair_item(const LevelDesc& d, int strip, int seg, int lane) {
  using PL = PairLanes<DIR>;
  PairItem it;
  it.W = d.W; it.H = d.H;
  it.ns_w = (d.W + 1) >> 1; it.nd_w = d.W >> 1;
  it.ns_h = (d.H + 1) >> 1; it.nd_h = d.H >> 1;
  it.ns_w1 = (it.ns_w + 1) >> 1; it.nd_w1 = it.ns_w >> 1;
  it.ns_h1 = (it.ns_h + 1) >> 1; it.nd_h1 = it.ns_h >> 1;
  it.Q = PL::count * strip + lane - PL::base;
  it.qL = 2 * it.Q;
  it.J0 = seg * d.seg;
  it.J1 = min(it.J0 + d.seg, it.ns_h1);
  it.own = lane >= PL::base && lane < PL::base + PL::count;
  return it;
}

// Whether an item's lanes reach outside the image on the left (strip 0) or
// the right: then they read folded single elements instead of vectors.
template <int DIR>
__device__ __forceinline__ bool pair_edge(const PairItem& it, int strip) {
  using PL = PairLanes<DIR>;
  const int q_first = 2 * (PL::count * strip - PL::base);
  return q_first < 0 || q_first + 2 * kWave > it.nd_w;
}

// Element offset that no buffer holds (its store or load is dropped).
constexpr int kOff = -1;

// Load policy of the pair kernels: the default (caching) one.  Neighbouring
// strips load the same columns for their overlapping lanes, and vertically
// adjacent segments the same rows for their halos, at about the same time;
// cached loads let one of them hit in L2.  With non-temporal loads the
// pairs fetched 1.29-1.33x their input bytes from memory, and measured
// 8-11 % slower (8192^2 float, six levels: forward 137.7 vs 133.1 us,
// inverse 137.2 vs 126.2, adjoint 140.6 vs 130.6).
constexpr int kLdPol = 0;

// Pixel-row loads of level k: four pixels per lane, one 16-byte load (or,
// EDGE, four folded single elements).
template <typename T, bool EDGE>
struct PairPx {
  const T* base;
  int64_t stride;
  int W, H, c0;
  int pc[4];
  __device__ __forceinline__ void load(int r, V4<T>& m) const {
    const Rsrc rs = row_rsrc(base + (int64_t)fold_idx(r, H) * stride, (int64_t)W * 4);
    if constexpr (EDGE) {
      m.x = bld1<T, kLdPol>(rs, pc[0]);
      m.y = bld1<T, kLdPol>(rs, pc[1]);
      m.z = bld1<T, kLdPol>(rs, pc[2]);
      m.w = bld1<T, kLdPol>(rs, pc[3]);
    } else {
      bld4<kLdPol>(rs, c0, m);
    }
  }
};

// One-element store helper (level k+1 writes one value per lane and row).
template <int POL, typename T>
__device__ __forceinline__ void bst1(T v, Rsrc r, int e) {
  __builtin_amdgcn_raw_buffer_store_b32(ubits(v), r, (unsigned)e * 4u, 0, POL);
}

// ---------------------------------------------------------------------------
// Forward pair: levels k and k+1.
// ---------------------------------------------------------------------------
// Level-(k+1) columns a workgroup of the forward pair stages through LDS,
// and the staging array's layout: per buffer, the workgroup's run of each
// of the three level-k bands on two level-k rows (kPairStageK elements
// each), then its run of each of the four level-(k+1) bands (kPairGroupQ).
constexpr int kPairGroupQ = kWavesPerBlock * PairLanes<kFwd>::count;
constexpr int kPairStageK = 2 * kPairGroupQ;
constexpr int kPairStageBuf = 6 * kPairStageK + 4 * kPairGroupQ;

// stage_lds: the workgroup's staging array, 2 x kPairStageBuf elements
// (one array for every wave of the workgroup, whichever variant it runs).
template <typename T, int CP, bool EDGE, bool STAGED>
__device__ void fwd_pair(const LevelDesc& d, const T* __restrict__ px, T* __restrict__ ll2, T* __restrict__ band,
                         const PairItem& it, T* stage_lds) {
  using O = Ops<T>;
  PairPx<T, EDGE> L;
  L.base = px; L.stride = d.pix_stride; L.W = it.W; L.H = it.H; L.c0 = 2 * it.qL;
  for (int k = 0; k < 4; ++k) L.pc[k] = fold_idx(L.c0 + k, it.W);
  const int64_t bs = d.band_stride, ls = d.ll_stride;
  // Stores.  Direct: each lane writes its own values -- its two level-k
  // quadruples' band values (8 bytes per band row, owned lanes only) with
  // the streaming policy, its level-(k+1) values (4 bytes) with the
  // write-back policy.  A strip's level-k runs are 448 bytes long, so every
  // other strip starts in the middle of a 128-byte line, and the level-(k+1)
  // runs (224 bytes) split lines at most strip edges.
  // STAGED: through LDS.  The four waves of a workgroup hold four adjacent
  // strips of one segment (the host pads the strip count to a multiple of
  // four), so together they own 448 adjacent level-k and 224 level-(k+1)
  // columns: 1792 and 896 bytes of each band row, from a 128-byte boundary
  // on.  Each wave puts its values of the two level-k rows and the
  // level-(k+1) row of a step into LDS, and after one barrier the waves
  // write whole runs with 16-byte stores: wave w the halves (w & 1) of the
  // level-k band rows w >> 1, 2 + (w >> 1), 4 + (w >> 1) of the six, and
  // level-(k+1) band w.  The prologue's level-k row goes out directly.
  // Split lines cost: the staged pair takes 107.8 us on 8192^2 float, the
  // direct one 110.8 us.
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int lane = threadIdx.x & (kWave - 1);
  const int slot = w * PairLanes<kFwd>::count + lane - PairLanes<kFwd>::base;  // this lane's column in the group
  const int Q0 = it.Q - slot;                // the group's first level-(k+1) column
  int buf = 0;
  bool direct_k = true;                      // level-k rows of the prologue
  // level-k band stores: owned lanes only, rows [2 J0, min(2 J1, ns_h))
  const int qst = it.own ? it.qL : kOff;
  const int krow_lo = 2 * it.J0, krow_hi = min(2 * it.J1, it.ns_h);
  // level-k band row `bnd` (0 HL, 1 LH, 2 HH) of row i, and whether it is stored
  auto krow_rsrc = [&](int i, int bnd) {
    const bool real = i >= krow_lo && i < krow_hi, real2 = real && i < it.nd_h;
    T* row = bnd == 0 ? band + (int64_t)i * bs + it.ns_w
                      : band + (int64_t)(it.ns_h + i) * bs + (bnd == 2 ? it.ns_w : 0);
    const bool ok = bnd == 0 ? real : real2;
    return row_rsrc(row, ok ? (bnd == 1 ? it.ns_w : it.nd_w) * 4 : 0);
  };
  auto store_k = [&](int i, T hlL, T hlR, T lhL, T lhR, T hhL, T hhR) {
    if constexpr (STAGED) {
      if (!direct_k) {
        if (it.own) {  // row 2j+1 -> slot 0, row 2j+2 -> slot 1
          T* sk = stage_lds + buf * kPairStageBuf + ((i + 1) & 1) * 3 * kPairStageK + 2 * slot;
          sk[0] = hlL; sk[1] = hlR;
          sk[kPairStageK] = lhL; sk[kPairStageK + 1] = lhR;
          sk[2 * kPairStageK] = hhL; sk[2 * kPairStageK + 1] = hhR;
        }
        return;
      }
    }
    bst2<kNT>(hlL, hlR, krow_rsrc(i, 0), qst);
    bst2<kNT>(lhL, lhR, krow_rsrc(i, 1), qst);
    bst2<kNT>(hhL, hhR, krow_rsrc(i, 2), qst);
  };
  const int Qst = it.own ? it.Q : kOff;
  auto store_k1 = [&](int j, T ll, T hl, T lh, T hh) {
    if constexpr (!STAGED) {
      const bool real = j >= it.J0 && j < it.J1, real2 = real && j < it.nd_h1;
      const Rsrc rl = row_rsrc(ll2 + (int64_t)j * ls, real ? it.ns_w1 * 4 : 0);
      const Rsrc rh = row_rsrc(band + (int64_t)j * bs + it.ns_w1, real ? it.nd_w1 * 4 : 0);
      T* row2 = band + (int64_t)(it.ns_h1 + j) * bs;
      const Rsrc rlh = row_rsrc(row2, real2 ? it.ns_w1 * 4 : 0);
      const Rsrc rhh = row_rsrc(row2 + it.ns_w1, real2 ? it.nd_w1 * 4 : 0);
      bst1<0>(ll, rl, Qst);
      bst1<0>(hl, rh, Qst);
      bst1<0>(lh, rlh, Qst);
      bst1<0>(hh, rhh, Qst);
      return;
    }
    T* sb = stage_lds + buf * kPairStageBuf;
    if (it.own) {
      T* s1 = sb + 6 * kPairStageK + slot;
      s1[0] = ll;
      s1[kPairGroupQ] = hl;
      s1[2 * kPairGroupQ] = lh;
      s1[3 * kPairGroupQ] = hh;
    }
    __syncthreads();
    // level-k rows 2j+1 (band rows 0..2) and 2j+2 (3..5)
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      const int rb = 2 * t + (w >> 1), half = w & 1;
      const int r = rb >= 3 ? 1 : 0;
      const int e = half * 4 * kWave + 4 * lane;  // element of the group's run
      const bool st = e < kPairStageK;
      const T* src = sb + rb * kPairStageK + (st ? e : 0);
      V4<T> v;
      v.x = src[0]; v.y = src[1]; v.z = src[2]; v.w = src[3];
      bst4<kNT>(v, krow_rsrc(2 * j + 1 + r, rb - 3 * r), st ? 2 * Q0 + e : kOff);
    }
    // level k+1: wave w stores band w (0 LL_{k+1}, 1 HL, 2 LH, 3 HH) of row j
    const bool real = j >= it.J0 && j < it.J1, real2 = real && j < it.nd_h1;
    const bool hpar = w == 1 || w == 3;
    const bool ok = w < 2 ? real : real2;
    T* row = w == 0 ? ll2 + (int64_t)j * ls
                    : band + (int64_t)(w < 2 ? j : it.ns_h1 + j) * bs + (hpar ? it.ns_w1 : 0);
    const Rsrc rs = row_rsrc(row, ok ? (hpar ? it.nd_w1 : it.ns_w1) * 4 : 0);
    const int qs = 4 * lane;                 // the columns this lane stores: Q0 + qs .. Q0 + qs + 3
    const bool st_lane = qs < kPairGroupQ;
    const T* src = sb + 6 * kPairStageK + w * kPairGroupQ + (st_lane ? qs : 0);
    V4<T> v;
    v.x = src[0]; v.y = src[1]; v.z = src[2]; v.w = src[3];
    // the group's columns before 0 (strip 0's left lanes) are not stored:
    // Q0 >= 0 always, since the first group starts at column 0
    // LL_{k+1} keeps the caching policy when a later launch reads it
    if (w == 0 && d.keep_out) bst4<0>(v, rs, st_lane ? Q0 + qs : kOff);
    else bst4<kNT>(v, rs, st_lane ? Q0 + qs : kOff);
    buf ^= 1;
  };

  // ---- level k: one quadruple row from pixel rows E (2i), O (2i+1), E1 (2i+2)
  V4<T> E;                       // pixel row 2i of the row being computed
  T p1U_L, p1U_R, p2U_L, p2U_R, p2U_P;  // predicted c, d of the row above (P: left neighbour's R)
  auto krow = [&](int i, const V4<T>& O_, const V4<T>& E1, T& llL, T& llR) {
    T p0L, p1L, p2L, p0R, p1R, p2R;
    O::predict(E.x, E.z, E1.x, E1.z, E.y, E1.y, O_.x, O_.z, O_.y, p0L, p1L, p2L);
    O::predict(E.z, from_next(E.x), E1.z, from_next(E1.x), E.w, E1.w, O_.z, from_next(O_.x), O_.w, p0R, p1R, p2R);
    const T p0P = from_prev(p0R), p2P = from_prev(p2R);
    T hlL, lhL, hlR, lhR;
    O::update(E.x, p0P, p0L, p1U_L, p1L, p2U_P, p2U_L, p2P, p2L, llL, hlL, lhL);
    O::update(E.z, p0L, p0R, p1U_R, p1R, p2U_L, p2U_R, p2L, p2R, llR, hlR, lhR);
    store_k(i, hlL, hlR, lhL, lhR, p2L, p2R);
    p1U_L = p1L; p1U_R = p1R; p2U_L = p2L; p2U_R = p2R; p2U_P = p2P;
    E = E1;
  };
  // the predicted values of a row only (the prologue row above the first)
  auto kpredict = [&](const V4<T>& O_, const V4<T>& E1) {
    T p0L, p0R;
    O::predict(E.x, E.z, E1.x, E1.z, E.y, E1.y, O_.x, O_.z, O_.y, p0L, p1U_L, p2U_L);
    O::predict(E.z, from_next(E.x), E1.z, from_next(E1.x), E.w, E1.w, O_.z, from_next(O_.x), O_.w, p0R, p1U_R,
               p2U_R);
    p2U_P = from_prev(p2U_R);
    E = E1;
  };

  // ---- level k+1 on LL_k rows: X' quadruple (xa, xb / xc, xd) per lane
  const int W1 = it.ns_w, H1 = it.ns_h;
  // right edge of LL_k (EDGE items): the lane whose right neighbour column
  // 2Q+2 is W1 (W1 even) reuses its own column 2Q; the lane whose column
  // 2Q+1 is W1 (W1 odd) takes columns W1-2, W1-3 from its left neighbour
  const bool rx_even = EDGE && 2 * it.Q + 2 == W1;
  const bool rx_odd = EDGE && 2 * it.Q + 1 == W1;
  T q1U, q2U, q2UP;  // predicted c', d' of the level-(k+1) row above (P: left neighbour)
  auto k1predict = [&](T xa, T xb, T xc, T xd, T xaD, T xbD, T& q0, T& q1, T& q2) {
    T aR = from_next(xa), aDR = from_next(xaD), cR = from_next(xc);
    if constexpr (EDGE) {
      const T pa = from_prev(xa), pb = from_prev(xb), pc = from_prev(xc), pd = from_prev(xd);
      const T paD = from_prev(xaD), pbD = from_prev(xbD);
      aR = rx_even ? xa : (rx_odd ? pa : aR);
      aDR = rx_even ? xaD : (rx_odd ? paD : aDR);
      cR = rx_even ? xc : (rx_odd ? pc : cR);
      xb = rx_odd ? pb : xb;
      xbD = rx_odd ? pbD : xbD;
      xd = rx_odd ? pd : xd;
    }
    O::predict(xa, aR, xaD, aDR, xb, xbD, xc, cR, xd, q0, q1, q2);
  };
  // X' rows held: the even row 2p (ea, eb), the odd row 2p+1 (oc, od), and
  // the pair before (pea, peb, poc, pod) for the bottom fold of odd H1
  T ea, eb, oc, od, pea, peb, poc, pod;

  struct Buf {
    V4<T> v[CP][4];
  };
  auto load_chunk = [&](Buf& b, int p0) {
#pragma unroll
    for (int m = 0; m < CP; ++m)
#pragma unroll
      for (int k = 0; k < 4; ++k) L.load(4 * (p0 + m) + 3 + k, b.v[m][k]);
  };
  Buf A, B;

  // ---- prologue: level-k rows 2 J0 - 3 (predicted only) .. 2 J0, level-(k+1)
  // predicted row J0 - 1.  The first chunk's loads go out right after the
  // prologue's, before its arithmetic: a work item waits for memory once
  // before its first pair, not twice.
  const int r0 = 4 * it.J0 - 6;  // first pixel row read
  {
    V4<T> v[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) L.load(r0 + k, v[k]);
    load_chunk(A, it.J0);
    E = v[0];
    kpredict(v[1], v[2]);
    T l0, r0_, l1, r1, l2, r2;
    krow(2 * it.J0 - 2, v[3], v[4], l0, r0_);
    krow(2 * it.J0 - 1, v[5], v[6], l1, r1);
    krow(2 * it.J0, v[7], v[8], l2, r2);
    T q0;
    k1predict(l0, r0_, l1, r1, l2, r2, q0, q1U, q2U);
    q2UP = from_prev(q2U);
    pea = l0; peb = r0_; poc = l1; pod = r1;
    ea = l2; eb = r2;
    oc = l1; od = r1;  // replaced before use
  }
  direct_k = false;

  // ---- pairs p = J0 .. J1-1: level-k rows 2p+1, 2p+2; level-(k+1) row p
  auto pair = [&](const Buf& b, int m, int p) {
    T xc, xd, xaD, xbD;
    krow(2 * p + 1, b.v[m][0], b.v[m][1], xc, xd);
    krow(2 * p + 2, b.v[m][2], b.v[m][3], xaD, xbD);
    // bottom of LL_k: row 2p+2 == H1 (H1 even) mirrors to row 2p; rows
    // 2p+1 == H1 and 2p+2 (H1 odd) mirror to rows 2p-1 and 2p-2
    const bool vD = 2 * p + 2 == H1, vO = 2 * p + 1 == H1;
    const T uc = vO ? poc : xc, ud = vO ? pod : xd;
    const T uaD = vD ? ea : (vO ? pea : xaD), ubD = vD ? eb : (vO ? peb : xbD);
    T q0, q1, q2;
    k1predict(ea, eb, uc, ud, uaD, ubD, q0, q1, q2);
    const T q0P = from_prev(q0), q2P = from_prev(q2);
    T ll, hl, lh;
    O::update(ea, q0P, q0, q1U, q1, q2UP, q2U, q2P, q2, ll, hl, lh);
    store_k1(p, ll, hl, lh, q2);
    q1U = q1; q2U = q2; q2UP = q2P;
    pea = ea; peb = eb; poc = xc; pod = xd;
    ea = xaD; eb = xbD;
  };
  run_rows<CP>(it.J0, it.J1, A, B, load_chunk, pair);
}

// ---------------------------------------------------------------------------
// Band loads of one level (inverse and adjoint): per lane, one element (level
// k+1) or two (level k, an 8-byte load) of a band row.  MIRROR (inverse):
// rows and columns go through the symmetric extension of the interleaved
// coefficient array, so every load is in range; otherwise (adjoint) values
// outside a band read as zero (row: a size-0 resource; column: the range
// check).  Columns of EDGE lanes are folded per element.
// ---------------------------------------------------------------------------
template <typename T, bool MIRROR, bool EDGE, int N>  // N: elements per lane (1 or 2)
struct PairBands {
  const T* band;   // packed array origin
  const T* ll;     // LL of this level (k+1: LL_{k+1}; unused at level k)
  int64_t bs, ls;
  int W, H, ns_w, nd_w, ns_h, nd_h;
  int q;           // the lane's first quadruple column (raw)
  int cl[N], ch[N];  // EDGE: folded (MIRROR) columns of the L and H parity
  __device__ __forceinline__ int erow(int r) const { return MIRROR ? (fold_idx(2 * r, H) >> 1) : r; }
  __device__ __forceinline__ int orow(int r) const { return MIRROR ? ((fold_idx(2 * r + 1, H) - 1) >> 1) : r; }
  __device__ __forceinline__ void ld(const T* row, bool valid, int width, bool hpar, T* v) const {
    const Rsrc rs = row_rsrc(row, (MIRROR || valid) ? width * 4 : 0);
    if constexpr (N == 1) {
      v[0] = bld1<T, kLdPol>(rs, EDGE ? (hpar ? ch[0] : cl[0]) : q);
    } else if constexpr (EDGE) {
      v[0] = bld1<T, kLdPol>(rs, hpar ? ch[0] : cl[0]);
      v[1] = bld1<T, kLdPol>(rs, hpar ? ch[1] : cl[1]);
    } else {
      bld2<kLdPol>(rs, q, v[0], v[1]);
    }
  }
  // row r of LL (level k+1 only) and HL
  __device__ __forceinline__ void even(int r, T* vll, T* vhl) const {
    const int re = erow(r);
    const bool valid = r >= 0 && r < ns_h;
    if (vll) ld(ll + (int64_t)re * ls, valid, ns_w, false, vll);
    ld(band + (int64_t)re * bs + ns_w, valid, nd_w, true, vhl);
  }
  // row r of LH and HH
  __device__ __forceinline__ void odd(int r, T* vlh, T* vhh) const {
    const int ro = orow(r);
    const bool valid = r >= 0 && r < nd_h;
    const T* row = band + (int64_t)(ns_h + ro) * bs;
    ld(row, valid, ns_w, false, vlh);
    ld(row + ns_w, valid, nd_w, true, vhh);
  }
};

template <typename T, bool MIRROR, bool EDGE, int N>
__device__ __forceinline__ PairBands<T, MIRROR, EDGE, N> pair_bands(const T* band, int64_t bs, const T* ll, int64_t ls,
                                                                    int W, int H, int q) {
  PairBands<T, MIRROR, EDGE, N> B;
  B.band = band; B.bs = bs; B.ll = ll; B.ls = ls;
  B.W = W; B.H = H;
  B.ns_w = (W + 1) >> 1; B.nd_w = W >> 1; B.ns_h = (H + 1) >> 1; B.nd_h = H >> 1;
  B.q = q;
  for (int k = 0; k < N; ++k) {
    B.cl[k] = MIRROR ? band_idx(q + k, W, 0) : q + k;
    B.ch[k] = MIRROR ? band_idx(q + k, W, 1) : q + k;
  }
  return B;
}

// Pixel-row stores of level k (inverse / adjoint): four pixels per lane,
// owned lanes only, rows [lo, hi).
template <typename T, int POL>
struct PairPxStore {
  T* base;
  int64_t stride;
  int W, c0, lo, hi;
  __device__ __forceinline__ void row(int r, const V4<T>& v) const {
    const Rsrc rs = row_rsrc(base + (int64_t)r * stride, (r >= lo && r < hi) ? W * 4 : 0);
    bst4<POL>(v, rs, c0);
  }
};

// ---------------------------------------------------------------------------
// Inverse pair: level k+1 (LL_{k+1} and its bands -> LL_k), then level k
// (LL_k and its bands -> pixels).
// ---------------------------------------------------------------------------
template <typename T, int CP, bool EDGE, int PPX>  // PPX: store policy of the output pixels
__device__ void inv_pair(const LevelDesc& d, const T* __restrict__ ll2, const T* __restrict__ band,
                         T* __restrict__ px, const PairItem& it) {
  using O = Ops<T>;
  const int W1 = it.ns_w, H1 = it.ns_h;
  const PairBands<T, true, EDGE, 1> B1 = pair_bands<T, true, EDGE, 1>(band, d.band_stride, ll2, d.ll_stride, W1, H1,
                                                                      it.Q);
  const PairBands<T, true, EDGE, 2> B0 = pair_bands<T, true, EDGE, 2>(band, d.band_stride, nullptr, 0, it.W, it.H,
                                                                      it.qL);
  const PairPxStore<T, PPX> S{px, d.pix_stride, it.W, it.own ? 2 * it.qL : kOff, 4 * it.J0, min(4 * it.J1, it.H)};

  // ---- level k+1: coefficient rows of LL', HL' (even) and LH', HH' (odd)
  T lhU1, hhU1;             // odd part of the row above
  T v0, v1, v2, hh1;        // undone update of the current row: (u0, u1, u2), and its HH'
  auto k1undo = [&](T ll, T hl, T lh, T hh, T& u0, T& u1, T& u2) {
    O::inv_update(ll, from_prev(hl), hl, lhU1, lh, from_prev(hhU1), hhU1, from_prev(hh), hh, u0, u1, u2);
    lhU1 = lh;
    hhU1 = hh;
  };
  // ---- level k: LL_k from level k+1, bands from memory
  T lhU_L, lhU_R, hhU_L, hhU_R;               // odd part of the row above
  T a_L, a_R, b_L, b_R, c_L, c_R, hh_L, hh_R;  // undone update of the previous row and its HH
  // right edge: LL_k columns past W1 take the level-k extension of the
  // interleaved array, not level k+1's (see the file comment)
  const int W = it.W;
  const bool lx_virt = EDGE && it.qL == W1, rx_virt = EDGE && it.qL + 1 == W1;
  auto fix_ll = [&](T& lL, T& lR) {
    if constexpr (EDGE) {
      const T pL = from_prev(lL), pR = from_prev(lR);
      const bool weven = (W & 1) == 0;
      // column W1 is band_idx(W1, W, 0): W1 - 1 (W even) or W1 - 2 (W odd)
      const T vL = weven ? pR : pL;        // lane whose L quadruple is W1
      const T vR = weven ? lL : pR;        // lane whose R quadruple is W1
      lL = lx_virt ? vL : lL;
      lR = rx_virt ? vR : lR;
    }
  };
  // undo the update of level-k row i (LL_k values lL, lR), then undo the
  // predict of row i - 1 and store its two pixel rows
  auto krow = [&](int i, T lL, T lR, const T* hl, const T* lh, const T* hh) {
    fix_ll(lL, lR);
    T u0L, u1L, u2L, u0R, u1R, u2R;
    const T hlP = from_prev(hl[1]), hhP = from_prev(hh[1]), hhUP = from_prev(hhU_R);
    O::inv_update(lL, hlP, hl[0], lhU_L, lh[0], hhUP, hhU_L, hhP, hh[0], u0L, u1L, u2L);
    O::inv_update(lR, hl[0], hl[1], lhU_R, lh[1], hhU_L, hhU_R, hh[0], hh[1], u0R, u1R, u2R);
    V4<T> e, o;
    e.x = a_L;
    e.z = a_R;
    O::inv_predict(a_L, a_R, u0L, u0R, b_L, u1L, c_L, c_R, hh_L, e.y, o.x, o.y);
    O::inv_predict(a_R, from_next(a_L), u0R, from_next(u0L), b_R, u1R, c_R, from_next(c_L), hh_R, e.w, o.z, o.w);
    S.row(2 * i - 2, e);
    S.row(2 * i - 1, o);
    lhU_L = lh[0]; lhU_R = lh[1]; hhU_L = hh[0]; hhU_R = hh[1];
    a_L = u0L; a_R = u0R; b_L = u1L; b_R = u1R; c_L = u2L; c_R = u2R; hh_L = hh[0]; hh_R = hh[1];
  };
  // LL_k rows held for the bottom substitution: the level-k walk reads LL_k
  // row H1 (virtual) as row H1 - 1 (H even) or H1 - 2 (H odd)
  T xa_p, xb_p, xc_p, xd_p;  // LL_k rows 2p - 2 (xa, xb) and 2p - 1 (xc, xd)

  // chunks of the pair loop (below)
  struct Buf {
    T ll1[CP], hl1[CP], lh1[CP], hh1[CP];
    T hl[CP][2][2], lh[CP][2][2], hh[CP][2][2];
  };
  auto load_chunk = [&](Buf& b, int p0) {
#pragma unroll
    for (int m = 0; m < CP; ++m) {
      const int p = p0 + m;
      B1.even(p + 1, &b.ll1[m], &b.hl1[m]);
      B1.odd(p + 1, &b.lh1[m], &b.hh1[m]);
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        B0.even(2 * p + r, nullptr, b.hl[m][r]);
        B0.odd(2 * p + r, b.lh[m][r], b.hh[m][r]);
      }
    }
  };
  Buf A, Bb;

  // ---- prologue: level-(k+1) odd part of row J0 - 1 and undone update of
  // row J0; level-k odd part of row 2 J0 - 1.  The first chunk's loads go
  // out right after the prologue's, before its arithmetic.
  {
    T lh0, hh0, ll1, hl1, lh1, hh1_;
    B1.odd(it.J0 - 1, &lh0, &hh0);
    B1.even(it.J0, &ll1, &hl1);
    B1.odd(it.J0, &lh1, &hh1_);
    T lh[2], hh[2];
    B0.odd(2 * it.J0 - 1, lh, hh);
    load_chunk(A, it.J0);
    lhU1 = lh0;
    hhU1 = hh0;
    k1undo(ll1, hl1, lh1, hh1_, v0, v1, v2);
    hh1 = hh1_;
    lhU_L = lh[0]; lhU_R = lh[1]; hhU_L = hh[0]; hhU_R = hh[1];
    a_L = a_R = b_L = b_R = c_L = c_R = hh_L = hh_R = T(0);  // row 2 J0 - 1: not stored
    xa_p = xb_p = xc_p = xd_p = T(0);
  }

  // ---- pairs p = J0 .. J1: level-(k+1) row p+1 undone, row p reconstructed
  // (LL_k rows 2p, 2p+1); level-k rows 2p and 2p+1 undone, rows 2p-1 and 2p
  // reconstructed (pixel rows 4p-2 .. 4p+1)
  auto pair = [&](const Buf& b, int m, int p) {
    T n0, n1, n2;
    k1undo(b.ll1[m], b.hl1[m], b.lh1[m], b.hh1[m], n0, n1, n2);
    T xb, xc, xd;
    O::inv_predict(v0, from_next(v0), n0, from_next(n0), v1, n1, v2, from_next(v2), hh1, xb, xc, xd);
    const T xa = v0;
    v0 = n0; v1 = n1; v2 = n2; hh1 = b.hh1[m];
    // virtual LL_k rows: 2p == H1 or 2p + 1 == H1
    const bool weven = (it.H & 1) == 0;
    const bool vE = 2 * p == H1, vO = 2 * p + 1 == H1;
    // row H1 - 1 is 2p - 1 (vE) or 2p (vO); row H1 - 2 is 2p - 2 (vE) or 2p - 1 (vO)
    const T ea = vE ? (weven ? xc_p : xa_p) : xa, eb = vE ? (weven ? xd_p : xb_p) : xb;
    const T oc = vO ? (weven ? xa : xc_p) : xc, od = vO ? (weven ? xb : xd_p) : xd;
    krow(2 * p, ea, eb, b.hl[m][0], b.lh[m][0], b.hh[m][0]);
    krow(2 * p + 1, oc, od, b.hl[m][1], b.lh[m][1], b.hh[m][1]);
    xa_p = ea; xb_p = eb; xc_p = oc; xd_p = od;
  };
  run_rows<CP>(it.J0, it.J1 + 1, A, Bb, load_chunk, pair);
}

// ---------------------------------------------------------------------------
// Adjoint pair: W^T of levels k+1 then k (float).  Coefficient gradients
// outside their bands are zero, and the transposed boundary weights of each
// axis carry the edges (as in the single-level kernel); the LL_k gradient
// the first level hands to the second is zero outside LL_k.
// ---------------------------------------------------------------------------
template <int CP, bool EDGE, int PPX>
__device__ void bwd_pair(const LevelDesc& d, const float* __restrict__ ll2, const float* __restrict__ band,
                         float* __restrict__ px, const PairItem& it) {
  const int W1 = it.ns_w, H1 = it.ns_h;
  const PairBands<float, false, EDGE, 1> B1 =
      pair_bands<float, false, EDGE, 1>(band, d.band_stride, ll2, d.ll_stride, W1, H1, it.Q);
  const PairBands<float, false, EDGE, 2> B0 =
      pair_bands<float, false, EDGE, 2>(band, d.band_stride, nullptr, 0, it.W, it.H, it.qL);
  const PairPxStore<float, PPX> S{px, d.pix_stride, it.W, it.own ? 2 * it.qL : kOff, 4 * it.J0,
                                  min(4 * it.J1, it.H)};
  // horizontal weights; all lanes away from the left and right borders:
  // plain sums (bit-identical, see wsum)
  const AxisW h1 = axis_weights(it.Q, W1);
  const AxisW hL = axis_weights(it.qL, it.W), hR = axis_weights(it.qL + 1, it.W);
  const bool unit_h1 = __all(unit_weights(h1));
  const bool unit_h = __all(unit_weights(hL) && unit_weights(hR));
  // LL_k gradient columns inside LL_k (else zero)
  const bool colL_in = it.qL >= 0 && it.qL < W1, colR_in = it.qL + 1 >= 0 && it.qL + 1 < W1;

  // ---- level k+1: step A (transposed update) of row J needs rows J, J+1
  float ga1, gb1, gc1, gd1;      // coefficients of the current row J
  float sc1U, sd1U, sd1UP;        // step A of the row above (P: left neighbour)
  float sb1, sc1, sd1;           // step A of the current row
  auto k1stepA = [&](int j, float gaN, float gbN) {
    const AxisW v = axis_weights(j, H1);
    const float gaR = from_next(ga1), gaDR = from_next(gaN), gcR = from_next(gc1);
    if (unit_h1 && unit_weights(v)) f32_adj_a<true>(ga1, gaR, gaN, gaDR, gb1, gbN, gc1, gcR, gd1, h1, v, sb1, sc1, sd1);
    else f32_adj_a(ga1, gaR, gaN, gaDR, gb1, gbN, gc1, gcR, gd1, h1, v, sb1, sc1, sd1);
  };
  // step B of row J: the LL_k gradient rows 2J (xa, xb) and 2J+1 (xc, xd)
  auto k1stepB = [&](int j, float& xa, float& xb, float& xc, float& xd) {
    const AxisW v = axis_weights(j, H1);
    const float sbP = from_prev(sb1), sdP = from_prev(sd1);
    if (unit_h1 && unit_weights(v)) f32_adj_b<true>(ga1, sbP, sb1, sc1U, sc1, sd1UP, sd1U, sdP, sd1, h1, v, xa, xb, xc);
    else f32_adj_b(ga1, sbP, sb1, sc1U, sc1, sd1UP, sd1U, sdP, sd1, h1, v, xa, xb, xc);
    xd = sd1;
    sc1U = sc1; sd1U = sd1; sd1UP = sdP;
    // zero outside LL_k
    const bool rE = 2 * j >= 0 && 2 * j < H1, rO = 2 * j + 1 >= 0 && 2 * j + 1 < H1;
    xa = (rE && colL_in) ? xa : 0.f;
    xb = (rE && colR_in) ? xb : 0.f;
    xc = (rO && colL_in) ? xc : 0.f;
    xd = (rO && colR_in) ? xd : 0.f;
  };

  // ---- level k: step A of row i needs LL_k-gradient rows i, i+1
  float ka_L, ka_R, kb_L, kb_R, kc_L, kc_R, kd_L, kd_R;  // row i (LL_k grad and bands)
  float tc_UL, tc_UR, td_UL, td_UR, td_UP;               // step A of the row above
  auto krow = [&](int i, float naL, float naR, const float* nb, const float* nc, const float* nd) {
    const AxisW v = axis_weights(i, it.H);
    const bool unit = unit_h && unit_weights(v);
    float sbL, scL, sdL, sbR, scR, sdR;
    const float gaN = from_next(ka_L), gaDN = from_next(naL), gcN = from_next(kc_L);
    if (unit) {
      f32_adj_a<true>(ka_L, ka_R, naL, naR, kb_L, nb[0], kc_L, kc_R, kd_L, hL, v, sbL, scL, sdL);
      f32_adj_a<true>(ka_R, gaN, naR, gaDN, kb_R, nb[1], kc_R, gcN, kd_R, hR, v, sbR, scR, sdR);
    } else {
      f32_adj_a(ka_L, ka_R, naL, naR, kb_L, nb[0], kc_L, kc_R, kd_L, hL, v, sbL, scL, sdL);
      f32_adj_a(ka_R, gaN, naR, gaDN, kb_R, nb[1], kc_R, gcN, kd_R, hR, v, sbR, scR, sdR);
    }
    const float sbP = from_prev(sbR), sdP = from_prev(sdR);
    V4<float> e, o;
    if (unit) {
      f32_adj_b<true>(ka_L, sbP, sbL, tc_UL, scL, td_UP, td_UL, sdP, sdL, hL, v, e.x, e.y, o.x);
      f32_adj_b<true>(ka_R, sbL, sbR, tc_UR, scR, td_UL, td_UR, sdL, sdR, hR, v, e.z, e.w, o.z);
    } else {
      f32_adj_b(ka_L, sbP, sbL, tc_UL, scL, td_UP, td_UL, sdP, sdL, hL, v, e.x, e.y, o.x);
      f32_adj_b(ka_R, sbL, sbR, tc_UR, scR, td_UL, td_UR, sdL, sdR, hR, v, e.z, e.w, o.z);
    }
    o.y = sdL;
    o.w = sdR;
    S.row(2 * i, e);
    S.row(2 * i + 1, o);
    tc_UL = scL; tc_UR = scR; td_UL = sdL; td_UR = sdR; td_UP = sdP;
    ka_L = naL; ka_R = naR; kb_L = nb[0]; kb_R = nb[1]; kc_L = nc[0]; kc_R = nc[1]; kd_L = nd[0]; kd_R = nd[1];
  };

  // chunks of the pair loop (below)
  struct Buf {
    float a1[CP], b1[CP], c1[CP], d1[CP];
    float hb[CP][2][2], hc[CP][2][2], hd[CP][2][2];
  };
  auto load_chunk = [&](Buf& b, int p0) {
#pragma unroll
    for (int m = 0; m < CP; ++m) {
      const int p = p0 + m;
      B1.even(p + 1, &b.a1[m], &b.b1[m]);
      B1.odd(p + 1, &b.c1[m], &b.d1[m]);
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        B0.even(2 * p + r, nullptr, b.hb[m][r]);
        B0.odd(2 * p + r, b.hc[m][r], b.hd[m][r]);
      }
    }
  };
  Buf A, Bb;

  // ---- prologue: level-(k+1) rows J0 - 2 .. J0 loaded, step A of J0 - 2
  // and J0 - 1, step B of J0 - 1 (LL_k-gradient rows 2 J0 - 2, 2 J0 - 1);
  // level-k row 2 J0 - 1 current, its step A needs LL_k-gradient row 2 J0.
  // The first chunk's loads go out right after the prologue's, before its
  // arithmetic.
  {
    float a0, b0, c0, d0, a1, b1_, c1, d1, a2, b2, c2, d2;
    B1.even(it.J0 - 2, &a0, &b0);
    B1.odd(it.J0 - 2, &c0, &d0);
    B1.even(it.J0 - 1, &a1, &b1_);
    B1.odd(it.J0 - 1, &c1, &d1);
    B1.even(it.J0, &a2, &b2);
    B1.odd(it.J0, &c2, &d2);
    float hb[2], hc[2], hd[2];
    B0.even(2 * it.J0 - 1, nullptr, hb);
    B0.odd(2 * it.J0 - 1, hc, hd);
    load_chunk(A, it.J0);
    ga1 = a0; gb1 = b0; gc1 = c0; gd1 = d0;
    k1stepA(it.J0 - 2, a1, b1_);
    sc1U = sc1; sd1U = sd1; sd1UP = from_prev(sd1);
    ga1 = a1; gb1 = b1_; gc1 = c1; gd1 = d1;
    k1stepA(it.J0 - 1, a2, b2);
    float xa, xb, xc, xd;
    k1stepB(it.J0 - 1, xa, xb, xc, xd);
    ga1 = a2; gb1 = b2; gc1 = c2; gd1 = d2;
    // level k: row 2 J0 - 1 (LL_k gradient xc, xd) is the current row
    ka_L = xc; ka_R = xd; kb_L = hb[0]; kb_R = hb[1]; kc_L = hc[0]; kc_R = hc[1]; kd_L = hd[0]; kd_R = hd[1];
    tc_UL = tc_UR = td_UL = td_UR = td_UP = 0.f;  // row 2 J0 - 2: its outputs are not stored
  }

  // ---- pairs p = J0 .. J1: level-(k+1) step A of row p (needs row p+1),
  // step B of row p (LL_k-gradient rows 2p, 2p+1); level-k rows 2p - 1 and
  // 2p (pixel rows 4p - 2 .. 4p + 1)
  auto pair = [&](const Buf& b, int m, int p) {
    k1stepA(p, b.a1[m], b.b1[m]);
    float xa, xb, xc, xd;
    k1stepB(p, xa, xb, xc, xd);
    ga1 = b.a1[m]; gb1 = b.b1[m]; gc1 = b.c1[m]; gd1 = b.d1[m];
    krow(2 * p - 1, xa, xb, b.hb[m][0], b.hc[m][0], b.hd[m][0]);
    krow(2 * p, xc, xd, b.hb[m][1], b.hc[m][1], b.hd[m][1]);
  };
  run_rows<CP>(it.J0, it.J1 + 1, A, Bb, load_chunk, pair);
}

// ---------------------------------------------------------------------------
// Pair kernel: one wave per work item (image, segment, strip) of a pair of
// levels; the descriptor's W, H are level k's input, seg counts level-(k+1)
// quadruple rows, ll is LL_{k+1} (output of the forward, input of the
// inverse and adjoint).
// ---------------------------------------------------------------------------
// One work item of a pair launch: strip `strip` of segment `seg`, with the
// image's element offsets from the descriptor's pointers.  STAGE_OK: the
// launch may stage the forward's stores (d.stage; four adjacent strips per
// workgroup, `stage` the workgroup's LDS array); otherwise d.stage is 0.
template <int DIR, typename T, int CP, bool STAGE_OK>
__device__ __forceinline__ void pair_run(const LevelDesc& d, int64_t pix_off, int64_t ll_off, int64_t band_off,
                                         int strip, int seg, int lane, T* stage) {
  const PairItem it = make_pair_item<DIR>(d, strip, seg, lane);
  const bool edge = pair_edge<DIR>(it, strip);
  if constexpr (DIR == kFwd) {
    const T* px = static_cast<const T*>(d.pix_in) + pix_off;
    T* ll2 = static_cast<T*>(d.ll_out) + ll_off;
    T* band = static_cast<T*>(d.band_out) + band_off;
    if constexpr (STAGE_OK) {
      if (d.stage) {
        if (edge) fwd_pair<T, CP, true, true>(d, px, ll2, band, it, stage);
        else fwd_pair<T, CP, false, true>(d, px, ll2, band, it, stage);
        return;
      }
    }
    if (edge) fwd_pair<T, CP, true, false>(d, px, ll2, band, it, stage);
    else fwd_pair<T, CP, false, false>(d, px, ll2, band, it, stage);
  } else {
    const T* ll2 = static_cast<const T*>(d.ll_in) + ll_off;
    const T* band = static_cast<const T*>(d.band_in) + band_off;
    T* px = static_cast<T*>(d.pix_out) + pix_off;
    if constexpr (DIR == kInv) {
      if (d.keep_out) {
        if (edge) inv_pair<T, CP, true, 0>(d, ll2, band, px, it);
        else inv_pair<T, CP, false, 0>(d, ll2, band, px, it);
      } else {
        if (edge) inv_pair<T, CP, true, kNT>(d, ll2, band, px, it);
        else inv_pair<T, CP, false, kNT>(d, ll2, band, px, it);
      }
    } else {
      if (d.keep_out) bwd_pair<CP, false, 0>(d, ll2, band, px, it);
      else bwd_pair<CP, false, kNT>(d, ll2, band, px, it);
    }
  }
}

template <int DIR, typename T, int CP>
__global__ __launch_bounds__(kBlock) void pair_kernel(LevelLaunch a) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int64_t item = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * kWavesPerBlock + wave;
  if (item >= a.items) return;
  const int img = (int)(item / a.items_per_image);
  const int rem = (int)(item - (int64_t)img * a.items_per_image);
  const int seg = rem / a.d.nstrips;
  const int strip = rem - seg * a.d.nstrips;
  T* stage = nullptr;
  if constexpr (DIR == kFwd) {
    __shared__ T stage_lds[2 * kPairStageBuf];
    stage = stage_lds;
  }
  pair_run<DIR, T, CP, true>(a.d, img * a.pix_bstride, img * a.ll_bstride, img * a.band_bstride, strip, seg, lane,
                             stage);
}

// One pair step of a ragged batch (level-synchronous schedule): one wave per
// work item, the item's image descriptor found through the device item ->
// descriptor table, as in table_kernel.  The descriptors never stage.
template <int DIR, typename T, int CP>
__global__ __launch_bounds__(kBlock) void pair_table_kernel(TableArgs a) {
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
  pair_run<DIR, T, CP, false>(jd.d, img * jd.pix_bstride, img * jd.ll_bstride, img * jd.band_bstride, strip, seg,
                              lane, (T*)nullptr);
}

template <int DIR, typename T>
hipError_t launch_pair_t(int chunk, const LevelLaunch& a, hipStream_t s) {
  const dim3 grid((unsigned)((a.items + kWavesPerBlock - 1) / kWavesPerBlock));
  if (chunk >= 2) hipLaunchKernelGGL((pair_kernel<DIR, T, 2>), grid, dim3(kBlock), 0, s, a);
  else hipLaunchKernelGGL((pair_kernel<DIR, T, 1>), grid, dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

}  // namespace

// Launches one pair of levels (declared in dwt2_internal.h); each
// fused_*.hip instantiates it for its direction.
template <int DIR>
int launch_pair_dir(int mode, int chunk, const LevelLaunch& a, void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (a.items <= 0) return hipSuccess;
  if (mode == DWT2_F32) return launch_pair_t<DIR, float>(chunk, a, s);
  if constexpr (DIR != kBwd) return launch_pair_t<DIR, int>(chunk, a, s);
  return hipErrorInvalidValue;
}

template <int DIR, typename T>
hipError_t launch_pair_table_t(const TableArgs& a, hipStream_t s) {
  const dim3 grid((unsigned)((a.items + kWavesPerBlock - 1) / kWavesPerBlock));
  hipLaunchKernelGGL((pair_table_kernel<DIR, T, 1>), grid, dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

template <int DIR>
int launch_pair_table_dir(int mode, const TableArgs& a, void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (a.items <= 0) return hipSuccess;
  if (mode == DWT2_F32) return launch_pair_table_t<DIR, float>(a, s);
  if constexpr (DIR != kBwd) return launch_pair_table_t<DIR, int>(a, s);
  return hipErrorInvalidValue;
}

#define DWT2_INSTANTIATE_PAIR(DIR)                                                 \
  template int launch_pair_dir<DIR>(int, int, const LevelLaunch&, void*);         \
  template int launch_pair_table_dir<DIR>(int, const TableArgs&, void*);

}  // namespace dwt2
