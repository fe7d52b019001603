// CDF 9/7 (float32) with the non-separable lifting scheme, one launch per
// level.  The wavelet's two lifting pairs (§2, eq. (2)) are treated in turn,
// each as one spatial predict and one spatial update (§3, eq. (5)), so a
// level is four spatial steps followed by the scaling of the quadrants.
// Coefficients: the Daubechies-Sweldens lifting factorisation, normalised as
// JPEG 2000's irreversible transform (lowpass gain 1 at DC, highpass gain 2
// at Nyquist), so that the quadrants scale as LL / K^2, HL and LH by 1,
// HH * K^2.
//
// Each 256-thread workgroup owns 64 x 16 output quadruples.  It copies them
// into LDS with two quadruples of halo on every side, split into the planes
// a, b, c, d (even/odd row x even/odd column).  Each step reaches one
// quadruple to one side, so four steps need two on each side.  The copy
// reads through the symmetric extension: of the pixels (forward), or of the
// interleaved coefficients (inverse).  The extension keeps every index's
// parity, so it commutes with lifting, and each step can run on a fixed
// local range that shrinks by one quadruple per step.  The steps ping-pong
// b and c between two sets of planes, with a workgroup barrier between
// steps, so that no step overwrites a value another thread of the same step
// still reads.  d needs one plane: a predict step reads it only at its own
// quadruple.  Six planes (32640 bytes) leave room for five workgroups per CU.
#include <hip/hip_runtime.h>

#include "fused.h"

namespace dwt2 {
namespace {

constexpr float kAlpha = -1.586134342059924f, kBeta = -0.052980118572961f;
constexpr float kGamma = 0.882911075530934f, kDelta = 0.443506852043971f;
constexpr double kK = 1.230174104914001;
constexpr float kAlpha2 = (float)(-1.586134342059924 * -1.586134342059924);
constexpr float kBeta2 = (float)(-0.052980118572961 * -0.052980118572961);
constexpr float kGamma2 = (float)(0.882911075530934 * 0.882911075530934);
constexpr float kDelta2 = (float)(0.443506852043971 * 0.443506852043971);
constexpr float kLLScale = (float)(1.0 / (kK * kK)), kHHScale = (float)(kK * kK);

constexpr int kQX = 64, kQY = 16;                    // output quadruples per tile
constexpr int kNX = kQX + 4, kNY = kQY + 4, kNP = kNX * kNY;
constexpr int kBlk = 256, kWv = kBlk / kWave;

// Whole-sample symmetric fold of p onto [0, n), n >= 2.
__device__ __forceinline__ int fold97(int p, int n) {
  if ((unsigned)p < (unsigned)n) return p;
  const int m = 2 * (n - 1);
  p %= m;
  if (p < 0) p += m;
  return p >= n ? m - p : p;
}

// Consecutive logical tiles on one XCD (workgroups are dealt round-robin
// over the 8 XCDs), so vertically adjacent tiles share halo rows in one L2.
__device__ __forceinline__ int tile_remap(int b, int nb) {
  const int q = nb >> 3, r = nb & 7, x = b & 7, s = b >> 3;
  return (x < r) ? x * (q + 1) + s : r * (q + 1) + (x - r) * q + s;
}

// f(i, q) for rows i in [i0, i1) and quadruple columns q in
// [q0, q0 + 64 + EXTRA): one wave per row for the first 64 columns, then
// the EXTRA last columns of every row in one pass of the block.
template <int EXTRA, typename F>
__device__ __forceinline__ void walk(int i0, int i1, int q0, int lane, int wv, F&& f) {
  for (int i = i0 + wv; i < i1; i += kWv) f(i, q0 + lane);
  if constexpr (EXTRA > 0) {
    const int t = threadIdx.x;
    if (t < EXTRA * (i1 - i0)) f(i0 + t / EXTRA, q0 + kWave + t % EXTRA);
  }
}

// Spatial predict with P = p (1 + z): R / D = next quadruple column / row.
__device__ __forceinline__ void sp_pred(float p, float pp, float a, float aR, float aD, float aDR, float b, float bD,
                                        float c, float cR, float d, float& bo, float& co, float& dout) {
  const float sh = a + aR;
  bo = __fmaf_rn(p, sh, b);
  co = __fmaf_rn(p, a + aD, c);
  dout = __fmaf_rn(pp, sh + (aD + aDR), __fmaf_rn(p, b + bD, __fmaf_rn(p, c + cR, d)));
}

// Spatial update with U = u (1 + z^-1): L / U = previous column / row.
__device__ __forceinline__ void sp_upd(float u, float uu, float a, float bL, float b, float cU, float c, float dUL,
                                       float dU, float dL, float d, float& ao, float& bo, float& co) {
  bo = __fmaf_rn(u, dU + d, b);
  co = __fmaf_rn(u, dL + d, c);
  ao = __fmaf_rn(uu, (dUL + dU) + (dL + d), __fmaf_rn(u, cU + c, __fmaf_rn(u, bL + b, a)));
}

// Inverse of sp_upd, solved so that it reads only the step's outputs.
__device__ __forceinline__ void sp_inv_upd(float u, float uu, float ll, float hlL, float hl, float lhU, float lh,
                                           float dUL, float dU, float dL, float d, float& a, float& b, float& c) {
  b = __fmaf_rn(-u, dU + d, hl);
  c = __fmaf_rn(-u, dL + d, lh);
  a = __fmaf_rn(uu, (dUL + dU) + (dL + d), __fmaf_rn(-u, (hlL + hl) + (lhU + lh), ll));
}

// Inverse of sp_pred, likewise.
__device__ __forceinline__ void sp_inv_pred(float p, float pp, float a, float aR, float aD, float aDR, float b1,
                                            float b1D, float c1, float c1R, float d1, float& b, float& c, float& d) {
  const float sh = a + aR;
  b = __fmaf_rn(-p, sh, b1);
  c = __fmaf_rn(-p, a + aD, c1);
  d = __fmaf_rn(pp, sh + (aD + aDR), __fmaf_rn(-p, b1 + b1D, __fmaf_rn(-p, c1 + c1R, d1)));
}

// Forward level: pixels in, LL_k and the three H bands out.
__global__ __launch_bounds__(kBlk, 5) void fwd97(Level97 a, int tiles_x) {
  __shared__ float S[6 * kNP];
  float* A0 = S;
  float* B0 = S + kNP;
  float* C0 = S + 2 * kNP;
  float* D0 = S + 3 * kNP;
  float* B1 = S + 4 * kNP;
  float* C1 = S + 5 * kNP;
  float* D1 = D0;  // d is read only at its own quadruple by the step that rewrites it
  // the wave index is uniform: as a scalar, row folds and row pointers are
  // scalar code, not per-lane branches
  const int lane = threadIdx.x & (kWave - 1), wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int tile = tile_remap(blockIdx.x, gridDim.x);
  const int ty = tile / tiles_x, tx = tile - ty * tiles_x;
  const int W = a.W, H = a.H;
  const int ns_w = (W + 1) >> 1, ns_h = (H + 1) >> 1, nd_w = W >> 1, nd_h = H >> 1;
  const int px0 = 2 * (tx * kQX - 2), py0 = 2 * (ty * kQY - 2);  // image pixel of local pixel (0, 0)
  // the tile's 2 kNX = 136 pixel columns: lane, 64 + lane, and 128 + lane % 8
  // (stored by lanes 0..7; the others reload one of those eight)
  static_assert(2 * kNX == 2 * kWave + 8, "tile width");
  const int gc0 = fold97(px0 + lane, W), gc1 = fold97(px0 + kWave + lane, W);
  const int gc2 = fold97(px0 + 2 * kWave + (lane & 7), W);
  // plane and quadruple column of those pixel columns (even columns: a / c)
  const int s0 = (lane & 1) * kNP + (lane >> 1);
  const int s1 = (lane & 1) * kNP + kWave / 2 + (lane >> 1);
  const int s2 = (lane & 1) * kNP + kWave + ((lane & 7) >> 1);
  constexpr int kRowsPerWave = 2 * kNY / kWv;
  static_assert(2 * kNY % kWv == 0, "tile height");
  const int gqx = tx * kQX + lane;
  for (int img = blockIdx.y; img < a.batch; img += gridDim.y) {
    const float* src = static_cast<const float*>(a.in) + img * a.in_bstride;
    float* ll = static_cast<float*>(a.ll) + img * a.ll_bstride;
    float* band = static_cast<float*>(a.out) + img * a.out_bstride;
    {
      float v0[kRowsPerWave], v1[kRowsPerWave], v2[kRowsPerWave];
#pragma unroll
      for (int k = 0; k < kRowsPerWave; ++k) {
        const float* row = src + (int64_t)fold97(py0 + wv + k * kWv, H) * a.in_stride;
        v0[k] = row[gc0];
        v1[k] = row[gc1];
        v2[k] = row[gc2];
      }
#pragma unroll
      for (int k = 0; k < kRowsPerWave; ++k) {
        const int r = wv + k * kWv;
        float* x = S + (r & 1) * 2 * kNP + (r >> 1) * kNX;  // odd rows: planes c, d
        x[s0] = v0[k];
        x[s1] = v1[k];
        if (lane < 8) x[s2] = v2[k];
      }
    }
    __syncthreads();
    // pair 1 predict (alpha): rows [0, kNY - 1), columns [0, kNX - 1)
    walk<3>(0, kNY - 1, 0, lane, wv, [&](int i, int q) {
      const int o = i * kNX + q;
      sp_pred(kAlpha, kAlpha2, A0[o], A0[o + 1], A0[o + kNX], A0[o + kNX + 1], B0[o], B0[o + kNX], C0[o],
              C0[o + 1], D0[o], B1[o], C1[o], D1[o]);
    });
    __syncthreads();
    // pair 1 update (beta): rows [1, kNY - 1), columns [1, kNX - 1)
    walk<2>(1, kNY - 1, 1, lane, wv, [&](int i, int q) {
      const int o = i * kNX + q;
      sp_upd(kBeta, kBeta2, A0[o], B1[o - 1], B1[o], C1[o - kNX], C1[o], D1[o - kNX - 1], D1[o - kNX], D1[o - 1],
             D1[o], A0[o], B0[o], C0[o]);
    });
    __syncthreads();
    // pair 2 predict (gamma): rows [1, kNY - 2), columns [1, kNX - 2)
    walk<1>(1, kNY - 2, 1, lane, wv, [&](int i, int q) {
      const int o = i * kNX + q;
      sp_pred(kGamma, kGamma2, A0[o], A0[o + 1], A0[o + kNX], A0[o + kNX + 1], B0[o], B0[o + kNX], C0[o],
              C0[o + 1], D1[o], B1[o], C1[o], D0[o]);
    });
    __syncthreads();
    // pair 2 update (delta) on the tile's own quadruples, scaling, store
#pragma unroll
    for (int k = 0; k < kQY / kWv; ++k) {
      const int i = 2 + wv + k * kWv;
      const int o = i * kNX + 2 + lane;
      float vll, vhl, vlh;
      sp_upd(kDelta, kDelta2, A0[o], B1[o - 1], B1[o], C1[o - kNX], C1[o], D0[o - kNX - 1], D0[o - kNX], D0[o - 1],
             D0[o], vll, vhl, vlh);
      const float vhh = D0[o] * kHHScale;
      vll *= kLLScale;
      const int gqy = ty * kQY + i - 2;
      // H bands (and a last level's LL) are final: streamed, so that they do
      // not evict the next tiles' inputs (8192^2, six levels: 188 -> 178 us)
      if (gqx < ns_w && gqy < ns_h) {
        float* pll = ll + (int64_t)gqy * a.ll_stride + gqx;
        if (a.final_out) __builtin_nontemporal_store(vll, pll);
        else *pll = vll;
        if (gqx < nd_w) __builtin_nontemporal_store(vhl, band + (int64_t)gqy * a.out_stride + ns_w + gqx);
        if (gqy < nd_h) {
          __builtin_nontemporal_store(vlh, band + (int64_t)(ns_h + gqy) * a.out_stride + gqx);
          if (gqx < nd_w) __builtin_nontemporal_store(vhh, band + (int64_t)(ns_h + gqy) * a.out_stride + ns_w + gqx);
        }
      }
    }
    if (img + (int)gridDim.y < a.batch) __syncthreads();  // S is reused for the next image
  }
}

// Inverse level: LL_k and the H bands in, the level input's pixels out.
__global__ __launch_bounds__(kBlk, 5) void inv97(Level97 a, int tiles_x) {
  __shared__ float S[6 * kNP];
  float* A0 = S;
  float* B0 = S + kNP;
  float* C0 = S + 2 * kNP;
  float* D0 = S + 3 * kNP;
  float* B1 = S + 4 * kNP;
  float* C1 = S + 5 * kNP;
  float* D1 = D0;  // d is read only at its own quadruple by the step that rewrites it
  // the wave index is uniform: as a scalar, row folds and row pointers are
  // scalar code, not per-lane branches
  const int lane = threadIdx.x & (kWave - 1), wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int tile = tile_remap(blockIdx.x, gridDim.x);
  const int ty = tile / tiles_x, tx = tile - ty * tiles_x;
  const int W = a.W, H = a.H;
  const int ns_w = (W + 1) >> 1, ns_h = (H + 1) >> 1;
  const int qx0 = tx * kQX - 2, qy0 = ty * kQY - 2;  // image quadruple of local quadruple (0, 0)
  const int gqx = tx * kQX + lane;
  // pixel pairs (even column, next column) are 8-byte aligned in every row
  // and image: store them as one float2
  const bool pairs = ((reinterpret_cast<uintptr_t>(a.out) | (uintptr_t)(a.out_stride << 2) |
                       (uintptr_t)(a.out_bstride << 2)) & 7) == 0;
  for (int img = blockIdx.y; img < a.batch; img += gridDim.y) {
    const float* lls = static_cast<const float*>(a.in) + img * a.in_bstride;
    const float* bands = static_cast<const float*>(a.bands) + img * a.bands_bstride;
    float* out = static_cast<float*>(a.out) + img * a.out_bstride;
    // coefficients of quadruples [0, kNX) x [0, kNY), through the symmetric
    // extension of the interleaved array: the L (even) and H (odd) positions
    // of a quadruple fold onto band indices of their own parity; the scaling
    // is undone as they are stored
    // (all of a wave's loads are issued before its first LDS store)
    {
      constexpr int kR = kNY / kWv;  // rows per wave in the first 64 columns
      static_assert(kNY % kWv == 0 && (kNX - kWave) * kNY <= kBlk, "inverse load mapping");
      float vll[kR + 1], vhl[kR + 1], vlh[kR + 1], vhh[kR + 1];
      int slot[kR + 1];
#pragma unroll
      for (int k = 0; k <= kR; ++k) {
        // k < kR: row wv + k kWv, column lane; k = kR: one of the last
        // kNX - 64 columns, for threads below (kNX - 64) kNY
        const bool extra = k == kR;
        const int t = threadIdx.x;
        const bool live = !extra || t < (kNX - kWave) * kNY;
        const int i = extra ? (live ? t / (kNX - kWave) : 0) : wv + k * kWv;
        const int q = extra ? kWave + t % (kNX - kWave) : lane;
        const int gx = qx0 + q, gy = qy0 + i;
        const int bx0 = fold97(2 * gx, W) >> 1, bx1 = (fold97(2 * gx + 1, W) - 1) >> 1;
        const int by0 = fold97(2 * gy, H) >> 1, by1 = (fold97(2 * gy + 1, H) - 1) >> 1;
        vll[k] = lls[(int64_t)by0 * a.in_stride + bx0];
        vhl[k] = bands[(int64_t)by0 * a.bands_stride + ns_w + bx1];
        vlh[k] = bands[(int64_t)(ns_h + by1) * a.bands_stride + bx0];
        vhh[k] = bands[(int64_t)(ns_h + by1) * a.bands_stride + ns_w + bx1];
        slot[k] = live ? i * kNX + q : -1;
      }
#pragma unroll
      for (int k = 0; k <= kR; ++k) {
        const int o = slot[k];
        if (o >= 0) {
          A0[o] = vll[k] * kHHScale;
          B0[o] = vhl[k];
          C0[o] = vlh[k];
          D0[o] = vhh[k] * kLLScale;
        }
      }
    }
    __syncthreads();
    // undo pair 2 update (delta): rows [1, kNY), columns [1, kNX)
    walk<3>(1, kNY, 1, lane, wv, [&](int i, int q) {
      const int o = i * kNX + q;
      sp_inv_upd(kDelta, kDelta2, A0[o], B0[o - 1], B0[o], C0[o - kNX], C0[o], D0[o - kNX - 1], D0[o - kNX],
                 D0[o - 1], D0[o], A0[o], B1[o], C1[o]);
    });
    __syncthreads();
    // undo pair 2 predict (gamma): rows [1, kNY - 1), columns [1, kNX - 1)
    walk<2>(1, kNY - 1, 1, lane, wv, [&](int i, int q) {
      const int o = i * kNX + q;
      sp_inv_pred(kGamma, kGamma2, A0[o], A0[o + 1], A0[o + kNX], A0[o + kNX + 1], B1[o], B1[o + kNX], C1[o],
                  C1[o + 1], D0[o], B0[o], C0[o], D1[o]);
    });
    __syncthreads();
    // undo pair 1 update (beta): rows [2, kNY - 1), columns [2, kNX - 1)
    walk<1>(2, kNY - 1, 2, lane, wv, [&](int i, int q) {
      const int o = i * kNX + q;
      sp_inv_upd(kBeta, kBeta2, A0[o], B0[o - 1], B0[o], C0[o - kNX], C0[o], D1[o - kNX - 1], D1[o - kNX],
                 D1[o - 1], D1[o], A0[o], B1[o], C1[o]);
    });
    __syncthreads();
    // undo pair 1 predict (alpha) on the tile's own quadruples; store pixels
#pragma unroll
    for (int k = 0; k < kQY / kWv; ++k) {
      const int i = 2 + wv + k * kWv;
      const int o = i * kNX + 2 + lane;
      float pb, pc, pd;
      sp_inv_pred(kAlpha, kAlpha2, A0[o], A0[o + 1], A0[o + kNX], A0[o + kNX + 1], B1[o], B1[o + kNX], C1[o],
                  C1[o + 1], D1[o], pb, pc, pd);
      const float pa = A0[o];
      const int gqy = ty * kQY + i - 2;
      const int x0 = 2 * gqx, y0 = 2 * gqy;
      if (x0 < W && y0 < H) {
        float* r0 = out + (int64_t)y0 * a.out_stride;
        float* r1 = r0 + a.out_stride;
        if (pairs && x0 + 1 < W && a.final_out) {  // the image: streamed
          typedef float F2 __attribute__((ext_vector_type(2)));
          __builtin_nontemporal_store(F2{pa, pb}, reinterpret_cast<F2*>(r0 + x0));
          if (y0 + 1 < H) __builtin_nontemporal_store(F2{pc, pd}, reinterpret_cast<F2*>(r1 + x0));
        } else if (pairs && x0 + 1 < W) {
          *reinterpret_cast<float2*>(r0 + x0) = make_float2(pa, pb);
          if (y0 + 1 < H) *reinterpret_cast<float2*>(r1 + x0) = make_float2(pc, pd);
        } else {
          r0[x0] = pa;
          if (x0 + 1 < W) r0[x0 + 1] = pb;
          if (y0 + 1 < H) {
            r1[x0] = pc;
            if (x0 + 1 < W) r1[x0 + 1] = pd;
          }
        }
      }
    }
    if (img + (int)gridDim.y < a.batch) __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Forward level as a register-resident strip kernel (the default for level
// inputs of at least kStrip97Min pixels on each axis).  The mapping is the
// 5/3 pair kernels': a wave covers 128 quadruple columns, lane l holding two
// adjacent quadruples (one 16-byte vector per pixel row), and owns the 112
// columns of lanes 4..59.  The four spatial steps run in registers, row by
// row: the first pair (alpha, beta) on quadruple row r, then the second
// (gamma, delta) on row r - 1, which by then has its lower neighbour.  Each
// step reaches one quadruple to one side, the predicts to the right and the
// updates to the left, so after the four steps lanes 1..62 hold exact
// values and every neighbour crosses lanes by DPP; the edge lanes of a strip
// recompute its neighbours' columns instead of exchanging them.  Reads go
// through the symmetric fold of the pixels, which commutes with the lifting
// (it keeps every index's parity), exactly as in the tiled kernel, and each
// output comes from the same step functions on the same operands: results
// are bit-identical to fwd97.
// ---------------------------------------------------------------------------
constexpr int kStrip97Min = 16;
// STAGED stores: the four waves of a workgroup hold four adjacent strips of
// one segment (the host pads the strip count to a multiple of four); per
// output row each wave puts its 112 values of each band into LDS and, after
// one barrier, wave w writes band w's 448-value run (1792 bytes from a
// 128-byte boundary) with 16-byte stores, instead of four 448-byte runs
// that split a line at every other strip edge.
constexpr int kStage97 = kWavesPerBlock * 2 * 56;  // one band row of a workgroup

template <bool EDGE, int CP, bool STAGED>
__device__ void fwd97_strip_item(const Level97& a, const float* __restrict__ px, float* __restrict__ ll,
                                 float* __restrict__ band, int strip, int seg, int segh, int lane, float* stage) {
  using PL = PairLanes<kFwd>;
  const int W = a.W, H = a.H;
  const int ns_w = (W + 1) >> 1, ns_h = (H + 1) >> 1, nd_w = W >> 1, nd_h = H >> 1;
  const int Q = PL::count * strip + lane - PL::base;  // the lane's quadruple pair
  const int qL = 2 * Q;                                 // its first quadruple column
  const bool own = lane >= PL::base && lane < PL::base + PL::count;
  const int I0 = seg * segh, I1 = min(I0 + segh, ns_h);  // quadruple rows written
  PairPx<float, EDGE> L;
  L.base = px; L.stride = a.in_stride; L.W = W; L.H = H; L.c0 = 2 * qL;
  for (int k = 0; k < 4; ++k) L.pc[k] = fold_idx(L.c0 + k, W);
  const int qst = own ? qL : kOff;
  const int64_t bs = a.out_stride, ls = a.ll_stride;
  const bool keep_ll = !a.final_out;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int slot = w * PL::count + lane - PL::base;  // the lane's quadruple pair in the workgroup's run
  const int q0 = qL - 2 * slot;                        // the run's first quadruple column
  int buf = 0;
  // output row r: LL, HL, LH, HH of the lane's two quadruples
  auto store = [&](int r, float llL, float llR, float hlL, float hlR, float lhL, float lhR, float hhL, float hhR) {
    const bool real = r >= I0 && r < I1, real2 = real && r < nd_h;
    if constexpr (STAGED) {
      float* sb = stage + buf * 4 * kStage97;
      if (own) {
        sb[2 * slot] = llL * kLLScale; sb[2 * slot + 1] = llR * kLLScale;
        sb[kStage97 + 2 * slot] = hlL; sb[kStage97 + 2 * slot + 1] = hlR;
        sb[2 * kStage97 + 2 * slot] = lhL; sb[2 * kStage97 + 2 * slot + 1] = lhR;
        sb[3 * kStage97 + 2 * slot] = hhL * kHHScale; sb[3 * kStage97 + 2 * slot + 1] = hhR * kHHScale;
      }
      __syncthreads();
      // wave w: band w (0 LL, 1 HL, 2 LH, 3 HH) of row r
      const bool hpar = w == 1 || w == 3;
      const bool ok = w < 2 ? real : real2;
      float* row = w == 0 ? ll + (int64_t)r * ls : band + (int64_t)(w < 2 ? r : ns_h + r) * bs + (hpar ? ns_w : 0);
      const Rsrc rs = row_rsrc(row, ok ? (hpar ? nd_w : ns_w) * 4 : 0);
      const float* src = sb + w * kStage97;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int e = h * 4 * kWave + 4 * lane;  // element of the run
        const bool st = e < kStage97;
        const float* v = src + (st ? e : 0);
        V4<float> o;
        o.x = v[0]; o.y = v[1]; o.z = v[2]; o.w = v[3];
        if (w == 0 && keep_ll) bst4<0>(o, rs, st ? q0 + e : kOff);
        else bst4<kNT>(o, rs, st ? q0 + e : kOff);
      }
      buf ^= 1;
    } else {
      const Rsrc rl = row_rsrc(ll + (int64_t)r * ls, real ? ns_w * 4 : 0);
      const Rsrc rh = row_rsrc(band + (int64_t)r * bs + ns_w, real ? nd_w * 4 : 0);
      float* row2 = band + (int64_t)(ns_h + r) * bs;
      const Rsrc rlh = row_rsrc(row2, real2 ? ns_w * 4 : 0);
      const Rsrc rhh = row_rsrc(row2 + ns_w, real2 ? nd_w * 4 : 0);
      if (keep_ll) bst2<0>(llL * kLLScale, llR * kLLScale, rl, qst);
      else bst2<kNT>(llL * kLLScale, llR * kLLScale, rl, qst);
      bst2<kNT>(hlL, hlR, rh, qst);
      bst2<kNT>(lhL, lhR, rlh, qst);
      bst2<kNT>(hhL * kHHScale, hhR * kHHScale, rhh, qst);
    }
  };

  V4<float> E;                                  // pixel row 2r of the row being computed
  float p1U_L, p1U_R, p2U_L, p2U_R, p2U_P;      // first predict (c', d') of the row above
  float a1L = 0.f, b1L = 0.f, c1L = 0.f, d1L = 0.f, a1R = 0.f, b1R = 0.f, c1R = 0.f, d1R = 0.f;  // first pair, row r-1
  float q1U_L = 0.f, q1U_R = 0.f, q2U_L = 0.f, q2U_R = 0.f, q2U_P = 0.f;  // second predict of row r-2
  // first pair (alpha, beta) on row r from pixel rows 2r (E), 2r+1 (O), 2r+2 (E1)
  auto pair1 = [&](const V4<float>& O, const V4<float>& E1, float& aL, float& bL, float& cL, float& dL, float& aR,
                   float& bR, float& cR, float& dR) {
    float p0L, p1L, p2L, p0R, p1R, p2R;
    sp_pred(kAlpha, kAlpha2, E.x, E.z, E1.x, E1.z, E.y, E1.y, O.x, O.z, O.y, p0L, p1L, p2L);
    sp_pred(kAlpha, kAlpha2, E.z, from_next(E.x), E1.z, from_next(E1.x), E.w, E1.w, O.z, from_next(O.x), O.w, p0R,
            p1R, p2R);
    const float p0P = from_prev(p0R), p2P = from_prev(p2R);
    sp_upd(kBeta, kBeta2, E.x, p0P, p0L, p1U_L, p1L, p2U_P, p2U_L, p2P, p2L, aL, bL, cL);
    sp_upd(kBeta, kBeta2, E.z, p0L, p0R, p1U_R, p1R, p2U_L, p2U_R, p2L, p2R, aR, bR, cR);
    dL = p2L;
    dR = p2R;
    p1U_L = p1L; p1U_R = p1R; p2U_L = p2L; p2U_R = p2R; p2U_P = p2P;
    E = E1;
  };
  // chunks of the row loop (below)
  struct Buf {
    V4<float> v[CP][2];
  };
  auto load_chunk = [&](Buf& b, int r0) {
#pragma unroll
    for (int m = 0; m < CP; ++m) {
      L.load(2 * (r0 + m) + 1, b.v[m][0]);
      L.load(2 * (r0 + m) + 2, b.v[m][1]);
    }
  };
  Buf A, B;
  // prologue: pixel rows 2 I0 - 4 .. 2 I0; the first predict of row I0 - 2
  // and the first pair of row I0 - 1; the first chunk's loads go out right
  // after these, before the arithmetic
  {
    V4<float> v[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) L.load(2 * I0 - 4 + k, v[k]);
    load_chunk(A, I0);
    E = v[0];
    float p0L, p0R;
    sp_pred(kAlpha, kAlpha2, E.x, E.z, v[2].x, v[2].z, E.y, v[2].y, v[1].x, v[1].z, v[1].y, p0L, p1U_L, p2U_L);
    sp_pred(kAlpha, kAlpha2, E.z, from_next(E.x), v[2].z, from_next(v[2].x), E.w, v[2].w, v[1].z, from_next(v[1].x),
            v[1].w, p0R, p1U_R, p2U_R);
    p2U_P = from_prev(p2U_R);
    E = v[2];
    pair1(v[3], v[4], a1L, b1L, c1L, d1L, a1R, b1R, c1R, d1R);
  }
  // row r: the first pair of row r, then the second pair of row r - 1
  auto row = [&](const Buf& b, int m, int r) {
    float aL, bL, cL, dL, aR, bR, cR, dR;
    pair1(b.v[m][0], b.v[m][1], aL, bL, cL, dL, aR, bR, cR, dR);
    float q0L, q1L, q2L, q0R, q1R, q2R;
    sp_pred(kGamma, kGamma2, a1L, a1R, aL, aR, b1L, bL, c1L, c1R, d1L, q0L, q1L, q2L);
    sp_pred(kGamma, kGamma2, a1R, from_next(a1L), aR, from_next(aL), b1R, bR, c1R, from_next(c1L), d1R, q0R, q1R,
            q2R);
    const float q0P = from_prev(q0R), q2P = from_prev(q2R);
    float llL, hlL, lhL, llR, hlR, lhR;
    sp_upd(kDelta, kDelta2, a1L, q0P, q0L, q1U_L, q1L, q2U_P, q2U_L, q2P, q2L, llL, hlL, lhL);
    sp_upd(kDelta, kDelta2, a1R, q0L, q0R, q1U_R, q1R, q2U_L, q2U_R, q2L, q2R, llR, hlR, lhR);
    store(r - 1, llL, llR, hlL, hlR, lhL, lhR, q2L, q2R);
    q1U_L = q1L; q1U_R = q1R; q2U_L = q2L; q2U_R = q2R; q2U_P = q2P;
    a1L = aL; b1L = bL; c1L = cL; d1L = dL; a1R = aR; b1R = bR; c1R = cR; d1R = dR;
  };
  run_rows<CP>(I0, I1 + 1, A, B, load_chunk, row);
}

// Inverse level as a strip kernel, the same mapping: per quadruple row r it
// undoes the second update (delta) on row r, the second predict (gamma) on
// row r - 1, the first update (beta) on row r - 1 and the first predict
// (alpha) on row r - 2, whose pixels it then writes.  The undone updates
// reach up and left, the undone predicts down and right, so lanes 1..62 end
// exact.  Coefficients are read through the symmetric extension of the
// interleaved array (PairBands), as the tiled kernel reads them, and the
// results are bit-identical to inv97.
template <bool EDGE, int CP>
__device__ void inv97_strip_item(const Level97& a, const float* __restrict__ lls, const float* __restrict__ bands,
                                 float* __restrict__ px, int strip, int seg, int segh, int lane) {
  using PL = PairLanes<kInv>;
  const int W = a.W, H = a.H;
  const int ns_h = (H + 1) >> 1;
  const int qL = 2 * (PL::count * strip + lane - PL::base);
  const bool own = lane >= PL::base && lane < PL::base + PL::count;
  const int I0 = seg * segh, I1 = min(I0 + segh, ns_h);
  const PairBands<float, true, EDGE, 2> B =
      pair_bands<float, true, EDGE, 2>(bands, a.bands_stride, lls, a.in_stride, W, H, qL);
  const int c0 = own ? 2 * qL : kOff;
  const int lo = 2 * I0, hi = min(2 * I1, H);
  auto store = [&](int r, const V4<float>& v) {  // pixel row r
    const Rsrc rs = row_rsrc(px + (int64_t)r * a.out_stride, (r >= lo && r < hi) ? W * 4 : 0);
    if (a.final_out) bst4<kNT>(v, rs, c0);
    else bst4<0>(v, rs, c0);
  };
  // carried state: the scaled LH, HH of coefficient row r-1; the first
  // undone step (U1) of row r-1; the second (P1, its c and d) of row r-2;
  // the third (U2) of row r-2 with its d
  float lhU_L, lhU_R, hhU_L, hhU_R, hhU_P;
  float A1L, A1R, B1L, B1R, C1L, C1R, D1L, D1R;
  float pcU_L = 0.f, pcU_R = 0.f, pdU_L = 0.f, pdU_R = 0.f, pdU_P = 0.f;
  float A2L = 0.f, A2R = 0.f, B2L = 0.f, B2R = 0.f, C2L = 0.f, C2R = 0.f, D2L = 0.f, D2R = 0.f;
  // U1 (undo delta) of a coefficient row
  auto undo1 = [&](const float* ll, const float* hl, const float* lh, const float* hh, float& aL, float& bL, float& cL,
                   float& dL, float& aR, float& bR, float& cR, float& dR) {
    const float llL = ll[0] * kHHScale, llR = ll[1] * kHHScale;
    const float hhL = hh[0] * kLLScale, hhR = hh[1] * kLLScale;
    const float hlP = from_prev(hl[1]), hhP = from_prev(hhR);
    sp_inv_upd(kDelta, kDelta2, llL, hlP, hl[0], lhU_L, lh[0], hhU_P, hhU_L, hhP, hhL, aL, bL, cL);
    sp_inv_upd(kDelta, kDelta2, llR, hl[0], hl[1], lhU_R, lh[1], hhU_L, hhU_R, hhL, hhR, aR, bR, cR);
    dL = hhL;
    dR = hhR;
    lhU_L = lh[0]; lhU_R = lh[1]; hhU_L = hhL; hhU_R = hhR; hhU_P = hhP;
  };
  // chunks of the row loop (below)
  struct Buf {
    float ll[CP][2], hl[CP][2], lh[CP][2], hh[CP][2];
  };
  auto load_chunk = [&](Buf& b, int r0) {
#pragma unroll
    for (int m = 0; m < CP; ++m) {
      B.even(r0 + m, b.ll[m], b.hl[m]);
      B.odd(r0 + m, b.lh[m], b.hh[m]);
    }
  };
  Buf A, Bb;
  // prologue: coefficient rows I0 - 2 (the up neighbours) and I0 - 1 (U1);
  // the first chunk's loads go out right after these, before the arithmetic
  {
    float ll0[2], hl0[2], lh0[2], hh0[2], ll1[2], hl1[2], lh1[2], hh1[2];
    B.even(I0 - 2, ll0, hl0);
    B.odd(I0 - 2, lh0, hh0);
    B.even(I0 - 1, ll1, hl1);
    B.odd(I0 - 1, lh1, hh1);
    load_chunk(A, I0);
    lhU_L = lh0[0]; lhU_R = lh0[1];
    hhU_L = hh0[0] * kLLScale; hhU_R = hh0[1] * kLLScale;
    hhU_P = from_prev(hhU_R);
    undo1(ll1, hl1, lh1, hh1, A1L, B1L, C1L, D1L, A1R, B1R, C1R, D1R);
  }
  auto row = [&](const Buf& b, int m, int r) {
    float a1L, b1L, c1L, d1L, a1R, b1R, c1R, d1R;
    undo1(b.ll[m], b.hl[m], b.lh[m], b.hh[m], a1L, b1L, c1L, d1L, a1R, b1R, c1R, d1R);
    // P1 (undo gamma) of row r-1
    float pbL, pcL, pdL, pbR, pcR, pdR;
    sp_inv_pred(kGamma, kGamma2, A1L, A1R, a1L, a1R, B1L, b1L, C1L, C1R, D1L, pbL, pcL, pdL);
    sp_inv_pred(kGamma, kGamma2, A1R, from_next(A1L), a1R, from_next(a1L), B1R, b1R, C1R, from_next(C1L), D1R, pbR,
                pcR, pdR);
    // U2 (undo beta) of row r-1
    const float pbP = from_prev(pbR), pdP = from_prev(pdR);
    float a2L, b2L, c2L, a2R, b2R, c2R;
    sp_inv_upd(kBeta, kBeta2, A1L, pbP, pbL, pcU_L, pcL, pdU_P, pdU_L, pdP, pdL, a2L, b2L, c2L);
    sp_inv_upd(kBeta, kBeta2, A1R, pbL, pbR, pcU_R, pcR, pdU_L, pdU_R, pdL, pdR, a2R, b2R, c2R);
    pcU_L = pcL; pcU_R = pcR; pdU_L = pdL; pdU_R = pdR; pdU_P = pdP;
    // P2 (undo alpha) of row r-2: its pixels
    float xbL, xcL, xdL, xbR, xcR, xdR;
    sp_inv_pred(kAlpha, kAlpha2, A2L, A2R, a2L, a2R, B2L, b2L, C2L, C2R, D2L, xbL, xcL, xdL);
    sp_inv_pred(kAlpha, kAlpha2, A2R, from_next(A2L), a2R, from_next(a2L), B2R, b2R, C2R, from_next(C2L), D2R, xbR,
                xcR, xdR);
    V4<float> e, o;
    e.x = A2L; e.y = xbL; e.z = A2R; e.w = xbR;
    o.x = xcL; o.y = xdL; o.z = xcR; o.w = xdR;
    store(2 * (r - 2), e);
    store(2 * (r - 2) + 1, o);
    A1L = a1L; B1L = b1L; C1L = c1L; D1L = d1L; A1R = a1R; B1R = b1R; C1R = c1R; D1R = d1R;
    A2L = a2L; B2L = b2L; C2L = c2L; D2L = pdL; A2R = a2R; B2R = b2R; C2R = c2R; D2R = pdR;
  };
  run_rows<CP>(I0, I1 + 2, A, Bb, load_chunk, row);
}

template <int CP>
__global__ __launch_bounds__(kBlock) void inv97_strip(Level97 a, int nstrips, int nsegs, int segh, int64_t items) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t item = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * kWavesPerBlock +
                       __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  if (item >= items) return;
  const int per_img = nstrips * nsegs;
  const int img = (int)(item / per_img);
  const int rem = (int)(item - (int64_t)img * per_img);
  const int seg = rem / nstrips;
  const int strip = rem - seg * nstrips;
  const float* lls = static_cast<const float*>(a.in) + img * a.in_bstride;
  const float* bands = static_cast<const float*>(a.bands) + img * a.bands_bstride;
  float* px = static_cast<float*>(a.out) + img * a.out_bstride;
  // the wave's quadruple columns 2 (56 strip - 4) .. + 127: all with both
  // band parities inside the bands?
  const int q_first = 2 * (PairLanes<kInv>::count * strip - PairLanes<kInv>::base);
  if (q_first < 0 || q_first + 2 * kWave > (a.W >> 1)) inv97_strip_item<true, CP>(a, lls, bands, px, strip, seg, segh, lane);
  else inv97_strip_item<false, CP>(a, lls, bands, px, strip, seg, segh, lane);
}

// One wave per (image, segment, strip) item; items past the grid's last
// full workgroup return at once (no barrier in this kernel).
template <int CP, bool STAGED>
__global__ __launch_bounds__(kBlock) void fwd97_strip(Level97 a, int nstrips, int nsegs, int segh, int64_t items) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t item = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * kWavesPerBlock +
                       __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  if (item >= items) return;
  const int per_img = nstrips * nsegs;
  const int img = (int)(item / per_img);
  const int rem = (int)(item - (int64_t)img * per_img);
  const int seg = rem / nstrips;
  const int strip = rem - seg * nstrips;
  const float* px = static_cast<const float*>(a.in) + img * a.in_bstride;
  float* ll = static_cast<float*>(a.ll) + img * a.ll_bstride;
  float* band = static_cast<float*>(a.out) + img * a.out_bstride;
  // the wave's pixel columns 4 (112 strip - 4) .. + 255, all inside the image?
  const int c_first = 4 * (PairLanes<kFwd>::count * strip - PairLanes<kFwd>::base);
  float* stage = nullptr;
  if constexpr (STAGED) {
    __shared__ float stage_lds[2 * 4 * kStage97];
    stage = stage_lds;
  }
  if (c_first < 0 || c_first + 4 * kWave > a.W)
    fwd97_strip_item<true, CP, STAGED>(a, px, ll, band, strip, seg, segh, lane, stage);
  else
    fwd97_strip_item<false, CP, STAGED>(a, px, ll, band, strip, seg, segh, lane, stage);
}

// Separable comparison kernel on the same tiles: per level and per pair,
// horizontal predict, vertical predict, horizontal update, vertical update
// (eq. (3)), eight steps with a workgroup barrier between steps, then the
// scaling.  The 136 x 40-pixel tile (a 4-pixel halo around the 128 x 32
// output pixels) is lifted in place: a step changes one parity class and
// reads only the other.  Each step reads one pixel to each side on its
// axis, so the valid region shrinks by one pixel per step and four steps per
// axis use up the halo exactly; steps run on every position whose
// neighbours lie in the tile.
constexpr int kSX = 2 * kNX, kSY = 2 * kNY;  // 136 x 40

__global__ __launch_bounds__(kBlk) void fwd97_sep(Level97 a, int tiles_x) {
  __shared__ float X[kSX * kSY];
  const int lane = threadIdx.x & (kWave - 1), wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int tile = tile_remap(blockIdx.x, gridDim.x);
  const int ty = tile / tiles_x, tx = tile - ty * tiles_x;
  const int W = a.W, H = a.H;
  const int ns_w = (W + 1) >> 1, ns_h = (H + 1) >> 1, nd_w = W >> 1, nd_h = H >> 1;
  const int px0 = 2 * (tx * kQX - 2), py0 = 2 * (ty * kQY - 2);
  const int gc0 = fold97(px0 + lane, W), gc1 = fold97(px0 + kWave + lane, W);
  const int gc2 = fold97(px0 + 2 * kWave + (lane & 7), W);
  constexpr int kRowsPerWave = kSY / kWv;
  const int gqx = tx * kQX + lane;
  constexpr float kCoef[4] = {kAlpha, kBeta, kGamma, kDelta};
  for (int img = blockIdx.y; img < a.batch; img += gridDim.y) {
    const float* src = static_cast<const float*>(a.in) + img * a.in_bstride;
    float* ll = static_cast<float*>(a.ll) + img * a.ll_bstride;
    float* band = static_cast<float*>(a.out) + img * a.out_bstride;
    {
      float v0[kRowsPerWave], v1[kRowsPerWave], v2[kRowsPerWave];
#pragma unroll
      for (int k = 0; k < kRowsPerWave; ++k) {
        const float* row = src + (int64_t)fold97(py0 + wv + k * kWv, H) * a.in_stride;
        v0[k] = row[gc0];
        v1[k] = row[gc1];
        v2[k] = row[gc2];
      }
#pragma unroll
      for (int k = 0; k < kRowsPerWave; ++k) {
        float* x = X + (wv + k * kWv) * kSX;
        x[lane] = v0[k];
        x[kWave + lane] = v1[k];
        if (lane < 8) x[2 * kWave + lane] = v2[k];
      }
    }
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const float cf = kCoef[st];
      const int par = (st & 1) ? 0 : 1;  // predicts change odd samples, updates even ones
      __syncthreads();
      // horizontal: columns of parity `par` in [1, kSX - 1), every row
      for (int e = threadIdx.x; e < kSY * (kSX / 2 - 1); e += kBlk) {
        const int r = e / (kSX / 2 - 1), k = e - r * (kSX / 2 - 1);
        float* x = X + r * kSX + 2 * k + par + (par ? 0 : 2);
        x[0] = __fmaf_rn(cf, x[-1] + x[1], x[0]);
      }
      __syncthreads();
      // vertical: rows of parity `par` in [1, kSY - 1), every column
      for (int e = threadIdx.x; e < (kSY / 2 - 1) * kSX; e += kBlk) {
        const int j = e / kSX, c = e - j * kSX;
        float* x = X + (2 * j + par + (par ? 0 : 2)) * kSX + c;
        x[0] = __fmaf_rn(cf, x[-kSX] + x[kSX], x[0]);
      }
    }
    __syncthreads();
    // scaling and store of the tile's own quadruples (local pixels [4, 132) x [4, 36))
#pragma unroll
    for (int k = 0; k < kQY / kWv; ++k) {
      const int i = wv + k * kWv;
      const float* x = X + (2 * i + 4) * kSX + 2 * lane + 4;
      const float vll = x[0] * kLLScale, vhl = x[1], vlh = x[kSX], vhh = x[kSX + 1] * kHHScale;
      const int gqy = ty * kQY + i;
      if (gqx < ns_w && gqy < ns_h) {
        ll[(int64_t)gqy * a.ll_stride + gqx] = vll;
        if (gqx < nd_w) band[(int64_t)gqy * a.out_stride + ns_w + gqx] = vhl;
        if (gqy < nd_h) {
          band[(int64_t)(ns_h + gqy) * a.out_stride + gqx] = vlh;
          if (gqx < nd_w) band[(int64_t)(ns_h + gqy) * a.out_stride + ns_w + gqx] = vhh;
        }
      }
    }
    if (img + (int)gridDim.y < a.batch) __syncthreads();
  }
}


// ---------------------------------------------------------------------------
// Fused forward tail: the last n (2 or 3) levels, whose inputs are small,
// in one launch.  Each workgroup owns a kT97 x kT97 tile of the first tail
// level's input and runs every level on that tile plus a recompute halo in
// LDS.  A level reaches two quadruples (four pixels) to each side, so level
// m of the tail needs 4 (2^(n-m) - 1) pixels of halo and its region, minus
// two quadruples on each side, is the next level's region.  Each region is
// filled through the symmetric fold of its own level (the first from
// memory, the others from the LL the level before left in LDS), so every
// value past an edge is the one the per-level kernels read, and far-out
// positions that no in-image output reaches take any in-region value.  The
// four steps are the tiled kernel's on the same operands: the results are
// bit-identical to the per-level launches.
// ---------------------------------------------------------------------------
constexpr int kT97 = 64;
__host__ __device__ constexpr int tail97_halo(int n, int m) { return 4 * ((1 << (n - m)) - 1); }
constexpr int kTail97Q = (kT97 + 2 * tail97_halo(kTailMaxLevels, 0)) / 2;  // largest region, quadruples per side
constexpr int kTail97N = kT97 / 2 + 2 * tail97_halo(kTailMaxLevels, 1);    // largest LL hand-off, pixels per side
constexpr int kTail97Lds = 6 * kTail97Q * kTail97Q + kTail97N * kTail97N;   // floats (96.6 KiB)
constexpr int kTail97Block = 1024;
static_assert(kTail97Q - 4 == kTail97N, "level 1's region is level 0's, less two quadruples per side");

// f(i, q) for i in [i0, i1), q in [q0, q1): consecutive threads take
// consecutive columns.
template <typename F>
__device__ __forceinline__ void tail97_walk(int i0, int i1, int q0, int q1, F&& f) {
  const int cols = q1 - q0, cnt = (i1 - i0) * cols;
  for (int e = (int)threadIdx.x; e < cnt; e += kTail97Block) {
    const int r = e / cols;
    f(i0 + r, q0 + e - r * cols);
  }
}

__global__ __launch_bounds__(kTail97Block) void tail97_fwd(TailArgs a) {
  __shared__ float S[kTail97Lds];
  float* N = S + 6 * kTail97Q * kTail97Q;  // LL of the level just done, over the next region
  const int t = threadIdx.x;
  const int ty = blockIdx.x / a.tiles_x, tx = blockIdx.x - ty * a.tiles_x;
  const int n = a.n;
  // level-0 loads per thread: all issued before the first LDS store
  constexpr int kLoads = (4 * kTail97Q * kTail97Q + kTail97Block - 1) / kTail97Block;
  for (int img = blockIdx.y; img < a.batch; img += gridDim.y) {
    const float* src = static_cast<const float*>(a.in) + img * a.in_bstride;
    float* dst = static_cast<float*>(a.out) + img * a.out_bstride;
    for (int m = 0; m < n; ++m) {
      const int T = kT97 >> m, h = tail97_halo(n, m);
      const int R = T + 2 * h, Q = R / 2, P = Q * Q;
      const int W = a.W[m], H = a.H[m];
      const int ox = tx * T - h, oy = ty * T - h;  // level-m pixel of the region's local (0, 0)
      float* A = S;
      float* B = S + P;
      float* C = S + 2 * P;
      float* D = S + 3 * P;
      float* B1 = S + 4 * P;
      float* C1 = S + 5 * P;
      __syncthreads();  // the previous level's LL is in N; S is free
      if (m == 0) {
        float v[kLoads];
#pragma unroll
        for (int k = 0; k < kLoads; ++k) {
          const int e = t + k * kTail97Block < R * R ? t + k * kTail97Block : 0;
          const int r = e / R, c = e - r * R;
          v[k] = src[(int64_t)fold97(oy + r, H) * a.in_stride + fold97(ox + c, W)];
        }
#pragma unroll
        for (int k = 0; k < kLoads; ++k) {
          const int e = t + k * kTail97Block;
          if (e < R * R) {
            const int r = e / R, c = e - r * R;
            S[((r & 1) * 2 + (c & 1)) * P + (r >> 1) * Q + (c >> 1)] = v[k];
          }
        }
      } else {
        for (int e = t; e < R * R; e += kTail97Block) {
          const int r = e / R, c = e - r * R;
          const int fr = min(max(fold97(oy + r, H) - oy, 0), R - 1);
          const int fc = min(max(fold97(ox + c, W) - ox, 0), R - 1);
          S[((r & 1) * 2 + (c & 1)) * P + (r >> 1) * Q + (c >> 1)] = N[fr * R + fc];
        }
      }
      __syncthreads();
      // pair 1 predict (alpha), update (beta); pair 2 predict (gamma)
      tail97_walk(0, Q - 1, 0, Q - 1, [&](int i, int q) {
        const int o = i * Q + q;
        sp_pred(kAlpha, kAlpha2, A[o], A[o + 1], A[o + Q], A[o + Q + 1], B[o], B[o + Q], C[o], C[o + 1], D[o], B1[o],
                C1[o], D[o]);
      });
      __syncthreads();
      tail97_walk(1, Q - 1, 1, Q - 1, [&](int i, int q) {
        const int o = i * Q + q;
        sp_upd(kBeta, kBeta2, A[o], B1[o - 1], B1[o], C1[o - Q], C1[o], D[o - Q - 1], D[o - Q], D[o - 1], D[o], A[o],
               B[o], C[o]);
      });
      __syncthreads();
      tail97_walk(1, Q - 2, 1, Q - 2, [&](int i, int q) {
        const int o = i * Q + q;
        sp_pred(kGamma, kGamma2, A[o], A[o + 1], A[o + Q], A[o + Q + 1], B[o], B[o + Q], C[o], C[o + 1], D[o], B1[o],
                C1[o], D[o]);
      });
      __syncthreads();
      // pair 2 update (delta) and the scaling over the next region; the
      // tile's own quadruples go out (their H bands, and the last level's LL)
      const bool last = m == n - 1;
      const int ns_w = (W + 1) >> 1, ns_h = (H + 1) >> 1, nd_w = W >> 1, nd_h = H >> 1;
      const int own0 = h / 2, Tq = T / 2, Rn = Q - 4;
      tail97_walk(2, Q - 2, 2, Q - 2, [&](int i, int q) {
        const int o = i * Q + q;
        float vll, vhl, vlh;
        sp_upd(kDelta, kDelta2, A[o], B1[o - 1], B1[o], C1[o - Q], C1[o], D[o - Q - 1], D[o - Q], D[o - 1], D[o], vll,
               vhl, vlh);
        const float vhh = D[o] * kHHScale;
        vll *= kLLScale;
        if (!last) N[(i - 2) * Rn + (q - 2)] = vll;
        const int li = i - own0, lq = q - own0;
        const int gqy = ty * Tq + li, gqx = tx * Tq + lq;
        if (li >= 0 && li < Tq && lq >= 0 && lq < Tq && gqx < ns_w && gqy < ns_h) {
          if (last) __builtin_nontemporal_store(vll, dst + (int64_t)gqy * a.out_stride + gqx);
          if (gqx < nd_w) __builtin_nontemporal_store(vhl, dst + (int64_t)gqy * a.out_stride + ns_w + gqx);
          if (gqy < nd_h) {
            __builtin_nontemporal_store(vlh, dst + (int64_t)(ns_h + gqy) * a.out_stride + gqx);
            if (gqx < nd_w) __builtin_nontemporal_store(vhh, dst + (int64_t)(ns_h + gqy) * a.out_stride + ns_w + gqx);
          }
        }
      });
    }
  }
}

}  // namespace

int cdf97_tail_tiles(int W, int H, int& tiles_x, int& tiles_y) {
  tiles_x = (W + kT97 - 1) / kT97;
  tiles_y = (H + kT97 - 1) / kT97;
  return (int64_t)tiles_x * tiles_y <= 0x7fffffff;
}

int launch_cdf97_tail(const TailArgs& a, void* stream) {
  int tx, ty;
  if (a.n < 2 || a.n > kTailMaxLevels || !cdf97_tail_tiles(a.W[0], a.H[0], tx, ty) || tx != a.tiles_x ||
      ty != a.tiles_y)
    return hipErrorInvalidValue;
  for (int m = 0; m < a.n; ++m)
    if (a.W[m] < 2 || a.H[m] < 2) return hipErrorInvalidValue;  // the fold needs two samples
  const dim3 grid((unsigned)(tx * ty), (unsigned)(a.batch < 65535 ? a.batch : 65535));
  hipLaunchKernelGGL(tail97_fwd, grid, dim3(kTail97Block), 0, static_cast<hipStream_t>(stream), a);
  return hipGetLastError();
}

int cdf97_tiles(int W, int H, int& tiles_x, int& tiles_y) {
  tiles_x = (((W + 1) >> 1) + kQX - 1) / kQX;
  tiles_y = (((H + 1) >> 1) + kQY - 1) / kQY;
  return (int64_t)tiles_x * tiles_y <= 0x7fffffff;
}

int cdf97_strip_geometry(int W, int H, int& nstrips) {
  nstrips = (((W + 1) >> 1) + 2 * PairLanes<kFwd>::count - 1) / (2 * PairLanes<kFwd>::count);
  return W >= kStrip97Min && H >= kStrip97Min;
}

int launch_cdf97_strip(int dir, const Level97& a, int segh, int chunk, bool staged, void* stream) {
  int nstrips;
  if (!cdf97_strip_geometry(a.W, a.H, nstrips) || segh < 1) return hipErrorInvalidValue;
  staged = staged && dir == kFwd;
  if (staged) nstrips = (nstrips + kWavesPerBlock - 1) / kWavesPerBlock * kWavesPerBlock;  // whole workgroups
  const int nsegs = (((a.H + 1) >> 1) + segh - 1) / segh;
  const int64_t items = (int64_t)nstrips * nsegs * a.batch;
  const dim3 grid((unsigned)((items + kWavesPerBlock - 1) / kWavesPerBlock));
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (dir == kFwd) {
    if (staged && chunk >= 2)
      hipLaunchKernelGGL((fwd97_strip<2, true>), grid, dim3(kBlock), 0, s, a, nstrips, nsegs, segh, items);
    else if (staged)
      hipLaunchKernelGGL((fwd97_strip<1, true>), grid, dim3(kBlock), 0, s, a, nstrips, nsegs, segh, items);
    else if (chunk >= 2)
      hipLaunchKernelGGL((fwd97_strip<2, false>), grid, dim3(kBlock), 0, s, a, nstrips, nsegs, segh, items);
    else
      hipLaunchKernelGGL((fwd97_strip<1, false>), grid, dim3(kBlock), 0, s, a, nstrips, nsegs, segh, items);
  } else if (dir == kInv) {
    if (chunk >= 2) hipLaunchKernelGGL(inv97_strip<2>, grid, dim3(kBlock), 0, s, a, nstrips, nsegs, segh, items);
    else hipLaunchKernelGGL(inv97_strip<1>, grid, dim3(kBlock), 0, s, a, nstrips, nsegs, segh, items);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int launch_cdf97_level(int dir, bool separable, const Level97& a, void* stream) {
  int tx, ty;
  if (!cdf97_tiles(a.W, a.H, tx, ty)) return hipErrorInvalidValue;
  const dim3 grid((unsigned)(tx * ty), (unsigned)(a.batch < 65535 ? a.batch : 65535));
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (dir == kFwd && separable) hipLaunchKernelGGL(fwd97_sep, grid, dim3(kBlk), 0, s, a, tx);
  else if (dir == kFwd) hipLaunchKernelGGL(fwd97, grid, dim3(kBlk), 0, s, a, tx);
  else if (!separable) hipLaunchKernelGGL(inv97, grid, dim3(kBlk), 0, s, a, tx);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace dwt2
