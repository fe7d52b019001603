// LDS-tiled comparison kernels (the separable and non-separable schemes with
// equal data movement, and the adapted scheme).
#include "lift.h"

namespace dwt2 {
namespace {

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

}  // namespace

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

}  // namespace dwt2
