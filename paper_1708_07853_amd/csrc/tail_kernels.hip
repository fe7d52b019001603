// Fused tail kernels: the small last levels of a forward, or the small first
// levels of an inverse or adjoint, in one launch (tail_fwd, tail_inv,
// tail_bwd), and the fill kernel that clears synchronisation words.
#include "lift.h"

namespace dwt2 {
namespace {

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
  const int lx = threadIdx.x & (kTailRowT - 1);
  const int ly = __builtin_amdgcn_readfirstlane(threadIdx.x / kTailRowT);  // one wave per row: uniform
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
  const int lx = threadIdx.x & (kTailRowT - 1);
  const int ly = __builtin_amdgcn_readfirstlane(threadIdx.x / kTailRowT);  // one wave per row: uniform
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
  const int lx = threadIdx.x & (kTailRowT - 1);
  const int ly = __builtin_amdgcn_readfirstlane(threadIdx.x / kTailRowT);  // one wave per row: uniform
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

__global__ void zero_kernel(uint32_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

}  // namespace

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

int launch_zero(uint32_t* p, int64_t n, void* stream) {
  const int64_t blocks = n < 256 * 256 ? (n + 255) / 256 : 256;
  hipLaunchKernelGGL(zero_kernel, dim3((unsigned)(blocks > 0 ? blocks : 1)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), p, n);
  return hipGetLastError();
}

}  // namespace dwt2
