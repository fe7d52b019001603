// Strip kernels of one direction: one launch per level (level_kernel), the
// persistent job that chains levels (job_kernel) and the level-synchronous
// launch over a ragged batch's item table (table_kernel), with their host
// launchers.  Each direction's level kernels (strip_*.hip) and job / table
// kernels (job_*.hip) are instantiated in translation units of their own, so
// they compile in parallel.
#pragma once

#include "lift.h"

namespace dwt2 {
namespace {

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
// deadlock.  A wait that exceeds its poll budget gives up rather than hang:
// it sets the error word in the workspace and the library's host-visible
// error word (pinned host memory, read by the next library call on the
// host), and the item skips its arithmetic -- its inputs may not exist -- but
// still publishes its counter so that its dependants do not wait in turn.
// ---------------------------------------------------------------------------
// s_sleep(16) pauses about 16 * 64 clocks (~0.43 us at 2.4 GHz); a poll
// backs off to at most kNapCap of them (~1.7 us), so a waiter sees a finished
// producer within about that time, and gives up after kSpinLimit polls (~2 s)
// unless the launch sets a smaller budget.
constexpr uint32_t kNapCap = 4;
constexpr uint32_t kSpinLimit = 1u << 20;

// Wait until rows [r_lo, r_hi] of the output of step p (image img) exist;
// false if the wait gave up.  `pixels`: the rows are pixel rows of p's output
// (inverse / adjoint, two per quadruple row); otherwise they are p's LL rows
// (forward, one per row).  `unreachable` (a test setting) asks for one
// completion more than a segment has, so every wait runs out its budget.
__device__ __forceinline__ bool wait_rows(const JobDesc& p, const JobArgs& a, int img, int r_lo, int r_hi,
                                          bool pixels) {
  const int ns_h = (p.d.H + 1) >> 1;
  int q_lo = pixels ? (r_lo >> 1) : r_lo, q_hi = pixels ? (r_hi >> 1) : r_hi;
  q_lo = q_lo < 0 ? 0 : q_lo;
  q_hi = q_hi > ns_h - 1 ? ns_h - 1 : q_hi;
  const int g_lo = q_lo / p.d.seg, g_hi = q_hi / p.d.seg;
  uint32_t* ctr = a.sync + kSyncCounters + (int64_t)kCounterStride * (p.cbase + img * p.d.nsegs);
  const uint32_t limit = a.max_polls ? a.max_polls : kSpinLimit;
  const uint32_t need = (uint32_t)p.d.nstrips + (a.unreachable ? 1u : 0u);
  bool ok = true;
  for (int g = g_lo; g <= g_hi && ok; ++g) {
    uint32_t spins = 0, nap = 1;
    // every lane reads the same word; readfirstlane makes the loop wave-uniform
    while (__builtin_amdgcn_readfirstlane(__hip_atomic_load(ctr + (int64_t)kCounterStride * g, __ATOMIC_RELAXED,
                                                            __HIP_MEMORY_SCOPE_AGENT)) < need) {
      if (++spins > limit) {
        ok = false;
        break;
      }
      for (uint32_t k = 0; k < nap; ++k) __builtin_amdgcn_s_sleep(16);
      nap = nap < kNapCap ? 2 * nap : kNapCap;
    }
  }
  if (!ok) {
    __hip_atomic_store(a.sync + kSyncError, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (a.host_err) __hip_atomic_store(a.host_err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
  // the item's loads of the producers' rows are coherent (sc0 sc1) and are
  // issued only after the counters were seen; the fence keeps the compiler
  // from moving them above the wait
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  return ok;
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
    bool ready = true;
    if (jd.prev >= 0) {
      const JobDesc p = D[jd.prev];
      const int I0 = seg * jd.d.seg;
      const int I1 = min(I0 + jd.d.seg, (jd.d.H + 1) >> 1);
      // rows this item reads from p's output, with a margin that covers the
      // symmetric folds at the image edges
      if (DIR == kFwd) ready = wait_rows(p, a, img, 2 * I0 - 4, 2 * I1 + 2, false);
      else ready = wait_rows(p, a, img, I0 - 3, I1 + 2, true);
    }
    if (ready)
      run_item<DIR, T, CH, true>(jd.d, jd.coh, img * jd.pix_bstride, img * jd.ll_bstride, img * jd.band_bstride,
                                 strip, seg, lane);
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

// The persistent job and the table kernel run with a prefetch chunk of two
// quadruple rows (the batched plans use no other); a call that forces
// another chunk keeps it for the per-level launches only.
constexpr int kJobCh = 2;

template <int DIR, typename T, int CH>
hipError_t launch_level_t(const LevelLaunch& a, hipStream_t s) {
  const int64_t blocks = (a.items + kWavesPerBlock - 1) / kWavesPerBlock;
  hipLaunchKernelGGL((level_kernel<DIR, T, CH>), dim3((unsigned)blocks), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

template <int DIR, typename T>
hipError_t launch_level_ch(int chunk, const LevelLaunch& a, hipStream_t s) {
  if (chunk >= 4) return launch_level_t<DIR, T, 4>(a, s);
  if (chunk >= 2) return launch_level_t<DIR, T, 2>(a, s);
  return launch_level_t<DIR, T, 1>(a, s);
}

// Cooperative launch: the runtime places every block at once or fails.
template <int DIR, typename T>
hipError_t launch_job_t(const JobArgs& a, int blocks, hipStream_t s) {
  void* args[] = {const_cast<JobArgs*>(&a)};
  const void* f = a.descs ? reinterpret_cast<const void*>(&job_kernel<DIR, T, kJobCh, true>)
                          : reinterpret_cast<const void*>(&job_kernel<DIR, T, kJobCh, false>);
  return hipLaunchCooperativeKernel(f, dim3((unsigned)blocks), dim3(kBlock), args, 0, s);
}

// Resident blocks per CU of the job kernel variant that a launch uses
// (TABLE: descriptors in device memory); the cooperative launch fails if
// the grid exceeds what this variant can hold at once.
template <int DIR, typename T>
int occ_job_t(bool table) {
  int n = 0;
  const void* f = table ? reinterpret_cast<const void*>(&job_kernel<DIR, T, kJobCh, true>)
                        : reinterpret_cast<const void*>(&job_kernel<DIR, T, kJobCh, false>);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, kBlock, 0) != hipSuccess) n = 0;
  return n;
}

template <int DIR, typename T>
hipError_t launch_table_t(const TableArgs& a, hipStream_t s) {
  const dim3 grid((unsigned)((a.items + kWavesPerBlock - 1) / kWavesPerBlock));
  hipLaunchKernelGGL((table_kernel<DIR, T, kJobCh>), grid, dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

}  // namespace

// The direction's entry points (declared in dwt2_internal.h); each
// strip_*.hip / job_*.hip instantiates them for its direction.  The adjoint has no
// integer mode.
template <int DIR>
int launch_level_dir(int mode, int chunk, const LevelLaunch& a, void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (mode == DWT2_F32) return launch_level_ch<DIR, float>(chunk, a, s);
  if constexpr (DIR != kBwd) return launch_level_ch<DIR, int>(chunk, a, s);
  return hipErrorInvalidValue;
}

template <int DIR>
int launch_job_dir(int mode, const JobArgs& a, int blocks, void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (mode == DWT2_F32) return launch_job_t<DIR, float>(a, blocks, s);
  if constexpr (DIR != kBwd) return launch_job_t<DIR, int>(a, blocks, s);
  return hipErrorInvalidValue;
}

template <int DIR>
int job_blocks_per_cu_dir(int mode, bool table) {
  if (mode == DWT2_F32) return occ_job_t<DIR, float>(table);
  if constexpr (DIR != kBwd) return occ_job_t<DIR, int>(table);
  return 0;
}

template <int DIR>
int launch_table_dir(int mode, const TableArgs& a, void* stream) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (a.items <= 0) return hipSuccess;
  if (mode == DWT2_F32) return launch_table_t<DIR, float>(a, s);
  if constexpr (DIR != kBwd) return launch_table_t<DIR, int>(a, s);
  return hipErrorInvalidValue;
}

#define DWT2_INSTANTIATE_LEVEL(DIR) template int launch_level_dir<DIR>(int, int, const LevelLaunch&, void*);
#define DWT2_INSTANTIATE_JOB(DIR)                                                    \
  template int launch_job_dir<DIR>(int, const JobArgs&, int, void*);                 \
  template int job_blocks_per_cu_dir<DIR>(int, bool);                                \
  template int launch_table_dir<DIR>(int, const TableArgs&, void*);

}  // namespace dwt2
