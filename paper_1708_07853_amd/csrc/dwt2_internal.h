// Internal types shared by the host API (api.cpp, batched.cpp) and the HIP
// kernels (strip_*.hip, tail_kernels.hip, lds_kernels.hip, separable.hip,
// cdf97.hip).  Not part of the public interface.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "../../include/dwt2.h"

namespace dwt2 {

// A wave (64 lanes) owns a vertical strip of 128 quadruple columns; each lane
// owns two adjacent quadruples (four pixel columns, one 16-byte vector per
// pixel row), so strip s covers quadruple columns [128 s, 128 s + 128).
constexpr int kWave = 64;
constexpr int kStripQuads = 128;
constexpr int kWavesPerBlock = 4;
constexpr int kBlock = kWave * kWavesPerBlock;

enum Dir : int32_t { kFwd = 0, kInv = 1, kBwd = 2 };

// One level of one image.  "Pixels" is the level input region X_{k-1}
// (w_{k-1} x h_{k-1}); "ll" is LL_k; "band" is the origin of the packed
// coefficient array, whose [0, h_{k-1}) x [0, w_{k-1}) corner holds this
// level's quadruple (LL_k at the origin unless ll points elsewhere).
//   forward : reads pixels, writes ll and the three H bands into band
//   inverse : reads ll and the H bands, writes pixels
//   adjoint : like inverse (gradients)
struct LevelDesc {
  const void* pix_in;   // forward input pixels
  void* pix_out;        // inverse/adjoint output pixels
  const void* ll_in;    // inverse/adjoint LL_k input
  void* ll_out;         // forward LL_k output
  const void* band_in;  // inverse/adjoint H-band source (packed array origin)
  void* band_out;       // forward H-band destination (packed array origin)
  int64_t pix_stride;
  int64_t ll_stride;
  int64_t band_stride;
  int32_t W, H;         // level input size
  int32_t seg;          // quadruple rows per work item
  int32_t nstrips;
  int32_t nsegs;
  int32_t keep_out;     // a later launch reads this level's LL output (cache it)
  int32_t stage;        // forward pair: stage its stores through LDS (whole 128-byte lines)
  int32_t pad_;
};

// Plain (uniform-geometry) launch of one level over a batch of images.
struct LevelLaunch {
  LevelDesc d;
  int64_t pix_bstride;   // element strides between consecutive images
  int64_t ll_bstride;
  int64_t band_bstride;
  int64_t items;         // batch * nsegs * nstrips
  int32_t items_per_image;
  int32_t pad_;
};

inline int ceil_half(int n) { return (n + 1) >> 1; }

inline int num_strips(int W) { return (ceil_half(W) + kStripQuads - 1) / kStripQuads; }

inline int64_t ll_pitch(int w) {  // padded row pitch (elements) of an LL buffer
  return ((int64_t)w + 63) & ~(int64_t)63;
}

// One step of a persistent job: one level of one image, or of a batch of
// equally sized images (nimg > 1, images `*_bstride` elements apart).
// Work items of the step occupy queue slots [item_start, item_start + items)
// in (image, segment, strip) order.  Each (image, segment) has a completion
// counter at sync[kSyncCounters + kCounterStride * (cbase + image * nsegs +
// segment)], one per 64-byte line so that polls of different counters do not
// queue behind each other.
struct JobDesc {
  LevelDesc d;
  int64_t pix_bstride, ll_bstride, band_bstride;
  int32_t nimg;
  int32_t item_start;
  int32_t items;
  int32_t cbase;
  int32_t prev;   // step this one reads from (same images), or -1
  int32_t coh;    // bit 0: input LL rows come from step `prev`; bit 1: a later step reads the LL output
  int32_t pad_[2];
};

// Largest intermediate LL (bytes over a launch) stored with the caching
// policy: half of MI355X's 256 MB Infinity Cache.
constexpr int64_t kKeepBytes = 128ll << 20;

constexpr int kInlineDescs = 20;
constexpr int kSyncError = 1;     // set when a dependency wait gives up
constexpr int kSyncCounters = 16; // first completion counter
constexpr int kCounterStride = 16; // words between counters (one 64-byte line each)

struct JobArgs {
  const JobDesc* descs;       // device table, or null: use inl[]
  const uint32_t* item_desc;  // device queue-slot -> desc table, or null: scan
  uint32_t* sync;             // zeroed before every launch
  uint32_t* host_err;         // pinned host word set when a wait gives up (may be null)
  int32_t ndesc;
  int32_t total_items;
  uint32_t max_polls;         // poll budget of one wait (0: kSpinLimit, about 2 s)
  uint32_t unreachable;       // test setting: every wait runs out its budget
  JobDesc inl[kInlineDescs];
};

// Wait settings of later persistent launches (dwt2_set_job_wait) and the
// device's host-visible error word (api.cpp).
void job_wait_settings(uint32_t& max_polls, uint32_t& unreachable);
uint32_t* host_error_word();  // device pointer of the current device's word, or null

// One level-synchronous launch over items [item_begin, item_begin + items)
// of a ragged batch's item table.
struct TableArgs {
  const JobDesc* descs;
  const uint32_t* item_desc;
  int32_t item_begin;
  int32_t items;
};

// One level of the separable baseline (separable.hip): the level input, a
// work array of the level's size, and the LL / band destinations.
struct SepLevel {
  const void* src;
  int64_t src_stride, src_bstride;
  void* work;
  int64_t work_pitch, work_bstride;
  void* ll;
  int64_t ll_stride, ll_bstride;
  void* band;
  int64_t band_stride, band_bstride;
  int32_t W, H, batch, pad_;
};
int launch_separable_level(int mode, const SepLevel& a, void* stream);

// Tail kernels (the last 2..kTailMaxLevels levels of a plain forward or
// inverse call in one launch): tile edge at the first tail level's input, workgroup size, LDS
// elements (region arrays of the n levels plus three predict arrays, n = 3),
// and the largest first-tail-level input (pixels over the batch) it takes.
constexpr int kTailMaxLevels = 3;
constexpr int kTailS = 64;
constexpr int kTailBlock = 1024;
constexpr int kTailLds = 17024;
constexpr int64_t kTailArea = 1024 * 1024;
struct TailArgs {
  const void* in;        // forward: the finest tail level's pixels (image or LL buffer);
                         // inverse: the packed coefficient array
  int64_t in_stride, in_bstride;
  void* out;             // forward: the packed coefficient array; inverse: the finest
                         // tail level's pixels
  int64_t out_stride, out_bstride;
  int32_t n, batch, tiles_x, tiles_y;
  int32_t W[kTailMaxLevels + 1], H[kTailMaxLevels + 1];  // level sizes from the first tail input
};
int launch_tail(int dir, int mode, const TailArgs& a, void* stream);
// LDS-tiled forward level (comparison kernels): scheme DWT2_SCHEME_*, the
// separable steps of eq. (3), the spatial steps of eq. (5) or the adapted
// scheme of §3 (float only), a workgroup barrier between steps.  Uses src,
// ll, band and the sizes of a; work is unused.  lds_tiles gives the grid's
// tile counts (returns 0 if they exceed a launch).
int lds_tiles(int W, int H, int& tiles_x, int& tiles_y);
int launch_lds_level(int scheme, int mode, const SepLevel& a, void* stream);

// One CDF 9/7 level (float32; cdf97.hip).  W, H: the level input's size.
struct Level97 {
  const void* in;      // forward: the level input's pixels; inverse: LL_k
  int64_t in_stride, in_bstride;
  const void* bands;   // inverse: the packed array holding level k's H bands
  int64_t bands_stride, bands_bstride;
  void* ll;            // forward: LL_k
  int64_t ll_stride, ll_bstride;
  void* out;           // forward: the packed array (H bands); inverse: the pixels
  int64_t out_stride, out_bstride;
  int32_t W, H, batch;
  int32_t final_out;   // 1: LL_k (forward) or the pixels (inverse) are final results
};
int cdf97_tiles(int W, int H, int& tiles_x, int& tiles_y);
// separable: the comparison kernel with the eight separable steps (forward only)
int launch_cdf97_level(int dir, bool separable, const Level97& a, void* stream);
// A forward or inverse level as a register-resident strip kernel: nstrips
// for width W, and whether the level takes it (inputs of at least 16 x 16).
// segh = quadruple rows per work item, chunk = prefetch rows (1 or 2),
// staged = the forward writes whole lines through LDS.
int cdf97_strip_geometry(int W, int H, int& nstrips);
int launch_cdf97_strip(int dir, const Level97& a, int segh, int chunk, bool staged, void* stream);
// The last a.n (2..kTailMaxLevels) levels of a CDF 9/7 forward in one
// launch (a.in: the first tail level's input; a.out: the packed array,
// which takes every tail level's bands and the last LL); tiles of 64 x 64
// pixels of the first tail level's input; every tail level at least 2 x 2.
int cdf97_tail_tiles(int W, int H, int& tiles_x, int& tiles_y);
int launch_cdf97_tail(const TailArgs& a, void* stream);

// Strip-kernel launchers, instantiated per direction (level kernels in
// strip_fwd.hip, strip_inv.hip, strip_bwd.hip; job and table kernels in
// job_fwd.hip, job_inv.hip, job_bwd.hip).  Return hipError_t as int.
template <int DIR> int launch_level_dir(int mode, int chunk, const LevelLaunch& a, void* stream);
template <int DIR> int launch_job_dir(int mode, const JobArgs& a, int blocks, void* stream);
template <int DIR> int job_blocks_per_cu_dir(int mode, bool table);
template <int DIR> int launch_table_dir(int mode, const TableArgs& a, void* stream);

// Each direction's instantiation lives in its own translation unit; the
// others only refer to it.
#define DWT2_EXTERN_STRIP(DIR)                                                        \
  extern template int launch_level_dir<DIR>(int, int, const LevelLaunch&, void*);     \
  extern template int launch_job_dir<DIR>(int, const JobArgs&, int, void*);           \
  extern template int job_blocks_per_cu_dir<DIR>(int, bool);                          \
  extern template int launch_table_dir<DIR>(int, const TableArgs&, void*);
DWT2_EXTERN_STRIP(kFwd)
DWT2_EXTERN_STRIP(kInv)
DWT2_EXTERN_STRIP(kBwd)
#undef DWT2_EXTERN_STRIP

// One level of a plain call; `chunk`: prefetch chunk (1, 2 or 4 quadruple rows).
inline int launch_level(int dir, int mode, int chunk, const LevelLaunch& a, void* stream) {
  if (dir == kFwd) return launch_level_dir<kFwd>(mode, chunk, a, stream);
  if (dir == kInv) return launch_level_dir<kInv>(mode, chunk, a, stream);
  return launch_level_dir<kBwd>(mode, chunk, a, stream);
}
// Resident blocks per CU of the persistent job kernel (TABLE variant or not).
inline int job_blocks_per_cu(int dir, int mode, bool table) {
  if (dir == kFwd) return job_blocks_per_cu_dir<kFwd>(mode, table);
  if (dir == kInv) return job_blocks_per_cu_dir<kInv>(mode, table);
  return job_blocks_per_cu_dir<kBwd>(mode, table);
}
// The persistent job (cooperative launch of `blocks` blocks).
inline int launch_job(int dir, int mode, const JobArgs& a, int blocks, void* stream) {
  if (dir == kFwd) return launch_job_dir<kFwd>(mode, a, blocks, stream);
  if (dir == kInv) return launch_job_dir<kInv>(mode, a, blocks, stream);
  return launch_job_dir<kBwd>(mode, a, blocks, stream);
}
// One level-synchronous launch over a ragged batch's item range.
inline int launch_table(int dir, int mode, const TableArgs& a, void* stream) {
  if (dir == kFwd) return launch_table_dir<kFwd>(mode, a, stream);
  if (dir == kInv) return launch_table_dir<kInv>(mode, a, stream);
  return launch_table_dir<kBwd>(mode, a, stream);
}
// Two levels in one pass (fused_fwd.hip, fused_inv.hip, fused_bwd.hip):
// the descriptor's W, H are the finer level's input, seg counts rows of
// quadruples of the coarser level, ll is the coarser level's LL, nstrips
// counts strips of pair_strip_q(dir) owned quadruple columns of the finer
// level.
constexpr int pair_strip_q(int) { return 112; }
template <int DIR> int launch_pair_dir(int mode, int chunk, const LevelLaunch& a, void* stream);
extern template int launch_pair_dir<kFwd>(int, int, const LevelLaunch&, void*);
extern template int launch_pair_dir<kInv>(int, int, const LevelLaunch&, void*);
extern template int launch_pair_dir<kBwd>(int, int, const LevelLaunch&, void*);
inline int launch_pair(int dir, int mode, int chunk, const LevelLaunch& a, void* stream) {
  if (dir == kFwd) return launch_pair_dir<kFwd>(mode, chunk, a, stream);
  if (dir == kInv) return launch_pair_dir<kInv>(mode, chunk, a, stream);
  return launch_pair_dir<kBwd>(mode, chunk, a, stream);
}
// One pair step of a ragged batch over the items [item_begin, item_begin +
// items) of a table (level-synchronous schedule; descriptors never stage).
template <int DIR> int launch_pair_table_dir(int mode, const TableArgs& a, void* stream);
extern template int launch_pair_table_dir<kFwd>(int, const TableArgs&, void*);
extern template int launch_pair_table_dir<kInv>(int, const TableArgs&, void*);
extern template int launch_pair_table_dir<kBwd>(int, const TableArgs&, void*);
inline int launch_pair_table(int dir, int mode, const TableArgs& a, void* stream) {
  if (dir == kFwd) return launch_pair_table_dir<kFwd>(mode, a, stream);
  if (dir == kInv) return launch_pair_table_dir<kInv>(mode, a, stream);
  return launch_pair_table_dir<kBwd>(mode, a, stream);
}
// Clears n synchronisation words with a fill kernel (tail_kernels.hip).
int launch_zero(uint32_t* p, int64_t n, void* stream);

}  // namespace dwt2
