/*
 * dwt2.h -- multi-level 2-D CDF 5/3 discrete wavelet transform on AMD
 * Instinct MI355X (gfx950), computed with the non-separable lifting scheme of
 * Barina et al., "The Parallel Algorithm for the 2-D Discrete Wavelet
 * Transform" (§3, eq. (5)).
 *
 * Mathematical definition (what every entry point computes)
 * ---------------------------------------------------------
 * One level splits a w x h region X into the quadruple (LL, HL, LH, HH) of
 * §2 by sample parity: a = X[2i][2j], b = X[2i][2j+1], c = X[2i+1][2j],
 * d = X[2i+1][2j+1].  The CDF 5/3 lifting pair of §2, eq. (2) (K = 1) uses
 * predict P(z) = -1/2 (1 + z) and update U(z) = 1/4 (1 + z^-1), without
 * scaling.  The level applies the spatial predict and then the spatial
 * update of §3, eq. (5); in exact arithmetic this equals the separable
 * sequence of §2, eq. (3) (horizontal predict, vertical predict, horizontal
 * update, vertical update).  Samples outside the region are taken from its
 * whole-sample symmetric extension (x[-i] = x[i], x[N-1+i] = x[N-1-i]).
 * Even 0-based indices are L: a length-N axis keeps ceil(N/2) L and
 * floor(N/2) H coefficients.  Levels recurse on LL (Mallat).
 *
 * Modes
 *   DWT2_F32      float32 samples; results within 2e-4 absolute of the
 *                 float64 definition for 8-bit-range inputs.
 *   DWT2_I32_REV  int32 samples, reversible integer 5/3: predict
 *                 d -= floor((l + r) / 2), update s += floor((l + r + 2) / 4),
 *                 rounded separable steps composed in the eq. (3) order
 *                 inside each spatial step.  Bit-exact and exactly
 *                 invertible.  Inputs must keep every intermediate sum in
 *                 int32 range (|x| <= 2^24 is always safe).
 *
 * Output layout ("Mallat-packed", same w x h shape as the image), with
 * w_0 = w, w_k = ceil(w_{k-1} / 2) (likewise h):
 *   LL_L   rows [0, h_L),          cols [0, w_L)
 *   HL_k   rows [0, h_k),          cols [w_k, w_{k-1})
 *   LH_k   rows [h_k, h_{k-1}),    cols [0, w_k)
 *   HH_k   rows [h_k, h_{k-1}),    cols [w_k, w_{k-1})
 *
 * Conventions for every call
 *   - Image, coefficient and workspace pointers are DEVICE pointers of the
 *     current HIP device; strides are in ELEMENTS (4-byte samples).
 *   - stream is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls are asynchronous and stream-ordered; the return value covers
 *     argument validation and launch only, execution errors surface at the
 *     caller's next synchronisation.
 *   - Ownership: the caller owns src, dst and workspace; the library never
 *     frees or retains them beyond the call's stream work.  The library owns
 *     only its batched-plan cache (released by dwt2_clear_plan_cache).
 *   - Errors are negative status codes; validation happens before any HIP
 *     call, so a failing call has no side effects.  No C++ exception crosses
 *     this interface.  dwt2_last_error() gives a thread-local detail string.
 *   - The transforms are out of place: src and dst must not overlap, and the
 *     workspace must overlap neither.
 *   - Calls on different streams need distinct workspaces.
 */
#ifndef DWT2_H
#define DWT2_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* modes */
enum { DWT2_F32 = 0, DWT2_I32_REV = 1 };
/* boundary extension: whole-sample symmetric is the only one */
enum { DWT2_EXT_SYMMETRIC = 0 };
/* status codes */
enum {
  DWT2_OK = 0,
  DWT2_ERR_ARG = -1,       /* null pointer, pointer not 4-byte aligned,
                              width/height < 2, stride < width, batch < 1,
                              batch stride too small, bad boundary */
  DWT2_ERR_SIZE = -2,      /* levels < 1, a level input below 2 x 2, or a
                              dimension above DWT2_MAX_DIM */
  DWT2_ERR_MODE = -3,      /* unknown mode, or integer mode in dwt2_bwd */
  DWT2_ERR_WORKSPACE = -4, /* workspace smaller than the queried size */
  DWT2_ERR_ALIAS = -5,     /* src, dst and workspace byte ranges overlap */
  DWT2_ERR_HIP = -6,       /* HIP runtime / launch failure (detail in last_error) */
  DWT2_ERR_NOMEM = -7      /* host or plan-cache allocation failed */
};

#define DWT2_MAX_DIM (1 << 28)
#define DWT2_MAX_LEVELS 24

/* Bytes of device workspace that dwt2_fwd / dwt2_inv / dwt2_bwd need for
 * `batch` images of width x height with `levels` levels (0 when one level
 * suffices, since no intermediate LL is stored).  Returns 0 as well for
 * invalid arguments; the transform call then reports the error. */
size_t dwt2_workspace_size(int32_t width, int32_t height, int32_t batch,
                           int32_t levels, int32_t mode);

/* Forward transform (§3, eq. (5), per level; levels chained on LL).
 *   src   image(s): width x height samples, row stride src_stride, image b
 *         at src + b * src_batch_stride (elements).  Read only.
 *   dst   Mallat-packed coefficients, same geometry convention.  Written.
 *   mode  DWT2_F32 (float*) or DWT2_I32_REV (int32_t*).
 *   boundary must be DWT2_EXT_SYMMETRIC.
 *   workspace / workspace_bytes: device scratch of at least
 *         dwt2_workspace_size(...) bytes (may be NULL when that is 0). */
int dwt2_fwd(const void* src, int64_t src_stride, int64_t src_batch_stride,
             void* dst, int64_t dst_stride, int64_t dst_batch_stride,
             int32_t width, int32_t height, int32_t batch, int32_t levels,
             int32_t mode, int32_t boundary, void* workspace,
             size_t workspace_bytes, void* stream);

/* Inverse transform: src holds Mallat-packed coefficients, dst receives the
 * image.  Per level, coarsest first, the eq. (5) steps are undone (update
 * first); the integer mode undoes the composed rounded steps exactly. */
int dwt2_inv(const void* src, int64_t src_stride, int64_t src_batch_stride,
             void* dst, int64_t dst_stride, int64_t dst_batch_stride,
             int32_t width, int32_t height, int32_t batch, int32_t levels,
             int32_t mode, int32_t boundary, void* workspace,
             size_t workspace_bytes, void* stream);

/* Adjoint (transpose) of the float forward transform: src holds a gradient
 * with respect to the packed coefficients, dst receives W^T src, the
 * gradient with respect to the image.  Per level, coarsest first, the
 * transposed spatial update and then the transposed spatial predict are
 * applied with the boundary weights that transpose the symmetric extension.
 * mode must be DWT2_F32 (DWT2_ERR_MODE otherwise). */
int dwt2_bwd(const void* src, int64_t src_stride, int64_t src_batch_stride,
             void* dst, int64_t dst_stride, int64_t dst_batch_stride,
             int32_t width, int32_t height, int32_t batch, int32_t levels,
             int32_t mode, int32_t boundary, void* workspace,
             size_t workspace_bytes, void* stream);

/* Baseline for comparison, not the product path: the same forward
 * transform computed with the separable lifting scheme of §2, eq. (3), that
 * the non-separable scheme of §3, eq. (5), regroups.  Every lifting step of
 * a level (horizontal predict, vertical predict, horizontal update, vertical
 * update, in that order) is its own kernel launch and its own pass over the
 * level in HBM, the last one writing the Mallat layout.  Arguments, layout,
 * ownership and errors are those of dwt2_fwd, except that the workspace
 * must hold dwt2_separable_workspace_size bytes (it adds one work array of
 * the image's size per image).  Integer results are identical to
 * dwt2_fwd's; float results agree up to rounding, since eq. (5) regroups the
 * same arithmetic. */
size_t dwt2_separable_workspace_size(int32_t width, int32_t height,
                                     int32_t batch, int32_t levels,
                                     int32_t mode);
int dwt2_fwd_separable(const void* src, int64_t src_stride,
                       int64_t src_batch_stride, void* dst, int64_t dst_stride,
                       int64_t dst_batch_stride, int32_t width, int32_t height,
                       int32_t batch, int32_t levels, int32_t mode,
                       int32_t boundary, void* workspace,
                       size_t workspace_bytes, void* stream);

/* Second baseline for comparison, not the product path: the forward
 * transform with one launch per level in which each 256-thread workgroup
 * copies a 128 x 32-pixel tile of the level input plus a 2-pixel halo
 * (through the symmetric extension) into LDS, lifts it there and stores its
 * 64 x 16 quadruples' coefficients.  Consecutive lifting steps are separated
 * by a workgroup barrier, the GPU form of the paper's synchronisation
 * steps, so the two schemes differ only in their step count:
 *   scheme DWT2_SCHEME_SEPARABLE:    horizontal predict, vertical predict,
 *       horizontal update, vertical update (§2, eq. (3)): four steps;
 *   scheme DWT2_SCHEME_NONSEPARABLE: spatial predict, spatial update (§3,
 *       eq. (5)): two steps;
 *   scheme DWT2_SCHEME_ADAPTED: the adapted non-separable scheme of §3, float
 *       only: each filter split into its constant term and the rest
 *       (P = P0 + P1, U = U0 + U1); the constant terms, which touch only a
 *       quadruple's own samples, run separably without an exchange, so the
 *       two steps need fewer operations.
 * Arguments, layout, ownership and errors are those of dwt2_fwd, with the
 * workspace of dwt2_workspace_size; an unknown scheme is DWT2_ERR_ARG, an
 * integer mode with the adapted scheme DWT2_ERR_MODE.  Integer results equal
 * dwt2_fwd's for both other schemes.  Float results of the non-separable
 * scheme equal dwt2_fwd's bit for bit; those of the separable scheme equal
 * dwt2_fwd_separable's bit for bit; those of the adapted scheme agree with
 * both up to rounding. */
enum { DWT2_SCHEME_SEPARABLE = 0, DWT2_SCHEME_NONSEPARABLE = 1, DWT2_SCHEME_ADAPTED = 2 };
int dwt2_fwd_lds(const void* src, int64_t src_stride, int64_t src_batch_stride,
                 void* dst, int64_t dst_stride, int64_t dst_batch_stride,
                 int32_t width, int32_t height, int32_t batch, int32_t levels,
                 int32_t mode, int32_t boundary, int32_t scheme,
                 void* workspace, size_t workspace_bytes, void* stream);

/* CDF 9/7 (float32 only), computed with the non-separable scheme: the
 * wavelet's two lifting pairs (§2, eq. (2)) are treated in turn, each as a
 * spatial predict and a spatial update (§3, eq. (5)), and the quadrants are
 * then scaled.  The paper prints no 9/7 coefficients, so these are the
 * Daubechies-Sweldens lifting factorisation with JPEG 2000's normalisation
 * of the irreversible transform (lowpass gain 1 at DC, highpass gain 2 at
 * Nyquist): predict -1.586134342059924, update -0.052980118572961, predict
 * 0.882911075530934, update 0.443506852043971, then L / K and H * K with
 * K = 1.230174104914001.  Boundary, Mallat layout, level rule, arguments,
 * ownership and errors are those of dwt2_fwd / dwt2_inv, with the workspace
 * of dwt2_workspace_size.  mode must be DWT2_F32 (DWT2_ERR_MODE otherwise).
 * One launch per level; each workgroup lifts a tile of 64 x 16 quadruples
 * in LDS (two quadruples of halo), with a barrier between the four spatial
 * steps. */
int dwt2_fwd_cdf97(const void* src, int64_t src_stride, int64_t src_batch_stride,
                   void* dst, int64_t dst_stride, int64_t dst_batch_stride,
                   int32_t width, int32_t height, int32_t batch, int32_t levels,
                   int32_t mode, int32_t boundary, void* workspace,
                   size_t workspace_bytes, void* stream);
/* Baseline for comparison, not the product path: the same CDF 9/7 forward
 * with the separable lifting of §2, eq. (3), applied to each pair in turn:
 * horizontal predict, vertical predict, horizontal update, vertical update,
 * that is eight steps per level instead of the non-separable scheme's four.
 * It uses the same tiles and workgroups as dwt2_fwd_cdf97, lifting each
 * tile in place in LDS with a barrier between steps, so the two differ in
 * their step count.  Arguments, layout, ownership and errors are those of
 * dwt2_fwd_cdf97; results agree with it up to rounding. */
int dwt2_fwd_cdf97_separable(const void* src, int64_t src_stride,
                             int64_t src_batch_stride, void* dst,
                             int64_t dst_stride, int64_t dst_batch_stride,
                             int32_t width, int32_t height, int32_t batch,
                             int32_t levels, int32_t mode, int32_t boundary,
                             void* workspace, size_t workspace_bytes,
                             void* stream);
/* Inverse of dwt2_fwd_cdf97: src = Mallat-packed 9/7 coefficients, dst =
 * image. */
int dwt2_inv_cdf97(const void* src, int64_t src_stride, int64_t src_batch_stride,
                   void* dst, int64_t dst_stride, int64_t dst_batch_stride,
                   int32_t width, int32_t height, int32_t batch, int32_t levels,
                   int32_t mode, int32_t boundary, void* workspace,
                   size_t workspace_bytes, void* stream);

/* One image of a ragged batch (all pointers device pointers). */
typedef struct {
  const void* src;
  void* dst;
  int64_t src_stride;
  int64_t dst_stride;
  int32_t width;
  int32_t height;
} dwt2_image_t;

/* Workspace bytes for dwt2_fwd_batched over this list of images.  Only the
 * width and height of each entry are read; returns 0 if n < 1, levels or
 * mode are invalid, or an image is too small for the levels. */
size_t dwt2_batched_workspace_size(const dwt2_image_t* images, int32_t n,
                                   int32_t levels, int32_t mode);

/* Forward transform of n images of unequal sizes (Mallat recursion of §2
 * with the spatial steps of §3, eq. (5), per image), replayed from a HIP
 * graph that is cached per shape set and workspace.
 *   images  HOST array of n descriptors; every image is validated like a
 *           dwt2_fwd call (the detail string names the failing image).
 * The work items (image, level, strip, segment) of all images run under one
 * of three schedules, picked per shape set by timing them on the first call:
 * one cooperative persistent launch in which an item waits only for the
 * rows of the previous level of its own image; one launch per level over
 * every image; or the same with levels 1 and 2 of every image in one launch
 * of the two-level kernels (when levels >= 2 and every image is at least
 * 8 x 8).  The environment variables DWT2_BATCH_SCHEDULE (0 persistent,
 * 1 per level, 2 with the two-level launch; DWT2_ERR_ARG when it does not
 * apply) and DWT2_BATCH_SEG (level-1 segment height) force a policy, and
 * DWT2_TUNE_CACHE names a file that keeps tuning results.
 * Results are bit-identical to n separate dwt2_fwd calls under every
 * policy.  The first call for a new shape set builds the plan (tuning,
 * schedule, graph); later calls with the same shapes and workspace only
 * rewrite the descriptor table in pinned staging memory and launch the
 * graph on `stream`.  Batched calls are not capture-safe: the graph copies
 * the staging memory when it runs, and the next eager call rewrites it.
 * The library keeps at most 16 plans and evicts the least recently used
 * one; reusing one workspace per shape set avoids rebuilding plans.  Calls
 * sharing a workspace must be stream-ordered. */
int dwt2_fwd_batched(const dwt2_image_t* images, int32_t n, int32_t levels,
                     int32_t mode, int32_t boundary, void* workspace,
                     size_t workspace_bytes, void* stream);

/* Inverse (dwt2_inv per image: src = packed coefficients, dst = image) and
 * adjoint (dwt2_bwd per image, DWT2_F32 only: src = coefficient gradient,
 * dst = image gradient) of a ragged set, with the plans, schedules, tuning,
 * workspace (dwt2_batched_workspace_size) and rules of dwt2_fwd_batched;
 * levels run coarsest first.  Results are bit-identical to the per-image
 * calls.  dwt2_bwd_batched returns DWT2_ERR_MODE for integer mode. */
int dwt2_inv_batched(const dwt2_image_t* images, int32_t n, int32_t levels,
                     int32_t mode, int32_t boundary, void* workspace,
                     size_t workspace_bytes, void* stream);
int dwt2_bwd_batched(const dwt2_image_t* images, int32_t n, int32_t levels,
                     int32_t mode, int32_t boundary, void* workspace,
                     size_t workspace_bytes, void* stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): dwt2_fwd with the
 * workspace taken from a device array the library holds (96 MiB per GPU it
 * runs on, kept until the process ends; enough for one 8192 x 8192 image at
 * six levels) instead of a caller's buffer.  Arguments other than the
 * workspace, layout, ownership, results and errors are those of dwt2_fwd;
 * a call whose dwt2_workspace_size exceeds 96 MiB returns
 * DWT2_ERR_WORKSPACE.  It always runs the per-level path (path 0 of
 * dwt2_set_path), allocates nothing and issues no memset.  Every call on a
 * GPU shares that GPU's array: calls that overlap in time on one GPU (two
 * streams, two threads) race and must be serialised by the caller. */
int dwt2_fwd_noalloc(const void* src, int64_t src_stride, int64_t src_batch_stride,
                     void* dst, int64_t dst_stride, int64_t dst_batch_stride,
                     int32_t width, int32_t height, int32_t batch, int32_t levels,
                     int32_t mode, int32_t boundary, void* stream);

/* Process-wide tiling override, for tuning sweeps and tests: seg = quadruple
 * rows per work item (0 = automatic), chunk = quadruple rows per prefetch
 * chunk (1, 2 or 4; 0 = automatic).  Results are bit-identical for every
 * setting; only speed changes.  Must not race with running calls.
 * Returns DWT2_OK, or DWT2_ERR_ARG for values outside those ranges. */
int dwt2_set_tiling(int32_t seg, int32_t chunk);

/* Per-shape tuning of the work-item height of the per-level path (a
 * performance aid; results never change).  Runs the call that dwt2_fwd
 * (dir 0), dwt2_inv (dir 1), dwt2_bwd (dir 2), dwt2_fwd_cdf97 (dir 3) or
 * dwt2_inv_cdf97 (dir 4) would run with these arguments -- same meaning,
 * layout, validation and errors -- several times: for each single-level or
 * pair launch of the current path (for the CDF 9/7: each level that runs in
 * a strip kernel), in execution order, it times that launch (events on
 * `stream`) at a few candidate heights and records the fastest for the
 * launch's shape (launch kind, direction, mode, level input size, batch)
 * when it beats the automatic choice by more than 2 %.  Later calls of any entry point
 * on the per-level path that launch the same shape use the recorded
 * height, unless dwt2_set_tiling forces one.  dst and the workspace are
 * overwritten (dst ends holding the call's result); src is only read.
 * Blocks the host until the timed calls finish; not capturable into a
 * graph; must not race with other calls.  Does nothing more than one call
 * when a tiling is forced or the persistent path is selected.  Returns
 * DWT2_OK or the status of the first failing call (DWT2_ERR_ARG also for
 * dir outside 0..4, DWT2_ERR_HIP for event failures). */
int dwt2_tune(int32_t dir, const void* src, int64_t src_stride, int64_t src_batch_stride,
              void* dst, int64_t dst_stride, int64_t dst_batch_stride,
              int32_t width, int32_t height, int32_t batch, int32_t levels,
              int32_t mode, int32_t boundary, void* workspace, size_t workspace_bytes,
              void* stream);

/* Number of launch shapes with a recorded height (dwt2_tune). */
int32_t dwt2_tune_entries(void);

/* Forgets every recorded height; always DWT2_OK.  Must not race with
 * running calls. */
int dwt2_tune_clear(void);

/* Process-wide choice of how levels are chained, for tests and
 * measurements.  The building blocks: single-level launches; pair launches
 * (levels k and k+1 in one launch that keeps LL_k on chip, from the finest
 * level, where the level-k input is at least 8 x 8); and the fused coarsest
 * levels (the 2-3 coarsest levels -- at most 2 for dwt2_inv -- when their
 * inputs hold at most
 * 1024 x 1024 pixels over the batch, in one launch in which each workgroup
 * runs them in LDS on its tile plus a recompute halo; the inverse also
 * needs the coarsest input at least 4 x 4).
 *   0 (default): pairs for dwt2_inv and dwt2_bwd, and for dwt2_fwd where
 *     the pair's strips (112 quadruple columns each) would be at least 60 %
 *     filled by the level-k input's ceil(w/2) quadruple columns or the
 *     level-k input holds at most 2 x 1024 x 1024 pixels over the batch, single
 *     levels elsewhere, and the fused coarsest levels only where they take
 *     fewer launches than pairs and single levels (what measured fastest
 *     on MI355X);
 *   1: every level of a call in one cooperative persistent launch whose
 *     work items wait only for the rows they read;
 *   2: one launch per level throughout;
 *   3: pairs in every direction, then the fused coarsest levels;
 *   4: pairs in every direction, single levels where no pair applies, no
 *     fused coarsest levels;
 *   5: single levels in every direction, then the fused coarsest levels.
 * Results are bit-identical.  Returns DWT2_OK or DWT2_ERR_ARG. */
int dwt2_set_path(int32_t path);

/* Process-wide timing probe, a measurement aid: while set, every
 * dwt2_fwd (dir 0), dwt2_inv (dir 1) or dwt2_bwd (dir 2) call on the
 * per-level path records ev_begin on its stream just before the launch of
 * level `level` (1 = finest) and ev_end just after it, so hipEventElapsedTime
 * of the pair is that one kernel's duration.  ev_begin / ev_end are
 * hipEvent_t handles owned by the caller, created on the device of the
 * calls.  A probe on any level of a launch that covers several levels
 * (see dwt2_launch_levels) records around that launch; the persistent path
 * has no per-level launches and records nothing.  dir < 0 clears the probe.  Must not race with running calls.
 * Returns DWT2_OK, or DWT2_ERR_ARG for a dir above 2, a level outside
 * 1..DWT2_MAX_LEVELS or a null event. */
int dwt2_set_probe(int32_t dir, int32_t level, void* ev_begin, void* ev_end);

/* Persistent-launch wait settings, for tests of the failure path: every
 * later persistent launch (path 1 of dwt2_set_path, and batched plans built
 * afterwards with the persistent schedule) gives a dependency wait at most
 * max_polls polls (0 = the default budget, about 2 s), and with
 * unreachable = 1 every wait asks for one completion more than can happen,
 * so each one runs out its budget.  A wait that gives up never hangs the
 * GPU: its work item skips its arithmetic, the launch finishes, and the
 * library records the failure for the device (see dwt2_synchronize).  Must
 * not race with running calls.  Returns DWT2_OK, or DWT2_ERR_ARG for
 * max_polls < 0 or unreachable other than 0 or 1. */
int dwt2_set_job_wait(int32_t max_polls, int32_t unreachable);

/* Waits for the work on `stream` (a hipStream_t as void*, NULL = the null
 * stream) and reports failures that surfaced while it ran: DWT2_ERR_HIP if
 * the synchronisation fails, or if a persistent launch on the current
 * device gave up a dependency wait since the last report (its results are
 * then invalid); DWT2_OK otherwise.  Such a give-up is also reported, once,
 * by the next transform call on the device (dwt2_fwd ... dwt2_bwd_batched),
 * which then returns DWT2_ERR_HIP without running. */
int dwt2_synchronize(void* stream);

/* Measurement aid: the launches a plain call of this geometry makes on the
 * current path (dwt2_set_path), in execution order.  dir: 0 dwt2_fwd,
 * 1 dwt2_inv, 2 dwt2_bwd.  Launch i covers levels first[i] .. last[i]
 * (1 = finest); a probe (dwt2_set_probe) on any of those levels times that
 * launch.  first / last are HOST arrays of `cap` entries (may be NULL with
 * cap 0).  Returns the number of launches (>= 1), or DWT2_ERR_ARG /
 * DWT2_ERR_SIZE for an invalid geometry, batch or dir. */
int32_t dwt2_launch_levels(int32_t width, int32_t height, int32_t batch,
                           int32_t levels, int32_t dir, int32_t* first,
                           int32_t* last, int32_t cap);

/* Static description of a status code. */
const char* dwt2_status_string(int status);
/* Thread-local detail of the last failing call on this thread ("" if none). */
const char* dwt2_last_error(void);
/* Releases every cached batched plan (graphs, device tables, pinned staging).
 * Must not race with dwt2_fwd_batched calls. */
void dwt2_clear_plan_cache(void);
/* Number of batched plans currently cached (at most 16). */
int32_t dwt2_plan_cache_size(void);

#ifdef __cplusplus
}
#endif

#endif /* DWT2_H */
