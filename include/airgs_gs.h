/*
 * airgs_gs.h -- C ABI of the MI355X (gfx950) Gaussian-splatting rasterizer.
 *
 * The library renders one frame of a dynamic Gaussian scene and
 * differentiates it.  A frame is an anchor Gaussian set plus an accumulated,
 * pruned attribute delta (AirGS, Eq. (2), Eq. (5), Eq. (12)); attribute
 * deltas travel as multi-channel 2D images with one texel per Gaussian
 * (Eq. (3), Sec. III-C); each Gaussian carries mean, opacity, colour as
 * spherical harmonics, rotation and scale (Sec. II).  The renderer itself is
 * the differentiable splatting rasterizer the paper cites in Sec. II: EWA
 * projection, 16x16-tile binning, a depth-ordered front-to-back composite,
 * and its backward pass.  Around it sit the terms the paper trains and
 * delivers with: the Eq. (1) loss, Adam, usage counts for pruning, the
 * temporal and keyframe terms, low-opacity culling, and the bookkeeping and
 * quantisation of sent updates.
 *
 * Conventions shared by every call
 *   - All array pointers are DEVICE pointers unless a parameter says "host".
 *   - The caller owns every buffer.  The library keeps no pointer after a
 *     call returns, except that enqueued kernels read and write them on the
 *     given stream until they complete.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream).
 *     Only gs_bin_sort and gs_cull_low_opacity block the host (they read a
 *     count back through the context's pinned slot).
 *   - Argument checks are synchronous; a failed check returns an error code
 *     and enqueues nothing.  Kernel faults surface at the next synchronising
 *     HIP call.  gs_last_error() returns the text of the latest error.
 *   - No C++ exception crosses this boundary.
 *   - One gs_ctx per host thread; calls on one context are not reentrant.
 *   - Parameters are FP32 structure-of-arrays planes with a common plane
 *     stride `ld` (>= n, a multiple of 64); Gaussian i of plane k of a
 *     (P, ld) array is element k*ld + i.
 */
#ifndef AIRGS_GS_H
#define AIRGS_GS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gs_status;
#define GS_OK 0
#define GS_ERR_INVALID_ARG 1 /* null pointer, bad size, bad degree, bad stride */
#define GS_ERR_CAPACITY 2    /* instance buffers too small; count holds the need */
#define GS_ERR_OOM 3         /* workspace smaller than the *_workspace_size() */
#define GS_ERR_HIP 4         /* a HIP runtime call failed */

/* Every `workspace` argument is device memory aligned to 256 bytes (as
 * hipMalloc returns it); a misaligned one is GS_ERR_INVALID_ARG. */

#define GS_TILE 16           /* tile side in pixels */
#define GS_MAX_SH_DEGREE 3
/* Largest instance capacity and largest n_views * ld that gs_bin_sort takes:
 * the binning's instance indices, offsets and counts are 32-bit, and this
 * bound keeps them and the sums formed from them clear of overflow. */
#define GS_MAX_INSTANCES (((int64_t)1 << 30) - 1)

typedef struct gs_ctx gs_ctx;

/* Gaussian set, FP32 planes of stride ld:
 *   mean (3, ld); log_scale (3, ld) (scale = exp); quat (4, ld) as (w, x, y, z),
 *   any nonzero norm; opacity (ld) as a logit (opacity = sigmoid);
 *   sh (K, 3, ld), K = (sh_degree + 1)^2, coefficient index l*l + l + m.
 * As a gradient set (gs_render_bwd output) the same planes hold dL/d(.). */
typedef struct gs_gaussians {
  int32_t n;
  int32_t sh_degree;
  int32_t ld;
  int32_t reserved;
  float* mean;
  float* log_scale;
  float* quat;
  float* opacity;
  float* sh;
} gs_gaussians;

/* Pinhole camera: x_cam = R * x_world + t (R row-major, OpenCV frame: x
 * right, y down, z forward); pixel (u, v) samples the image plane at integer
 * coordinates, u = fx * x/z + cx.  144 bytes, FP64. */
typedef struct gs_camera {
  double R[9];
  double t[3];
  double fx, fy, cx, cy;
  int32_t width, height;
  int32_t reserved[2];
} gs_camera;

/* Render options: background colour added with the final transmittance;
 * usage (device, n uint32, nullable): when set, gs_render_fwd ADDS to
 * usage[i] the number of (view, pixel) pairs that composite Gaussian i --
 * the rendering usage frequency by which the paper prunes updates
 * (Sec. III-C).  Ignored by gs_render_fwd_batched and gs_render_bwd.
 * grad2d_norm, visible_views (device, n, nullable, used by gs_render_bwd):
 * densification statistics for keyframe reconstruction (Sec. III-B, cloning
 * and splitting where gradients are high): gs_render_bwd ADDS, per
 * Gaussian, the sum over the views where it is visible of the Euclidean
 * norm of dL/d(screen mean) in pixels, and the number of those views. */
typedef struct gs_opts {
  float bg[3];
  float reserved;
  uint32_t* usage;
  float* grad2d_norm;
  uint32_t* visible_views;
} gs_opts;

/* Per (view, Gaussian) projection records, index v*ld + i:
 *   splat (V, ld, 16) FP32 words, 64 B per record:
 *       [px, py, A, B, C, opacity, r, g, b, depth, Q, 0, o, w, e, s]
 *       screen mean, conic (power = -(A dx^2 + C dy^2)/2 - B dx dy), opacity
 *       sigmoid(logit), clamped SH colour, camera-space depth, and the conic
 *       determinant Q = A C - B^2 (from FP64, used for cancellation-free
 *       evaluation of the quadratic form); words 12..15 are uint32 bit
 *       patterns: o = tx0 | ty0 << 16 and w = tx1 - tx0 of the tile rectangle
 *       (written by gs_project; w has bit 31 set when the record carries
 *       tile spans, see GS_PROJECT_TILE_SPANS), e = the first instance of
 *       the pair in the binning's emission order (written by gs_bin_sort,
 *       read by gs_render_bwd), s = the tile spans or 0;
 *   rect (V, ld, 4) int32: tile rectangle [tx0, ty0, tx1, ty1), all 0 if culled;
 *       with GS_PROJECT_TIGHT_RECT in `options` it is narrowed to the tiles
 *       that meet the bounding box of the ellipse where alpha could reach
 *       1/255 (with the quadrant test's margin): the lists then hold fewer
 *       instances, every one dropped is skipped by every pixel of its tile,
 *       so images and final_T are unchanged and n_contrib counts positions
 *       in the shorter lists; a Gaussian whose opacity cannot reach 1/255
 *       anywhere gets no tiles;
 *       with GS_PROJECT_TILE_SPANS (which implies the narrowed rectangle),
 *       a pair whose rectangle is at most 4 tile rows tall and 15 tiles wide
 *       keeps, in each tile row r, only the columns [tx0 + a_r, tx0 + b_r)
 *       whose 16x16 pixel box meets that ellipse (computed exactly per row
 *       band, with 1e-3 px of slack); byte r of record word 15 is
 *       a_r | b_r << 4 (0 for an empty row), and the same reasoning keeps
 *       images and final_T unchanged;
 *   tiles_touched (V, ld) int32: the pair's instance count: (tx1 - tx0) *
 *       (ty1 - ty0), or the sum of its spans, 0 if culled;
 *   depth_bits (V, ld) uint32: bits of FP32(z);
 *   flags (V, ld) uint8: 1,2,4 colour channel clamped at 0; 8, 16 guard band
 *       clamp of x/z, y/z; 32 visible. */
#define GS_PROJECT_TIGHT_RECT 1  /* gs_projected.options: opacity-aware rectangles */
#define GS_PROJECT_TILE_SPANS 2  /* gs_projected.options: ... and per-row tile spans */

typedef struct gs_projected {
  int32_t n_views;
  int32_t n;       /* Gaussians per view (records i >= n are never read) */
  int32_t ld;
  int32_t options; /* 0 or GS_PROJECT_TIGHT_RECT | GS_PROJECT_TILE_SPANS
                      (read by gs_project) */
  float* splat;
  int32_t* rect;
  int32_t* tiles_touched;
  uint32_t* depth_bits;
  uint8_t* flags;
} gs_projected;

/* Sorted tile lists.  Views are concatenated: view v's tiles are segments
 * seg_base(v) .. seg_base(v) + TX_v*TY_v - 1 in row-major tile order, with
 * seg_base(v) the sum of the tile counts of the views before it.
 *   keys (capacity) uint64, optional (NULL = not written):
 *       (segment << 32) | depth_bits, ascending;
 *   vals (capacity) uint32: Gaussian id of each instance, in key order, ties
 *       (equal segment and depth) in ascending id;
 *   ranges (n_segments, 2) uint32: [start, end) of each segment in vals;
 *   gv_base (gv_capacity >= n_views * ld) uint32, optional (NULL = not
 *       written): for each (view v, Gaussian i) with tiles_touched > 0, at
 *       v*ld + i, the index of its first instance in the binning's emission
 *       order (its tiles row by row over its tile rectangle or its spans,
 *       consecutive).
 *       The same index is always written to word 14 of the pair's projected
 *       record, where gs_render_bwd reads it: the backward writes one
 *       gradient row per instance in that order and sums each pair's rows
 *       without atomics.
 * capacity (in) bounds the instance count; count (out) is the instance count
 * M; n_segments (out) is the total tile count. */
typedef struct gs_tile_lists {
  int64_t capacity;
  int64_t count;
  int64_t n_segments;
  uint64_t* keys;
  uint32_t* vals;
  uint32_t* ranges;
  int64_t gv_capacity;
  uint32_t* gv_base;
} gs_tile_lists;

/* Frame update for the backward pass to the delta images.
 * temporal_weight: lambda_t of Eq. (7); when nonzero the temporal term of
 *   Eq. (6), lambda_t * sum_{i<n} |delta_i - e| over the 8 channels with e =
 *   (0,0,0,1,0,0,0,0) the no-motion update, is fused into the delta gradient
 *   (ADDED: lambda_t * sign(delta - e), sign(0) = 0, at every texel i < n
 *   whatever its mask) and its value ACCUMULATED in FP64 into *temporal_loss
 *   (device, nullable).  delta (8, gh, gw) is then required. */
typedef struct gs_frame_update {
  const float* anchor_quat; /* (4, ld) anchor quaternions */
  int32_t ld;
  int32_t gw, gh;           /* texel grid, gw * gh >= n */
  float temporal_weight;
  const uint8_t* mask;      /* (gh, gw), 1 = the texel's update was applied */
  const float* delta;       /* (8, gh, gw), read when temporal_weight != 0 */
  double* temporal_loss;
} gs_frame_update;

/* ---- support ------------------------------------------------------------ */

int gs_version(void);

/* Create a context bound to HIP device `device` (allocates a small pinned
 * host buffer for the instance-count readback).  *out is NULL on failure. */
gs_status gs_create(gs_ctx** out, int device);
void gs_destroy(gs_ctx* ctx);

/* Text of the last error on this context (static storage if ctx is NULL). */
const char* gs_last_error(const gs_ctx* ctx);

/* Total number of tile segments of n_views host cameras. */
int64_t gs_num_segments(const gs_camera* cams_host, int n_views);

/* Workspace bytes for gs_bin_sort with the given views, stride, instance
 * capacity and total segment count; 0 when an argument is out of range
 * (capacity or n_views * ld above GS_MAX_INSTANCES, or n_segments >= 2^31). */
size_t gs_bin_sort_workspace_size(int n_views, int ld, int64_t capacity, int64_t n_segments);

/* Workspace bytes for gs_render_bwd over lists of `instances` entries.  Its
 * first n_views*ld*12 floats hold the per-(view, Gaussian) screen-space
 * gradients after the call (entries i < n):
 * [d px, d py, d A, d B, d C, d opacity, d r, d g, d b, 0, 0, 0]; then one
 * 9-float gradient row per instance. */
size_t gs_render_bwd_workspace_size(int n_views, int ld, int64_t instances);

/* Device-time measurement.  With timing enabled, every kernel stage a call
 * enqueues is bracketed by HIP events on the call's stream.  Stages:
 *   0 apply, 1 project, 2 depth sort, 3 count scan, 4 emit, 5 segment sort,
 *   6 ranges, 7 render fwd, 8 render bwd, 9 project bwd, 10 apply bwd,
 *   11 l1, 12 adam, 13 fill, 14 dssim, 15 compact (culling, gathers),
 *   16 residual (bookkeeping, quantisation, quantised apply), 17 grad gather
 *   (per-Gaussian sums of the backward's instance rows). */
#define GS_STAGE_COUNT 18
gs_status gs_set_timing(gs_ctx* ctx, int enable);
/* Timing of the stages whose bit (1 << stage) is set only (0 = off): each
 * pair of event records adds device-side gaps, so a timed region can bracket
 * just the stages it needs. */
gs_status gs_set_timing_mask(gs_ctx* ctx, uint32_t stage_mask);
/* Sum of event-measured milliseconds and number of launches per stage since
 * the previous collection (host arrays of GS_STAGE_COUNT); blocks until the
 * recorded events have completed, then resets the counters. */
gs_status gs_collect_timing(gs_ctx* ctx, double* ms, int64_t* launches);
const char* gs_stage_name(int stage);

/* Work counting for roofline accounting.  With `counters` non-NULL (a device
 * array of GS_WORK_COUNTERS uint64 values that the caller zeroes and owns),
 * the compositing calls gs_render_fwd, gs_render_fwd_l1 and gs_render_bwd
 * on this context launch counting instances of their kernels: the same
 * arithmetic and the same per-entry decisions, plus per-tile tallies added
 * to the array at each tile's end.  A wave evaluates one "slot" (an 8x8
 * pixel quadrant of its 16x16 tile, one pixel per lane) per (entry, slot)
 * pair it does not skip, so 64 x slots is the number of (pixel, entry)
 * pairs it executes.  Counters:
 *   0 fwd entries staged, 1 fwd entries visited (some slot evaluated),
 *   2 fwd slot evaluations, 3 fwd pairs with T > 0 and alpha >= 1/255,
 *   4 bwd entries staged, 5 bwd entries visited, 6 bwd slot evaluations,
 *   7 bwd pairs inside the pixel's list prefix with alpha >= 1/255.
 * The counting kernels are slower (one 64-bit atomic per counter per tile)
 * and are meant for runs outside any timed region.  NULL switches counting
 * off.  Other calls ignore the setting. */
#define GS_WORK_COUNTERS 8
gs_status gs_set_work_counters(gs_ctx* ctx, uint64_t* counters);

/* Peak-rate probes for the roofline (measurement support, not the hot
 * path).  Runs one launch of probe `kind` on `stream`, waits for it, and
 * returns its event-timed duration in *ms and its work in *work:
 *   GS_PEAK_COPY      device copy of the first half of `buf` into the second
 *                     half; work = bytes read + written;
 *   GS_PEAK_READ      read of `buf` (its tail holds 4 MiB of per-thread
 *                     sums); work = bytes read;
 *   GS_PEAK_LDS       `iters` sweeps over 64 KB of LDS per workgroup, 16-byte
 *                     conflict-free reads; work = LDS bytes read;
 *   GS_PEAK_FMA       16 independent FP32 FMA chains per lane, `iters`
 *                     rounds; work = FLOP (an FMA counted as 2);
 *   GS_PEAK_EXP       8 independent exp2 chains per lane; work = exp2 count;
 *   GS_PEAK_ATOMIC_SPREAD / GS_PEAK_ATOMIC_SAME
 *                     float atomic adds without return, `iters` per thread,
 *                     each thread on its own address / on one of 64
 *                     addresses; work = atomics (buf receives the sums).
 * 1,048,576 threads (4,096 workgroups of 256) in every probe.  `buf` is
 * device memory of `bytes` bytes, at least gs_peak_min_bytes(kind); its
 * contents are overwritten.  GS_ERR_INVALID_ARG for an unknown kind, a
 * short buffer or iters < 1. */
#define GS_PEAK_COPY 0
#define GS_PEAK_READ 1
#define GS_PEAK_LDS 2
#define GS_PEAK_FMA 3
#define GS_PEAK_EXP 4
#define GS_PEAK_ATOMIC_SPREAD 5
#define GS_PEAK_ATOMIC_SAME 6
size_t gs_peak_min_bytes(int kind);
gs_status gs_peak_run(gs_ctx* ctx, int kind, void* buf, size_t bytes, int iters, double* ms,
                      double* work, void* stream);

/* ---- hot path ----------------------------------------------------------- */

/* Apply a decoded frame update to anchor Gaussians (Eq. (2)/(5)/(12): frame
 * = anchor + accumulated delta; Eq. (3): one texel per Gaussian; Eq. (11):
 * the pruning mask drops updates).  delta (8, gh, gw) FP32 planar channels
 * [dx, dy, dz, dq_w, dq_x, dq_y, dq_z, d_opacity_logit]; Gaussian i reads
 * texel (i / gw, i % gw); requires gw * gh >= anchor->n.  Where mask = 1:
 * mean' = mean + d_mu, quat' = dq (x) quat (Hamilton product), logit' =
 * logit + d_o; elsewhere the anchor values are copied.  Each result is
 * computed in FP64 and rounded once to FP32.  Writes frame->mean, quat,
 * opacity only (its log_scale and sh may alias the anchor's planes). */
gs_status gs_apply_frame_update(gs_ctx* ctx, const gs_gaussians* anchor, const float* delta,
                                const uint8_t* mask, int gw, int gh, gs_gaussians* frame,
                                void* stream);

/* EWA projection (Sec. II renderer): camera transform, near cull (z <= 0.2,
 * a fixed plane: the paper names none),
 * 3D covariance R_q diag(exp s)^2 R_q^T, 2D covariance J W Sigma W^T J^T
 * with a 1.3x guard band on J and +0.3 px^2 dilation, conic, screen mean,
 * radius ceil(3 sqrt(lambda_max)) (eigenvalue floor 0.1), 16x16 tile
 * rectangle, SH colour + 0.5 clamped at 0, sigmoid opacity, depth.  The
 * binning quantities (depth, radius, rectangle) are computed in FP64.
 * cams_host and cams_dev hold the same n_views cameras (host copy for
 * validation and launch sizes, device copy for the kernels). */
gs_status gs_project(gs_ctx* ctx, const gs_gaussians* g, const gs_camera* cams_host,
                     const gs_camera* cams_dev, int n_views, gs_projected* out, void* stream);

/* Binning and depth ordering of the splatting renderer the paper cites in
 * Sec. II (its tile-based rasterizer sorts splats per 16x16 tile by depth):
 * every (visible Gaussian, tile of its
 * rectangle, or of its per-row spans when the record carries them, see
 * GS_PROJECT_TILE_SPANS) pair is an instance; instances are ordered by
 * (segment, FP32 depth, Gaussian id) with LDS-resident radix sorts that
 * run inside each view.  Reads the instance count back to the host
 * (blocking).  Returns GS_ERR_CAPACITY with lists->count = M when
 * M > lists->capacity (nothing else is written).
 * Besides the lists it writes word 14 of each listed record of proj->splat
 * (the pair's first instance in emission order, also stored in
 * lists->gv_base when that is given).
 * workspace must hold gs_bin_sort_workspace_size() bytes. */
gs_status gs_bin_sort(gs_ctx* ctx, const gs_projected* proj, const gs_camera* cams_host,
                      const gs_camera* cams_dev, int n_views, gs_tile_lists* lists,
                      void* workspace, size_t ws_bytes, void* stream);

/* Front-to-back alpha compositing per pixel over its tile's list (the
 * renderer of Sec. II, run for every training view and every delivered
 * view, Sec. IV-B):
 * alpha = min(0.99, opacity * exp(power)); skip if power > 0 or alpha <
 * 1/255; stop before compositing an entry that would take the
 * transmittance below 1e-4.  Views must share width and height.
 * image (V, 3, H, W), final_T (V, H, W), n_contrib (V, H, W) = 1 + index
 * (within the tile list) of the last composited entry, 0 if none. */
gs_status gs_render_fwd(gs_ctx* ctx, const gs_projected* proj, const gs_tile_lists* lists,
                        const gs_camera* cams_host, const gs_camera* cams_dev, int n_views,
                        const gs_opts* opts, float* image, float* final_T, int32_t* n_contrib,
                        void* stream);

/* gs_render_fwd with the L1 term of Eq. (1) evaluated on the composited
 * pixels, as gs_l1_loss_grad would on the written image: with
 * count = n_views * 3 * H * W and d = image - target (target (V, 3, H, W)),
 * dL_dimage = sign(d) / count is WRITTEN (sign(0) = 0) and mean |d| is
 * ACCUMULATED in FP64 into *loss_dev (device; caller zeroes).  image may be
 * NULL (then it is not written); final_T and n_contrib are required.
 * opts->usage must be NULL.  workspace: gs_render_fwd_l1_workspace_size
 * bytes (one FP64 partial sum per tile). */
size_t gs_render_fwd_l1_workspace_size(int n_views, int width, int height);
gs_status gs_render_fwd_l1(gs_ctx* ctx, const gs_projected* proj, const gs_tile_lists* lists,
                           const gs_camera* cams_host, const gs_camera* cams_dev, int n_views,
                           const gs_opts* opts, const float* target, float* image,
                           float* final_T, int32_t* n_contrib, float* dL_dimage,
                           double* loss_dev, void* workspace, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * gs_render_fwd_l1 without the workspace argument, same kernels and results.
 * The per-tile FP64 partial sums live in a fixed device array of
 * GS_NOALLOC_MAX_TILES doubles (2 MiB) that the library holds on each device
 * from gs_create until the process ends; a call whose views have more tiles
 * in total is GS_ERR_INVALID_ARG.  The call allocates nothing (no hipMalloc,
 * no host allocation) and is not timed by gs_set_timing.  Every call on one
 * device shares that array, which keeps the last call's partials (each is
 * written before it is read, so nothing needs clearing): calls that overlap
 * on one device (other streams, contexts or host threads) race and must be
 * serialised by the caller. */
#define GS_NOALLOC_MAX_TILES (1 << 18)
gs_status gs_render_fwd_l1_noalloc(gs_ctx* ctx, const gs_projected* proj,
                                   const gs_tile_lists* lists, const gs_camera* cams_host,
                                   const gs_camera* cams_dev, int n_views, const gs_opts* opts,
                                   const float* target, float* image, float* final_T,
                                   int32_t* n_contrib, float* dL_dimage, double* loss_dev,
                                   void* stream);

/* Batched rendering of n_views requests of (possibly) different sizes in one
 * persistent launch: workgroups take (request, tile) items from a shared
 * device-wide queue until it is drained (view delivery, Sec. IV-B: the
 * client applies the update and renders the frame).  Same compositing as
 * gs_render_fwd.  images: packed FP32 planes, request v's (3, H_v, W_v)
 * image starting at float offset 3 * sum_{u<v} W_u H_u.  final_T and
 * n_contrib are not produced.  workspace: gs_render_batched_workspace_size
 * bytes; the queue state lives there, so concurrent calls need distinct
 * workspaces. */
size_t gs_render_batched_workspace_size(int n_views);
gs_status gs_render_fwd_batched(gs_ctx* ctx, const gs_projected* proj,
                                const gs_tile_lists* lists, const gs_camera* cams_host,
                                const gs_camera* cams_dev, int n_views, const gs_opts* opts,
                                float* images, void* workspace, size_t ws_bytes, void* stream);

/* ---- view server ------------------------------------------------------ */

/* A resident dynamic scene: frame f = anchor + masked delta images f (Eq.
 * (12); one texel per Gaussian, Eq. (3)).  All pointers are device memory
 * owned by the caller and must outlive the server:
 *   deltas (n_frames, 8, gh, gw) FP32 channels as in gs_apply_frame_update,
 *   masks (n_frames, gh, gw) uint8, 1 = apply. */
typedef struct gs_sequence {
  gs_gaussians anchor;
  const float* deltas;
  const uint8_t* masks;
  int32_t n_frames;
  int32_t gw, gh;
  int32_t reserved;
} gs_sequence;

/* One view request: host camera (its width and height are the resolution),
 * frame index, arrival time in seconds after gs_server_run starts. */
typedef struct gs_request {
  gs_camera cam;
  int32_t frame;
  int32_t reserved;
  double arrival_s;
} gs_request;

/* max_batch: requests per batch (1..4096); n_workers: batches in flight
 * (1..16), each on its own host thread, context and stream; options:
 * gs_projected.options of the projections (tile sets); inline_singletons:
 * nonzero lets the scheduler's thread render a lone request itself while
 * the server is idle and arrivals are sparse (mean gap above 2.5 times the
 * render time of a lone request); budget_bytes: device-memory budget for
 * admission (each request is charged an estimate: projected records and
 * sort buffers per Gaussian, 1.5x the observed instances per tile times its
 * tiles, its image; one request is always admitted when nothing is in
 * flight); bg: background colour. */
typedef struct gs_server_config {
  int32_t max_batch;
  int32_t n_workers;
  int32_t options;
  int32_t inline_singletons;
  int64_t budget_bytes;
  float bg[3];
  float reserved;
} gs_server_config;

typedef struct gs_server gs_server;

/* Continuous-batching server (view delivery, Sec. IV-B; the renderer of
 * Sec. II): create it on `device` for `seq` (contexts, streams and pinned
 * camera slots are made here; device buffers grow on demand and are held
 * until gs_server_destroy).  GS_ERR_INVALID_ARG for a bad configuration or
 * sequence; GS_ERR_HIP / GS_ERR_OOM if resources cannot be made. */
gs_status gs_server_create(gs_server** out, int device, const gs_sequence* seq,
                           const gs_server_config* cfg);
void gs_server_destroy(gs_server* server);
const char* gs_server_last_error(const gs_server* server);

/* Serve n requests (host array, arrival_s non-decreasing) in real time on
 * the calling thread's clock, returning when all are done.  plain = 0:
 * continuous batching (requests that arrive while batches are on the device
 * join later batches; batches overlap on the device).  plain = 1: the
 * comparison renderer, one request at a time in arrival order, each with
 * its own apply, projection, binning and compositing launches.  t_start,
 * t_done (host, n): seconds after the start when the request's batch began
 * and when its image was complete (INFINITY if its batch failed).  images
 * (host array of n device pointers, nullable, entries nullable): request
 * i's (3, H, W) image is copied to images[i].  Both modes wait for an
 * arrival by sleeping until 200 us before it and then polling the clock,
 * so the calling thread spins for up to that long per arrival.  Returns
 * the first error of any batch (text via gs_server_last_error); the other
 * requests are still served.  Not reentrant on one server. */
gs_status gs_server_run(gs_server* server, const gs_request* reqs, int n, int plain,
                        double* t_start, double* t_done, float* const* images);

/* Statistics of the last run (host array of 5): batches formed, requests
 * rendered by worker threads, requests rendered inline, largest batch,
 * peak estimated bytes in flight. */
gs_status gs_server_stats(const gs_server* server, int64_t* out);

/* Backward of gs_project + gs_render_fwd for dL/dimage (V, 3, H, W) (the
 * differentiable renderer of Sec. II through which Eq. (1) trains the
 * Gaussians and, with `upd`, the delta images of Eq. (12)):
 * transmittance is recovered by walking each pixel's list back from
 * n_contrib.  proj and lists must be the ones gs_bin_sort last processed
 * together (the backward reads the emission bases that call stores in the
 * projected records).  Gradients w.r.t. the frame's mean, log_scale, quat, opacity
 * logit and SH, summed over views, are WRITTEN to `grad` (same shape as
 * `frame`) for i < n.  If `upd` is non-NULL, dL/d(delta images) (8, gh,
 * gw) is WRITTEN to dL_ddelta (zero at masked and padding texels). */
gs_status gs_render_bwd(gs_ctx* ctx, const gs_gaussians* frame, const gs_projected* proj,
                        const gs_tile_lists* lists, const gs_camera* cams_host,
                        const gs_camera* cams_dev, int n_views, const gs_opts* opts,
                        const float* final_T, const int32_t* n_contrib, const float* dL_dimage,
                        gs_gaussians* grad, const gs_frame_update* upd, float* dL_ddelta,
                        void* workspace, size_t ws_bytes, void* stream);

/* ---- training support ----------------------------------------------------- */

/* L1 photometric term (Eq. (1)): loss = mean |image - target| over count
 * values, ACCUMULATED in FP64 into *loss_dev (device; caller zeroes);
 * grad = sign(image - target) / count (sign(0) = 0) WRITTEN. */
gs_status gs_l1_loss_grad(gs_ctx* ctx, const float* image, const float* target, int64_t count,
                          float* grad, double* loss_dev, void* stream);

/* Full photometric loss of Eq. (1): (1 - lambda) L1 + lambda (1 - SSIM) over
 * `planes` image planes of H x W (V*3 for V RGB views), SSIM with an 11x11
 * Gaussian window (sigma 1.5, weights summing to 1), zero padding, C1 =
 * 0.01^2, C2 = 0.03^2, averaged over all values; lambda = 0.2 in the paper's
 * setting (Sec. IV-A).  The loss is ACCUMULATED in FP64 into *loss_dev
 * (device; caller zeroes); its gradient w.r.t. the image is WRITTEN to grad.
 * workspace: gs_l1_dssim_workspace_size bytes. */
size_t gs_l1_dssim_workspace_size(int planes, int H, int W);
gs_status gs_l1_dssim_loss_grad(gs_ctx* ctx, const float* image, const float* target, int planes,
                                int H, int W, float lambda, float* grad, double* loss_dev,
                                void* workspace, size_t ws_bytes, void* stream);

/* Sum of squared differences over count values, ACCUMULATED in FP64 into
 * *sum_dev (device; caller zeroes).  mean = sum / count gives the MSE behind
 * the PSNR quality measure of the pruning-level sweep (Sec. III-C, Alg. 1). */
gs_status gs_sq_error(gs_ctx* ctx, const float* a, const float* b, int64_t count,
                      double* sum_dev, void* stream);

/* One Adam step (Kingma & Ba 2015, Alg. 1) over count FP32 values, in
 * place, bias-corrected for step number `step` >= 1. */
gs_status gs_adam_step(gs_ctx* ctx, float* param, const float* grad, float* m, float* v,
                       int64_t count, int step, float lr, float beta1, float beta2, float eps,
                       void* stream);

/* ---- keyframe reconstruction (Sec. III-B) ------------------------------- */

/* Keyframe temporal term (Eq. (9) with its weight from Eq. (10)): over
 * `rows` FP32 planes of stride ld (e.g. all parameter planes of a Gaussian
 * set) and their first `bound` columns (the Gaussians carried over from the
 * previous frame, U in the paper), ADDS weight * sign(x - x_prev) (sign(0) =
 * 0) to grad and ACCUMULATES weight * sum |x - x_prev| in FP64 into
 * *loss_dev (device, nullable). */
gs_status gs_keyframe_temporal_l1(gs_ctx* ctx, const float* x, const float* x_prev, int rows,
                                  int bound, int64_t ld, float weight, float* grad,
                                  double* loss_dev, void* stream);

/* Low-opacity culling (Sec. III-B: Gaussians whose opacity falls below a
 * threshold are discarded during keyframe training).  Gaussian i < n is kept
 * iff sigmoid(opacity_logit[i]) >= min_opacity, decided as logit >=
 * log(m / (1 - m)) in FP64.  WRITES the kept indices in increasing order to
 * kept_index (device, capacity n) and their number to *kept_host; blocks
 * until the count has been read back.  workspace: gs_cull_workspace_size(n)
 * bytes.  min_opacity must lie in (0, 1). */
size_t gs_cull_workspace_size(int n);
gs_status gs_cull_low_opacity(gs_ctx* ctx, const float* opacity_logit, int n, float min_opacity,
                              int32_t* kept_index, int32_t* kept_host, void* workspace,
                              size_t ws_bytes, void* stream);

/* dst[p * dst_ld + j] = src[p * src_ld + index[j]] for planes p < `planes`
 * and j < m: applies a kept-index list to parameter planes, gradients or
 * optimizer moments.  Indices must lie in [0, src_ld); dst must not overlap
 * src. */
gs_status gs_gather_planes(gs_ctx* ctx, const float* src, int64_t src_ld, int planes,
                           const int32_t* index, int m, float* dst, int64_t dst_ld,
                           void* stream);

/* ---- sent updates (Sec. III-C, Eq. (11), (12)) --------------------------- */
/* All planes are (8, gh, gw) FP32 delta images as in gs_apply_frame_update;
 * D' starts as the no-motion update (0,0,0,1,0,0,0,0) at every texel. */

/* Eq. (11): d' = mask ? D_t - D'_(t-1) : 0 at texels i < n (0 at padding),
 * WRITTEN to d_out; the per-channel max |d'| over i < n is ACCUMULATED by
 * max into absmax (device, 8 floats; caller zeroes). */
gs_status gs_residual_delta(gs_ctx* ctx, const float* D_t, const float* Dp_prev,
                            const uint8_t* mask, int n, int gw, int gh, float* d_out,
                            float* absmax, void* stream);

/* Symmetric per-channel quantisation of d to signed `bits`-bit codes (bits
 * 8: int8, 16: int16, layout of d): scale_c = absmax_c / (2^(bits-1) - 1)
 * (0 if absmax_c is 0), code = round-half-even(d / scale_c) clamped to
 * +-(2^(bits-1) - 1), 0 at padding texels i >= n.  scale_out (device, 8)
 * WRITTEN.  If Dp is non-NULL, the server-side sum is advanced in place,
 * Dp += code * scale_c (Eq. (12)), with the same FP32 rounding as the
 * client's gs_apply_quantized_update. */
gs_status gs_quantize_delta(gs_ctx* ctx, const float* d, const float* absmax, int bits, int n,
                            int gw, int gh, void* q_out, float* scale_out, float* Dp,
                            void* stream);

/* Client side of Eq. (12): Dp += code * scale at texels i < n (in place),
 * then frame = anchor with Dp applied, as gs_apply_frame_update with every
 * texel kept (mean, quat, opacity of `frame` WRITTEN). */
gs_status gs_apply_quantized_update(gs_ctx* ctx, const gs_gaussians* anchor, const void* q,
                                    int bits, const float* scale, float* Dp, int gw, int gh,
                                    gs_gaussians* frame, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* AIRGS_GS_H */
