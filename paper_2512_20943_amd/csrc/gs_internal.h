// Internal declarations of the HIP rasterizer: constants, the projected
// record layout, and the host-side launchers each kernel file provides.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "airgs_gs.h"

namespace gs {

constexpr int kTile = GS_TILE;
constexpr double kNear = 0.2;       // cull when camera-space z <= kNear
constexpr double kDilate = 0.3;     // screen-space low-pass, px^2
constexpr double kGuard = 1.3;      // guard band on x/z, y/z in the Jacobian
constexpr float kAlphaMax = 0.99f;  // opacity cap per composited entry
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kTStop = 1e-4f;     // stop before T would fall below this

constexpr uint8_t kClampR = 1, kClampG = 2, kClampB = 4, kClampU = 8, kClampV = 16,
                  kVisible = 32;

constexpr int kSplatFloats = 12;    // projected record stride (3 x float4)
constexpr int kGrad2dFloats = 12;   // screen-space gradient record stride
constexpr int kSplatF4 = 4;         // float4s per projected record (64 B)

// Per-row tile spans (GS_PROJECT_TILE_SPANS): a record whose opacity-aware
// rectangle is at most kSpanRows tile rows tall and kSpanWidth tiles wide
// keeps, per tile row r, only the columns [tx0 + a_r, tx0 + b_r) whose pixel
// box meets the ellipse; byte r of record word 15 holds a_r | b_r << 4
// (a_r = b_r = 0 for an empty row) and kSpanFlag is set in word 13.  Its
// instances are emitted row by row over these spans.
constexpr int kSpanRows = 4;
constexpr int kSpanWidth = 15;
constexpr double kSpanEps = 1e-3;   // px of slack on every span edge
constexpr uint32_t kSpanFlag = 0x80000000u;

__host__ __device__ inline int tiles_across(int px) { return (px + kTile - 1) / kTile; }

// ---------------------------------------------------------------- timing
// Stages whose device time the context can measure with HIP events.
enum Stage {
  kStApply = 0, kStProject, kStDepthSort, kStCountScan, kStEmit, kStSegmentSort, kStRanges,
  kStRenderFwd, kStRenderBwd, kStProjectBwd, kStApplyBwd, kStL1, kStAdam, kStFill, kStDssim,
  kStCompact, kStResidual, kStGradGather, kStageCount
};
static_assert(kStageCount == GS_STAGE_COUNT, "stage table out of sync with the header");

struct StageTimer {
  virtual void begin(int stage, hipStream_t s) = 0;
  virtual void end(int stage, hipStream_t s) = 0;
  virtual ~StageTimer() = default;
};
// Active timer of the C ABI call running on this host thread (or null).
extern thread_local StageTimer* g_timer;

// Work counters of the counting render instances (GS_WORK_COUNTERS device
// words, or null: the plain kernels run).
enum WorkCounter {
  kWkFwdStaged = 0, kWkFwdVisits, kWkFwdSlots, kWkFwdUsed, kWkBwdStaged, kWkBwdVisits,
  kWkBwdSlots, kWkBwdUsed, kWorkCount
};
static_assert(kWorkCount == GS_WORK_COUNTERS, "work counter table out of sync with the header");
extern thread_local unsigned long long* g_work;

struct StageScope {
  int stage;
  hipStream_t stream;
  StageScope(int st, hipStream_t s) : stage(st), stream(s) {
    if (g_timer) g_timer->begin(stage, stream);
  }
  ~StageScope() {
    if (g_timer) g_timer->end(stage, stream);
  }
};

// ---------------------------------------------------------------- launchers
// apply
void launch_apply(const gs_gaussians& anchor, const float* delta, const uint8_t* mask, int gw,
                  int gh, gs_gaussians& frame, hipStream_t s);
void launch_apply_bwd(int n, const gs_frame_update& upd, const gs_gaussians& grad,
                      float* dL_ddelta, hipStream_t s);
// project
void launch_project(const gs_gaussians& g, const gs_camera* cams_dev, int n_views,
                    const gs_projected& out, hipStream_t s);
void launch_project_bwd(const gs_gaussians& g, const gs_camera* cams_dev, int n_views,
                        const gs_projected& proj, const float* grad2d, gs_gaussians& grad,
                        float* st_norm, uint32_t* st_views, hipStream_t s);
// sort / binning
struct BinSortPlan {
  int n_views;
  int n;
  int ld;
  int64_t capacity;
  int64_t n_segments;
  int max_tiles;  // most tiles of one view
};
size_t bin_sort_workspace_bytes(int n_views, int ld, int64_t capacity, int64_t n_segments);
// Stage 1 reduces the visible pairs' depth-bit range and instance count
// into 4 device words {min bits, max bits, count (u64)}; the second stage,
// once the host has read them, depth-sorts, emits, sorts by tile and builds
// ranges.
hipError_t bin_sort_stage1(const BinSortPlan& p, const gs_projected& proj,
                           const gs_camera* cams_dev, void* ws, hipStream_t s,
                           uint32_t** d_stats);
hipError_t bin_sort_stage2(const BinSortPlan& p, const gs_projected& proj,
                           const gs_camera* cams_dev, uint32_t M, uint32_t dmin, uint32_t dmax,
                           uint32_t n_visible, gs_tile_lists& lists, void* ws, hipStream_t s);
// render
void launch_render_fwd(const gs_projected& proj, const gs_tile_lists& lists, int n_views, int W,
                       int H, const float bg[3], float* image, float* final_T,
                       int32_t* n_contrib, uint32_t* usage, hipStream_t s);
size_t render_fwd_l1_workspace_bytes(int V, int W, int H);
void launch_render_fwd_l1(const gs_projected& proj, const gs_tile_lists& lists, int V, int W,
                          int H, const float bg[3], const float* target, float* image,
                          float* final_T, int32_t* n_contrib, float* grad, double* loss,
                          void* ws, hipStream_t s);
size_t render_batched_workspace_bytes(int V);
void launch_render_batched(const gs_projected& proj, const gs_tile_lists& lists,
                           const gs_camera* cams_dev, int V, int64_t total_segments,
                           const float bg[3], float* images, void* ws, hipStream_t s);
void launch_render_bwd(const gs_projected& proj, const gs_tile_lists& lists, int V, int W, int H,
                       const float bg[3], const float* final_T, const int32_t* n_contrib,
                       const float* dL_dimage, float* rows, float* grad2d, hipStream_t s);
// training support
void launch_l1(const float* image, const float* target, int64_t count, float* grad,
               double* loss, hipStream_t s);
// low-opacity culling and plane gathers
size_t keep_workspace_bytes(int n);
double opacity_logit_threshold(float min_opacity);
const uint32_t* launch_keep_low_opacity(const float* logit, int n, double thr, int32_t* index,
                                        void* ws, hipStream_t s);
void launch_gather(const float* src, int64_t src_ld, int planes, const int32_t* index, int m,
                   float* dst, int64_t dst_ld, hipStream_t s);
void launch_l1_penalty(const float* x, const float* ref, int rows, int bound, int64_t ld, float w,
                       float* grad, double* loss, hipStream_t s);
// residual bookkeeping and quantised updates
void launch_residual(const float* D, const float* P, const uint8_t* mask, int n, int gw, int gh,
                     float* d, float* absmax, hipStream_t s);
void launch_quantize(const float* d, const float* absmax, int bits, int n, int gw, int gh,
                     void* q, float* scale, float* P, hipStream_t s);
void launch_apply_quantized(const gs_gaussians& a, const void* q, int bits, const float* scale,
                            float* P, int gw, int gh, gs_gaussians& f, hipStream_t s);
size_t l1_dssim_workspace_bytes(int planes, int H, int W);
void launch_l1_dssim(const float* image, const float* target, int planes, int H, int W,
                     float lambda, float* grad, double* loss, void* ws, hipStream_t s);
void launch_sq_error(const float* a, const float* b, int64_t count, double* sum, hipStream_t s);
void launch_adam(float* p, const float* g, float* m, float* v, int64_t count, float lr, float b1,
                 float b2, float eps, float bc1, float bc2, hipStream_t s);
// peak-rate probes
hipError_t launch_peak(int kind, void* buf, size_t bytes, int iters, double* work,
                       hipStream_t s);
size_t peak_min_bytes(int kind, int iters);
void launch_fill_u32(uint32_t* p, uint32_t value, int64_t count, hipStream_t s);
void launch_fill_f32(float* p, float value, int64_t count, hipStream_t s);

}  // namespace gs
