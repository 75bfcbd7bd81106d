// C ABI of the rasterizer: argument validation, workspace accounting and
// kernel launches.  No C++ exception crosses this boundary.
#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cmath>
#include <cstring>
#include <new>

#include <vector>

#include "gs_internal.h"

namespace gs {
thread_local StageTimer* g_timer = nullptr;
thread_local unsigned long long* g_work = nullptr;
}

namespace {

// HIP-event brackets around each stage a call enqueues.
struct EventTimer final : gs::StageTimer {
  struct Rec {
    int stage;
    hipEvent_t a, b;
  };
  std::vector<hipEvent_t> pool;
  std::vector<Rec> recs;
  std::vector<size_t> open;
  uint32_t mask = ~0u;  // stages that are timed

  hipEvent_t take() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  void begin(int stage, hipStream_t s) override {
    if (!(mask >> stage & 1u)) return;
    Rec r{stage, take(), take()};
    if (r.a) hipEventRecord(r.a, s);
    open.push_back(recs.size());
    recs.push_back(r);
  }
  void end(int stage, hipStream_t s) override {
    if (!(mask >> stage & 1u)) return;
    if (open.empty()) return;
    Rec& r = recs[open.back()];
    open.pop_back();
    if (r.b) hipEventRecord(r.b, s);
  }
  hipError_t collect(double* ms, int64_t* launches) {
    for (int k = 0; k < gs::kStageCount; ++k) {
      ms[k] = 0.0;
      launches[k] = 0;
    }
    hipError_t err = hipSuccess;
    for (Rec& r : recs) {
      float t = 0.f;
      if (r.a && r.b) {
        hipError_t e = hipEventSynchronize(r.b);
        if (e == hipSuccess) e = hipEventElapsedTime(&t, r.a, r.b);
        if (e != hipSuccess) err = e;
      }
      ms[r.stage] += t;
      launches[r.stage] += 1;
      if (r.a) pool.push_back(r.a);
      if (r.b) pool.push_back(r.b);
    }
    recs.clear();
    open.clear();
    return err;
  }
  ~EventTimer() override {
    for (Rec& r : recs) {
      if (r.a) hipEventDestroy(r.a);
      if (r.b) hipEventDestroy(r.b);
    }
    for (hipEvent_t e : pool) hipEventDestroy(e);
  }
};

}  // namespace

// Partial sums of gs_render_fwd_l1_noalloc: one FP64 value per tile, in a
// fixed device array that each device holds until the process ends.  In host
// code this name is only a host-side stand-in for the symbol: its device
// address comes from hipGetSymbolAddress (gs_create, per device), and only
// that address is passed to kernels.
static __device__ __align__(256) double scratch[GS_NOALLOC_MAX_TILES];

struct gs_ctx {
  int device;
  uint32_t* pinned;  // host-visible readback slot for the instance count
  bool timing;
  EventTimer timer;
  double* scratch_dev;  // device address of `scratch` on this context's device
  unsigned long long* work;  // GS_WORK_COUNTERS device words, or null
  char err[512];
};

namespace {
// Makes the context's timer and work counters active for the duration of
// one C ABI call.
struct TimerGuard {
  gs::StageTimer* prev;
  unsigned long long* prev_work;
  explicit TimerGuard(gs_ctx* c) : prev(gs::g_timer), prev_work(gs::g_work) {
    gs::g_timer = (c && c->timing) ? &c->timer : nullptr;
    gs::g_work = c ? c->work : nullptr;
  }
  ~TimerGuard() {
    gs::g_timer = prev;
    gs::g_work = prev_work;
  }
};
}  // namespace

namespace {

char g_err[512] = "";

gs_status fail(gs_ctx* c, gs_status code, const char* fmt, ...) {
  char* dst = c ? c->err : g_err;
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(dst, 512, fmt, ap);
  va_end(ap);
  return code;
}

gs_status hip_fail(gs_ctx* c, hipError_t e, const char* where) {
  return fail(c, GS_ERR_HIP, "%s: %s", where, hipGetErrorString(e));
}

gs_status check_gaussians(gs_ctx* c, const gs_gaussians* g, const char* what) {
  if (!g) return fail(c, GS_ERR_INVALID_ARG, "%s is NULL", what);
  if (g->n < 0) return fail(c, GS_ERR_INVALID_ARG, "%s: n = %d < 0", what, g->n);
  if (g->sh_degree < 0 || g->sh_degree > GS_MAX_SH_DEGREE)
    return fail(c, GS_ERR_INVALID_ARG, "%s: sh_degree %d not in 0..3", what, g->sh_degree);
  if (g->ld < g->n || g->ld <= 0 || (g->ld % 64) != 0)
    return fail(c, GS_ERR_INVALID_ARG, "%s: ld %d must be >= n (%d) and a positive multiple of 64",
                what, g->ld, g->n);
  if (g->n > 0 && (!g->mean || !g->log_scale || !g->quat || !g->opacity || !g->sh))
    return fail(c, GS_ERR_INVALID_ARG, "%s: NULL parameter plane", what);
  return GS_OK;
}

gs_status check_cams(gs_ctx* c, const gs_camera* h, const gs_camera* d, int V) {
  if (V <= 0) return fail(c, GS_ERR_INVALID_ARG, "n_views = %d must be > 0", V);
  if (!h || !d) return fail(c, GS_ERR_INVALID_ARG, "camera array is NULL");
  for (int v = 0; v < V; ++v) {
    const gs_camera& k = h[v];
    if (k.width <= 0 || k.height <= 0 || k.width > 65536 || k.height > 65536)
      return fail(c, GS_ERR_INVALID_ARG, "camera %d: size %dx%d out of range", v, k.width,
                  k.height);
    if (!(k.fx > 0.0) || !(k.fy > 0.0))
      return fail(c, GS_ERR_INVALID_ARG, "camera %d: focal lengths must be > 0", v);
  }
  return GS_OK;
}

gs_status check_projected(gs_ctx* c, const gs_projected* p, int V, int ld) {
  if (!p) return fail(c, GS_ERR_INVALID_ARG, "projected is NULL");
  if (p->n_views != V || p->ld != ld)
    return fail(c, GS_ERR_INVALID_ARG, "projected: n_views/ld (%d, %d) != (%d, %d)", p->n_views,
                p->ld, V, ld);
  if (p->n < 0 || p->n > p->ld || p->ld <= 0 || (p->ld % 64) != 0)
    return fail(c, GS_ERR_INVALID_ARG, "projected: n %d / ld %d invalid", p->n, p->ld);
  if (!p->splat || !p->rect || !p->tiles_touched || !p->depth_bits || !p->flags)
    return fail(c, GS_ERR_INVALID_ARG, "projected: NULL buffer");
  return GS_OK;
}

gs_status use_device(gs_ctx* c) {
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return hip_fail(c, e, "hipGetDevice");
  if (cur != c->device) {
    e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
  }
  return GS_OK;
}

// Sizes gs_bin_sort accepts: its instance indices, offsets and counts are
// 32-bit, so the instance capacity (which bounds the count that is sorted)
// and the number of (view, Gaussian) depth keys stay below 2^30, clear of
// overflow in the sums formed from them; segment ids are 31-bit.
bool bin_sort_sizes_ok(int V, int ld, int64_t capacity, int64_t n_segments) {
  return V > 0 && ld > 0 && capacity >= 0 && capacity <= GS_MAX_INSTANCES &&
         (int64_t)V * ld <= GS_MAX_INSTANCES && n_segments >= 0 &&
         n_segments < ((int64_t)1 << 31);
}

int64_t segments_of(const gs_camera* h, int V) {
  int64_t s = 0;
  for (int v = 0; v < V; ++v)
    s += (int64_t)gs::tiles_across(h[v].width) * gs::tiles_across(h[v].height);
  return s;
}

int max_tiles_of(const gs_camera* h, int V) {
  int64_t m = 0;
  for (int v = 0; v < V; ++v)
    m = std::max<int64_t>(m, (int64_t)gs::tiles_across(h[v].width) * gs::tiles_across(h[v].height));
  return (int)m;
}

#define GS_TRY(expr)              \
  do {                            \
    const gs_status st_ = (expr); \
    if (st_ != GS_OK) return st_; \
  } while (0)

#define GS_LAUNCHED(ctx, where)                          \
  do {                                                   \
    const hipError_t e_ = hipGetLastError();             \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, where); \
  } while (0)

}  // namespace

extern "C" {

int gs_version(void) { return 100; }

gs_status gs_create(gs_ctx** out, int device) {
  if (!out) return fail(nullptr, GS_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetDeviceCount");
  if (device < 0 || device >= count)
    return fail(nullptr, GS_ERR_INVALID_ARG, "device %d not in [0, %d)", device, count);
  gs_ctx* c = new (std::nothrow) gs_ctx();
  if (!c) return fail(nullptr, GS_ERR_OOM, "context allocation failed");
  c->device = device;
  c->timing = false;
  c->work = nullptr;
  c->err[0] = 0;
  int prev = 0;
  hipGetDevice(&prev);
  hipSetDevice(device);
  e = hipHostMalloc(reinterpret_cast<void**>(&c->pinned), 64, hipHostMallocDefault);
  if (e != hipSuccess) {
    hipSetDevice(prev);
    delete c;
    return hip_fail(nullptr, e, "hipHostMalloc");
  }
  // the allocation-free entry points use this device's copy of `scratch`
  c->scratch_dev = nullptr;
  e = hipGetSymbolAddress(reinterpret_cast<void**>(&c->scratch_dev), HIP_SYMBOL(scratch));
  hipSetDevice(prev);
  if (e != hipSuccess || !c->scratch_dev) {
    hipHostFree(c->pinned);
    delete c;
    return hip_fail(nullptr, e, "hipGetSymbolAddress(scratch)");
  }
  *out = c;
  return GS_OK;
}

void gs_destroy(gs_ctx* c) {
  if (!c) return;
  if (c->pinned) hipHostFree(c->pinned);
  delete c;
}

const char* gs_last_error(const gs_ctx* c) { return c ? c->err : g_err; }

gs_status gs_set_timing(gs_ctx* c, int enable) {
  if (!c) return fail(nullptr, GS_ERR_INVALID_ARG, "ctx is NULL");
  c->timing = enable != 0;
  c->timer.mask = ~0u;
  return GS_OK;
}

gs_status gs_set_timing_mask(gs_ctx* c, uint32_t stage_mask) {
  if (!c) return fail(nullptr, GS_ERR_INVALID_ARG, "ctx is NULL");
  c->timing = stage_mask != 0;
  c->timer.mask = stage_mask;
  return GS_OK;
}

gs_status gs_set_work_counters(gs_ctx* c, uint64_t* counters) {
  if (!c) return fail(nullptr, GS_ERR_INVALID_ARG, "ctx is NULL");
  if (reinterpret_cast<uintptr_t>(counters) % 8 != 0)
    return fail(c, GS_ERR_INVALID_ARG, "work counters must be 8-byte aligned");
  c->work = reinterpret_cast<unsigned long long*>(counters);
  return GS_OK;
}

size_t gs_peak_min_bytes(int kind) { return gs::peak_min_bytes(kind, 1); }

gs_status gs_peak_run(gs_ctx* c, int kind, void* buf, size_t bytes, int iters, double* ms,
                      double* work, void* stream) {
  if (!c) return fail(nullptr, GS_ERR_INVALID_ARG, "ctx is NULL");
  if (!buf || !ms || !work) return fail(c, GS_ERR_INVALID_ARG, "NULL argument");
  const size_t need = gs::peak_min_bytes(kind, iters);
  if (need == 0) return fail(c, GS_ERR_INVALID_ARG, "unknown probe %d", kind);
  if (bytes < need)
    return fail(c, GS_ERR_INVALID_ARG, "probe %d needs %zu bytes, got %zu", kind, need, bytes);
  if (iters < 1) return fail(c, GS_ERR_INVALID_ARG, "iters must be >= 1");
  GS_TRY(use_device(c));
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  if (e == hipSuccess) e = hipEventRecord(a, s);
  if (e == hipSuccess) e = gs::launch_peak(kind, buf, bytes, iters, work, s);
  if (e == hipSuccess) e = hipEventRecord(b, s);
  if (e == hipSuccess) e = hipEventSynchronize(b);
  float t = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
  if (a) hipEventDestroy(a);
  if (b) hipEventDestroy(b);
  if (e != hipSuccess) return hip_fail(c, e, "peak probe");
  *ms = (double)t;
  return GS_OK;
}

gs_status gs_collect_timing(gs_ctx* c, double* ms, int64_t* launches) {
  if (!c || !ms || !launches) return fail(c, GS_ERR_INVALID_ARG, "NULL argument");
  const hipError_t e = c->timer.collect(ms, launches);
  if (e != hipSuccess) return hip_fail(c, e, "timing events");
  return GS_OK;
}

const char* gs_stage_name(int stage) {
  static const char* names[GS_STAGE_COUNT] = {
      "apply",  "project",    "depth_sort",  "count_scan", "emit", "segment_sort", "ranges",
      "render_fwd", "render_bwd", "project_bwd", "apply_bwd", "l1",   "adam",         "fill",
      "dssim", "compact", "residual", "grad_gather"};
  return (stage >= 0 && stage < GS_STAGE_COUNT) ? names[stage] : "?";
}

int64_t gs_num_segments(const gs_camera* cams, int V) {
  if (!cams || V <= 0) return 0;
  return segments_of(cams, V);
}

size_t gs_bin_sort_workspace_size(int V, int ld, int64_t capacity, int64_t n_segments) {
  if (!bin_sort_sizes_ok(V, ld, capacity, n_segments)) return 0;
  return gs::bin_sort_workspace_bytes(V, ld, capacity, n_segments);
}

size_t gs_render_bwd_workspace_size(int V, int ld, int64_t instances) {
  if (V <= 0 || ld <= 0 || instances < 0) return 0;
  const size_t g2d = (size_t)V * (size_t)ld * gs::kGrad2dFloats * sizeof(float);
  return g2d + (size_t)instances * 9 * sizeof(float);
}

gs_status gs_apply_frame_update(gs_ctx* c, const gs_gaussians* anchor, const float* delta,
                                const uint8_t* mask, int gw, int gh, gs_gaussians* frame,
                                void* stream) {
  if (!c) return fail(nullptr, GS_ERR_INVALID_ARG, "ctx is NULL");
  TimerGuard timer_guard(c);
  GS_TRY(check_gaussians(c, anchor, "anchor"));
  if (!frame) return fail(c, GS_ERR_INVALID_ARG, "frame is NULL");
  if (frame->n != anchor->n || frame->ld != anchor->ld)
    return fail(c, GS_ERR_INVALID_ARG, "frame n/ld differ from the anchor's");
  if (gw <= 0 || gh <= 0 || (int64_t)gw * gh < anchor->n)
    return fail(c, GS_ERR_INVALID_ARG, "texel grid %dx%d cannot hold %d Gaussians", gw, gh,
                anchor->n);
  if (anchor->n > 0 && (!delta || !mask || !frame->mean || !frame->quat || !frame->opacity))
    return fail(c, GS_ERR_INVALID_ARG, "NULL delta, mask or frame plane");
  GS_TRY(use_device(c));
  gs::launch_apply(*anchor, delta, mask, gw, gh, *frame, (hipStream_t)stream);
  GS_LAUNCHED(c, "apply");
  return GS_OK;
}

gs_status gs_project(gs_ctx* c, const gs_gaussians* g, const gs_camera* ch, const gs_camera* cd,
                     int V, gs_projected* out, void* stream) {
  if (!c) return fail(nullptr, GS_ERR_INVALID_ARG, "ctx is NULL");
  TimerGuard timer_guard(c);
  GS_TRY(check_gaussians(c, g, "gaussians"));
  GS_TRY(check_cams(c, ch, cd, V));
  GS_TRY(check_projected(c, out, V, g->ld));
  if (out->n != g->n) return fail(c, GS_ERR_INVALID_ARG, "projected n != gaussians n");
  if (out->options & ~(GS_PROJECT_TIGHT_RECT | GS_PROJECT_TILE_SPANS))
    return fail(c, GS_ERR_INVALID_ARG, "unknown projection options %d", out->options);
  GS_TRY(use_device(c));
  gs::launch_project(*g, cd, V, *out, (hipStream_t)stream);
  GS_LAUNCHED(c, "project");
  return GS_OK;
}

// Workspaces are carved into 256-byte aligned sub-buffers that kernels read
// with 16-byte vector loads, so the base must keep that alignment.
static gs_status check_ws_align(gs_ctx* c, const void* ws) {
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0)
    return fail(c, GS_ERR_INVALID_ARG, "workspace %p is not 256-byte aligned", ws);
  return GS_OK;
}

gs_status gs_bin_sort(gs_ctx* c, const gs_projected* proj, const gs_camera* ch,
                      const gs_camera* cd, int V, gs_tile_lists* lists, void* ws, size_t ws_bytes,
                      void* stream) {
  if (!c) return fail(nullptr, GS_ERR_INVALID_ARG, "ctx is NULL");
  TimerGuard timer_guard(c);
  GS_TRY(check_cams(c, ch, cd, V));
  if (!proj) return fail(c, GS_ERR_INVALID_ARG, "projected is NULL");
  GS_TRY(check_projected(c, proj, V, proj->ld));
  if (!lists || !lists->vals || !lists->ranges)
    return fail(c, GS_ERR_INVALID_ARG, "tile lists (vals, ranges) are NULL");
  if (lists->gv_base && lists->gv_capacity < (int64_t)V * proj->ld)
    return fail(c, GS_ERR_INVALID_ARG, "gv_base holds %lld entries, n_views * ld = %lld",
                (long long)lists->gv_capacity, (long long)V * proj->ld);
  const int64_t nseg = segments_of(ch, V);
  if (!bin_sort_sizes_ok(V, proj->ld, lists->capacity, nseg))
    return fail(c, GS_ERR_INVALID_ARG,
                "capacity %lld or n_views * ld = %lld outside [0, 2^30 - 1], or %lld segments",
                (long long)lists->capacity, (long long)V * proj->ld, (long long)nseg);
  if (!ws) return fail(c, GS_ERR_INVALID_ARG, "workspace is NULL");
  GS_TRY(check_ws_align(c, ws));
  gs::BinSortPlan plan{V, proj->n, proj->ld, lists->capacity, nseg, max_tiles_of(ch, V)};
  const size_t need = gs::bin_sort_workspace_bytes(V, proj->ld, lists->capacity, nseg);
  if (ws_bytes < need)
    return fail(c, GS_ERR_OOM, "bin_sort workspace %zu < %zu bytes", ws_bytes, need);
  GS_TRY(use_device(c));
  hipStream_t s = (hipStream_t)stream;
  lists->n_segments = nseg;
  uint32_t* d_stats = nullptr;
  hipError_t e = gs::bin_sort_stage1(plan, *proj, cd, ws, s, &d_stats);
  if (e != hipSuccess) return hip_fail(c, e, "bin_sort (count)");
  e = hipMemcpyAsync(c->pinned, d_stats, 5 * sizeof(uint32_t), hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return hip_fail(c, e, "instance count readback");
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
  const uint32_t dmin = c->pinned[0], dmax = c->pinned[1];
  const uint64_t M = (uint64_t)c->pinned[2] | ((uint64_t)c->pinned[3] << 32);
  lists->count = (int64_t)M;
  if (M > (uint64_t)lists->capacity)
    return fail(c, GS_ERR_CAPACITY, "instance count %llu exceeds capacity %lld",
                (unsigned long long)M, (long long)lists->capacity);
  const uint32_t n_visible = c->pinned[4];
  e = gs::bin_sort_stage2(plan, *proj, cd, (uint32_t)M, dmin, dmax, n_visible, *lists, ws, s);
  if (e != hipSuccess) return hip_fail(c, e, "bin_sort (sort)");
  return GS_OK;
}

gs_status gs_render_fwd(gs_ctx* c, const gs_projected* proj, const gs_tile_lists* lists,
                        const gs_camera* ch, const gs_camera* cd, int V, const gs_opts* opts,
                        float* image, float* final_T, int32_t* n_contrib, void* stream) {
  if (!c) return fail(nullptr, GS_ERR_INVALID_ARG, "ctx is NULL");
  TimerGuard timer_guard(c);
  GS_TRY(check_cams(c, ch, cd, V));
  if (!proj) return fail(c, GS_ERR_INVALID_ARG, "projected is NULL");
  GS_TRY(check_projected(c, proj, V, proj->ld));
  if (!lists || !lists->vals || !lists->ranges)
    return fail(c, GS_ERR_INVALID_ARG, "tile lists are NULL");
  if (lists->n_segments != segments_of(ch, V))
    return fail(c, GS_ERR_INVALID_ARG, "tile lists were built for other cameras");
  for (int v = 1; v < V; ++v)
    if (ch[v].width != ch[0].width || ch[v].height != ch[0].height)
      return fail(c, GS_ERR_INVALID_ARG, "views must share width and height");
  if (!image || !final_T || !n_contrib)
    return fail(c, GS_ERR_INVALID_ARG, "NULL output buffer");
  GS_TRY(use_device(c));
  const float zero[3] = {0.f, 0.f, 0.f};
  gs::launch_render_fwd(*proj, *lists, V, ch[0].width, ch[0].height, opts ? opts->bg : zero, image,
                        final_T, n_contrib, opts ? opts->usage : nullptr, (hipStream_t)stream);
  GS_LAUNCHED(c, "render_fwd");
  return GS_OK;
}

size_t gs_render_fwd_l1_workspace_size(int V, int W, int H) {
  if (V <= 0 || W <= 0 || H <= 0) return 0;
  return gs::render_fwd_l1_workspace_bytes(V, W, H);
}

gs_status gs_render_fwd_l1(gs_ctx* c, const gs_projected* proj, const gs_tile_lists* lists,
                           const gs_camera* ch, const gs_camera* cd, int V, const gs_opts* opts,
                           const float* target, float* image, float* final_T,
                           int32_t* n_contrib, float* dL_dimage, double* loss_dev, void* ws,
                           size_t ws_bytes, void* stream) {
  if (!c) return fail(nullptr, GS_ERR_INVALID_ARG, "ctx is NULL");
  TimerGuard timer_guard(c);
  GS_TRY(check_cams(c, ch, cd, V));
  if (!proj) return fail(c, GS_ERR_INVALID_ARG, "projected is NULL");
  GS_TRY(check_projected(c, proj, V, proj->ld));
  if (!lists || !lists->vals || !lists->ranges)
    return fail(c, GS_ERR_INVALID_ARG, "tile lists are NULL");
  if (lists->n_segments != segments_of(ch, V))
    return fail(c, GS_ERR_INVALID_ARG, "tile lists were built for other cameras");
  for (int v = 1; v < V; ++v)
    if (ch[v].width != ch[0].width || ch[v].height != ch[0].height)
      return fail(c, GS_ERR_INVALID_ARG, "views must share width and height");
  if (!target || !final_T || !n_contrib || !dL_dimage || !loss_dev)
    return fail(c, GS_ERR_INVALID_ARG, "NULL buffer");
  if (opts && opts->usage)
    return fail(c, GS_ERR_INVALID_ARG, "usage counts are not produced by the fused L1 forward");
  const size_t need = gs::render_fwd_l1_workspace_bytes(V, ch[0].width, ch[0].height);
  if (!ws || ws_bytes < need)
    return fail(c, GS_ERR_OOM, "render_fwd_l1 workspace %zu < %zu bytes", ws_bytes, need);
  GS_TRY(check_ws_align(c, ws));
  GS_TRY(use_device(c));
  const float zero[3] = {0.f, 0.f, 0.f};
  gs::launch_render_fwd_l1(*proj, *lists, V, ch[0].width, ch[0].height, opts ? opts->bg : zero,
                           target, image, final_T, n_contrib, dL_dimage, loss_dev, ws,
                           (hipStream_t)stream);
  GS_LAUNCHED(c, "render_fwd_l1");
  return GS_OK;
}

gs_status gs_render_fwd_l1_noalloc(gs_ctx* c, const gs_projected* proj,
                                   const gs_tile_lists* lists, const gs_camera* ch,
                                   const gs_camera* cd, int V, const gs_opts* opts,
                                   const float* target, float* image, float* final_T,
                                   int32_t* n_contrib, float* dL_dimage, double* loss_dev,
                                   void* stream) {
  // No TimerGuard: the stage timer records events into growing host vectors,
  // and this entry point allocates nothing.
  if (!c) return fail(nullptr, GS_ERR_INVALID_ARG, "ctx is NULL");
  if (!c->scratch_dev) return fail(c, GS_ERR_INVALID_ARG, "context has no scratch array");
  GS_TRY(check_cams(c, ch, cd, V));
  if (!proj) return fail(c, GS_ERR_INVALID_ARG, "projected is NULL");
  GS_TRY(check_projected(c, proj, V, proj->ld));
  if (!lists || !lists->vals || !lists->ranges)
    return fail(c, GS_ERR_INVALID_ARG, "tile lists are NULL");
  const int64_t nseg = segments_of(ch, V);
  if (lists->n_segments != nseg)
    return fail(c, GS_ERR_INVALID_ARG, "tile lists were built for other cameras");
  for (int v = 1; v < V; ++v)
    if (ch[v].width != ch[0].width || ch[v].height != ch[0].height)
      return fail(c, GS_ERR_INVALID_ARG, "views must share width and height");
  if (!target || !final_T || !n_contrib || !dL_dimage || !loss_dev)
    return fail(c, GS_ERR_INVALID_ARG, "NULL buffer");
  if (opts && opts->usage)
    return fail(c, GS_ERR_INVALID_ARG, "usage counts are not produced by the fused L1 forward");
  if (nseg > GS_NOALLOC_MAX_TILES)
    return fail(c, GS_ERR_INVALID_ARG,
                "%lld tiles over all views exceed the fixed scratch of %d tiles",
                (long long)nseg, GS_NOALLOC_MAX_TILES);
  GS_TRY(use_device(c));
  const float zero[3] = {0.f, 0.f, 0.f};
  // every tile writes its partial before the sum kernel reads it, so the
  // array needs no clearing between calls
  gs::launch_render_fwd_l1(*proj, *lists, V, ch[0].width, ch[0].height, opts ? opts->bg : zero,
                           target, image, final_T, n_contrib, dL_dimage, loss_dev,
                           c->scratch_dev, (hipStream_t)stream);
  GS_LAUNCHED(c, "render_fwd_l1_noalloc");
  return GS_OK;
}

size_t gs_render_batched_workspace_size(int V) {
  if (V <= 0) return 0;
  return gs::render_batched_workspace_bytes(V);
}

gs_status gs_render_fwd_batched(gs_ctx* c, const gs_projected* proj, const gs_tile_lists* lists,
                                const gs_camera* ch, const gs_camera* cd, int V,
                                const gs_opts* opts, float* images, void* ws, size_t ws_bytes,
                                void* stream) {
  if (!c) return fail(nullptr, GS_ERR_INVALID_ARG, "ctx is NULL");
  TimerGuard timer_guard(c);
  GS_TRY(check_cams(c, ch, cd, V));
  if (!proj) return fail(c, GS_ERR_INVALID_ARG, "projected is NULL");
  GS_TRY(check_projected(c, proj, V, proj->ld));
  if (!lists || !lists->vals || !lists->ranges)
    return fail(c, GS_ERR_INVALID_ARG, "tile lists are NULL");
  const int64_t nseg = segments_of(ch, V);
  if (lists->n_segments != nseg)
    return fail(c, GS_ERR_INVALID_ARG, "tile lists were built for other cameras");
  if (!images) return fail(c, GS_ERR_INVALID_ARG, "images is NULL");
  const size_t need = gs::render_batched_workspace_bytes(V);
  if (!ws || ws_bytes < need)
    return fail(c, GS_ERR_OOM, "batched render workspace %zu < %zu bytes", ws_bytes, need);
  GS_TRY(check_ws_align(c, ws));
  GS_TRY(use_device(c));
  const float zero[3] = {0.f, 0.f, 0.f};
  gs::launch_render_batched(*proj, *lists, cd, V, nseg, opts ? opts->bg : zero, images, ws,
                            (hipStream_t)stream);
  GS_LAUNCHED(c, "render_fwd_batched");
  return GS_OK;
}

gs_status gs_render_bwd(gs_ctx* c, const gs_gaussians* frame, const gs_projected* proj,
                        const gs_tile_lists* lists, const gs_camera* ch, const gs_camera* cd,
                        int V, const gs_opts* opts, const float* final_T, const int32_t* n_contrib,
                        const float* dL_dimage, gs_gaussians* grad, const gs_frame_update* upd,
                        float* dL_ddelta, void* ws, size_t ws_bytes, void* stream) {
  if (!c) return fail(nullptr, GS_ERR_INVALID_ARG, "ctx is NULL");
  TimerGuard timer_guard(c);
  GS_TRY(check_gaussians(c, frame, "frame"));
  GS_TRY(check_gaussians(c, grad, "grad"));
  if (grad->n != frame->n || grad->ld != frame->ld || grad->sh_degree != frame->sh_degree)
    return fail(c, GS_ERR_INVALID_ARG, "grad shape differs from frame shape");
  GS_TRY(check_cams(c, ch, cd, V));
  GS_TRY(check_projected(c, proj, V, frame->ld));
  if (proj->n != frame->n) return fail(c, GS_ERR_INVALID_ARG, "projected n != frame n");
  if (!lists || !lists->vals || !lists->ranges)
    return fail(c, GS_ERR_INVALID_ARG, "tile lists are NULL");
  if (lists->n_segments != segments_of(ch, V))
    return fail(c, GS_ERR_INVALID_ARG, "tile lists were built for other cameras");
  for (int v = 1; v < V; ++v)
    if (ch[v].width != ch[0].width || ch[v].height != ch[0].height)
      return fail(c, GS_ERR_INVALID_ARG, "views must share width and height");
  if (!final_T || !n_contrib || !dL_dimage)
    return fail(c, GS_ERR_INVALID_ARG, "NULL forward state or image gradient");
  if (upd) {
    if (!dL_ddelta || !upd->anchor_quat || !upd->mask)
      return fail(c, GS_ERR_INVALID_ARG, "frame update given without its buffers");
    if (upd->ld != frame->ld || upd->gw <= 0 || upd->gh <= 0 ||
        (int64_t)upd->gw * upd->gh < frame->n)
      return fail(c, GS_ERR_INVALID_ARG, "frame update grid/stride mismatch");
    if (!std::isfinite(upd->temporal_weight))
      return fail(c, GS_ERR_INVALID_ARG, "temporal_weight is not finite");
    if (upd->temporal_weight != 0.f && !upd->delta)
      return fail(c, GS_ERR_INVALID_ARG, "temporal term needs the delta images");
  }
  if (opts && ((opts->grad2d_norm == nullptr) != (opts->visible_views == nullptr)))
    return fail(c, GS_ERR_INVALID_ARG, "grad2d_norm and visible_views go together");
  if (lists->count < 0 || lists->count > lists->capacity)
    return fail(c, GS_ERR_INVALID_ARG, "tile list count out of range");
  const size_t need = gs_render_bwd_workspace_size(V, frame->ld, lists->count);
  if (!ws || ws_bytes < need)
    return fail(c, GS_ERR_OOM, "render_bwd workspace %zu < %zu bytes", ws_bytes, need);
  GS_TRY(check_ws_align(c, ws));
  GS_TRY(use_device(c));
  hipStream_t s = (hipStream_t)stream;
  float* grad2d = static_cast<float*>(ws);
  float* rows = grad2d + (size_t)V * (size_t)frame->ld * gs::kGrad2dFloats;
  const float zero[3] = {0.f, 0.f, 0.f};
  gs::launch_render_bwd(*proj, *lists, V, ch[0].width, ch[0].height, opts ? opts->bg : zero,
                        final_T, n_contrib, dL_dimage, rows, grad2d, s);
  GS_LAUNCHED(c, "render_bwd");
  float* st_norm = opts ? opts->grad2d_norm : nullptr;
  uint32_t* st_views = opts ? opts->visible_views : nullptr;
  gs::launch_project_bwd(*frame, cd, V, *proj, grad2d, *grad, st_norm, st_views, s);
  GS_LAUNCHED(c, "project_bwd");
  if (upd) {
    gs::launch_apply_bwd(frame->n, *upd, *grad, dL_ddelta, s);
    GS_LAUNCHED(c, "apply_bwd");
  }
  return GS_OK;
}

gs_status gs_l1_loss_grad(gs_ctx* c, const float* image, const float* target, int64_t count,
                          float* grad, double* loss_dev, void* stream) {
  if (!c) return fail(nullptr, GS_ERR_INVALID_ARG, "ctx is NULL");
  TimerGuard timer_guard(c);
  if (count < 0) return fail(c, GS_ERR_INVALID_ARG, "count < 0");
  if (count > 0 && (!image || !target || !grad || !loss_dev))
    return fail(c, GS_ERR_INVALID_ARG, "NULL buffer");
  GS_TRY(use_device(c));
  gs::launch_l1(image, target, count, grad, loss_dev, (hipStream_t)stream);
  GS_LAUNCHED(c, "l1");
  return GS_OK;
}

size_t gs_l1_dssim_workspace_size(int planes, int H, int W) {
  if (planes <= 0 || H <= 0 || W <= 0) return 0;
  return gs::l1_dssim_workspace_bytes(planes, H, W);
}

gs_status gs_l1_dssim_loss_grad(gs_ctx* c, const float* image, const float* target, int planes,
                                int H, int W, float lambda, float* grad, double* loss_dev,
                                void* ws, size_t ws_bytes, void* stream) {
  if (!c) return fail(nullptr, GS_ERR_INVALID_ARG, "ctx is NULL");
  TimerGuard timer_guard(c);
  if (planes <= 0 || H <= 0 || W <= 0 || planes > 65535)
    return fail(c, GS_ERR_INVALID_ARG, "planes/H/W out of range");
  if (!(lambda >= 0.f && lambda <= 1.f)) return fail(c, GS_ERR_INVALID_ARG, "lambda not in [0,1]");
  if (!image || !target || !grad || !loss_dev) return fail(c, GS_ERR_INVALID_ARG, "NULL buffer");
  const size_t need = gs::l1_dssim_workspace_bytes(planes, H, W);
  if (!ws || ws_bytes < need)
    return fail(c, GS_ERR_OOM, "l1_dssim workspace %zu < %zu bytes", ws_bytes, need);
  GS_TRY(check_ws_align(c, ws));
  GS_TRY(use_device(c));
  gs::launch_l1_dssim(image, target, planes, H, W, lambda, grad, loss_dev, ws, (hipStream_t)stream);
  GS_LAUNCHED(c, "l1_dssim");
  return GS_OK;
}

gs_status gs_sq_error(gs_ctx* c, const float* a, const float* b, int64_t count, double* sum_dev,
                      void* stream) {
  if (!c) return fail(nullptr, GS_ERR_INVALID_ARG, "ctx is NULL");
  TimerGuard timer_guard(c);
  if (count < 0) return fail(c, GS_ERR_INVALID_ARG, "count < 0");
  if (count > 0 && (!a || !b || !sum_dev)) return fail(c, GS_ERR_INVALID_ARG, "NULL buffer");
  GS_TRY(use_device(c));
  gs::launch_sq_error(a, b, count, sum_dev, (hipStream_t)stream);
  GS_LAUNCHED(c, "sq_error");
  return GS_OK;
}

gs_status gs_adam_step(gs_ctx* c, float* param, const float* grad, float* m, float* v,
                       int64_t count, int step, float lr, float b1, float b2, float eps,
                       void* stream) {
  if (!c) return fail(nullptr, GS_ERR_INVALID_ARG, "ctx is NULL");
  TimerGuard timer_guard(c);
  if (count < 0 || step < 1) return fail(c, GS_ERR_INVALID_ARG, "count < 0 or step < 1");
  if (!(b1 >= 0.f && b1 < 1.f) || !(b2 >= 0.f && b2 < 1.f) || !(eps > 0.f))
    return fail(c, GS_ERR_INVALID_ARG, "Adam hyper-parameters out of range");
  if (count > 0 && (!param || !grad || !m || !v))
    return fail(c, GS_ERR_INVALID_ARG, "NULL buffer");
  GS_TRY(use_device(c));
  const double bc1 = 1.0 - std::pow((double)b1, (double)step);
  const double bc2 = 1.0 - std::pow((double)b2, (double)step);
  gs::launch_adam(param, grad, m, v, count, lr, b1, b2, eps, (float)bc1, (float)bc2,
                  (hipStream_t)stream);
  GS_LAUNCHED(c, "adam");
  return GS_OK;
}

gs_status gs_keyframe_temporal_l1(gs_ctx* c, const float* x, const float* x_prev, int rows,
                                  int bound, int64_t ld, float weight, float* grad,
                                  double* loss_dev, void* stream) {
  if (!c) return fail(nullptr, GS_ERR_INVALID_ARG, "ctx is NULL");
  TimerGuard timer_guard(c);
  if (rows < 0 || bound < 0 || (int64_t)bound > ld)
    return fail(c, GS_ERR_INVALID_ARG, "rows/bound/ld out of range");
  if (!std::isfinite(weight)) return fail(c, GS_ERR_INVALID_ARG, "weight is not finite");
  if ((int64_t)rows * bound > 0 && (!x || !x_prev || !grad))
    return fail(c, GS_ERR_INVALID_ARG, "NULL buffer");
  GS_TRY(use_device(c));
  gs::launch_l1_penalty(x, x_prev, rows, bound, ld, weight, grad, loss_dev, (hipStream_t)stream);
  GS_LAUNCHED(c, "keyframe_temporal_l1");
  return GS_OK;
}

size_t gs_cull_workspace_size(int n) { return n < 0 ? 0 : gs::keep_workspace_bytes(n); }

gs_status gs_cull_low_opacity(gs_ctx* c, const float* logit, int n, float min_opacity,
                              int32_t* kept_index, int32_t* kept_host, void* ws, size_t ws_bytes,
                              void* stream) {
  if (!c) return fail(nullptr, GS_ERR_INVALID_ARG, "ctx is NULL");
  TimerGuard timer_guard(c);
  if (n < 0) return fail(c, GS_ERR_INVALID_ARG, "n < 0");
  if (!(min_opacity > 0.f && min_opacity < 1.f))
    return fail(c, GS_ERR_INVALID_ARG, "min_opacity must lie in (0, 1)");
  if (!kept_host || (n > 0 && (!logit || !kept_index)))
    return fail(c, GS_ERR_INVALID_ARG, "NULL buffer");
  const size_t need = gs::keep_workspace_bytes(n);
  if (!ws || ws_bytes < need)
    return fail(c, GS_ERR_OOM, "cull workspace %zu < %zu bytes", ws_bytes, need);
  GS_TRY(check_ws_align(c, ws));
  GS_TRY(use_device(c));
  hipStream_t s = (hipStream_t)stream;
  const uint32_t* d_total = gs::launch_keep_low_opacity(
      logit, n, gs::opacity_logit_threshold(min_opacity), kept_index, ws, s);
  GS_LAUNCHED(c, "cull_low_opacity");
  hipError_t e = hipMemcpyAsync(c->pinned, d_total, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return hip_fail(c, e, "kept count readback");
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(c, e, "hipStreamSynchronize");
  *kept_host = (int32_t)*c->pinned;
  return GS_OK;
}

gs_status gs_gather_planes(gs_ctx* c, const float* src, int64_t src_ld, int planes,
                           const int32_t* index, int m, float* dst, int64_t dst_ld,
                           void* stream) {
  if (!c) return fail(nullptr, GS_ERR_INVALID_ARG, "ctx is NULL");
  TimerGuard timer_guard(c);
  if (planes < 0 || m < 0 || src_ld < 0 || dst_ld < m || (m > src_ld))
    return fail(c, GS_ERR_INVALID_ARG, "planes/m/stride out of range");
  if (planes > 0 && m > 0 && (!src || !dst || !index))
    return fail(c, GS_ERR_INVALID_ARG, "NULL buffer");
  GS_TRY(use_device(c));
  gs::launch_gather(src, src_ld, planes, index, m, dst, dst_ld, (hipStream_t)stream);
  GS_LAUNCHED(c, "gather_planes");
  return GS_OK;
}

namespace {
gs_status check_grid(gs_ctx* c, int n, int gw, int gh) {
  if (n < 0 || gw <= 0 || gh <= 0 || (int64_t)gw * gh < n || (int64_t)gw * gh > (1ll << 31))
    return fail(c, GS_ERR_INVALID_ARG, "texel grid %dx%d cannot hold %d Gaussians", gw, gh, n);
  return GS_OK;
}
}  // namespace

gs_status gs_residual_delta(gs_ctx* c, const float* D, const float* Dp, const uint8_t* mask,
                            int n, int gw, int gh, float* d_out, float* absmax, void* stream) {
  if (!c) return fail(nullptr, GS_ERR_INVALID_ARG, "ctx is NULL");
  TimerGuard timer_guard(c);
  GS_TRY(check_grid(c, n, gw, gh));
  if (!D || !Dp || !mask || !d_out || !absmax) return fail(c, GS_ERR_INVALID_ARG, "NULL buffer");
  GS_TRY(use_device(c));
  gs::launch_residual(D, Dp, mask, n, gw, gh, d_out, absmax, (hipStream_t)stream);
  GS_LAUNCHED(c, "residual_delta");
  return GS_OK;
}

gs_status gs_quantize_delta(gs_ctx* c, const float* d, const float* absmax, int bits, int n,
                            int gw, int gh, void* q_out, float* scale_out, float* Dp,
                            void* stream) {
  if (!c) return fail(nullptr, GS_ERR_INVALID_ARG, "ctx is NULL");
  TimerGuard timer_guard(c);
  GS_TRY(check_grid(c, n, gw, gh));
  if (bits != 8 && bits != 16) return fail(c, GS_ERR_INVALID_ARG, "bits must be 8 or 16");
  if (!d || !absmax || !q_out || !scale_out) return fail(c, GS_ERR_INVALID_ARG, "NULL buffer");
  GS_TRY(use_device(c));
  gs::launch_quantize(d, absmax, bits, n, gw, gh, q_out, scale_out, Dp, (hipStream_t)stream);
  GS_LAUNCHED(c, "quantize_delta");
  return GS_OK;
}

gs_status gs_apply_quantized_update(gs_ctx* c, const gs_gaussians* anchor, const void* q,
                                    int bits, const float* scale, float* Dp, int gw, int gh,
                                    gs_gaussians* frame, void* stream) {
  if (!c) return fail(nullptr, GS_ERR_INVALID_ARG, "ctx is NULL");
  TimerGuard timer_guard(c);
  GS_TRY(check_gaussians(c, anchor, "anchor"));
  if (!frame) return fail(c, GS_ERR_INVALID_ARG, "frame is NULL");
  if (frame->n != anchor->n || frame->ld != anchor->ld)
    return fail(c, GS_ERR_INVALID_ARG, "frame n/ld differ from the anchor's");
  GS_TRY(check_grid(c, anchor->n, gw, gh));
  if (bits != 8 && bits != 16) return fail(c, GS_ERR_INVALID_ARG, "bits must be 8 or 16");
  if (anchor->n > 0 && (!q || !scale || !Dp || !frame->mean || !frame->quat || !frame->opacity))
    return fail(c, GS_ERR_INVALID_ARG, "NULL buffer");
  GS_TRY(use_device(c));
  gs::launch_apply_quantized(*anchor, q, bits, scale, Dp, gw, gh, *frame, (hipStream_t)stream);
  GS_LAUNCHED(c, "apply_quantized_update");
  return GS_OK;
}

}  // extern "C"
