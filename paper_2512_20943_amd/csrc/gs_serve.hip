// Native continuous-batching view server over a resident dynamic scene
// (view delivery, Sec. IV-B: a client applies a frame's update and renders
// it; here a server renders requested (frame, viewpoint, resolution) views
// of a sequence whose frames are anchor + delta images, Eq. (12)).
//
// The caller's thread schedules: it admits arrived requests while their
// estimated device memory fits the budget, forms a batch whenever a worker
// is free, and hands it to that worker's thread.  A worker owns a context,
// a stream and growable device buffers, and renders a batch with the
// library's own calls: one apply per distinct frame, one projection per
// frame group into consecutive view slots, one joint binning over all
// requests, and one persistent compositing launch over the shared (request,
// tile) queue (a batch of one takes the single-view compositing call, the
// same image bit for bit).  While arrivals are sparse, a lone request on an
// idle server is rendered on the scheduler's thread by a renderer of its
// own, which saves the wake-up of a worker thread.  The plain mode serves
// the same requests one at a time in arrival order on that renderer: the
// one-request-per-launch comparison.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "gs_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

template <typename T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  hipError_t ensure(size_t want) {
    if (want <= n && p) return hipSuccess;
    if (p) {
      hipError_t e = hipFree(p);
      if (e != hipSuccess) return e;
      p = nullptr;
      n = 0;
    }
    const size_t m = want > 0 ? want : 1;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&p), m * sizeof(T));
    if (e != hipSuccess) {
      p = nullptr;
      return e;
    }
    n = m;
    return hipSuccess;
  }
  ~DevBuf() {
    if (p) hipFree(p);
  }
};

int64_t tiles_of(int W, int H) {
  return (int64_t)gs::tiles_across(W) * (int64_t)gs::tiles_across(H);
}

// One rendering pipeline: context, stream and buffers for batches of up to
// max_batch requests.  Used by one host thread at a time.
struct Renderer {
  int device = 0;
  const gs_sequence* seq = nullptr;
  gs_server_config cfg{};
  gs_ctx* ctx = nullptr;
  hipStream_t stream = nullptr;
  gs_camera* cams_host = nullptr;  // pinned, max_batch
  DevBuf<gs_camera> cams_dev;
  std::vector<std::unique_ptr<DevBuf<float>>> fmean, fquat, fopac;
  DevBuf<float> splat;
  DevBuf<int32_t> rect, tiles;
  DevBuf<uint32_t> depth;
  DevBuf<uint8_t> flags;
  DevBuf<uint32_t> vals, ranges;
  int64_t capacity = 1 << 22;
  DevBuf<char> ws_sort, ws_batch;
  DevBuf<float> images, final_T;
  DevBuf<int32_t> n_contrib;
  double inst_per_tile = 600.0;
  char err[256] = "";

  gs_status init(int dev, const gs_sequence* s, const gs_server_config& c) {
    device = dev;
    seq = s;
    cfg = c;
    if (hipSetDevice(dev) != hipSuccess) return fail("hipSetDevice");
    gs_status st = gs_create(&ctx, dev);
    if (st != GS_OK) return fail("gs_create");
    if (hipStreamCreate(&stream) != hipSuccess) return fail("hipStreamCreate");
    if (hipHostMalloc(reinterpret_cast<void**>(&cams_host),
                      sizeof(gs_camera) * (size_t)cfg.max_batch, hipHostMallocDefault) !=
        hipSuccess) {
      cams_host = nullptr;
      return fail("hipHostMalloc");
    }
    if (cams_dev.ensure((size_t)cfg.max_batch) != hipSuccess) return fail("camera buffer");
    return GS_OK;
  }
  ~Renderer() {
    if (stream) hipStreamSynchronize(stream);
    if (cams_host) hipHostFree(cams_host);
    if (stream) hipStreamDestroy(stream);
    if (ctx) gs_destroy(ctx);
  }
  gs_status fail(const char* what) {
    snprintf(err, sizeof(err), "%s: %s", what, ctx ? gs_last_error(ctx) : "");
    return GS_ERR_HIP;
  }
  gs_status check(gs_status st, const char* what) {
    if (st == GS_OK) return GS_OK;
    snprintf(err, sizeof(err), "%s: %s", what, gs_last_error(ctx));
    return st;
  }
#define GS_SRV_TRY(expr)             \
  do {                               \
    const gs_status st_ = (expr);    \
    if (st_ != GS_OK) return st_;    \
  } while (0)
#define GS_SRV_HIP(expr, what)                                      \
  do {                                                              \
    if ((expr) != hipSuccess) {                                     \
      snprintf(err, sizeof(err), "%s failed", what);                \
      return GS_ERR_HIP;                                            \
    }                                                               \
  } while (0)

  // Render requests reqs[idx[0..B)]; out (nullable) holds one device
  // pointer per request index for a copy of its (3, H, W) image.
  gs_status render(const gs_request* reqs, const int* idx, int B, float* const* out) {
    const int ld = seq->anchor.ld;
    const int n = seq->anchor.n;
    // requests grouped by frame (stable)
    std::vector<int> order(idx, idx + B);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return reqs[a].frame < reqs[b].frame; });
    for (int j = 0; j < B; ++j) cams_host[j] = reqs[order[j]].cam;
    GS_SRV_HIP(hipMemcpyAsync(cams_dev.p, cams_host, sizeof(gs_camera) * (size_t)B,
                              hipMemcpyHostToDevice, stream),
               "camera upload");
    GS_SRV_HIP(splat.ensure((size_t)B * ld * 16), "projected records");
    GS_SRV_HIP(rect.ensure((size_t)B * ld * 4), "rectangles");
    GS_SRV_HIP(tiles.ensure((size_t)B * ld), "tile counts");
    GS_SRV_HIP(depth.ensure((size_t)B * ld), "depth bits");
    GS_SRV_HIP(flags.ensure((size_t)B * ld), "flags");
    const size_t texels = (size_t)seq->gw * (size_t)seq->gh;
    int k = 0;
    for (int s = 0; s < B; ++k) {
      const int f = reqs[order[s]].frame;
      int e = s;
      while (e < B && reqs[order[e]].frame == f) ++e;
      if ((int)fmean.size() <= k) {
        fmean.emplace_back(new DevBuf<float>());
        fquat.emplace_back(new DevBuf<float>());
        fopac.emplace_back(new DevBuf<float>());
      }
      GS_SRV_HIP(fmean[k]->ensure((size_t)3 * ld), "frame means");
      GS_SRV_HIP(fquat[k]->ensure((size_t)4 * ld), "frame quaternions");
      GS_SRV_HIP(fopac[k]->ensure((size_t)ld), "frame opacities");
      gs_gaussians fr = seq->anchor;
      fr.mean = fmean[k]->p;
      fr.quat = fquat[k]->p;
      fr.opacity = fopac[k]->p;
      GS_SRV_TRY(check(gs_apply_frame_update(ctx, &seq->anchor, seq->deltas + (size_t)f * 8 * texels,
                                             seq->masks + (size_t)f * texels, seq->gw, seq->gh,
                                             &fr, stream),
                       "apply"));
      gs_projected pp{e - s, n, ld, cfg.options, splat.p + (size_t)s * ld * 16,
                      rect.p + (size_t)s * ld * 4, tiles.p + (size_t)s * ld,
                      depth.p + (size_t)s * ld, flags.p + (size_t)s * ld};
      GS_SRV_TRY(check(gs_project(ctx, &fr, cams_host + s, cams_dev.p + s, e - s, &pp, stream),
                       "project"));
      s = e;
    }
    gs_projected proj{B, n, ld, cfg.options, splat.p, rect.p, tiles.p, depth.p, flags.p};
    const int64_t nseg = gs_num_segments(cams_host, B);
    GS_SRV_HIP(ranges.ensure((size_t)2 * nseg), "tile ranges");
    gs_tile_lists lists{};
    for (;;) {
      GS_SRV_HIP(vals.ensure((size_t)capacity), "tile lists");
      const size_t need = gs_bin_sort_workspace_size(B, ld, capacity, nseg);
      GS_SRV_HIP(ws_sort.ensure(need), "binning workspace");
      lists = gs_tile_lists{capacity, 0, 0, nullptr, vals.p, ranges.p, 0, nullptr};
      const gs_status st = gs_bin_sort(ctx, &proj, cams_host, cams_dev.p, B, &lists, ws_sort.p,
                                       ws_sort.n, stream);
      if (st == GS_ERR_CAPACITY && lists.count <= GS_MAX_INSTANCES) {
        capacity = std::min<int64_t>(
            std::max<int64_t>((int64_t)((double)lists.count * 1.25) + 1024, 2 * capacity),
            GS_MAX_INSTANCES);
        continue;
      }
      GS_SRV_TRY(check(st, "bin_sort"));
      break;
    }
    gs_opts opts{};
    for (int c = 0; c < 3; ++c) opts.bg[c] = cfg.bg[c];
    int64_t px_total = 0, tiles_total = 0;
    for (int j = 0; j < B; ++j) {
      px_total += (int64_t)cams_host[j].width * cams_host[j].height;
      tiles_total += tiles_of(cams_host[j].width, cams_host[j].height);
    }
    GS_SRV_HIP(images.ensure((size_t)(3 * px_total)), "images");
    if (B == 1) {
      GS_SRV_HIP(final_T.ensure((size_t)px_total), "final transmittance");
      GS_SRV_HIP(n_contrib.ensure((size_t)px_total), "last contributors");
      GS_SRV_TRY(check(gs_render_fwd(ctx, &proj, &lists, cams_host, cams_dev.p, 1, &opts, images.p,
                                     final_T.p, n_contrib.p, stream),
                       "render"));
    } else {
      const size_t need = gs_render_batched_workspace_size(B);
      GS_SRV_HIP(ws_batch.ensure(need), "batch workspace");
      GS_SRV_TRY(check(gs_render_fwd_batched(ctx, &proj, &lists, cams_host, cams_dev.p, B, &opts,
                                             images.p, ws_batch.p, ws_batch.n, stream),
                       "batched render"));
    }
    if (out) {
      size_t off = 0;
      for (int j = 0; j < B; ++j) {
        const size_t cnt = (size_t)3 * cams_host[j].width * cams_host[j].height;
        float* dst = out[order[j]];
        if (dst)
          GS_SRV_HIP(hipMemcpyAsync(dst, images.p + off, cnt * sizeof(float),
                                    hipMemcpyDeviceToDevice, stream),
                     "image copy");
        off += cnt;
      }
    }
    GS_SRV_HIP(hipStreamSynchronize(stream), "stream synchronise");
    inst_per_tile = 0.8 * inst_per_tile + 0.2 * (double)lists.count / (double)std::max<int64_t>(tiles_total, 1);
    return GS_OK;
  }
#undef GS_SRV_TRY
#undef GS_SRV_HIP
};

}  // namespace

struct gs_server {
  int device = 0;
  gs_sequence seq{};
  gs_server_config cfg{};
  std::vector<std::unique_ptr<Renderer>> workers;
  std::unique_ptr<Renderer> solo;
  // statistics of the last run
  int64_t batches = 0, batched_requests = 0, inline_requests = 0, max_batch_seen = 0;
  int64_t max_in_flight = 0;
  char err[256] = "";
};

namespace {

// Device-memory estimate of one request in a batch: projected records and
// sort buffers per Gaussian, 1.5x the running instances per tile times its
// tiles for the lists and their sort buffers, and its image.
int64_t request_bytes(const gs_request& r, int ld, double inst_per_tile) {
  const int64_t t = tiles_of(r.cam.width, r.cam.height);
  const double inst = 1.5 * inst_per_tile * (double)t;
  return (int64_t)(89.0 * ld + 28.0 * ld + 24.0 * inst + 12.0 * (double)r.cam.width * r.cam.height);
}

}  // namespace

extern "C" {

static gs_status server_create(gs_server** out, int device, const gs_sequence* seq,
                               const gs_server_config* cfg) {
  if (!out || !seq || !cfg) return GS_ERR_INVALID_ARG;
  *out = nullptr;
  if (cfg->max_batch < 1 || cfg->max_batch > 4096 || cfg->n_workers < 1 || cfg->n_workers > 16 ||
      cfg->budget_bytes <= 0)
    return GS_ERR_INVALID_ARG;
  if (!seq->anchor.mean || !seq->anchor.quat || !seq->anchor.opacity || !seq->anchor.log_scale ||
      !seq->anchor.sh || !seq->deltas || !seq->masks || seq->n_frames < 1 || seq->anchor.n <= 0 ||
      seq->anchor.ld < seq->anchor.n || seq->anchor.ld % 64 != 0 ||
      (int64_t)seq->gw * seq->gh < seq->anchor.n)
    return GS_ERR_INVALID_ARG;
  gs_server* s = new (std::nothrow) gs_server();
  if (!s) return GS_ERR_OOM;
  s->device = device;
  s->seq = *seq;
  s->cfg = *cfg;
  for (int w = 0; w < cfg->n_workers; ++w) {
    s->workers.emplace_back(new (std::nothrow) Renderer());
    if (!s->workers.back() || s->workers.back()->init(device, &s->seq, s->cfg) != GS_OK) {
      delete s;
      return GS_ERR_HIP;
    }
  }
  s->solo.reset(new (std::nothrow) Renderer());
  if (!s->solo || s->solo->init(device, &s->seq, s->cfg) != GS_OK) {
    delete s;
    return GS_ERR_HIP;
  }
  *out = s;
  return GS_OK;
}

gs_status gs_server_create(gs_server** out, int device, const gs_sequence* seq,
                           const gs_server_config* cfg) {
  try {
    return server_create(out, device, seq, cfg);
  } catch (...) {
    return GS_ERR_OOM;
  }
}

void gs_server_destroy(gs_server* s) { delete s; }

const char* gs_server_last_error(const gs_server* s) { return s ? s->err : ""; }

gs_status gs_server_stats(const gs_server* s, int64_t* out) {
  if (!s || !out) return GS_ERR_INVALID_ARG;
  out[0] = s->batches;
  out[1] = s->batched_requests;
  out[2] = s->inline_requests;
  out[3] = s->max_batch_seen;
  out[4] = s->max_in_flight;
  return GS_OK;
}

// Sleeps until shortly before t, then polls the clock: a timed sleep alone
// wakes tens of microseconds late (timer slack and the thread's wake-up),
// which would add to every request's latency.  Both serving modes wait for
// arrivals this way.
constexpr auto kPollWindow = std::chrono::microseconds(200);
static void wait_until_precise(Clock::time_point t) {
  if (Clock::now() + kPollWindow < t) std::this_thread::sleep_until(t - kPollWindow);
  while (Clock::now() < t) {
  }
}

static gs_status server_run(gs_server* s, const gs_request* reqs, int n, int plain,
                           double* t_start, double* t_done, float* const* images) {
  if (!s || (n > 0 && (!reqs || !t_start || !t_done)) || n < 0) return GS_ERR_INVALID_ARG;
  for (int i = 0; i < n; ++i) {
    if (reqs[i].frame < 0 || reqs[i].frame >= s->seq.n_frames || reqs[i].cam.width <= 0 ||
        reqs[i].cam.height <= 0 || !(reqs[i].arrival_s >= 0.0) ||
        (i > 0 && reqs[i].arrival_s < reqs[i - 1].arrival_s)) {
      snprintf(s->err, sizeof(s->err), "request %d: bad frame, size or arrival order", i);
      return GS_ERR_INVALID_ARG;
    }
  }
  s->batches = s->batched_requests = s->inline_requests = s->max_batch_seen = 0;
  s->max_in_flight = 0;
  s->err[0] = 0;
  if (n == 0) return GS_OK;
  if (hipSetDevice(s->device) != hipSuccess) return GS_ERR_HIP;
  const auto t0 = Clock::now();
  auto since = [&](Clock::time_point t) {
    return std::chrono::duration<double>(t - t0).count();
  };
  auto at = [&](double sec) {
    return t0 + std::chrono::duration_cast<Clock::duration>(std::chrono::duration<double>(sec));
  };
  for (int i = 0; i < n; ++i) t_start[i] = t_done[i] = NAN;

  if (plain) {
    for (int i = 0; i < n; ++i) {
      wait_until_precise(at(reqs[i].arrival_s));
      t_start[i] = since(Clock::now());
      const gs_status st = s->solo->render(reqs, &i, 1, images);
      t_done[i] = since(Clock::now());
      if (st != GS_OK) {
        snprintf(s->err, sizeof(s->err), "request %d: %s", i, s->solo->err);
        return st;
      }
    }
    return GS_OK;
  }

  const int W = (int)s->workers.size();
  const int ld = s->seq.anchor.ld;
  std::mutex mu;
  std::condition_variable cv_sched;
  std::vector<std::condition_variable> cv_w(W);
  struct Job {
    std::vector<int> ids;
    int64_t bytes = 0;
    bool has = false;
  };
  std::vector<Job> job(W);
  std::vector<int> free_w;
  for (int w = 0; w < W; ++w) free_w.push_back(w);
  // instances per tile seen by each worker, copied under the lock
  std::vector<double> ipt_w(W, 600.0);
  int64_t in_flight = 0;
  int done = 0;
  bool stop = false;
  gs_status first_err = GS_OK;
  double solo_ms = 0.5, gap_ema = INFINITY;
  double last_arrival = -1.0;

  auto finish = [&](int w_or_solo, const std::vector<int>& ids, int64_t bytes, gs_status st,
                    const char* msg, double td) {
    for (int id : ids) t_done[id] = st == GS_OK ? td : INFINITY;
    if (st != GS_OK && first_err == GS_OK) {
      first_err = st;
      snprintf(s->err, sizeof(s->err), "%s", msg);
    }
    in_flight -= bytes;
    if (w_or_solo >= 0) free_w.push_back(w_or_solo);
    done += (int)ids.size();
  };

  std::vector<std::thread> threads;
  for (int w = 0; w < W; ++w) {
    threads.emplace_back([&, w]() {
      hipSetDevice(s->device);
      std::unique_lock<std::mutex> lk(mu);
      for (;;) {
        cv_w[w].wait(lk, [&] { return job[w].has || stop; });
        if (!job[w].has) return;
        Job j = std::move(job[w]);
        job[w] = Job();
        lk.unlock();
        const double ts = since(Clock::now());
        for (int id : j.ids) t_start[id] = ts;
        const gs_status st = s->workers[w]->render(reqs, j.ids.data(), (int)j.ids.size(), images);
        const double td = since(Clock::now());
        lk.lock();
        ipt_w[w] = s->workers[w]->inst_per_tile;
        finish(w, j.ids, j.bytes, st, s->workers[w]->err, td);
        cv_sched.notify_one();
      }
    });
  }

  {
    std::unique_lock<std::mutex> lk(mu);
    std::vector<int> pending;  // FIFO of arrived request indices
    pending.reserve((size_t)n);
    std::vector<int> batch;    // reused, so that forming a batch allocates nothing
    batch.reserve((size_t)s->cfg.max_batch);
    size_t head = 0;
    int next = 0;
    while (done < n) {
      const double now = since(Clock::now());
      while (next < n && reqs[next].arrival_s <= now) {
        if (last_arrival >= 0.0) {
          const double g = reqs[next].arrival_s - last_arrival;
          gap_ema = std::isinf(gap_ema) ? g : 0.9 * gap_ema + 0.1 * g;
        }
        last_arrival = reqs[next].arrival_s;
        pending.push_back(next++);
      }
      if (head < pending.size() && !free_w.empty()) {
        double ipt = 0.0;
        for (double v : ipt_w) ipt = std::max(ipt, v);
        batch.clear();
        int64_t bytes = 0;
        while (head < pending.size() && (int)batch.size() < s->cfg.max_batch) {
          const int64_t need = request_bytes(reqs[pending[head]], ld, ipt);
          if (in_flight + bytes + need > s->cfg.budget_bytes && (!batch.empty() || in_flight > 0))
            break;
          batch.push_back(pending[head++]);
          bytes += need;
        }
        if (!batch.empty()) {
          s->batches += 1;
          s->max_batch_seen = std::max<int64_t>(s->max_batch_seen, (int64_t)batch.size());
          in_flight += bytes;
          s->max_in_flight = std::max(s->max_in_flight, in_flight);
          const bool idle = (int)free_w.size() == W;
          if (s->cfg.inline_singletons && batch.size() == 1 && idle &&
              gap_ema > 2.5 * solo_ms * 1e-3) {
            s->inline_requests += 1;
            lk.unlock();
            const auto ta = Clock::now();
            t_start[batch[0]] = since(ta);
            const gs_status st = s->solo->render(reqs, batch.data(), 1, images);
            const auto tb = Clock::now();
            solo_ms = 0.8 * solo_ms + 0.2 * std::chrono::duration<double, std::milli>(tb - ta).count();
            lk.lock();
            ipt_w[0] = std::max(ipt_w[0], s->solo->inst_per_tile);
            finish(-1, batch, bytes, st, s->solo->err, since(tb));
          } else {
            s->batched_requests += (int64_t)batch.size();
            const int w = free_w.back();  // the most recently freed worker
            free_w.pop_back();
            job[w].ids.assign(batch.begin(), batch.end());
            job[w].bytes = bytes;
            job[w].has = true;
            cv_w[w].notify_one();
          }
          continue;
        }
      }
      if (next < n) {
        const auto t_next = at(reqs[next].arrival_s);
        // requests that wait for a worker are served when one finishes
        const bool queued = head < pending.size();
        if (!queued && Clock::now() + kPollWindow >= t_next) {
          // nothing queued and an arrival imminent: poll for it without the
          // lock
          lk.unlock();
          wait_until_precise(t_next);
          lk.lock();
        } else {
          // sleep until the poll window opens (or the arrival, with requests
          // queued), or a worker finishes
          const auto wake = queued ? t_next : t_next - kPollWindow;
          cv_sched.wait_until(lk, std::min(wake, Clock::now() + std::chrono::milliseconds(50)));
        }
      } else {
        cv_sched.wait_for(lk, std::chrono::milliseconds(50));
      }
    }
    stop = true;
    for (int w = 0; w < W; ++w) cv_w[w].notify_one();
  }
  for (auto& t : threads) t.join();
  return first_err;
}

gs_status gs_server_run(gs_server* s, const gs_request* reqs, int n, int plain, double* t_start,
                        double* t_done, float* const* images) {
  try {
    return server_run(s, reqs, n, plain, t_start, t_done, images);
  } catch (...) {
    // thread creation or a host allocation failed before any thread started
    if (s) snprintf(s->err, sizeof(s->err), "host resources exhausted");
    return GS_ERR_OOM;
  }
}

}  // extern "C"
