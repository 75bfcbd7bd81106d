"""Continuous-batching view server over a resident dynamic scene.

A sequence is an anchor Gaussian set plus one (8, gh, gw) delta-image set and
pruning mask per frame, all resident in HBM (frame t = anchor + D'_t, AirGS
Eq. (12); one texel per Gaussian, Eq. (3)).  A request asks for (frame,
viewpoint, resolution).  The server

* admits arrived requests while their estimated device memory fits an HBM
  budget (requests that do not fit wait for memory to be released);
* forms a batch from the admitted requests whenever one of its workers is
  free, so requests that arrive while others are on the GPU join the next
  batch;
* runs each batch on its worker's own HIP stream: one apply per distinct
  frame, projection per frame group, one joint bin + sort over all requests
  (the request is the high part of the segment id), and one persistent
  render launch over the shared (request, tile) queue;
* keeps two workers so one batch's projection and sorting overlap another
  batch's rendering on the device;
* renders a batch of one request with the plain kernel sequence (the same
  image bit for bit; it skips the batch bookkeeping launch and the shared
  queue, which only pay off when requests share a launch);
* when every worker is idle, a single request is waiting and arrivals are
  sparse (the observed mean gap between arrivals is more than 2.5 times
  the observed render time of a lone request), renders it on the
  scheduler's own thread with a plain renderer of its own: a lone request
  then pays no hand-off to another thread (measured at about 0.07 ms of
  extra render time there); at higher rates a request arriving during such
  a render would wait for it, so the workers take every batch.

``PlainRenderer`` is the comparison: one request at a time, each with its own
apply, project, bin_sort and render launches.

The scheduler and workers are host threads; every device step is a C ABI call
(the ctypes calls release the interpreter lock).
"""
from __future__ import annotations

import collections
import concurrent.futures
import math
import queue
import threading
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import gs, scenes
from .raster import Rasterizer, frame_of

RESOLUTIONS = ((640, 480), (1280, 720), (1920, 1080))


@dataclass
class Request:
    rid: int
    frame: int
    cam: tuple          # (R, t, f, (W, H)) host camera
    arrival: float      # seconds on the trace clock
    viewer: int = 0
    t_start: float = math.nan   # its batch began rendering (trace clock)
    t_done: float = math.nan
    image: torch.Tensor | None = field(default=None, repr=False)

    @property
    def wh(self):
        return self.cam[3]


class ResidentSequence:
    """Anchor + per-frame delta images and masks, resident on the device."""

    def __init__(self, anchor_scene: dict, n_frames: int, seed: int = 0,
                 levels=(0.1, 0.3, 0.5), device="cuda"):
        self.anchor = gs.Gaussians.from_scene(anchor_scene, device)
        n = anchor_scene["n"]
        self.n = n
        self.gw = self.gh = scenes.grid_side(n)
        self.n_frames = n_frames
        self.deltas = torch.empty(n_frames, 8, self.gh, self.gw, device=device)
        self.masks = torch.empty(n_frames, self.gh, self.gw, dtype=torch.uint8, device=device)
        self.levels = [levels[f % len(levels)] for f in range(n_frames)]
        self.seed = seed
        with concurrent.futures.ThreadPoolExecutor(max_workers=8) as ex:
            for f, (d, m) in enumerate(ex.map(self.frame_inputs, range(n_frames))):
                self.deltas[f].copy_(torch.from_numpy(d))
                self.masks[f].copy_(torch.from_numpy(m))

    def frame_inputs(self, f: int, seed: int | None = None):
        """Host copy of frame f's delta images and mask (same generator)."""
        seed = self.seed if seed is None else seed
        d = scenes.make_delta(self.n, self.gw, self.gh, 10_000 + seed * 1000 + f)
        m = scenes.prune_mask(d, self.n, self.levels[f])
        return d, m

    def device_bytes(self) -> int:
        return (self.deltas.numel() * 4 + self.masks.numel() +
                sum(t.numel() * 4 for t in self.anchor.planes()))


def make_trace(n_requests: int | None, rate: float, duration: float, n_viewers: int, n_frames: int,
               seed: int, resolutions=RESOLUTIONS, r_lo=4.0, r_hi=6.0):
    """Open-loop Poisson arrivals at aggregate ``rate`` from ``n_viewers``
    viewers; each request: frame uniform in [0, n_frames), viewpoint uniform
    on a sphere of radius U[r_lo, r_hi] looking at the origin, resolution
    uniform over ``resolutions``."""
    g = scenes.rng(seed)
    t = 0.0
    out = []
    while True:
        t += g.exponential(1.0 / rate)
        if (duration is not None and t > duration) or (n_requests is not None and
                                                       len(out) >= n_requests):
            break
        W, H = resolutions[int(g.integers(len(resolutions)))]
        cam = scenes.sphere_camera(g, r_lo, r_hi, W, H)
        out.append(Request(len(out), int(g.integers(n_frames)), cam, t,
                           viewer=int(g.integers(n_viewers))))
    return out


class BatchWorker:
    """Renders batches of requests on its own stream and context."""

    def __init__(self, seq: ResidentSequence, device="cuda", bg=(0.0, 0.0, 0.0)):
        self.seq = seq
        self.device = device
        self.bg = bg
        self.stream = torch.cuda.Stream(device=device)
        self.ctx = gs.Context(torch.cuda.current_device())
        # opacity-aware tile rectangles: same images, shorter lists
        self.raster = Rasterizer(ctx=self.ctx, capacity=1 << 22, tight_rect=True,
                                 tile_spans=True)
        self.frames: list[gs.Gaussians] = []
        self._proj = None
        self._ws = None
        self.plain = PlainRenderer(seq, device, bg, ctx=self.ctx, stream=self.stream)
        self.instances_per_tile = 600.0

    def _frame_buffers(self, k):
        while len(self.frames) < k:
            self.frames.append(frame_of(self.seq.anchor))
        return self.frames[:k]

    def _projected(self, B):
        if self._proj is None or self._proj.V < B:
            self._proj = gs.Projected.empty(max(B, 8), self.seq.n, self.seq.anchor.ld, self.device)
            self._proj.options = gs.GS_PROJECT_TIGHT_RECT | gs.GS_PROJECT_TILE_SPANS
        return self._proj.slice(0, B)

    def render_one(self, r: Request):
        """A batch of one request: the plain renderer's own sequence (apply,
        project, bin + sort, one compositing launch) on this worker's
        context and stream."""
        image = self.plain.render(r)
        w, h = r.wh
        tiles = math.ceil(w / 16) * math.ceil(h / 16)
        count = self.plain.raster._lists.count
        self.instances_per_tile = 0.8 * self.instances_per_tile + 0.2 * count / max(tiles, 1)
        return image, [image]

    def render(self, reqs: list[Request]):
        """Render a batch; returns the packed image buffer and per-request
        views (request order as given)."""
        if len(reqs) == 1:
            return self.render_one(reqs[0])
        seq = self.seq
        order = sorted(range(len(reqs)), key=lambda k: reqs[k].frame)
        reqs_o = [reqs[k] for k in order]
        with torch.cuda.stream(self.stream):
            frames = sorted({r.frame for r in reqs_o})
            bufs = self._frame_buffers(len(frames))
            slot = {}
            for fb, f in zip(bufs, frames):
                gs.gs_apply_frame_update(self.ctx, seq.anchor, seq.deltas[f], seq.masks[f], seq.gw,
                                         seq.gh, fb, self.stream)
                slot[f] = fb
            cams = gs.Cameras.from_list([r.cam for r in reqs_o], self.device)
            B = len(reqs_o)
            proj = self._projected(B)
            start = 0
            while start < B:
                f = reqs_o[start].frame
                end = start
                while end < B and reqs_o[end].frame == f:
                    end += 1
                gs.gs_project(self.ctx, slot[f], cams.slice(start, end - start),
                              proj.slice(start, end - start), self.stream)
                start = end
            lists = self.raster.bin_sort(proj, cams, self.stream)
            pix = [w * h for (w, h) in cams.wh]
            images = torch.empty(3 * sum(pix), device=self.device)
            need = gs.render_batched_workspace_size(B)
            if self._ws is None or self._ws.numel() < need:
                self._ws = torch.empty(need, dtype=torch.uint8, device=self.device)
            gs.gs_render_fwd_batched(self.ctx, proj, lists, cams, self.bg, images, self._ws,
                                     self.stream)
            done = torch.cuda.Event()
            done.record(self.stream)
        done.synchronize()
        tiles = sum(math.ceil(w / 16) * math.ceil(h / 16) for (w, h) in cams.wh)
        self.instances_per_tile = 0.8 * self.instances_per_tile + 0.2 * lists.count / max(tiles, 1)
        off = 0
        out = [None] * len(reqs)
        for k, r in zip(order, reqs_o):
            w, h = r.wh
            out[k] = images[off:off + 3 * w * h].view(3, h, w)
            off += 3 * w * h
        return images, out


class PlainRenderer:
    """One request per launch sequence: apply, project, bin_sort, render.
    ``ctx`` and ``stream`` default to ones of its own."""

    def __init__(self, seq: ResidentSequence, device="cuda", bg=(0.0, 0.0, 0.0), ctx=None,
                 stream=None):
        self.seq = seq
        self.device = device
        self.bg = bg
        self.stream = stream if stream is not None else torch.cuda.Stream(device=device)
        self.ctx = ctx if ctx is not None else gs.Context(torch.cuda.current_device())
        self.raster = Rasterizer(ctx=self.ctx, capacity=1 << 22, tight_rect=True,
                                 tile_spans=True)
        self.frame = frame_of(seq.anchor)

    def render(self, r: Request) -> torch.Tensor:
        seq = self.seq
        with torch.cuda.stream(self.stream):
            gs.gs_apply_frame_update(self.ctx, seq.anchor, seq.deltas[r.frame], seq.masks[r.frame],
                                     seq.gw, seq.gh, self.frame, self.stream)
            cams = gs.Cameras.from_list([r.cam], self.device)
            out = self.raster.forward(self.frame, cams, self.bg, self.stream)
            done = torch.cuda.Event()
            done.record(self.stream)
        done.synchronize()
        return out["image"][0]


def request_bytes(r: Request, n_ld: int, instances_per_tile: float) -> int:
    """Device-memory estimate of one request in a batch: projected records,
    instance lists with sort buffers, and its image."""
    w, h = r.wh
    tiles = math.ceil(w / 16) * math.ceil(h / 16)
    inst = 1.5 * instances_per_tile * tiles
    return int(89 * n_ld + 28 * n_ld + 24 * inst + 12 * w * h)


class Server:
    """Continuous batching: admission against an HBM budget, batches formed
    whenever a worker is free, ``n_workers`` batches in flight."""

    def __init__(self, seq: ResidentSequence, budget_bytes: int, max_batch: int = 32,
                 n_workers: int = 2, device="cuda", keep_images: bool = False, workers=None,
                 inline_singletons: bool = True):
        self.seq = seq
        self.budget = int(budget_bytes)
        self.max_batch = max_batch
        self.workers = workers if workers is not None else [BatchWorker(seq, device)
                                                            for _ in range(n_workers)]
        self.keep_images = keep_images
        self.inline_singletons = inline_singletons
        # the scheduler thread's own renderer for lone requests on an idle
        # server (its own context and stream)
        self.solo = (PlainRenderer(seq, device) if inline_singletons and workers is None
                     else None)
        self.solo_ms = 0.5  # running estimate of a lone request's render time
        self.lock = threading.Condition()
        self.in_flight_bytes = 0
        self.max_in_flight_bytes = 0
        self.batches = []
        self.errors = []

    def _estimate(self, r):
        ipt = max(w.instances_per_tile for w in self.workers)
        return request_bytes(r, self.seq.anchor.ld, ipt)

    def run(self, trace: list[Request], clock_start: float | None = None):
        """Serve ``trace`` in real time; fills each request's t_start and
        t_done.  One long-lived thread per worker blocks on its own queue, so
        handing it a batch wakes only that thread; a lone request on an idle
        server is rendered on this thread."""
        t0 = time.perf_counter() if clock_start is None else clock_start
        pending = collections.deque()
        free = collections.deque(self.workers)
        inbox = {id(w): queue.SimpleQueue() for w in self.workers}
        next_idx = 0
        done_count = [0]
        # mean gap between the arrivals seen so far (exponential average)
        gap_ema = [math.inf]
        last_arrival = [None]

        def render_batch(worker, batch, nbytes, solo=False):
            start = time.perf_counter() - t0
            for r in batch:
                r.t_start = start
            try:
                if solo:
                    t_solo = time.perf_counter()
                    imgs = [self.solo.render(batch[0])]
                    self.solo_ms = 0.8 * self.solo_ms + 0.2 * (time.perf_counter() - t_solo) * 1e3
                else:
                    _, imgs = worker.render(batch)
                now = time.perf_counter() - t0
                for r, im in zip(batch, imgs):
                    r.t_done = now
                    if self.keep_images:
                        r.image = im.clone()
            except Exception as e:  # noqa: BLE001 - reported after the run
                self.errors.append(e)
                for r in batch:
                    r.t_done = math.inf
            with self.lock:
                self.in_flight_bytes -= nbytes
                free.append(worker)
                done_count[0] += len(batch)
                self.lock.notify_all()

        def serve_loop(worker):
            box = inbox[id(worker)]
            while True:
                item = box.get()
                if item is None:
                    return
                render_batch(worker, *item)

        threads = [threading.Thread(target=serve_loop, args=(w,), daemon=True)
                   for w in self.workers]
        for th in threads:
            th.start()
        try:
            while True:
                inline = None
                with self.lock:
                    now = time.perf_counter() - t0
                    while next_idx < len(trace) and trace[next_idx].arrival <= now:
                        a = trace[next_idx].arrival
                        if last_arrival[0] is not None:
                            g = a - last_arrival[0]
                            gap_ema[0] = g if math.isinf(gap_ema[0]) else 0.9 * gap_ema[0] + 0.1 * g
                        last_arrival[0] = a
                        pending.append(trace[next_idx])
                        next_idx += 1
                    if done_count[0] >= len(trace):
                        break
                    launched = False
                    if pending and free:
                        batch, nbytes = [], 0
                        while pending and len(batch) < self.max_batch:
                            need = self._estimate(pending[0])
                            if self.in_flight_bytes + nbytes + need > self.budget and (
                                    batch or self.in_flight_bytes > 0):
                                break
                            batch.append(pending.popleft())
                            nbytes += need
                        if batch:
                            # the most recently freed worker: at low load one
                            # worker serves every request, so its buffers stay
                            # warm in the caches and its TLB entries resident
                            worker = free.pop()
                            self.in_flight_bytes += nbytes
                            self.max_in_flight_bytes = max(self.max_in_flight_bytes,
                                                           self.in_flight_bytes)
                            self.batches.append(len(batch))
                            if (self.inline_singletons and len(batch) == 1
                                    and len(free) == len(self.workers) - 1
                                    and gap_ema[0] > 2.5 * self.solo_ms * 1e-3):
                                inline = (worker, batch, nbytes, self.solo is not None)
                            else:
                                inbox[id(worker)].put((batch, nbytes))
                            launched = True
                    if not launched:
                        wait = 0.05
                        if next_idx < len(trace):
                            wait = min(wait, max(trace[next_idx].arrival - now, 0.0))
                        self.lock.wait(timeout=wait if wait > 0 else 0.0005)
                if inline is not None:
                    render_batch(*inline)
        finally:
            for w in self.workers:
                inbox[id(w)].put(None)
            for th in threads:
                th.join()
        if self.errors:
            raise self.errors[0]
        return trace


def run_plain(renderer: PlainRenderer, trace: list[Request], clock_start: float | None = None,
              keep_images: bool = False):
    """Serve the trace one request at a time, FIFO, in real time."""
    t0 = time.perf_counter() if clock_start is None else clock_start
    for r in trace:
        now = time.perf_counter() - t0
        if r.arrival > now:
            time.sleep(r.arrival - now)
        r.t_start = time.perf_counter() - t0
        img = renderer.render(r)
        r.t_done = time.perf_counter() - t0
        if keep_images:
            r.image = img.clone()
    return trace


def summarize(trace: list[Request], warmup: float = 0.0) -> dict:
    meas = [r for r in trace if r.arrival >= warmup]
    lat = np.array([r.t_done - r.arrival for r in meas]) * 1e3
    if len(meas) == 0:
        return dict(views=0)
    span = max(r.t_done for r in meas) - min(r.arrival for r in meas)
    out = dict(views=len(meas), views_per_s=round(len(meas) / span, 2),
               p50_ms=round(float(np.percentile(lat, 50)), 3),
               p99_ms=round(float(np.percentile(lat, 99)), 3),
               mean_ms=round(float(lat.mean()), 3))
    wait = np.array([r.t_start - r.arrival for r in meas]) * 1e3
    if np.all(np.isfinite(wait)):
        # arrival -> its batch starts, and the batch's own render time
        out["mean_wait_ms"] = round(float(wait.mean()), 3)
        out["mean_render_ms"] = round(float((lat - wait).mean()), 3)
    return out


class NativeServer:
    """The library's native server (gs_server_*): the scheduler runs in C++
    on the calling thread (the ctypes call releases the interpreter lock) and
    every worker is a native thread with its own context, stream and
    buffers; ``run(..., plain=True)`` is the one-request-at-a-time
    comparison on the same native path."""

    def __init__(self, seq: ResidentSequence, budget_bytes: int, max_batch: int = 32,
                 n_workers: int = 2, inline_singletons: bool = True, bg=(0.0, 0.0, 0.0),
                 options: int = gs.GS_PROJECT_TIGHT_RECT | gs.GS_PROJECT_TILE_SPANS):
        import ctypes
        self.ct = ctypes
        self.lib = gs.load()
        self.seq = seq  # keeps the resident device buffers alive
        sq = gs.GsSequence(seq.anchor.c(), ctypes.c_void_p(seq.deltas.data_ptr()),
                           ctypes.c_void_p(seq.masks.data_ptr()), seq.n_frames, seq.gw, seq.gh, 0)
        cfg = gs.GsServerConfig(int(max_batch), int(n_workers), int(options),
                                1 if inline_singletons else 0, int(budget_bytes),
                                (ctypes.c_float * 3)(*[float(x) for x in bg]), 0.0)
        h = ctypes.c_void_p()
        torch.cuda.synchronize()
        st = self.lib.gs_server_create(ctypes.byref(h), torch.cuda.current_device(),
                                       ctypes.byref(sq), ctypes.byref(cfg))
        if st != gs.GS_OK:
            raise gs.GsError(st, "gs_server_create failed")
        self.handle = h
        self.max_batch = max_batch

    @staticmethod
    def _camera(cam, c):
        R, t, f, (W, H) = cam
        c.R[:] = np.asarray(R, np.float64).reshape(9).tolist()
        c.t[:] = np.asarray(t, np.float64).reshape(3).tolist()
        c.fx, c.fy, c.cx, c.cy = (float(x) for x in np.asarray(f, np.float64).reshape(4))
        c.width, c.height = int(W), int(H)

    def run(self, trace: list[Request], plain: bool = False, keep_images: bool = False):
        """Serve ``trace`` (arrivals non-decreasing) in real time; fills each
        request's t_start and t_done (and image with ``keep_images``)."""
        ct = self.ct
        n = len(trace)
        reqs = (gs.GsRequest * n)()
        for k, r in enumerate(trace):
            self._camera(r.cam, reqs[k].cam)
            reqs[k].frame = int(r.frame)
            reqs[k].arrival_s = float(r.arrival)
        ts = (ct.c_double * n)()
        td = (ct.c_double * n)()
        imgs, ptrs = None, None
        if keep_images:
            imgs = [torch.empty(3, r.wh[1], r.wh[0], device="cuda") for r in trace]
            ptrs = (ct.c_void_p * n)(*[t.data_ptr() for t in imgs])
        torch.cuda.synchronize()
        st = self.lib.gs_server_run(self.handle, reqs, n, 1 if plain else 0, ts, td, ptrs)
        for k, r in enumerate(trace):
            r.t_start, r.t_done = ts[k], td[k]
            if keep_images:
                r.image = imgs[k]
        if st != gs.GS_OK:
            raise gs.GsError(st, self.lib.gs_server_last_error(self.handle).decode())
        return trace

    def stats(self) -> dict:
        out = (self.ct.c_int64 * 5)()
        self.lib.gs_server_stats(self.handle, out)
        b, wr, inl, mx, peak = (int(x) for x in out)
        return {"batches": b, "worker_requests": wr, "inline_requests": inl, "max_batch": mx,
                "mean_batch": round((wr + inl) / b, 3) if b else None,
                "peak_in_flight_bytes": peak}

    def close(self):
        if getattr(self, "handle", None):
            self.lib.gs_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass
