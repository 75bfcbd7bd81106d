#!/usr/bin/env python3
"""Benchmark of the MI355X Gaussian-splatting rasterizer.

Workload (timed step): the per-frame training step on a synthetic frame of
300,000 Gaussians (means U[-3,3]^3, log-scales N(-4,0.5), SH degree 3),
20 cameras on a 120-degree arc at radius 5, 1352x1014 images: project, bin +
depth sort, render forward, L1 loss, render backward, projection backward,
fused Adam over all 59 parameter planes.  Inputs are resident in HBM before
timing starts.  ``value`` = training iterations/s on one GPU.

The same JSON line also carries: the temporal frame-update step (apply the
548x548 delta images, render, L1 + the temporal term of Eq. (7) with
lambda_t = 1e-3, backward to the deltas, Adam on the deltas);
per-stage device times from HIP events; the roofline of the dominant kernel;
and the FP64 CPU oracle timed on a bounded sample of the same workload.

    python bench.py [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# Published MI355X FP32 vector peak.  The library is compiled without packed
# FP32 instructions, which caps the rate of executed FP32 arithmetic at half
# of it (78.6 TFLOP/s); the fraction is still reported against the published
# figure, and it counts the pairs the compositing definition evaluates, some
# of which the kernels skip cheaply (whole quadrants below alpha 1/255).
PEAK_ALU_TFLOPS = 157.3

# Algorithmic FP32 operations per (pixel, entry) pair, FMA counted as 2 and
# a transcendental as 1, on the definition's own formulas: forward = offsets,
# quadratic form, exp, alpha cap and the two tests, T update, weight and three
# colour FMAs; backward = that recompute plus the T recovery, colour, alpha
# and power gradients and their moments.
FLOP_PER_PAIR_FWD = 26
FLOP_PER_PAIR_BWD = 68


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-frame-step", action="store_true")
    # opacity-aware rectangles only, without the per-row spans (comparison)
    ap.add_argument("--no-tile-spans", action="store_true")
    ap.add_argument("--no-autograd-step", action="store_true")
    ap.add_argument("--views", type=int, default=20)
    ap.add_argument("--gaussians", type=int, default=300_000)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-dssim-step", action="store_true")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the pruning-sweep and sent-update codec legs")
    ap.add_argument("--serve-rates", default="500,2000,4000",
                    help="aggregate Poisson arrival rates (requests/s)")
    ap.add_argument("--serve-seconds", type=float, default=2.0)
    ap.add_argument("--serve-warmup", type=float, default=0.5)
    ap.add_argument("--serve-frames", type=int, default=300)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of known size (counter calibration)")
    return ap.parse_args()


def copy_calibration():
    import torch
    n = 1 << 28  # 1 GiB of FP32
    a = torch.ones(n, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 3}))


class TrainStep:
    """One per-frame training iteration on a fixed scene and camera set."""

    def __init__(self, scene, cams, target_scene, frame_update=None, loss="l1",
                 tile_spans=True):
        import torch

        from paper_2512_20943_amd import gs
        from paper_2512_20943_amd.raster import Rasterizer, frame_of
        self.torch = torch
        self.gs = gs
        self.ctx = gs.default_context()
        n, deg, ld = scene["n"], scene["deg"], scene["ld"]
        K = (deg + 1) ** 2
        # all parameter planes in one buffer so that Adam is one launch
        self.nparam = (3 + 3 + 4 + 1 + 3 * K) * ld
        self.flat = torch.empty(self.nparam, device="cuda")
        self.gflat = torch.zeros(self.nparam, device="cuda")
        self.m = torch.zeros(self.nparam, device="cuda")
        self.v = torch.zeros(self.nparam, device="cuda")

        def views(buf):
            o = 0
            out = []
            for shape in ((3, ld), (3, ld), (4, ld), (ld,), (K, 3, ld)):
                cnt = math.prod(shape)
                out.append(buf[o:o + cnt].view(*shape))
                o += cnt
            return out

        planes = views(self.flat)
        for t, key in zip(planes, ("mean", "log_scale", "quat", "opacity", "sh")):
            t.copy_(torch.from_numpy(scene[key]))
        self.g = gs.Gaussians(n, deg, ld, *planes)
        self.grad = gs.Gaussians(n, deg, ld, *views(self.gflat))
        self.cams = gs.Cameras(cams)
        # opacity-aware tile rectangles and per-row tile spans: the lists omit
        # (Gaussian, tile) pairs that no pixel of the tile can composite;
        # images and gradients are those of the full rectangles
        self.r = Rasterizer(capacity=1 << 25, tight_rect=True, tile_spans=tile_spans)
        tg = gs.Gaussians.from_scene(target_scene)
        self.target = self.r.forward(tg, self.cams)["image"].clone()
        self.dimg = torch.empty_like(self.target)
        self.loss = torch.zeros(1, dtype=torch.float64, device="cuda")
        self.loss_kind = loss
        if loss == "l1_dssim":
            planes = self.target.numel() // (self.target.shape[-1] * self.target.shape[-2])
            self.ws_ssim = torch.empty(
                gs.l1_dssim_workspace_size(planes, self.target.shape[-2], self.target.shape[-1]),
                dtype=torch.uint8, device="cuda")
        self.t = 0
        self.frame_update = frame_update
        if frame_update is not None:
            d, mask, gw, gh = frame_update
            self.delta = torch.from_numpy(d).cuda()
            self.mask = torch.from_numpy(mask).cuda()
            self.gw, self.gh = gw, gh
            self.frame = frame_of(self.g)
            self.dd = torch.zeros(8, gh, gw, device="cuda")
            self.dm = torch.zeros_like(self.dd)
            self.dv = torch.zeros_like(self.dd)
        self.last = None

    def step(self):
        gs = self.gs
        self.t += 1
        g = self.g
        if self.frame_update is not None:
            gs.gs_apply_frame_update(self.ctx, self.g, self.delta, self.mask, self.gw, self.gh,
                                     self.frame)
            g = self.frame
        self.loss.zero_()
        if self.loss_kind == "l1_dssim":
            out = self.r.forward(g, self.cams)
            gs.gs_l1_dssim_loss_grad(self.ctx, out["image"], self.target, self.dimg, self.loss,
                                     self.ws_ssim, 0.2)
        else:
            # the L1 term is evaluated where the forward composites its pixels
            out = self.r.forward_l1(g, self.cams, self.target, self.dimg, self.loss)
        if self.frame_update is None:
            self.r.backward(g, self.cams, out, self.dimg, self.grad)
            gs.gs_adam_step(self.ctx, self.flat, self.gflat, self.m, self.v, self.t)
        else:
            # Eq. (7): L1 + lambda_t L_temp on the deltas, lambda_t = 1e-3 (Sec. IV-A)
            self.r.backward(g, self.cams, out, self.dimg, self.grad,
                            upd=(self.g.quat, self.mask, self.gw, self.gh), dL_ddelta=self.dd,
                            temporal=(1e-3, self.delta, self.loss))
            gs.gs_adam_step(self.ctx, self.delta, self.dd, self.dm, self.dv, self.t)
        self.last = out


class AutogradTrainStep:
    """The same training step written as a user of torch.autograd would: the
    hand-written backward behind GSRender and the L1 term behind GSL1Loss,
    loss.backward(), then the Adam kernel on the flat parameter buffer."""

    def __init__(self, ts):
        import torch

        from paper_2512_20943_amd.raster import GSL1Loss, GSRender
        self.torch, self.gs, self.ts = torch, ts.gs, ts
        self.ctx = ts.ctx
        self.GSRender, self.GSL1Loss = GSRender, GSL1Loss
        self.flat = ts.flat.detach().clone().requires_grad_(True)
        self.m = torch.zeros_like(ts.m)
        self.v = torch.zeros_like(ts.v)
        self.t = 0
        g = ts.g
        self.meta = (ts.r, ts.cams, g.n, g.deg, (0.0, 0.0, 0.0))
        self.shapes = ((3, g.ld), (3, g.ld), (4, g.ld), (g.ld,), ((g.deg + 1) ** 2, 3, g.ld))
        self.last = None

    def step(self):
        self.t += 1
        self.flat.grad = None
        planes, o = [], 0
        for shape in self.shapes:
            cnt = math.prod(shape)
            planes.append(self.flat[o:o + cnt].view(*shape))
            o += cnt
        image = self.GSRender.apply(*planes, self.meta)
        loss = self.GSL1Loss.apply(image, self.ts.target, self.ctx)
        loss.backward()
        self.gs.gs_adam_step(self.ctx, self.flat.detach(), self.flat.grad, self.m, self.v,
                             self.t)


class SweepStep:
    """One pruning-level sweep of a frame (usage render, 11 masked frames,
    one batched render of every (level, view) pair, squared error per pair,
    level selection by Alg. 1 on the host)."""

    def __init__(self, scene, target_scene, n_views):
        import torch

        from paper_2512_20943_amd import gs, scenes
        from paper_2512_20943_amd.prune import PruningSweep
        from paper_2512_20943_amd.raster import Rasterizer
        self.torch, self.gs = torch, gs
        self.ctx = gs.default_context()
        n = scene["n"]
        gw = gh = scenes.grid_side(n)
        anchor = gs.Gaussians.from_scene(scene)
        delta = torch.from_numpy(scenes.make_delta(n, gw, gh, 2)).cuda()
        self.cams = gs.Cameras(scenes.arc_cameras(n_views, 5.0, 1352, 1014))
        self.sweep = PruningSweep(anchor, delta, gw, gh, self.cams, ctx=self.ctx)
        # the frame's reference views: the target scene's renders
        r = Rasterizer(ctx=self.ctx, capacity=1 << 25, tight_rect=True, tile_spans=True)
        self.reference = r.forward(gs.Gaussians.from_scene(target_scene), self.cams)["image"]
        self.reference = self.reference.clone()
        self.last = None

    def step(self):
        self.last = self.sweep.run(self.reference)


class CodecStep:
    """One frame of sent updates at the server and the client (Eq. (11),
    (12)): residual against what was sent, 8-bit quantisation with the
    server's running sum, and the client's dequantise + accumulate + apply."""

    # algorithmic bytes per texel: residual reads D, D' (32 B each) and the
    # mask (1 B) and writes d (32 B); quantisation reads d and D' and writes
    # the codes (8 B) and D'; the client reads the codes, D' and the anchor's
    # mean, quaternion and opacity (32 B) and writes D' and the frame's
    BYTES_PER_TEXEL = (32 + 32 + 1 + 32) + (32 + 32 + 8 + 32) + (8 + 32 + 32 + 32 + 32)

    def __init__(self, scene):
        import torch

        from paper_2512_20943_amd import gs, scenes
        from paper_2512_20943_amd.raster import frame_of
        self.torch, self.gs = torch, gs
        self.ctx = gs.default_context()
        n = scene["n"]
        self.n = n
        self.gw = self.gh = gw = scenes.grid_side(n)
        self.anchor = gs.Gaussians.from_scene(scene)
        self.frame = frame_of(self.anchor)
        ident = np.zeros((8, gw, gw), np.float32)
        ident[3] = 1.0
        d = scenes.make_delta(n, gw, gw, 3)
        self.D = torch.from_numpy(d).cuda()
        self.mask = torch.from_numpy(scenes.prune_mask(d, n, 0.3)).cuda()
        self.P_srv = torch.from_numpy(ident).cuda()
        self.P_cli = self.P_srv.clone()
        self.d = torch.empty_like(self.D)
        self.amax = torch.zeros(8, device="cuda")
        self.q = torch.empty((8, gw, gw), dtype=torch.int8, device="cuda")
        self.scale = torch.empty(8, device="cuda")

    def step(self):
        gs, c = self.gs, self.ctx
        self.amax.zero_()
        gs.gs_residual_delta(c, self.D, self.P_srv, self.mask, self.n, self.gw, self.gh, self.d,
                             self.amax)
        gs.gs_quantize_delta(c, self.d, self.amax, 8, self.n, self.gw, self.gh, self.q,
                             self.scale, self.P_srv)
        gs.gs_apply_quantized_update(c, self.anchor, self.q, 8, self.scale, self.P_cli, self.gw,
                                     self.gh, self.frame)


class CompactStep:
    """Keyframe compaction (Sec. III-B): cull the Gaussians whose opacity is
    below 0.005 (kept-index list, count read back) and gather all 59
    parameter planes of the kept ones into a dense set."""

    PLANES = 59
    EPS = 0.005

    def __init__(self, scene):
        import torch

        from paper_2512_20943_amd import gs
        self.torch, self.gs = torch, gs
        self.ctx = gs.default_context()
        self.n, ld = scene["n"], scene["ld"]
        rows = [np.asarray(scene[k], np.float32).reshape(-1, ld)
                for k in ("mean", "log_scale", "quat", "opacity", "sh")]
        self.src = torch.from_numpy(np.concatenate(rows, axis=0)).cuda()
        assert self.src.shape[0] == self.PLANES
        self.opacity = self.src[10]
        self.idx = torch.empty(self.n, dtype=torch.int32, device="cuda")
        self.dst = torch.empty_like(self.src)
        self.ws = torch.empty(max(gs.cull_workspace_size(self.n), 1), dtype=torch.uint8,
                              device="cuda")
        self.kept = 0

    def step(self):
        gs = self.gs
        self.kept = gs.gs_cull_low_opacity(self.ctx, self.opacity, self.n, self.EPS, self.idx,
                                           self.ws)
        gs.gs_gather_planes(self.ctx, self.src, self.idx, self.kept, self.dst)


def time_steps(ts, steps, warmup):
    torch = ts.torch
    for _ in range(warmup):
        ts.step()
    torch.cuda.synchronize()
    ts.ctx.set_timing(True)
    ts.ctx.collect_timing()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    for k in range(steps):
        ts.step()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stages = ts.ctx.collect_timing()
    ts.ctx.set_timing(False)
    return wall, e0.elapsed_time(e1) / 1e3, stages


def definition_pairs(ts):
    """Sum over pixels of n_contrib for full (3-sigma) tile rectangles: the
    (pixel, entry) pairs the compositing definition evaluates up to each
    pixel's last contributor.  The training step's opacity-aware rectangles
    leave out entries that every pixel skips, which shortens the lists and
    lowers n_contrib without changing the work the definition prescribes, so
    the count comes from one extra full-rectangle forward of the current
    parameters, outside the timed region."""
    if getattr(ts, "_def_pairs", None) is None:
        from paper_2512_20943_amd.raster import Rasterizer
        out = Rasterizer(capacity=1 << 26).forward(ts.g if ts.frame_update is None else ts.frame,
                                                   ts.cams)
        ts._def_pairs = float(out["n_contrib"].sum(dtype=ts.torch.float64).item())
        ts._def_instances = out["lists"].count
    return ts._def_pairs


def algorithmic_work(stage, ts, steps):
    """(amount per launch, unit, bound) for a stage of one step."""
    n, V, K = ts.g.n, ts.cams.V, (ts.g.deg + 1) ** 2
    M = ts.last["lists"].count
    pbytes = 4 * (11 + 3 * K)
    if stage == "render_fwd" or stage == "render_bwd":
        pairs = definition_pairs(ts)
        f = FLOP_PER_PAIR_FWD if stage == "render_fwd" else FLOP_PER_PAIR_BWD
        return pairs * f, "flop", "alu", pairs
    if stage == "project":
        return n * pbytes + V * n * 89.0, "byte", "hbm", None
    if stage == "project_bwd":
        return 2 * n * pbytes + V * n * (36.0 + 20 + 1), "byte", "hbm", None
    if stage == "segment_sort":
        passes = math.ceil(math.ceil(math.log2(max(ts.cams.n_segments(), 2))) / 8)
        return M * (16.0 * passes + 4.0), "byte", "hbm", None
    if stage == "depth_sort":
        passes = math.ceil((32 + math.ceil(math.log2(max(V, 1)) if V > 1 else 0)) / 8)
        return V * n * (24.0 * passes + 8 + 4 + 8 + 4), "byte", "hbm", None
    if stage == "adam":
        return 28.0 * ts.nparam, "byte", "hbm", None
    if stage == "l1":
        return 12.0 * ts.target.numel(), "byte", "hbm", None
    if stage == "dssim":
        return 44.0 * ts.target.numel(), "byte", "hbm", None
    if stage == "emit":
        return V * n * 8.0 + M * 8.0, "byte", "hbm", None
    return None


STAGE_SOURCE = {"render_fwd": "gs_render.hip", "render_bwd": "gs_render.hip",
                "project": "gs_project.hip", "project_bwd": "gs_project.hip",
                "depth_sort": "gs_sort.hip", "segment_sort": "gs_sort.hip", "emit": "gs_sort.hip",
                "adam": "gs_train.hip", "l1": "gs_train.hip",
                "dssim": "gs_ssim.hip"}


def counted_traffic(stage):
    """HBM bytes per launch of a stage's kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary (profiles/*.md, line 'traffic: ...'),
    scaled by the copy-kernel calibration recorded there; None when no
    summary exists or the kernel's source changed since it was taken."""
    import glob
    import hashlib
    src = STAGE_SOURCE.get(stage)
    if src is None:
        return None
    path = os.path.join(ROOT, "paper_2512_20943_amd", "csrc", src)
    digest = hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]
    for md in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        for line in open(md):
            if not line.startswith("traffic:"):
                continue
            kv = dict(tok.split("=", 1) for tok in line.split()[1:])
            if kv.get("stage") == stage and kv.get("source_sha256") == digest:
                return float(kv["bytes_per_launch"])
    return None


def roofline(stages, ts, steps):
    busy = {k: v for k, v in stages.items() if v[1] > 0}
    dom = max(busy, key=lambda k: busy[k][0])
    ms, launches = busy[dom]
    per_launch_s = ms / launches / 1e3
    w = algorithmic_work(dom, ts, steps)
    if w is None:
        return dom, None
    amount, unit, bound, pairs = w
    launches_per_step = launches / steps
    amount_per_launch = amount / launches_per_step
    if unit == "byte":
        achieved = amount_per_launch / per_launch_s / 1e9
        rf = dict(bound=bound, achieved=round(achieved, 2), peak=PEAK_HBM_GBS, unit="GB/s",
                  frac=round(achieved / PEAK_HBM_GBS, 4), traffic=counted_traffic(dom))
    else:
        achieved = amount_per_launch / per_launch_s / 1e12
        rf = dict(bound=bound, achieved=round(achieved, 3), peak=PEAK_ALU_TFLOPS, unit="TFLOP/s",
                  frac=round(achieved / PEAK_ALU_TFLOPS, 4), traffic=counted_traffic(dom))
    rf["kernel"] = dom
    rf["launch_ms"] = round(per_launch_s * 1e3, 4)
    if pairs is not None:
        rf["pairs_per_launch"] = pairs / launches_per_step
    return dom, rf


def cpu_baseline(scene, cams, target_scene):
    """FP64 oracle (as it stands) on one of the 20 views of the frame step:
    projection, bin + sort, render, L1, render backward, projection backward;
    plus Adam over all parameters once.  Scaled to a 20-view iteration."""
    import numpy as np

    import oracle
    oracle.build(force=False)
    cam1 = {k: v[:1] for k, v in cams.items()}
    t0 = time.perf_counter()
    _, _, timg = oracle.forward(target_scene, cam1)
    t_target = time.perf_counter() - t0
    t0 = time.perf_counter()
    P, L, img = oracle.forward(scene, cam1)
    _, gI = oracle.l1(img["image"], timg["image"])
    _, grads = oracle.backward(scene, cam1, P, L, gI)
    t_view = time.perf_counter() - t0
    t0 = time.perf_counter()
    flat = np.concatenate([scene[k].ravel() for k in ("mean", "log_scale", "quat", "opacity",
                                                        "sh")]).astype(np.float64)
    gflat = np.concatenate([grads[k].ravel() for k in ("mean", "log_scale", "quat", "opacity",
                                                         "sh")])
    oracle.adam(flat, gflat, np.zeros_like(flat), np.zeros_like(flat), 1)
    t_adam = time.perf_counter() - t0
    V = cams["R"].shape[0]
    t_iter = V * t_view + t_adam
    cores = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    return dict(value=round(1.0 / t_iter, 6), unit="iters/s", cores=cores, kind="oracle",
                sample=(f"1 of {V} views of the 300k-Gaussian frame step (project, bin+sort, "
                        f"render, L1, render bwd, project bwd: {t_view:.2f} s) x {V} + Adam over "
                        f"all parameters ({t_adam:.2f} s); target render {t_target:.2f} s "
                        f"not counted"))


def serving(args, scene):
    """Served views/s and p50/p99 latency of the continuous-batching server
    vs the plain one-request-per-launch renderer on the same Poisson trace:
    300 resident frames of the 300k-Gaussian sequence, 64 viewers, random
    viewpoints on a sphere of radius 4-6, resolutions 640x480 / 1280x720 /
    1920x1080."""
    import copy

    import torch

    from paper_2512_20943_amd import serve
    t0 = time.perf_counter()
    seq = serve.ResidentSequence(scene, args.serve_frames, seed=0)
    log(f"resident sequence: {args.serve_frames} frames, {seq.device_bytes() / 2**30:.2f} GiB "
        f"({time.perf_counter() - t0:.1f} s to generate)")
    budget = 32 << 30
    server = serve.Server(seq, budget_bytes=budget, max_batch=32)
    plain = serve.PlainRenderer(seq)
    # warm both paths (allocations, first launches)
    wt = serve.make_trace(64, 1e6, None, 64, seq.n_frames, 99)
    server.run(copy.deepcopy(wt))
    serve.run_plain(plain, copy.deepcopy(wt[:8]))
    out = {"frames": seq.n_frames, "viewers": 64, "budget_gib": budget / 2**30,
           "resident_gib": round(seq.device_bytes() / 2**30, 3), "max_batch": 32,
           "seconds": args.serve_seconds, "warmup_s": args.serve_warmup, "rates": {}}
    for rate in [float(x) for x in args.serve_rates.split(",")]:
        trace = serve.make_trace(None, rate, args.serve_warmup + args.serve_seconds, 64,
                                 seq.n_frames, int(rate))
        tb = copy.deepcopy(trace)
        server.batches.clear()
        server.run(tb)
        sb = serve.summarize(tb, args.serve_warmup)
        sb["mean_batch"] = round(float(np.mean(server.batches)), 2)
        tp = copy.deepcopy(trace)
        serve.run_plain(plain, tp)
        sp = serve.summarize(tp, args.serve_warmup)
        out["rates"][str(int(rate))] = {"requests": len(trace), "batched": sb, "plain": sp}
        log(f"serving @ {rate:.0f} req/s: batched {sb}  plain {sp}")
        torch.cuda.synchronize()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported (sharding "
              f"the views over several GPUs is not implemented)", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    import torch

    from paper_2512_20943_amd import scenes
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    log("generating the 300k-Gaussian frame workload")
    scene, cams, target_scene = scenes.workload_frame_300k(0, n=args.gaussians, n_views=args.views)
    ts = TrainStep(scene, cams, target_scene, tile_spans=not args.no_tile_spans)
    log(f"instances per step: {ts.r.forward(ts.g, ts.cams)['lists'].count}")
    wall, dev_s, stages = time_steps(ts, args.steps, args.warmup)
    ms_per_step = wall / args.steps * 1e3
    value = args.steps / wall
    log(f"train step: {ms_per_step:.2f} ms ({value:.2f} it/s)")
    dom, rf = roofline(stages, ts, args.steps)
    stage_ms = {k: round(v[0] / args.steps, 4) for k, v in stages.items() if v[1] > 0}
    result = {
        "metric": "fwd+bwd train iters/s", "value": round(value, 4), "unit": "iters/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"frame training step: {args.gaussians} Gaussians SH3, "
                               f"{args.views} views 1352x1014, L1 + Adam",
                   "gaussians": args.gaussians, "views": args.views, "width": 1352,
                   "height": 1014, "instances_per_step": ts.last["lists"].count,
                   "instances_full_rectangles": getattr(ts, "_def_instances", None),
                   "tile_spans": not args.no_tile_spans},
        "stage_ms_per_step": stage_ms,
        "roofline": rf,
    }
    if not args.no_autograd_step:
        ag = AutogradTrainStep(ts)
        k4 = max(args.steps // 2, 3)
        wall4, _, st4 = time_steps(ag, k4, 2)
        result["autograd_step"] = {
            "iters_per_s": round(k4 / wall4, 4), "ms_per_step": round(wall4 / k4 * 1e3, 3),
            "path": "GSRender and GSL1Loss torch.autograd.Functions, loss.backward(), Adam",
            "stage_ms_per_step": {k: round(v[0] / k4, 4) for k, v in st4.items() if v[1] > 0}}
        log(f"autograd step: {wall4 / k4 * 1e3:.2f} ms")
        del ag
    del ts
    torch.cuda.empty_cache()
    if not args.no_frame_step:
        n = args.gaussians
        gw = gh = scenes.grid_side(n)
        d = scenes.make_delta(n, gw, gh, 1)
        mask = scenes.prune_mask(d, n, 0.3)
        fs = TrainStep(scene, cams, target_scene, frame_update=(d, mask, gw, gh),
                       tile_spans=not args.no_tile_spans)
        wall2, _, st2 = time_steps(fs, max(args.steps // 2, 3), 2)
        k2 = max(args.steps // 2, 3)
        result["frame_update_step"] = {
            "iters_per_s": round(k2 / wall2, 4), "ms_per_step": round(wall2 / k2 * 1e3, 3),
            "grid": [gh, gw], "prune_level": 0.3, "loss": "L1 + 1e-3 L_temp (Eq. (7))",
            "stage_ms_per_step": {k: round(v[0] / k2, 4) for k, v in st2.items() if v[1] > 0}}
        log(f"frame-update step: {wall2 / k2 * 1e3:.2f} ms")
        del fs
    if not args.no_dssim_step:
        ds = TrainStep(scene, cams, target_scene, loss="l1_dssim",
                       tile_spans=not args.no_tile_spans)
        k3 = max(args.steps // 2, 3)
        wall3, _, st3 = time_steps(ds, k3, 2)
        ms3, n3 = st3.get("dssim", (0.0, 0))
        launch_s = ms3 / max(n3, 1) / 1e3
        bytes_per_launch = algorithmic_work("dssim", ds, k3)[0] * k3 / max(n3, 1)
        result["dssim_step"] = {
            "iters_per_s": round(k3 / wall3, 4), "ms_per_step": round(wall3 / k3 * 1e3, 3),
            "loss": "(1 - 0.2) L1 + 0.2 (1 - SSIM), 11x11 Gaussian window",
            "dssim_ms": round(launch_s * 1e3, 4),
            "dssim_GBps": round(bytes_per_launch / launch_s / 1e9, 1) if n3 else None,
            "stage_ms_per_step": {k: round(v[0] / k3, 4) for k, v in st3.items() if v[1] > 0}}
        log(f"Eq. (1) L1 + D-SSIM step: {wall3 / k3 * 1e3:.2f} ms")
        del ds
    if not args.no_sweep:
        sw = SweepStep(scene, target_scene, 4)
        k5 = 3
        wall5, _, st5 = time_steps(sw, k5, 1)
        last = sw.last
        result["pruning_sweep"] = {
            "sweeps_per_s": round(k5 / wall5, 4), "ms_per_sweep": round(wall5 / k5 * 1e3, 3),
            "levels": len(last["levels"]), "views": 4, "width": 1352, "height": 1014,
            "selected_level": last["levels"][last["selected"]],
            "stage_ms_per_sweep": {k: round(v[0] / k5, 4) for k, v in st5.items() if v[1] > 0}}
        log(f"pruning sweep: {wall5 / k5 * 1e3:.2f} ms")
        del sw
        cs = CodecStep(scene)
        k6 = 50
        wall6, dev6, st6 = time_steps(cs, k6, 3)
        nbytes = CodecStep.BYTES_PER_TEXEL * cs.n
        result["sent_update_codec"] = {
            "frames_per_s": round(k6 / wall6, 2), "device_ms_per_frame": round(dev6 / k6 * 1e3, 4),
            "grid": [cs.gh, cs.gw], "bits": 8, "prune_level": 0.3,
            "algorithmic_bytes_per_frame": nbytes,
            "device_GBps": round(nbytes / (dev6 / k6) / 1e9, 1),
            "stage_ms_per_frame": {k: round(v[0] / k6, 4) for k, v in st6.items() if v[1] > 0}}
        log(f"sent-update codec: {dev6 / k6 * 1e3:.3f} ms device time per frame")
        del cs
        kc = CompactStep(scene)
        k7 = 50
        wall7, dev7, st7 = time_steps(kc, k7, 3)
        # algorithmic bytes: the opacity plane read once per pass (count,
        # write), 59 planes gathered (read + write) per kept Gaussian, 4-B
        # indices written and read
        nb7 = 2 * 4 * kc.n + kc.kept * (CompactStep.PLANES * 8 + 8)
        result["keyframe_compaction"] = {
            "per_s": round(k7 / wall7, 2), "ms_wall": round(wall7 / k7 * 1e3, 4),
            "device_ms": round(dev7 / k7 * 1e3, 4), "gaussians": kc.n, "kept": int(kc.kept),
            "min_opacity": CompactStep.EPS, "planes": CompactStep.PLANES,
            "algorithmic_bytes": nb7, "device_GBps": round(nb7 / (dev7 / k7) / 1e9, 1),
            "stage_ms": {k: round(v[0] / k7, 4) for k, v in st7.items() if v[1] > 0}}
        log(f"keyframe compaction: {dev7 / k7 * 1e3:.3f} ms device time")
        del kc
    if not args.no_serve:
        result["serving"] = serving(args, scene)
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on one view")
        result["cpu_baseline"] = cpu_baseline(scene, cams, target_scene)
    print(json.dumps(result))


if __name__ == "__main__":
    main()
