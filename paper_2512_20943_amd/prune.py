"""Usage-frequency pruning and pruning-level selection (AirGS Sec. III-C).

* ``usage_keep_mask`` drops the updates of the least-used Gaussians: usage
  is the number of (view, pixel) pairs that composite a Gaussian, counted by
  the forward render (``gs_opts.usage``).
* ``PruningSweep`` builds the dense pruning-level space S_t^d of one frame:
  for each level it applies the pruned update, renders all evaluation views
  of all levels in one persistent batched launch, and measures quality as
  the PSNR of each level's renders against the frame's reference views
  (squared errors reduced on the device) and size as the bytes of the kept
  update texels.
* ``select_level`` is Alg. 1: the levels before the first quality cliff are
  the candidates, and the least pruned candidate whose size fits B / R wins.

Readings where the paper is silent: quality is the mean over views of the
PSNR (data range 1) against the reference views the frame is trained on (the
level-0 render is not a reference: its own error would be zero); a previous
drop of exactly 0 makes a level a cliff when its own drop is negative; when
no candidate fits B / R the cliff level is returned (the algorithm's own
fallthrough), and without a cliff the most pruned level.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import gs
from .raster import Rasterizer, frame_of

BYTES_PER_UPDATE = 8 * 4  # eight FP32 channels per kept texel


def usage_keep_mask(usage: np.ndarray, n: int, gw: int, gh: int, level: float) -> np.ndarray:
    """Keep-mask (gh, gw) that drops floor(level * n) updates of the least
    used Gaussians (equal usage: lower id dropped first); padding texels 0."""
    return usage_keep_masks(usage, n, gw, gh, [level])[0]


def usage_keep_masks(usage: np.ndarray, n: int, gw: int, gh: int, levels) -> list:
    """usage_keep_mask for every level, sharing one stable ordering."""
    u = np.asarray(usage[:n], dtype=np.int64)
    order = np.argsort(u, kind="stable")
    out = []
    for level in levels:
        m = np.zeros(gh * gw, np.uint8)
        m[:n] = 1
        m[order[: int(math.floor(level * n + 1e-9))]] = 0
        out.append(m.reshape(gh, gw))
    return out


def _is_cliff(drop: float, before: float, beta: float) -> bool:
    if before == 0.0:
        return drop < 0.0
    return drop / before > beta


def select_level(space, beta: float, bandwidth: float, rate: float) -> int:
    """Alg. 1 over ``space`` = [(quality, size), ...] in increasing pruning.

    Each level's quality drop is compared with the drop of the level before
    it (the first drop with itself); the first level whose drop exceeds beta
    times that is the cliff and bounds the candidates.  Sizes do not grow
    with the level, so the candidates that fit the budget B / R form a
    suffix of the candidate range, and a bisection finds its first (least
    pruned) member."""
    quality = np.array([q for q, _ in space], np.float64)
    size = np.array([sz for _, sz in space], np.float64)
    drops = np.diff(quality)
    before = np.concatenate([drops[:1], drops[:-1]])
    cliff = next((k + 1 for k in range(drops.size) if _is_cliff(drops[k], before[k], beta)),
                 None)
    end = len(space) if cliff is None else cliff
    budget = bandwidth / rate
    lo, hi = 0, end
    while lo < hi:
        mid = (lo + hi) // 2
        if size[mid] <= budget:
            hi = mid
        else:
            lo = mid + 1
    if lo < end:
        return lo
    return len(space) - 1 if cliff is None else cliff


class PruningSweep:
    """Quality/size of every pruning level of one frame, on the device."""

    def __init__(self, anchor: gs.Gaussians, delta: torch.Tensor, gw: int, gh: int,
                 cams: gs.Cameras, ctx: gs.Context | None = None, levels=None):
        self.ctx = ctx or gs.default_context()
        self.anchor = anchor
        self.delta = delta
        self.gw, self.gh = gw, gh
        self.cams = cams
        self.levels = np.linspace(0.0, 1.0, 11) if levels is None else np.asarray(levels)
        # opacity-aware tile rectangles: same images and usage, shorter lists
        self.raster = Rasterizer(ctx=self.ctx, capacity=1 << 22, tight_rect=True,
                                 tile_spans=True)
        self._proj = None  # projected records of every (level, view), reused

    def usage(self, bg=(0.0, 0.0, 0.0)):
        """Per-Gaussian usage: composited (view, pixel) pairs of the unpruned
        frame."""
        dev = self.anchor.mean.device
        full = frame_of(self.anchor)
        ones = torch.ones(self.gh, self.gw, dtype=torch.uint8, device=dev)
        gs.gs_apply_frame_update(self.ctx, self.anchor, self.delta, ones, self.gw, self.gh, full)
        usage = torch.zeros(self.anchor.ld, dtype=torch.int32, device=dev)
        self.raster.forward(full, self.cams, bg, usage=usage)
        return usage

    def run(self, reference: torch.Tensor, beta: float = 2.0, bandwidth: float = 1e6,
            rate: float = 30.0, bg=(0.0, 0.0, 0.0)):
        """``reference``: the frame's (V, 3, H, W) views that quality is
        measured against."""
        dev = self.anchor.mean.device
        V = self.cams.V
        if tuple(reference.shape[:2]) != (V, 3):
            raise ValueError("reference must hold (V, 3, H, W) views")
        usage = self.usage(bg)
        u = usage.cpu().numpy().view(np.uint32).astype(np.int64)
        n, L = self.anchor.n, len(self.levels)
        masks = usage_keep_masks(u, n, self.gw, self.gh, self.levels)
        frames = []
        for m in masks:
            f = frame_of(self.anchor)
            gs.gs_apply_frame_update(self.ctx, self.anchor, self.delta,
                                     torch.from_numpy(m).to(dev), self.gw, self.gh, f)
            frames.append(f)
        # one batched render of every (level, view) pair
        items = []
        for _ in range(L):
            for v in range(V):
                h = self.cams.host[v]
                items.append((np.array(h.R[:]).reshape(3, 3), np.array(h.t[:]),
                              np.array([h.fx, h.fy, h.cx, h.cy]), (h.width, h.height)))
        cams = gs.Cameras.from_list(items, dev)
        proj = self._proj
        if proj is None or proj.V != L * V:
            proj = self._proj = gs.Projected.empty(L * V, n, self.anchor.ld, dev)
        proj.options = gs.GS_PROJECT_TIGHT_RECT | gs.GS_PROJECT_TILE_SPANS
        for k, f in enumerate(frames):
            gs.gs_project(self.ctx, f, cams.slice(k * V, V), proj.slice(k * V, V))
        lists = self.raster.bin_sort(proj, cams)
        pix = [w * hh for (w, hh) in cams.wh]
        images = torch.empty(3 * sum(pix), device=dev)
        ws = torch.empty(gs.render_batched_workspace_size(L * V), dtype=torch.uint8, device=dev)
        gs.gs_render_fwd_batched(self.ctx, proj, lists, cams, bg, images, ws)
        sq = torch.zeros(L * V, dtype=torch.float64, device=dev)
        off = 0
        refs = reference.reshape(V, -1)
        for k in range(L * V):
            cnt = 3 * pix[k]
            gs.gs_sq_error(self.ctx, images[off:off + cnt], refs[k % V], sq[k:k + 1])
            off += cnt
        mse = (sq.cpu().numpy() / np.array([3 * p for p in pix])).reshape(L, V)
        if not (mse > 0).all():
            raise ValueError("a level renders its reference exactly: quality is undefined")
        psnr = (-10.0 * np.log10(mse)).mean(axis=1)
        sizes = np.array([int(m.sum()) * BYTES_PER_UPDATE for m in masks])
        space = list(zip(psnr.tolist(), sizes.tolist()))
        p = select_level(space, beta, bandwidth, rate)
        return dict(levels=self.levels.tolist(), psnr=psnr.tolist(), size=sizes.tolist(),
                    selected=int(p), usage=u[:n], masks=masks, images=images, pix=pix)
