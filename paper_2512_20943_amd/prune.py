"""Usage-frequency pruning and pruning-level selection (AirGS Sec. III-C).

* ``usage_keep_mask`` drops the updates of the least-used Gaussians: usage
  is the number of (view, pixel) pairs that composite a Gaussian, counted by
  the forward render (``gs_opts.usage``).
* ``PruningSweep`` builds the dense pruning-level space S_t^d of one frame:
  for each level it applies the pruned update, renders all evaluation views
  of all levels in one persistent batched launch, and measures quality as
  PSNR against the unpruned frame's render (squared errors reduced on the
  device) and size as the bytes of the kept update texels.
* ``select_level`` is Alg. 1: scan S_t^d for the first quality cliff (a drop
  more than beta times the previous drop), keep the levels before it, then
  binary-search the lowest kept level whose size fits B / R.

Readings where the paper is silent: quality is PSNR (data range 1) against
the unpruned render, capped at 100 dB where the two are identical; a drop
compared with a previous drop of exactly 0 counts as a cliff when it is
nonzero; when no candidate fits B / R the algorithm's own fallthrough is
kept (the cliff level if one was found), and without a cliff the most pruned
candidate is returned.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import gs
from .raster import Rasterizer, frame_of

BYTES_PER_UPDATE = 8 * 4  # eight FP32 channels per kept texel
PSNR_CAP = 100.0


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


def select_level(space, beta: float, bandwidth: float, rate: float) -> int:
    """Alg. 1 over ``space`` = [(quality, size), ...] in increasing pruning."""
    p = None
    previous = space[1][0] - space[0][0]
    S = [0]
    for i in range(1, len(space)):
        drop = space[i][0] - space[i - 1][0]
        if previous == 0.0:
            cliff = drop != 0.0
        else:
            cliff = drop / previous > beta
        if cliff:
            p = i
            break
        S.append(i)
        previous = drop
    C = bandwidth / rate
    low, high = 0, len(S) - 1
    while low <= high:
        mid = (low + high) // 2
        tmp = S[mid]
        if space[tmp][1] <= C:
            p = tmp
            high = mid - 1
        else:
            low = mid + 1
    return S[-1] if p is None else p


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
        """Reference render of the unpruned frame and per-Gaussian usage."""
        dev = self.anchor.mean.device
        full = frame_of(self.anchor)
        ones = torch.ones(self.gh, self.gw, dtype=torch.uint8, device=dev)
        gs.gs_apply_frame_update(self.ctx, self.anchor, self.delta, ones, self.gw, self.gh, full)
        usage = torch.zeros(self.anchor.ld, dtype=torch.int32, device=dev)
        out = self.raster.forward(full, self.cams, bg, usage=usage)
        return out["image"].clone(), usage

    def run(self, beta: float = 2.0, bandwidth: float = 1e6, rate: float = 30.0,
            bg=(0.0, 0.0, 0.0)):
        dev = self.anchor.mean.device
        ref, usage = self.usage(bg)
        u = usage.cpu().numpy().view(np.uint32).astype(np.int64)
        n, L, V = self.anchor.n, len(self.levels), self.cams.V
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
        refs = ref.reshape(V, -1)
        for k in range(L * V):
            cnt = 3 * pix[k]
            gs.gs_sq_error(self.ctx, images[off:off + cnt], refs[k % V], sq[k:k + 1])
            off += cnt
        mse = (sq.cpu().numpy() / np.array([3 * p for p in pix])).reshape(L, V)
        psnr = np.where(mse > 0, -10.0 * np.log10(np.maximum(mse, 1e-300)), PSNR_CAP)
        psnr = np.minimum(psnr, PSNR_CAP).mean(axis=1)
        sizes = np.array([int(m.sum()) * BYTES_PER_UPDATE for m in masks])
        space = list(zip(psnr.tolist(), sizes.tolist()))
        p = select_level(space, beta, bandwidth, rate)
        return dict(levels=self.levels.tolist(), psnr=psnr.tolist(), size=sizes.tolist(),
                    selected=int(p), usage=u[:n], masks=masks, images=images, pix=pix)
