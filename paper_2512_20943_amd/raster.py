"""Pipeline around the C ABI: workspaces, capacity growth and autograd.

``Rasterizer`` owns the per-call buffers of one (scene size, camera set)
shape and chains gs_project -> gs_bin_sort -> gs_render_fwd, and
gs_render_bwd for the backward.  ``GSRender`` and ``GSFrameRender`` are the
``torch.autograd.Function`` front ends: the first differentiates the images
w.r.t. means, log-scales, quaternions, opacity logits and SH coefficients;
the second w.r.t. the per-frame delta images applied to a frozen anchor
(frame = anchor + pruned delta, AirGS Eq. (12)).

Forward state.  The backward needs the projected records and tile lists of
its own forward (gs_bin_sort also stores each pair's emission base in the
record).  A plain ``forward`` reuses the rasterizer's buffers, so a second
forward overwrites the first one's state: every such forward carries a
generation number and ``backward`` refuses a state whose buffers have been
reused since.  ``forward(..., own_buffers=True)`` -- what the autograd
functions use -- gives the call buffers of its own, so any number of renders
can be differentiated together.
"""
from __future__ import annotations

import torch

from . import gs


class Rasterizer:
    def __init__(self, ctx: gs.Context | None = None, capacity: int = 1 << 20,
                 with_keys: bool = False, growth: float = 1.25,
                 emission_bases: bool = False, tight_rect: bool = False,
                 tile_spans: bool = False):
        self.ctx = ctx or gs.default_context()
        # opacity-aware tile rectangles: same images and gradients, shorter
        # lists (GS_PROJECT_TIGHT_RECT); with tile_spans also the per-row
        # spans of small rectangles (GS_PROJECT_TILE_SPANS)
        self.tight_rect = tight_rect
        self.tile_spans = tile_spans
        self.capacity = int(capacity)
        self.with_keys = with_keys
        # also store each pair's first instance index in lists.gv_base (the
        # backward reads it from the projected record; this copy is for
        # inspection)
        self.emission_bases = emission_bases
        self.growth = growth
        self._lists = None
        self._ws_sort = None
        self._proj = None
        self._ws_bwd = None
        self._ws_l1 = None
        # bumped whenever the shared projected records or tile lists are
        # handed out again; a forward state remembers the value it saw
        self._gen = 0

    # -- buffers ------------------------------------------------------------
    def _options(self):
        return ((gs.GS_PROJECT_TIGHT_RECT if self.tight_rect else 0)
                | (gs.GS_PROJECT_TILE_SPANS if self.tile_spans else 0))

    def _projected(self, V, n, ld, device, own=False):
        if own:
            p = gs.Projected.empty(V, n, ld, device)
            p.options = self._options()
            return p
        p = self._proj
        if p is None or p.V != V or p.n != n or p.ld != ld:
            self._proj = gs.Projected.empty(V, n, ld, device)
        self._proj.options = self._options()
        self._gen += 1
        return self._proj

    def _sort_workspace(self, V, ld, capacity, nseg, device):
        need = gs.bin_sort_workspace_size(V, ld, capacity, nseg)
        if self._ws_sort is None or self._ws_sort.numel() < need:
            self._ws_sort = torch.empty(need, dtype=torch.uint8, device=device)
        return self._ws_sort

    def _sort_buffers(self, V, ld, nseg, device, own=False):
        gv = V * ld if self.emission_bases else 0
        if own:
            lists = gs.TileLists(self.capacity, nseg, self.with_keys, device, gv=gv)
        else:
            L = self._lists
            if (L is None or L.capacity < self.capacity or L.n_segments != nseg
                    or L.gv < gv):
                self._lists = gs.TileLists(self.capacity, nseg, self.with_keys, device, gv=gv)
            lists = self._lists
            self._gen += 1
        return lists, self._sort_workspace(V, ld, lists.capacity, nseg, device)

    def bwd_workspace(self, V, ld, device, instances=None):
        # scratch of one backward call only (screen-space gradients and the
        # per-instance rows), so one buffer serves every forward state
        if instances is None:
            instances = self._lists.count if self._lists is not None else 0
        need = gs.render_bwd_workspace_size(V, ld, instances)
        if self._ws_bwd is None or self._ws_bwd.numel() < need:
            self._ws_bwd = torch.empty(need, dtype=torch.uint8, device=device)
        return self._ws_bwd

    # -- passes -------------------------------------------------------------
    def project(self, g: gs.Gaussians, cams: gs.Cameras, stream=None,
                own_buffers=False) -> gs.Projected:
        proj = self._projected(cams.V, g.n, g.ld, g.mean.device, own_buffers)
        gs.gs_project(self.ctx, g, cams, proj, stream)
        return proj

    def bin_sort(self, proj: gs.Projected, cams: gs.Cameras, stream=None,
                 own_buffers=False) -> gs.TileLists:
        device = proj.splat.device
        nseg = cams.n_segments()
        while True:
            lists, ws = self._sort_buffers(cams.V, proj.ld, nseg, device, own_buffers)
            try:
                gs.gs_bin_sort(self.ctx, proj, cams, lists, ws, stream)
                return lists
            except gs.GsError as e:
                if e.code != gs.GS_ERR_CAPACITY or lists.count > gs.GS_MAX_INSTANCES:
                    raise
                self.capacity = min(max(int(lists.count * self.growth) + 1024,
                                        self.capacity * 2), gs.GS_MAX_INSTANCES)

    def _state(self, own, **kw):
        kw["gen"] = None if own else self._gen
        return kw

    def forward(self, g: gs.Gaussians, cams: gs.Cameras, bg=(0.0, 0.0, 0.0), stream=None,
                usage=None, own_buffers=False):
        """Render; the returned dict is the state ``backward`` takes.  With
        ``own_buffers`` the state's projected records and lists belong to
        this call alone (see the module docstring)."""
        W, H = cams.wh[0]
        device = g.mean.device
        proj = self.project(g, cams, stream, own_buffers)
        lists = self.bin_sort(proj, cams, stream, own_buffers)
        image = torch.empty(cams.V, 3, H, W, device=device)
        final_T = torch.empty(cams.V, H, W, device=device)
        n_contrib = torch.empty(cams.V, H, W, dtype=torch.int32, device=device)
        gs.gs_render_fwd(self.ctx, proj, lists, cams, bg, image, final_T, n_contrib, stream,
                         usage=usage)
        return self._state(own_buffers, image=image, final_T=final_T, n_contrib=n_contrib,
                           proj=proj, lists=lists)

    def forward_l1(self, g: gs.Gaussians, cams: gs.Cameras, target: torch.Tensor,
                   dL_dimage: torch.Tensor, loss: torch.Tensor, bg=(0.0, 0.0, 0.0), stream=None,
                   keep_image=False, own_buffers=False):
        """Forward with the L1 term of Eq. (1) fused into the compositing:
        dL_dimage written, mean |image - target| added to ``loss``; the image
        itself is written only with ``keep_image``.  ``own_buffers`` as in
        ``forward``."""
        W, H = cams.wh[0]
        device = g.mean.device
        proj = self.project(g, cams, stream, own_buffers)
        lists = self.bin_sort(proj, cams, stream, own_buffers)
        image = torch.empty(cams.V, 3, H, W, device=device) if keep_image else None
        final_T = torch.empty(cams.V, H, W, device=device)
        n_contrib = torch.empty(cams.V, H, W, dtype=torch.int32, device=device)
        need = gs.render_fwd_l1_workspace_size(cams.V, W, H)
        if self._ws_l1 is None or self._ws_l1.numel() < need:
            self._ws_l1 = torch.empty(need, dtype=torch.uint8, device=device)
        gs.gs_render_fwd_l1(self.ctx, proj, lists, cams, bg, target.contiguous(), image, final_T,
                            n_contrib, dL_dimage, loss, self._ws_l1, stream)
        return self._state(own_buffers, image=image, final_T=final_T, n_contrib=n_contrib,
                           proj=proj, lists=lists)

    def check_state(self, state: dict):
        """Raise when a forward state's shared buffers were reused since."""
        gen = state.get("gen")
        if gen is not None and gen != self._gen:
            raise RuntimeError(
                "forward state is stale: a later forward, project or bin_sort on this "
                "Rasterizer reused its projected records and tile lists; run the backward "
                "first, or render with own_buffers=True")

    def backward(self, g: gs.Gaussians, cams: gs.Cameras, state: dict, dL_dimage: torch.Tensor,
                 grad: gs.Gaussians, bg=(0.0, 0.0, 0.0), upd=None, dL_ddelta=None, stream=None,
                 temporal=None):
        """``temporal`` = (weight, delta, loss) adds the temporal term of
        Eq. (6)/(7) to the delta gradient (with ``upd``); see gs_render_bwd."""
        self.check_state(state)
        ws = self.bwd_workspace(cams.V, g.ld, g.mean.device, state["lists"].count)
        gs.gs_render_bwd(self.ctx, g, state["proj"], state["lists"], cams, bg, state["final_T"],
                         state["n_contrib"], dL_dimage.contiguous(), grad, ws, upd, dL_ddelta,
                         stream, temporal=temporal)
        return ws


class GSRender(torch.autograd.Function):
    """images = render(mean, log_scale, quat, opacity, sh) for the cameras."""

    @staticmethod
    def forward(ctx, mean, log_scale, quat, opacity, sh, meta):
        raster, cams, n, deg, bg = meta
        planes = [t.contiguous() for t in (mean, log_scale, quat, opacity, sh)]
        g = gs.Gaussians(n, deg, mean.shape[-1], *planes)
        # buffers of its own: other renders may run before this backward
        out = raster.forward(g, cams, bg, own_buffers=True)
        ctx.meta = meta
        # saved through autograd, so in-place changes to the parameters
        # between this forward and its backward raise
        ctx.save_for_backward(*planes)
        ctx.state = out
        return out["image"]

    @staticmethod
    def backward(ctx, dimage):
        raster, cams, n, deg, bg = ctx.meta
        g = gs.Gaussians(n, deg, ctx.saved_tensors[0].shape[-1], *ctx.saved_tensors)
        grad = gs.Gaussians.zeros_like(g)
        raster.backward(g, cams, ctx.state, dimage, grad, bg)
        return grad.mean, grad.log_scale, grad.quat, grad.opacity, grad.sh, None


class GSL1Loss(torch.autograd.Function):
    """loss = mean |image - target| (the L1 term of Eq. (1)) and its gradient
    from gs_l1_loss_grad; the backward scales that gradient by the incoming
    one."""

    @staticmethod
    def forward(ctx, image, target, gs_ctx):
        grad = torch.empty_like(image)
        loss = torch.zeros(1, dtype=torch.float64, device=image.device)
        gs.gs_l1_loss_grad(gs_ctx, image.contiguous(), target.contiguous(), grad, loss)
        ctx.save_for_backward(grad)
        return loss[0]

    @staticmethod
    def backward(ctx, g):
        (grad,) = ctx.saved_tensors
        return grad * g.to(grad.dtype), None, None


class GSRenderL1(torch.autograd.Function):
    """loss = mean |render(mean, log_scale, quat, opacity, sh) - target|, the
    L1 term of Eq. (1), in one fused forward (gs_render_fwd_l1: the image is
    never written, dL/dimage comes out of the compositing epilogue); the
    backward scales that saved gradient by the incoming one and runs the
    render backward.  No gradient flows to ``target``."""

    @staticmethod
    def forward(ctx, mean, log_scale, quat, opacity, sh, target, meta):
        raster, cams, n, deg, bg = meta
        planes = [t.contiguous() for t in (mean, log_scale, quat, opacity, sh)]
        g = gs.Gaussians(n, deg, mean.shape[-1], *planes)
        W, H = cams.wh[0]
        dimage = torch.empty(cams.V, 3, H, W, device=mean.device)
        loss = torch.zeros(1, dtype=torch.float64, device=mean.device)
        out = raster.forward_l1(g, cams, target, dimage, loss, bg, own_buffers=True)
        ctx.meta = meta
        ctx.save_for_backward(*planes)
        ctx.state = out
        ctx.dimage = dimage
        return loss[0]

    @staticmethod
    def backward(ctx, gl):
        raster, cams, n, deg, bg = ctx.meta
        g = gs.Gaussians(n, deg, ctx.saved_tensors[0].shape[-1], *ctx.saved_tensors)
        grad = gs.Gaussians.zeros_like(g)
        dimage = ctx.dimage.mul_(gl.to(ctx.dimage.dtype))
        raster.backward(g, cams, ctx.state, dimage, grad, bg)
        return grad.mean, grad.log_scale, grad.quat, grad.opacity, grad.sh, None, None


class GSFrameRender(torch.autograd.Function):
    """images = render(apply(anchor, delta, mask)); gradient to the (8, gh, gw)
    delta images, anchor frozen.  meta = (rasterizer, cameras, anchor, mask,
    gw, gh, bg).  Each call applies the update into frame planes of its own
    (log-scale and SH shared with the anchor) and renders with buffers of its
    own, so several calls can be differentiated together."""

    @staticmethod
    def forward(ctx, delta, meta):
        raster, cams, anchor, mask, gw, gh, bg = meta
        frame = frame_of(anchor)
        gs.gs_apply_frame_update(raster.ctx, anchor, delta.contiguous(), mask, gw, gh, frame)
        out = raster.forward(frame, cams, bg, own_buffers=True)
        ctx.meta = meta
        ctx.frame = frame
        ctx.state = out
        return out["image"]

    @staticmethod
    def backward(ctx, dimage):
        raster, cams, anchor, mask, gw, gh, bg = ctx.meta
        frame = ctx.frame
        grad = gs.Gaussians.zeros_like(frame)
        dd = torch.empty(8, gh, gw, device=dimage.device)
        raster.backward(frame, cams, ctx.state, dimage, grad, bg,
                        upd=(anchor.quat, mask, gw, gh), dL_ddelta=dd)
        return dd, None


def frame_of(anchor: gs.Gaussians) -> gs.Gaussians:
    """Frame buffers for an anchor: new mean/quat/opacity planes, log-scale
    and SH shared with the anchor."""
    return gs.Gaussians(anchor.n, anchor.deg, anchor.ld, torch.empty_like(anchor.mean),
                        anchor.log_scale, torch.empty_like(anchor.quat),
                        torch.empty_like(anchor.opacity), anchor.sh)
