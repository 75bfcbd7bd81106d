"""HIP path vs the FP64 oracle, through the C ABI, on seeded inputs.

Bars: apply results bit-exact; projection within 1e-3 px (screen mean) and
1e-4 relative (conic, colour, opacity); tile lists, keys and ranges
bit-exact; images and final transmittance within 1e-4 absolute with equal
n_contrib, except at pixels where the oracle finds a skip/stop decision
within a small relative margin of its threshold (counted, must be rare);
gradients within 1e-3 relative.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2512_20943_amd import gs, scenes
from paper_2512_20943_amd.raster import GSFrameRender, GSRender, Rasterizer, frame_of
from tests.gpu_helpers import (IMG_ATOL, MEAN2D_ATOL, NEAR_ATOL, NEAR_FRAC_CAP, assert_close_rel,
                               assert_grad_close, compare_images, gpu_forward, lists_to_numpy,
                               projected_to_oracle, require_gpu, span_rows)

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def small_frame_workload(seed=0):
    """20,000 Gaussians of the 300k-frame distribution (SH 3) seen by 4 arc
    cameras at 200x150 (ragged in both directions: 12.5 x 9.4 tiles)."""
    scene = scenes.make_scene(20_000, seed, -3.0, 3.0, -4.0, 0.5, 3)
    cams = scenes.arc_cameras(4, 5.0, 200, 150)
    return scene, cams


def compare_projection(P_gpu, P_or, vis_only=True):
    fl_g, fl_o = P_gpu["flags"], P_or["flags"]
    np.testing.assert_array_equal(fl_g & 0x38, fl_o & 0x38)  # visible + guard-band bits
    vis = (fl_o & 32) > 0
    np.testing.assert_array_equal(P_gpu["rect"][vis], P_or["rect"][vis])
    np.testing.assert_array_equal(P_gpu["tiles"], P_or["tiles"])
    np.testing.assert_array_equal(P_gpu["depth_bits"][vis], P_or["depth_bits"][vis])
    d = np.abs(P_gpu["mean2d"][vis] - P_or["mean2d"][vis]).max(initial=0.0)
    assert d <= MEAN2D_ATOL, f"mean2d error {d}"
    assert_close_rel(P_gpu["conic"][vis], P_or["conic"][vis], what="conic")
    assert_close_rel(P_gpu["rgb"][vis], P_or["rgb"][vis], what="rgb")
    assert_close_rel(P_gpu["alpha_hat"][vis], P_or["alpha_hat"][vis], what="opacity")
    # colour clamp bits may differ only where the oracle colour is ~0
    cg, co = fl_g & 7, fl_o & 7
    diff = (cg != co) & vis
    if diff.any():
        assert P_or["rgb"][diff].max() < 1e-5
    return int(vis.sum())


# ---------------------------------------------------------------------------

def test_context_and_version():
    require_gpu()
    ctx = gs.default_context()
    assert ctx.lib.gs_version() >= 100


@pytest.mark.parametrize("n,level", [(5_000, 0.3), (300_000, 0.1)])
def test_apply_bit_exact(n, level):
    require_gpu()
    say(f"apply n={n} level={level}")
    gw = gh = scenes.grid_side(n)
    sc = scenes.make_scene(n, 3, -3, 3, -4, 0.5, 0)
    d = scenes.make_delta(n, gw, gh, 4)
    mask = scenes.prune_mask(d, n, level)
    ref = oracle.apply(sc, d, mask, gw, gh)
    g = gs.Gaussians.from_scene(sc)
    f = frame_of(g)
    gs.gs_apply_frame_update(gs.default_context(), g, torch.from_numpy(d).cuda(),
                             torch.from_numpy(mask).cuda(), gw, gh, f)
    torch.cuda.synchronize()
    for k, t in (("mean", f.mean), ("quat", f.quat), ("opacity", f.opacity)):
        np.testing.assert_array_equal(t.cpu().numpy()[..., :n], ref[k][..., :n])


@pytest.mark.parametrize("which", ["plain_10k", "frame_20k_4v"])
@pytest.mark.parametrize("tileset", ["rect", "tight", "spans"])
def test_projection_and_lists_bit_exact(which, tileset):
    """Projection records, tile sets (rectangles, or the opacity-aware
    rectangles and per-row spans the benchmark bins with), keys, lists and
    ranges against the oracle's; then images, final_T and n_contrib (list
    positions in these lists) against the oracle's render of the same lists."""
    require_gpu()
    say(f"projection+lists {which} {tileset}")
    if which == "plain_10k":
        scene, cams, _ = scenes.workload_plain_10k(0)
    else:
        scene, cams = small_frame_workload(1)
    g, gc, r, out = gpu_forward(scene, cams, tight_rect=tileset != "rect",
                                tile_spans=tileset == "spans")
    P_or = oracle.project(scene, cams, tileset)
    P_g = projected_to_oracle(out["proj"])
    nvis = compare_projection(P_g, P_or)
    assert nvis > 0
    sp_g, rows_g = span_rows(P_g)
    sp_o, rows_o = span_rows(P_or)
    np.testing.assert_array_equal(sp_g, sp_o)
    np.testing.assert_array_equal(rows_g, rows_o)
    assert sp_o.any() == (tileset == "spans")
    L_or = oracle.bin_sort(P_or, cams)
    L_g = lists_to_numpy(out["lists"])
    assert L_g["count"] == L_or["count"] > 0
    np.testing.assert_array_equal(L_g["keys"], L_or["keys"])
    np.testing.assert_array_equal(L_g["vals"], L_or["vals"])
    np.testing.assert_array_equal(L_g["ranges"], L_or["ranges"])
    img_or = oracle.render_fwd(P_or, L_or, cams)
    compare_images(out, img_or, which)


@pytest.mark.parametrize("which", ["plain_10k", "frame_20k_4v"])
@pytest.mark.parametrize("mode", ["tight", "spans"])
def test_tight_rectangles_keep_images_and_gradients(which, mode):
    """With GS_PROJECT_TIGHT_RECT the rectangles shrink to the tiles the
    alpha >= 1/255 ellipse can reach, and with GS_PROJECT_TILE_SPANS small
    rectangles keep, per tile row, only the columns that meet it: images and
    final_T are bit-identical to the full rectangles', the kept instances
    appear in the full lists in the same order, and the gradients agree up to
    FP32 summation order (only all-zero gradient rows are dropped)."""
    require_gpu()
    if which == "plain_10k":
        scene, cams, _ = scenes.workload_plain_10k(0)
    else:
        scene, cams = small_frame_workload(6)
    g = gs.Gaussians.from_scene(scene)
    gc = gs.Cameras(cams)
    outs, grads = [], []
    gen = torch.Generator(device="cuda").manual_seed(3)
    for tight, spans in ((False, False), (True, False), (True, mode == "spans")):
        r = Rasterizer(capacity=1 << 20, with_keys=True, tight_rect=tight, tile_spans=spans)
        out = r.forward(g, gc)
        if not outs:
            dimg = torch.randn(out["image"].shape, device="cuda", generator=gen)
        grad = gs.Gaussians.zeros_like(g)
        r.backward(g, gc, out, dimg, grad)
        torch.cuda.synchronize()
        outs.append(out)
        grads.append(grad)
    full, rect_only, tight = outs
    assert torch.equal(tight["image"], full["image"])
    assert torch.equal(tight["final_T"], full["final_T"])
    Lf, Lt = lists_to_numpy(full["lists"]), lists_to_numpy(tight["lists"])
    Lr = lists_to_numpy(rect_only["lists"])
    assert 0 < Lt["count"] <= Lr["count"] < Lf["count"]
    say(f"  {mode}: keep {Lt['count']} of {Lf['count']} instances")
    tt = tight["proj"].tiles_touched.cpu().numpy()[:, :g.n]
    assert int(tt.sum()) == Lt["count"]
    if mode == "spans":
        assert Lt["count"] < Lr["count"]
        w13 = tight["proj"].splat.view(torch.int32).cpu().numpy()[:, :g.n, 13]
        flagged = (w13 < 0) & (tt > 0)
        assert flagged.any()
    # kept instances, in order, among the full lists' (key, id) pairs
    kf = (Lf["keys"].astype(object) << 32) | Lf["vals"].astype(object)
    kt = (Lt["keys"].astype(object) << 32) | Lt["vals"].astype(object)
    pos = np.searchsorted(kf, kt)
    assert np.all(pos < len(kf)) and np.array_equal(kf[pos], kt)
    rf = full["proj"].rect.cpu().numpy()
    rt = tight["proj"].rect.cpu().numpy()
    vis = tt > 0
    inside = ((rt[:, :g.n, 0] >= rf[:, :g.n, 0]) & (rt[:, :g.n, 1] >= rf[:, :g.n, 1]) &
              (rt[:, :g.n, 2] <= rf[:, :g.n, 2]) & (rt[:, :g.n, 3] <= rf[:, :g.n, 3]))
    assert np.all(inside[vis])
    for name in ("mean", "log_scale", "quat", "opacity", "sh"):
        a = getattr(grads[2], name).cpu().numpy()
        b = getattr(grads[0], name).cpu().numpy()
        np.testing.assert_allclose(a, b, rtol=1e-4, atol=1e-6 * max(1.0, np.abs(b).max()),
                                   err_msg=name)


def _box_min_q(A, B, C, px, py, x0, x1, y0, y1):
    """Minimum over the box [x0, x1] x [y0, y1] of the conic's quadratic form
    q(d) = A dx^2 + 2 B dx dy + C dy^2 around (px, py): 0 inside, else the
    smallest value on its four edges (q is convex)."""
    def edge(xa, ya, xb, yb):
        ux, uy = xb - xa, yb - ya
        dx, dy = xa - px, ya - py
        a = A * ux * ux + 2 * B * ux * uy + C * uy * uy
        b = A * dx * ux + B * (dx * uy + dy * ux) + C * dy * uy
        t = np.clip(-b / np.maximum(a, 1e-300), 0.0, 1.0)
        ex, ey = dx + t * ux, dy + t * uy
        return A * ex * ex + 2 * B * ex * ey + C * ey * ey
    inside = (px >= x0) & (px <= x1) & (py >= y0) & (py <= y1)
    m = np.minimum.reduce([edge(x0, y0, x1, y0), edge(x0, y1, x1, y1),
                           edge(x0, y0, x0, y1), edge(x1, y0, x1, y1)])
    return np.where(inside, 0.0, m)


def test_spans_keep_only_tiles_the_ellipse_meets():
    """Every instance that per-row tile spans keep lies in a tile whose pixel
    columns, over its row's band (pixel centres +- 0.5 px in y), meet the
    ellipse where alpha reaches 1/255 (plus the quadrant test's margin), by
    the oracle's FP64 projection of the same scene: the spans drop only
    tiles outside it (that they drop all of those up to the band rounding is
    what the bit-identical images and shorter lists of the span tests show)."""
    require_gpu()
    scene, cams = small_frame_workload(7)
    g, gc, r, out = gpu_forward(scene, cams, capacity=1 << 20, tight_rect=True,
                                tile_spans=True)
    L = out["lists"]
    M = L.count
    vals = L.vals[:M].cpu().numpy().astype(np.int64)
    ranges = L.ranges[:L.n_segments].cpu().numpy().astype(np.int64)
    seg_of = np.repeat(np.arange(L.n_segments), ranges[:, 1] - ranges[:, 0])
    words = out["proj"].splat.cpu().numpy().view(np.uint32).reshape(gc.V, g.ld, 16)
    tpv = [((w + 15) // 16) * ((h + 15) // 16) for (w, h) in cams["wh"]]
    sb = np.concatenate([[0], np.cumsum(tpv)])
    v = np.searchsorted(sb, seg_of, side="right") - 1
    tile = seg_of - sb[v]
    TX = np.array([(w + 15) // 16 for (w, h) in cams["wh"]])[v]
    ty, tx = tile // TX, tile % TX
    sp = (words[v, vals, 13] >> 31).astype(bool)
    assert sp.sum() > 1000
    P = oracle.project(scene, cams)
    px, py = P["mean2d"][v, vals, 0], P["mean2d"][v, vals, 1]
    A, B, C = (P["conic"][v, vals, k] for k in range(3))
    qm = 2.0 * (np.log(255.0) + np.log(P["alpha_hat"][v, vals]))
    thr = qm + 2e-4 * np.abs(qm) + 1e-3
    x0, y0 = 16.0 * tx, 16.0 * ty - 0.5
    # the spans' own slack: 1e-3 px on every edge, rows kept when the band
    # comes within it of the ellipse
    qmin = _box_min_q(A, B, C, px, py, x0 - 2e-3, x0 + 15.0 + 2e-3, y0 - 2e-3, y0 + 16.0 + 2e-3)
    bad = sp & (qmin > thr * (1 + 1e-5) + 1e-4)
    assert not bad.any(), (int(bad.sum()), qmin[bad][:3], thr[bad][:3])


def test_many_small_views_bit_exact():
    """1,100 views of 16x16 pixels (one tile each) on an arc around 200
    Gaussians: more views than the depth-range and key kernels have grid
    rows below 1,024, and a (view, depth) range beyond 32-bit keys.  Lists
    are bit-exact and images match the oracle."""
    require_gpu()
    scene = scenes.make_scene(200, 31, log_scale_mu=-2.5)
    cams = scenes.arc_cameras(1100, 4.0, 16, 16, azimuth_deg=300.0)
    g, gc, r, out = gpu_forward(scene, cams, capacity=1 << 20)
    P_or, L_or, img_or = oracle.forward(scene, cams)
    L_g = lists_to_numpy(out["lists"])
    assert L_g["count"] == L_or["count"] > 0
    np.testing.assert_array_equal(L_g["keys"], L_or["keys"])
    np.testing.assert_array_equal(L_g["vals"], L_or["vals"])
    np.testing.assert_array_equal(L_g["ranges"], L_or["ranges"])
    compare_images(out, img_or, "many_views_1100")


@pytest.mark.parametrize("which", ["plain_10k", "frame_20k_4v"])
def test_render_forward_parity(which):
    require_gpu()
    say(f"render fwd {which}")
    if which == "plain_10k":
        scene, cams, _ = scenes.workload_plain_10k(0)
        bg = (0.0, 0.0, 0.0)
    else:
        scene, cams = small_frame_workload(2)
        bg = (0.25, 0.5, 0.75)
    g, gc, r, out = gpu_forward(scene, cams, bg)
    P_or, L_or, img_or = oracle.forward(scene, cams, bg)
    err, near = compare_images(out, img_or, which)
    say(f"  max image error {err:.2e}, {near} pixels near a threshold")


def test_render_forward_is_deterministic():
    require_gpu()
    scene, cams = small_frame_workload(3)
    _, _, _, a = gpu_forward(scene, cams)
    _, _, _, b = gpu_forward(scene, cams)
    assert torch.equal(a["image"], b["image"])
    assert torch.equal(a["n_contrib"], b["n_contrib"])


@pytest.mark.parametrize("bg", [(0.0, 0.0, 0.0), (0.25, 0.5, 0.75)])
def test_fused_forward_l1_equals_forward_then_l1(bg):
    """gs_render_fwd_l1 gives the image, final_T and n_contrib of
    gs_render_fwd and the gradient of gs_l1_loss_grad bit for bit (the same
    FP32 operations), the loss to FP64 summation order; the oracle's L1 of
    the oracle's own image pins the loss to the image tolerance."""
    require_gpu()
    scene, cams = small_frame_workload(4)
    g, gc, r, out = gpu_forward(scene, cams, bg)
    ctx = gs.default_context()
    rng = np.random.default_rng(5)
    target_np = rng.uniform(0, 1, size=tuple(out["image"].shape)).astype(np.float32)
    target = torch.from_numpy(target_np).cuda()
    d_ref = torch.empty_like(target)
    loss_ref = torch.zeros(1, dtype=torch.float64, device="cuda")
    gs.gs_l1_loss_grad(ctx, out["image"], target, d_ref, loss_ref)
    for keep in (True, False):
        d = torch.full_like(target, 7.0)
        loss = torch.zeros(1, dtype=torch.float64, device="cuda")
        out2 = r.forward_l1(g, gc, target, d, loss, bg, keep_image=keep)
        torch.cuda.synchronize()
        if keep:
            assert torch.equal(out2["image"], out["image"])
        else:
            assert out2["image"] is None
        assert torch.equal(out2["final_T"], out["final_T"])
        assert torch.equal(out2["n_contrib"], out["n_contrib"])
        assert torch.equal(d, d_ref)
        assert abs(loss.item() - loss_ref.item()) <= 1e-12 * max(1.0, loss_ref.item())
    # |mean|a - t| - mean|b - t|| <= mean|a - b|: images agree within 1e-4
    # except at the near-threshold pixels (at most the workload's cap),
    # within 5e-3 there
    _, _, img_or = oracle.forward(scene, cams, np.array(bg, np.float64))
    loss_or, _ = oracle.l1(img_or["image"], target_np)
    cap = NEAR_FRAC_CAP["frame_20k_4v"]
    assert img_or["near_threshold"].mean() <= cap
    assert abs(loss_ref.item() - loss_or) <= IMG_ATOL + cap * NEAR_ATOL


def test_fused_forward_l1_rejects_bad_arguments():
    require_gpu()
    scene, cams = small_frame_workload(4)
    g, gc, r, out = gpu_forward(scene, cams)
    ctx = gs.default_context()
    V, _, H, W = out["image"].shape
    target = torch.zeros_like(out["image"])
    d = torch.empty_like(target)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    need = gs.render_fwd_l1_workspace_size(V, W, H)
    assert need == V * ((W + 15) // 16) * ((H + 15) // 16) * 8
    ws = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
    proj, lists = out["proj"], out["lists"]

    def call(tgt, workspace):
        gs.gs_render_fwd_l1(ctx, proj, lists, gc, (0, 0, 0), tgt, None, out["final_T"],
                            out["n_contrib"], d, loss, workspace)

    for tgt, workspace, code in ((None, ws, gs.GS_ERR_INVALID_ARG),
                                 (target, ws[:need - 8], gs.GS_ERR_OOM),
                                 (target, ws[16:], gs.GS_ERR_INVALID_ARG)):
        with pytest.raises(gs.GsError) as ei:
            call(tgt, workspace)
        assert ei.value.code == code
    call(target, ws)
    torch.cuda.synchronize()


def _oracle_grads(scene, cams, P_or, L_or, img_or, seed):
    rng = np.random.default_rng(seed)
    target = rng.uniform(0, 1, size=img_or["image"].shape)
    _, gI = oracle.l1(img_or["image"], target)
    gI[np.broadcast_to(img_or["near_threshold"][:, None], gI.shape)] = 0.0
    g2d, grads = oracle.backward(scene, cams, P_or, L_or, gI)
    return gI, g2d, grads


@pytest.mark.parametrize("which", ["plain_10k", "frame_20k_4v"])
def test_render_backward_parity(which):
    require_gpu()
    say(f"render bwd {which}")
    if which == "plain_10k":
        scene, cams, _ = scenes.workload_plain_10k(0)
    else:
        scene, cams = small_frame_workload(4)
    g, gc, r, out = gpu_forward(scene, cams)
    P_or, L_or, img_or = oracle.forward(scene, cams)
    gI, g2d_or, gr_or = _oracle_grads(scene, cams, P_or, L_or, img_or, 5)
    grad = gs.Gaussians.zeros_like(g)
    ws = r.backward(g, gc, out, torch.from_numpy(gI.astype(np.float32)).cuda(), grad)
    torch.cuda.synchronize()
    n = scene["n"]
    g2d = ws.view(torch.float32)[: gc.V * g.ld * 12].view(gc.V, g.ld, 12)[:, :n, :9].cpu().numpy()
    assert_grad_close(g2d, g2d_or, "screen-space gradients")
    for name in ("mean", "log_scale", "quat", "opacity", "sh"):
        got = getattr(grad, name).cpu().numpy()[..., :n]
        assert_grad_close(got, gr_or[name][..., :n], name)


def test_render_backward_parity_with_background():
    """A non-black background enters dL/dalpha through the colour
    composited behind each entry; the oracle keeps that colour, the kernel
    only its dot product with dL/dcolour."""
    require_gpu()
    bg = (0.25, 0.5, 0.75)
    scene, cams = small_frame_workload(6)
    g, gc, r, out = gpu_forward(scene, cams, bg)
    P_or, L_or, img_or = oracle.forward(scene, cams, bg)
    rng = np.random.default_rng(17)
    _, gI = oracle.l1(img_or["image"], rng.uniform(0, 1, size=img_or["image"].shape))
    gI[np.broadcast_to(img_or["near_threshold"][:, None], gI.shape)] = 0.0
    g2d_or, gr_or = oracle.backward(scene, cams, P_or, L_or, gI, bg)
    grad = gs.Gaussians.zeros_like(g)
    ws = r.backward(g, gc, out, torch.from_numpy(gI.astype(np.float32)).cuda(), grad, bg)
    torch.cuda.synchronize()
    n = scene["n"]
    g2d = ws.view(torch.float32)[: gc.V * g.ld * 12].view(gc.V, g.ld, 12)[:, :n, :9].cpu().numpy()
    assert_grad_close(g2d, g2d_or, "screen-space gradients")
    for name in ("mean", "opacity", "sh"):
        got = getattr(grad, name).cpu().numpy()[..., :n]
        assert_grad_close(got, gr_or[name][..., :n], name)


def test_frame_update_gradient_parity():
    """Backward to the (8, gh, gw) delta images on the 2,000-Gaussian, 64x64
    subset of the temporal frame-update workload."""
    require_gpu()
    full = scenes.make_scene(300_000, 0, -3.0, 3.0, -4.0, 0.5, 3)
    sc = scenes.subset(full, 2000)
    n = 2000
    gw = gh = scenes.grid_side(n)
    d = scenes.make_delta(n, gw, gh, 7)
    mask = scenes.prune_mask(d, n, 0.3)
    cams = scenes.arc_cameras(1, 5.0, 64, 64)
    frame = oracle.apply(sc, d, mask, gw, gh)
    P_or, L_or, img_or = oracle.forward(frame, cams)
    gI, _, gr_or = _oracle_grads(frame, cams, P_or, L_or, img_or, 8)
    gd_or = oracle.apply_bwd(sc, mask, gw, gh, gr_or)
    anchor = gs.Gaussians.from_scene(sc)
    r = Rasterizer(capacity=1 << 16)
    gc = gs.Cameras(cams)
    delta = torch.from_numpy(d).cuda().requires_grad_(True)
    mask_t = torch.from_numpy(mask).cuda()
    img = GSFrameRender.apply(delta, (r, gc, anchor, mask_t, gw, gh, (0.0, 0.0, 0.0)))
    img.backward(torch.from_numpy(gI.astype(np.float32)).cuda())
    torch.cuda.synchronize()
    got = delta.grad.cpu().numpy()
    assert np.all(got.reshape(8, -1)[:, n:] == 0)
    assert np.all(got.reshape(8, -1)[:, :n][:, mask.reshape(-1)[:n] == 0] == 0)
    assert_grad_close(got, gd_or, "delta images")


@pytest.mark.parametrize("which", ["plain_10k", "frame_20k_4v"])
def test_autograd_render_matches_oracle_for_all_parameter_groups(which):
    """GSRender through torch.autograd: the image equals the oracle's and the
    gradients of means, log-scales, quaternions, opacity logits and SH
    coefficients match the oracle's analytic backward."""
    require_gpu()
    say(f"GSRender autograd {which}")
    if which == "plain_10k":
        scene, cams, _ = scenes.workload_plain_10k(1)
    else:
        scene, cams = small_frame_workload(9)
    P_or, L_or, img_or = oracle.forward(scene, cams)
    gI, _, gr_or = _oracle_grads(scene, cams, P_or, L_or, img_or, 21)
    g = gs.Gaussians.from_scene(scene)
    gc = gs.Cameras(cams)
    r = Rasterizer(capacity=1 << 16)
    leaves = [t.clone().requires_grad_(True) for t in g.planes()]
    img = GSRender.apply(*leaves, (r, gc, g.n, g.deg, (0.0, 0.0, 0.0)))
    keep = ~img_or["near_threshold"]
    err = np.abs(img.detach().cpu().numpy() - img_or["image"]).max(axis=1)[keep].max()
    assert err <= IMG_ATOL, f"image error {err:.3e}"
    img.backward(torch.from_numpy(gI.astype(np.float32)).cuda())
    torch.cuda.synchronize()
    n = scene["n"]
    for name, t in zip(("mean", "log_scale", "quat", "opacity", "sh"), leaves):
        assert t.grad is not None
        assert_grad_close(t.grad.cpu().numpy()[..., :n], gr_or[name][..., :n], name)


def test_two_renders_differentiated_together():
    """Two forwards on one rasterizer and one backward through both: each
    render keeps its own projected records and lists, so the gradient is the
    sum of the two separate backwards (up to FP32 addition order).  A plain
    forward state whose buffers a later forward reused is refused."""
    require_gpu()
    say("two renders, one backward")
    scene, cams = small_frame_workload(10)
    g = gs.Gaussians.from_scene(scene)
    gc = gs.Cameras(cams)
    rng = np.random.default_rng(3)
    gA = torch.from_numpy(rng.uniform(-1, 1, (4, 3, 150, 200)).astype(np.float32)).cuda()
    gB = torch.from_numpy(rng.uniform(-1, 1, (4, 3, 150, 200)).astype(np.float32)).cuda()
    shift = torch.zeros_like(g.mean)
    shift[0] = 0.05  # the second render sees every mean moved along x

    def grads(weights):
        leaves = [t.clone().requires_grad_(True) for t in g.planes()]
        r = Rasterizer(capacity=1 << 16)
        meta = (r, gc, g.n, g.deg, (0.0, 0.0, 0.0))
        loss = 0.0
        if weights[0]:
            loss = loss + (GSRender.apply(*leaves, meta) * gA).sum()
        if weights[1]:
            moved = [leaves[0] + shift] + leaves[1:]
            loss = loss + (GSRender.apply(*moved, meta) * gB).sum()
        loss.backward()
        torch.cuda.synchronize()
        return [t.grad.cpu().numpy()[..., :g.n].astype(np.float64) for t in leaves]

    both, a, b = grads((1, 1)), grads((1, 0)), grads((0, 1))
    for name, x, y, z in zip(("mean", "log_scale", "quat", "opacity", "sh"), both, a, b):
        assert_grad_close(x, y + z, name)
    # the plain path: a second forward makes the first state stale
    r = Rasterizer(capacity=1 << 16)
    s1 = r.forward(g, gc)
    s2 = r.forward(g, gc)
    grad = gs.Gaussians.zeros_like(g)
    with pytest.raises(RuntimeError, match="stale"):
        r.backward(g, gc, s1, gA, grad)
    r.backward(g, gc, s2, gA, grad)
    torch.cuda.synchronize()


def test_fused_render_l1_autograd_equals_render_then_l1():
    """GSRenderL1 (render with the L1 term fused into the compositing) gives
    the loss of GSRender followed by GSL1Loss to FP64 summation order and
    bit-identical parameter gradients, scaled by the incoming gradient; two
    fused calls differentiate together (each keeps its own buffers)."""
    require_gpu()
    say("fused render + L1 under autograd")
    from paper_2512_20943_amd.raster import GSL1Loss, GSRenderL1
    scene, cams = small_frame_workload(12)
    g = gs.Gaussians.from_scene(scene)
    gc = gs.Cameras(cams)
    rng = np.random.default_rng(12)
    target = torch.from_numpy(rng.uniform(0, 1, (4, 3, 150, 200)).astype(np.float32)).cuda()
    ctx = gs.default_context()

    def run(fused, scale, twice=False):
        leaves = [t.clone().requires_grad_(True) for t in g.planes()]
        meta = (Rasterizer(capacity=1 << 16), gc, g.n, g.deg, (0.0, 0.0, 0.0))
        if fused:
            loss = GSRenderL1.apply(*leaves, target, meta)
            if twice:
                loss = loss + GSRenderL1.apply(*leaves, target, meta)
        else:
            loss = GSL1Loss.apply(GSRender.apply(*leaves, meta), target, ctx)
        (scale * loss).backward()
        torch.cuda.synchronize()
        return float(loss.item()), [t.grad.cpu().numpy() for t in leaves]

    l_ref, g_ref = run(False, 1.0)
    l_fused, g_fused = run(True, 1.0)
    assert abs(l_fused - l_ref) <= 1e-12 * abs(l_ref)
    for x, y in zip(g_fused, g_ref):
        assert np.array_equal(x, y)
    # a scaled dL/dimage rounds differently inside the backward: compared
    # as gradients are everywhere else (relative to the norm)
    _, g_scaled = run(True, 3.0)
    for name, x, y in zip(("mean", "log_scale", "quat", "opacity", "sh"), g_scaled, g_ref):
        assert_grad_close(x[..., :g.n], 3.0 * y[..., :g.n], name)
    # two identical renders: autograd adds two identical gradients
    l_two, g_two = run(True, 1.0, twice=True)
    assert abs(l_two - 2 * l_ref) <= 1e-12 * abs(l_ref)
    for x, y in zip(g_two, g_ref):
        assert np.array_equal(x, 2.0 * y)


def test_l1_and_adam_match_closed_forms():
    require_gpu()
    ctx = gs.default_context()
    rng = np.random.default_rng(9)
    img = rng.uniform(0, 1, 5000).astype(np.float32)
    tgt = img.copy()
    tgt[::3] = rng.uniform(0, 1, tgt[::3].shape)
    loss_or, g_or = oracle.l1(img, tgt)
    grad = torch.empty(5000, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    gs.gs_l1_loss_grad(ctx, torch.from_numpy(img).cuda(), torch.from_numpy(tgt).cuda(), grad, loss)
    torch.cuda.synchronize()
    assert abs(loss.item() - loss_or) <= 1e-9
    np.testing.assert_allclose(grad.cpu().numpy(), g_or, rtol=1e-6, atol=0)
    th = rng.normal(size=4096).astype(np.float32)
    gg = rng.normal(size=4096).astype(np.float32)
    m = np.zeros(4096)
    v = np.zeros(4096)
    p_t, g_t = torch.from_numpy(th.copy()).cuda(), torch.from_numpy(gg).cuda()
    m_t, v_t = torch.zeros(4096, device="cuda"), torch.zeros(4096, device="cuda")
    ref = th.astype(np.float64)
    for step in range(1, 4):
        ref, m, v = oracle.adam(ref, gg, m, v, step)
        gs.gs_adam_step(ctx, p_t, g_t, m_t, v_t, step)
    torch.cuda.synchronize()
    np.testing.assert_allclose(p_t.cpu().numpy(), ref, rtol=0, atol=1e-6)


def test_l1_autograd_function_matches_oracle():
    """GSL1Loss returns mean |image - target| and hands sign(d) / count,
    scaled by the incoming gradient, back to the image."""
    require_gpu()
    from paper_2512_20943_amd.raster import GSL1Loss
    ctx = gs.default_context()
    rng = np.random.default_rng(10)
    img = rng.uniform(0, 1, (2, 3, 17, 23)).astype(np.float32)
    tgt = img.copy()
    tgt[:, :, ::2] = rng.uniform(0, 1, tgt[:, :, ::2].shape)
    loss_or, g_or = oracle.l1(img.ravel(), tgt.ravel())
    x = torch.from_numpy(img).cuda().requires_grad_(True)
    loss = GSL1Loss.apply(x, torch.from_numpy(tgt).cuda(), ctx)
    (2.5 * loss).backward()
    assert abs(loss.item() - loss_or) <= 1e-9
    np.testing.assert_allclose(x.grad.cpu().numpy().ravel(), 2.5 * g_or, rtol=1e-6, atol=0)


@pytest.mark.parametrize("count,offset", [(1, 0), (5003, 1), (4_112_537, 0)])
def test_sq_error_vector_and_scalar_paths(count, offset):
    """gs_sq_error adds sum (a - b)^2, each term formed in FP64 from the two
    FP32 values, to an FP64 scalar: 16-byte loads when both buffers are
    aligned, one value at a time otherwise and in the tail, at most 1024
    blocks striding over large counts."""
    require_gpu()
    ctx = gs.default_context()
    rng = np.random.default_rng(count)
    a = rng.uniform(0, 1, count + offset).astype(np.float32)
    b = (a + rng.normal(0, 0.1, a.shape)).astype(np.float32)
    ref = float(((a[offset:].astype(np.float64) - b[offset:].astype(np.float64)) ** 2).sum())
    s = torch.full((1,), 0.5, dtype=torch.float64, device="cuda")
    gs.gs_sq_error(ctx, torch.from_numpy(a).cuda()[offset:], torch.from_numpy(b).cuda()[offset:], s)
    torch.cuda.synchronize()
    assert abs(s.item() - 0.5 - ref) <= 1e-12 * max(1.0, ref) * max(1.0, np.log2(count))


@pytest.mark.parametrize("count,offset", [(5003, 0), (5003, 1), (3_000_001, 0)])
def test_l1_vector_and_scalar_paths(count, offset):
    """The L1 kernel takes four values per step when the three buffers are
    16-byte aligned and one at a time otherwise and in the tail; a grid of at
    most 1024 blocks strides over large counts."""
    require_gpu()
    ctx = gs.default_context()
    rng = np.random.default_rng(count + offset)
    img = rng.uniform(0, 1, count).astype(np.float32)
    tgt = img.copy()
    tgt[::3] = rng.uniform(0, 1, tgt[::3].shape)
    loss_or, g_or = oracle.l1(img, tgt)
    img_d = torch.empty(count + offset, device="cuda")
    tgt_d = torch.empty(count + offset, device="cuda")
    grad = torch.empty(count + offset, device="cuda")
    img_d[offset:] = torch.from_numpy(img).cuda()
    tgt_d[offset:] = torch.from_numpy(tgt).cuda()
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    gs.gs_l1_loss_grad(ctx, img_d[offset:], tgt_d[offset:], grad[offset:], loss)
    torch.cuda.synchronize()
    assert abs(loss.item() - loss_or) <= 1e-9
    np.testing.assert_allclose(grad[offset:].cpu().numpy(), g_or, rtol=1e-6, atol=0)


# ---------------------------------------------------------------------------
# edge cases
# ---------------------------------------------------------------------------

def test_empty_scene_renders_background():
    require_gpu()
    sc = scenes.make_scene(0, 0, sh_degree=1)
    cams = scenes.axis_camera(33, 17)
    g, gc, r, out = gpu_forward(sc, cams, bg=(0.1, 0.2, 0.3))
    assert out["lists"].count == 0
    im = out["image"].cpu().numpy()
    np.testing.assert_allclose(im[0, :, :, :], np.array([0.1, 0.2, 0.3])[:, None, None] *
                               np.ones((3, 17, 33)), atol=1e-7)
    assert (out["n_contrib"] == 0).all() and (out["final_T"] == 1).all()


def test_all_culled_and_tiny_images():
    require_gpu()
    sc = scenes.make_scene(500, 1, -1, 1, -3, 0.5, 0)
    behind = scenes.stack_cams([(np.eye(3), np.array([0.0, 0.0, -10.0]),
                                 np.array([50.0, 50.0, 0.5, 0.5]), (1, 1))])
    _, _, _, out = gpu_forward(sc, behind)
    assert out["lists"].count == 0
    for W, H in ((1, 1), (17, 33), (16, 16)):
        cams = scenes.axis_camera(W, H)
        _, _, _, out = gpu_forward(sc, cams)
        _, L_or, img_or = oracle.forward(sc, cams)
        assert out["lists"].count == L_or["count"]
        compare_images(out, img_or, "tiny")


def test_single_centred_gaussian_and_huge_gaussian():
    require_gpu()
    sc = scenes.make_scene(2, 0, 0, 0, -3, 0.0, 0)
    sc["mean"][:, :2] = 0.0
    sc["mean"][2, 1] = 0.5
    sc["log_scale"][:, 1] = 0.3  # sigma ~ 1.35 -> covers every tile
    sc["opacity"][:2] = [0.2, -1.0]
    cams = scenes.axis_camera(96, 80)
    g, gc, r, out = gpu_forward(sc, cams)
    _, L_or, img_or = oracle.forward(sc, cams)
    assert out["lists"].count == L_or["count"]
    compare_images(out, img_or, "single_and_huge")
    TX, TY = 6, 5
    assert (out["lists"].ranges[:TX * TY, 1] - out["lists"].ranges[:TX * TY, 0] >= 1).all()


def test_capacity_error_reports_the_need_and_retry_succeeds():
    require_gpu()
    scene, cams, _ = scenes.workload_plain_10k(0)
    g = gs.Gaussians.from_scene(scene)
    gc = gs.Cameras(cams)
    ctx = gs.default_context()
    proj = gs.Projected.empty(gc.V, g.n, g.ld)
    gs.gs_project(ctx, g, gc, proj)
    small = gs.TileLists(100, gc.n_segments())
    ws = torch.empty(gs.bin_sort_workspace_size(gc.V, g.ld, 100, gc.n_segments()),
                     dtype=torch.uint8, device="cuda")
    with pytest.raises(gs.GsError) as ei:
        gs.gs_bin_sort(ctx, proj, gc, small, ws)
    assert ei.value.code == gs.GS_ERR_CAPACITY
    need = small.count
    assert need > 100
    r = Rasterizer(capacity=100)
    lists = r.bin_sort(proj, gc)
    assert lists.count == need


def test_invalid_arguments_are_rejected():
    require_gpu()
    scene, cams, _ = scenes.workload_plain_10k(0)
    g = gs.Gaussians.from_scene(scene)
    gc = gs.Cameras(cams)
    ctx = gs.default_context()
    proj = gs.Projected.empty(gc.V, g.n, g.ld)
    bad = gs.Gaussians(g.n, 4, g.ld, *g.planes())
    with pytest.raises(gs.GsError) as ei:
        gs.gs_project(ctx, bad, gc, proj)
    assert ei.value.code == gs.GS_ERR_INVALID_ARG
    bad = gs.Gaussians(g.n, g.deg, g.ld + 1, *g.planes())
    with pytest.raises(gs.GsError):
        gs.gs_project(ctx, bad, gc, proj)
    two = gs.Cameras(scenes.stack_cams([
        (np.eye(3), np.array([0, 0, 4.0]), np.array([100.0, 100, 64, 64]), (128, 128)),
        (np.eye(3), np.array([0, 0, 4.0]), np.array([100.0, 100, 32, 32]), (64, 64))]))
    p2 = gs.Projected.empty(2, g.n, g.ld)
    gs.gs_project(ctx, g, two, p2)
    r = Rasterizer(capacity=1 << 16)
    lists = r.bin_sort(p2, two)
    with pytest.raises(gs.GsError):
        gs.gs_render_fwd(ctx, p2, lists, two, (0, 0, 0), torch.empty(2, 3, 128, 128, device="cuda"),
                         torch.empty(2, 128, 128, device="cuda"),
                         torch.empty(2, 128, 128, dtype=torch.int32, device="cuda"))
    ws = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(gs.GsError) as ei:
        gs.gs_bin_sort(ctx, proj, gc, gs.TileLists(1000, gc.n_segments()), ws)
    assert ei.value.code == gs.GS_ERR_OOM
    with pytest.raises(gs.GsError) as ei:  # emission-base copy shorter than V * ld
        gs.gs_bin_sort(ctx, proj, gc, gs.TileLists(1000, gc.n_segments(), gv=1), ws)
    assert ei.value.code == gs.GS_ERR_INVALID_ARG
    need = gs.bin_sort_workspace_size(gc.V, g.ld, 1000, gc.n_segments())
    big = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(gs.GsError) as ei:  # workspace off its 256-byte alignment
        gs.gs_bin_sort(ctx, proj, gc, gs.TileLists(1000, gc.n_segments()), big[16:])
    assert ei.value.code == gs.GS_ERR_INVALID_ARG


def _code(fn):
    with pytest.raises(gs.GsError) as ei:
        fn()
    return ei.value.code


def test_training_and_delivery_calls_reject_bad_arguments():
    """The loss, keyframe, culling and sent-update calls validate before
    enqueueing anything."""
    require_gpu()
    ctx = gs.default_context()
    dev = "cuda"
    img = torch.zeros(1, 3, 16, 16, device=dev)
    grad = torch.empty_like(img)
    loss = torch.zeros(1, dtype=torch.float64, device=dev)
    small_ws = torch.empty(8, dtype=torch.uint8, device=dev)
    assert _code(lambda: gs.gs_l1_dssim_loss_grad(ctx, img, img, grad, loss, small_ws)) == \
        gs.GS_ERR_OOM
    ws = torch.empty(gs.l1_dssim_workspace_size(3, 16, 16), dtype=torch.uint8, device=dev)
    assert _code(lambda: gs.gs_l1_dssim_loss_grad(ctx, img, img, grad, loss, ws, 1.5)) == \
        gs.GS_ERR_INVALID_ARG
    x = torch.zeros(4, 64, device=dev)
    assert _code(lambda: gs.gs_keyframe_temporal_l1(ctx, x, x, 65, 1e-3, x)) == \
        gs.GS_ERR_INVALID_ARG                       # bound beyond the plane stride
    logit = torch.zeros(100, device=dev)
    idx = torch.empty(100, dtype=torch.int32, device=dev)
    for bad in (0.0, 1.0, float("nan")):
        assert _code(lambda: gs.gs_cull_low_opacity(ctx, logit, 100, bad, idx)) == \
            gs.GS_ERR_INVALID_ARG
    assert _code(lambda: gs.gs_cull_low_opacity(ctx, logit, 100, 0.1, idx, small_ws[:0])) == \
        gs.GS_ERR_OOM
    d = torch.zeros(8, 4, 4, device=dev)
    m = torch.ones(4, 4, dtype=torch.uint8, device=dev)
    amax = torch.zeros(8, device=dev)
    assert _code(lambda: gs.gs_residual_delta(ctx, d, d, m, 17, 4, 4, d, amax)) == \
        gs.GS_ERR_INVALID_ARG                       # 17 Gaussians on a 4x4 grid
    q = torch.empty(8, 4, 4, dtype=torch.int16, device=dev)
    assert _code(lambda: gs.gs_quantize_delta(ctx, d, amax, 12, 16, 4, 4, q, amax)) == \
        gs.GS_ERR_INVALID_ARG                       # 12-bit codes
    sc = scenes.make_scene(16, 1, -1, 1, -4, 0.5, 0)
    a = gs.Gaussians.from_scene(sc)
    f = frame_of(a)
    assert _code(lambda: gs.gs_apply_quantized_update(ctx, a, q, 16, amax, d, 3, 3, f)) == \
        gs.GS_ERR_INVALID_ARG                       # grid too small for 16 Gaussians


# ---------------------------------------------------------------------------
# full-size frame workload: sampled checks
# ---------------------------------------------------------------------------

def test_full_frame_300k_20_views_sampled():
    """300,000 Gaussians, SH 3, 20 views at 1352x1014: every projection record
    is compared, view 0's tile lists bit for bit (full rectangles, as the
    definition bins), view 0's image in full; then the benchmark's binning
    (opacity-aware rectangles with per-row tile spans) must give the same
    images and final transmittance bit for bit from fewer instances."""
    require_gpu()
    say("full frame 300k x 20 views")
    scene, cams, _ = scenes.workload_frame_300k(0)
    g, gc, r, out = gpu_forward(scene, cams, capacity=1 << 26)
    say(f"  instances {out['lists'].count}")
    P_or = oracle.project(scene, cams)
    P_g = projected_to_oracle(out["proj"])
    compare_projection(P_g, P_or)
    cam0 = {k: v[:1] for k, v in cams.items()}
    P0 = {k: (v[:1] if isinstance(v, np.ndarray) else v) for k, v in P_or.items()}
    P0["V"] = 1
    L0 = oracle.bin_sort(P0, cam0)
    L_g = lists_to_numpy(out["lists"])
    nseg0 = L0["n_segments"]
    rg = L_g["ranges"][:nseg0]
    np.testing.assert_array_equal(rg, L0["ranges"])
    M0 = int(rg[:, 1].max())
    np.testing.assert_array_equal(L_g["vals"][:M0], L0["vals"])
    np.testing.assert_array_equal(L_g["keys"][:M0], L0["keys"])
    img0 = oracle.render_fwd(P0, L0, cam0)
    out0 = {k: out[k][:1] for k in ("image", "final_T", "n_contrib")}
    err, near = compare_images(out0, img0, "frame_300k_view0")
    say(f"  view 0 max image error {err:.2e}, {near} near-threshold pixels")
    _, _, _, out_s = gpu_forward(scene, cams, with_keys=False, capacity=1 << 26,
                                 tight_rect=True, tile_spans=True)
    say(f"  spans: {out_s['lists'].count} instances")
    assert 0 < out_s["lists"].count < out["lists"].count
    assert torch.equal(out_s["image"], out["image"])
    assert torch.equal(out_s["final_T"], out["final_T"])
    # the benchmark's tile sets: every record's spans, view 0's lists bit for
    # bit, and n_contrib as positions in those lists
    P_s = oracle.project(scene, cams, "spans")
    Pg_s = projected_to_oracle(out_s["proj"])
    np.testing.assert_array_equal(Pg_s["tiles"], P_s["tiles"])
    vis = (P_s["flags"] & 32) > 0
    np.testing.assert_array_equal(Pg_s["rect"][vis], P_s["rect"][vis])
    for a, b in zip(span_rows(Pg_s), span_rows(P_s)):
        np.testing.assert_array_equal(a, b)
    del Pg_s
    P0s = {k: (v[:1] if isinstance(v, np.ndarray) else v) for k, v in P_s.items()}
    P0s["V"] = 1
    del P_s
    L0s = oracle.bin_sort(P0s, cam0)
    L_s = lists_to_numpy(out_s["lists"])
    rg = L_s["ranges"][:nseg0]
    np.testing.assert_array_equal(rg, L0s["ranges"])
    np.testing.assert_array_equal(L_s["vals"][:int(rg[:, 1].max())], L0s["vals"])
    img0s = oracle.render_fwd(P0s, L0s, cam0)
    out0s = {k: out_s[k][:1] for k in ("image", "final_T", "n_contrib")}
    compare_images(out0s, img0s, "frame_300k_view0")


def _sparse_tile_gradient(img_shape, n_tiles, seed, W, H):
    """dL/dimage that is nonzero (random signs / count) only on n_tiles random
    16x16 tiles per view, so the oracle backward only walks those tiles."""
    rng = np.random.default_rng(seed)
    V = img_shape[0]
    g = np.zeros(img_shape)
    TX, TY = (W + 15) // 16, (H + 15) // 16
    count = float(np.prod(img_shape))
    for v in range(V):
        for t in rng.choice(TX * TY, size=min(n_tiles, TX * TY), replace=False):
            ty, tx = divmod(int(t), TX)
            blk = g[v, :, ty * 16:(ty + 1) * 16, tx * 16:(tx + 1) * 16]
            blk[...] = rng.choice([-1.0, 1.0], size=blk.shape) / count
    return g


def test_full_frame_backward_sparse_tiles():
    """Backward at the full 300k-Gaussian / 20-view / 1352x1014 size and in the
    benchmark's launch configuration (opacity-aware rectangles with per-row
    tile spans), with the image gradient restricted to 30 random tiles per
    view (the oracle, binning full rectangles, walks only those)."""
    require_gpu()
    say("full frame backward, sparse tiles")
    scene, cams, _ = scenes.workload_frame_300k(0)
    g, gc, r, out = gpu_forward(scene, cams, with_keys=False, capacity=1 << 26,
                                tight_rect=True, tile_spans=True)
    P_or, L_or, img_or = oracle.forward(scene, cams)
    gI = _sparse_tile_gradient(img_or["image"].shape, 30, 21, 1352, 1014)
    gI[np.broadcast_to(img_or["near_threshold"][:, None], gI.shape)] = 0.0
    g2d_or, gr_or = oracle.backward(scene, cams, P_or, L_or, gI)
    grad = gs.Gaussians.zeros_like(g)
    ws = r.backward(g, gc, out, torch.from_numpy(gI.astype(np.float32)).cuda(), grad)
    torch.cuda.synchronize()
    n = scene["n"]
    g2d = ws.view(torch.float32)[: gc.V * g.ld * 12].view(gc.V, g.ld, 12)[:, :n, :9].cpu().numpy()
    assert_grad_close(g2d, g2d_or, "screen-space gradients")
    for name in ("mean", "log_scale", "quat", "opacity", "sh"):
        assert_grad_close(getattr(grad, name).cpu().numpy()[..., :n], gr_or[name][..., :n], name)


def test_full_frame_update_delta_gradient_sparse_tiles():
    """Apply + render + backward to the (8, 548, 548) delta images at the full
    300k / 20-view size, pruning level 0.5, sparse-tile image gradient."""
    require_gpu()
    say("full frame update backward, sparse tiles")
    scene, cams, _ = scenes.workload_frame_300k(0)
    n = scene["n"]
    gw = gh = scenes.grid_side(n)
    d = scenes.make_delta(n, gw, gh, 12)
    mask = scenes.prune_mask(d, n, 0.5)
    frame = oracle.apply(scene, d, mask, gw, gh)
    P_or, L_or, img_or = oracle.forward(frame, cams)
    gI = _sparse_tile_gradient(img_or["image"].shape, 20, 22, 1352, 1014)
    gI[np.broadcast_to(img_or["near_threshold"][:, None], gI.shape)] = 0.0
    _, gr_or = oracle.backward(frame, cams, P_or, L_or, gI)
    gd_or = oracle.apply_bwd(scene, mask, gw, gh, gr_or)
    anchor = gs.Gaussians.from_scene(scene)
    r = Rasterizer(capacity=1 << 26, tight_rect=True, tile_spans=True)  # as benchmarked
    delta = torch.from_numpy(d).cuda().requires_grad_(True)
    img = GSFrameRender.apply(delta, (r, gs.Cameras(cams), anchor, torch.from_numpy(mask).cuda(),
                                      gw, gh, (0.0, 0.0, 0.0)))
    img.backward(torch.from_numpy(gI.astype(np.float32)).cuda())
    torch.cuda.synchronize()
    assert_grad_close(delta.grad.cpu().numpy(), gd_or, "delta images")


def test_large_2m_8_views_sampled():
    """2,000,000 Gaussians (means U[-6,6]^3, log-scales N(-4.5,0.7), SH 3), 8
    views at 1920x1080 from inside the cloud: every projection record, view 0's
    tile lists bit for bit and view 0's image."""
    require_gpu()
    say("large 2M x 8 views")
    scene, cams, _ = scenes.workload_large_2m(0)
    g, gc, r, out = gpu_forward(scene, cams, capacity=1 << 26)
    say(f"  instances {out['lists'].count}")
    P_or = oracle.project(scene, cams)
    compare_projection(projected_to_oracle(out["proj"]), P_or)
    cam0 = {k: v[:1] for k, v in cams.items()}
    P0 = {k: (v[:1] if isinstance(v, np.ndarray) else v) for k, v in P_or.items()}
    P0["V"] = 1
    del P_or
    L0 = oracle.bin_sort(P0, cam0)
    L_g = lists_to_numpy(out["lists"])
    rg = L_g["ranges"][:L0["n_segments"]]
    np.testing.assert_array_equal(rg, L0["ranges"])
    M0 = int(rg[:, 1].max())
    np.testing.assert_array_equal(L_g["vals"][:M0], L0["vals"])
    img0 = oracle.render_fwd(P0, L0, cam0)
    out0 = {k: out[k][:1] for k in ("image", "final_T", "n_contrib")}
    err, near = compare_images(out0, img0, "large_2m_view0")
    say(f"  view 0 max image error {err:.2e}, {near} near-threshold pixels")


@pytest.mark.parametrize("mode", ["rect", "spans"])
def test_emission_bases_index_every_instance_once(mode):
    """Emission bases: the instances of each (view, Gaussian) occupy rows
    base .. base + tiles_touched - 1 in row-major order over its tile
    rectangle, or over its per-row spans (record word 15, flagged in bit 31
    of word 13), and these rows, over all sorted instances, are a
    permutation of 0..M-1 (the backward writes one gradient row per instance
    there).  The base in the projected record (word 14, next to the packed
    rectangle in words 12, 13) and the optional gv_base copy agree."""
    require_gpu()
    scene, cams = small_frame_workload(3)
    spans = mode == "spans"
    g, gc, r, out = gpu_forward(scene, cams, emission_bases=True, tight_rect=spans,
                                tile_spans=spans)
    L = out["lists"]
    M = L.count
    vals = L.vals[:M].cpu().numpy().astype(np.int64)
    ranges = L.ranges[:L.n_segments].cpu().numpy().astype(np.int64)
    seg_of = np.repeat(np.arange(L.n_segments), ranges[:, 1] - ranges[:, 0])
    ld = g.ld
    base = L.gv_base[:gc.V * ld].cpu().numpy().view(np.uint32).astype(np.int64)
    words = out["proj"].splat.cpu().numpy().view(np.uint32).reshape(gc.V, ld, 16)
    rect = out["proj"].rect.cpu().numpy().reshape(gc.V, ld, 4)
    tiles = out["proj"].tiles_touched.cpu().numpy().reshape(gc.V, ld)
    touched = tiles > 0
    touched[:, g.n:] = False  # records past n are never written
    np.testing.assert_array_equal(words[..., 14][touched], base.reshape(gc.V, ld)[touched])
    np.testing.assert_array_equal(words[..., 12][touched],
                                  (rect[..., 0] | (rect[..., 1] << 16))[touched])
    flag = (words[..., 13] >> 31).astype(bool)
    np.testing.assert_array_equal((words[..., 13] & 0x7FFFFFFF)[touched],
                                  (rect[..., 2] - rect[..., 0])[touched])
    assert flag[touched].any() == spans
    tpv = [((w + 15) // 16) * ((h + 15) // 16) for (w, h) in cams["wh"]]
    sb = np.concatenate([[0], np.cumsum(tpv)])
    v = np.searchsorted(sb, seg_of, side="right") - 1
    tile = seg_of - sb[v]
    TX = np.array([(w + 15) // 16 for (w, h) in cams["wh"]])[v]
    ty, tx = tile // TX, tile % TX
    rc = rect[v, vals]
    dy, dx = ty - rc[:, 1], tx - rc[:, 0]
    local = dy * (rc[:, 2] - rc[:, 0]) + dx
    sp = flag[v, vals]
    if sp.any():
        # spans: byte r of word 15 = a_r | b_r << 4; an instance lies in its
        # row's span and follows the spans of the rows above it
        m = words[..., 15][v, vals].astype(np.int64)
        a = np.stack([(m >> (8 * k)) & 15 for k in range(4)], axis=1)
        b = np.stack([(m >> (8 * k + 4)) & 15 for k in range(4)], axis=1)
        assert np.all(dy[sp] < 4)
        rows_ = np.arange(len(vals))
        dyc = np.minimum(dy, 3)
        a_r, b_r = a[rows_, dyc], b[rows_, dyc]
        assert np.all((a_r[sp] <= dx[sp]) & (dx[sp] < b_r[sp]))
        pre = np.where(np.arange(4)[None, :] < dyc[:, None], b - a, 0).sum(axis=1)
        local = np.where(sp, pre + dx - a_r, local)
        cnt = (b - a).sum(axis=1)
        np.testing.assert_array_equal(cnt[sp], tiles[v, vals][sp])
    assert np.all((local >= 0) & (local < tiles[v, vals]))
    rows = base[v * ld + vals] + local
    assert np.array_equal(np.sort(rows), np.arange(M))


def test_large_2m_backward_sparse_tiles():
    """Forward + backward over the 2M-Gaussian, 8-view 1920x1080 batch in one
    launch each; the image gradient is nonzero on 20 random tiles of views 0
    and 1 only, so the oracle walks those tiles of those two views."""
    require_gpu()
    say("large 2M x 8 views backward, sparse tiles")
    scene, cams, _ = scenes.workload_large_2m(0)
    g, gc, r, out = gpu_forward(scene, cams, with_keys=False, capacity=1 << 26)
    cam01 = {k: v[:2] for k, v in cams.items()}
    P_or, L_or, img_or = oracle.forward(scene, cam01)
    g01 = _sparse_tile_gradient(img_or["image"].shape, 20, 23, 1920, 1080)
    g01[np.broadcast_to(img_or["near_threshold"][:, None], g01.shape)] = 0.0
    g2d_or, gr_or = oracle.backward(scene, cam01, P_or, L_or, g01)
    gI = np.zeros((8,) + g01.shape[1:], np.float32)
    gI[:2] = g01
    grad = gs.Gaussians.zeros_like(g)
    ws = r.backward(g, gc, out, torch.from_numpy(gI).cuda(), grad)
    torch.cuda.synchronize()
    n = scene["n"]
    g2d = ws.view(torch.float32)[: gc.V * g.ld * 12].view(gc.V, g.ld, 12)[:2, :n, :9].cpu().numpy()
    assert_grad_close(g2d, g2d_or, "screen-space gradients, views 0-1")
    for name in ("mean", "log_scale", "quat", "opacity", "sh"):
        assert_grad_close(getattr(grad, name).cpu().numpy()[..., :n], gr_or[name][..., :n], name)


def test_lists_bit_exact_with_a_depth_range_beyond_32_bit_keys():
    """Gaussians from z = 3 to z = 1e9 seen by 20 views: the view index does
    not fit above the bits of the depth-bit range in 32 bits, so the binning
    sorts 64-bit (view, depth) keys (on the depth bits only, inside each
    view); lists and keys stay bit-exact against the oracle."""
    require_gpu()
    base = scenes.subset(scenes.make_scene(10_000, 7, -1.0, 1.0, -4.0, 0.5, 0), 2000)
    far = [(0.0, 0.0, 1e9), (2e7, 1e7, 1e9), (-3e7, 0.0, 5e8), (0.0, 0.0, 2e9)]
    sc = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in base.items()}
    for j, (x, y, z) in enumerate(far):
        sc["mean"][:, j] = (x, y, z)
        sc["log_scale"][:, j] = np.log(1e6)
        sc["opacity"][j] = 3.0
    one = scenes.axis_camera(64, 48, 4.0)
    cams = {k: np.concatenate([v] * 20) for k, v in one.items()}
    g, gc, r, out = gpu_forward(sc, cams)
    P_or = oracle.project(sc, cams)
    db = P_or["depth_bits"][P_or["tiles"] > 0].astype(np.int64) & 0xFFFFFFFF
    dbits = (int(db.max()) - int(db.min())).bit_length()  # bits of the range
    assert (20 << dbits) > 2 ** 32
    L_or = oracle.bin_sort(P_or, cams)
    L_g = lists_to_numpy(out["lists"])
    assert L_g["count"] == L_or["count"] > 0
    np.testing.assert_array_equal(L_g["keys"], L_or["keys"])
    np.testing.assert_array_equal(L_g["vals"], L_or["vals"])
    np.testing.assert_array_equal(L_g["ranges"], L_or["ranges"])


@pytest.mark.parametrize("tileset", ["rect", "spans"])
def test_lists_bit_exact_with_views_that_see_nothing(tileset):
    """Six views, four of them turned away from the scene (first, last and two
    in a row): the binning sorts run inside each view, so views without a
    visible Gaussian leave empty ranges in both sorts and their neighbours'
    partitions must not shift.  Lists and keys are bit-exact against the
    oracle; the empty views' tiles have empty ranges."""
    require_gpu()
    say(f"lists with empty views {tileset}")
    scene = scenes.make_scene(8_000, 41, -1.0, 1.0, -4.0, 0.5, 0)
    seen = scenes.arc_cameras(2, 5.0, 96, 64, azimuth_deg=40.0)
    away = {k: v[:1].copy() for k, v in seen.items()}
    away["t"] = away["t"] * -3.0  # the scene lies behind this camera
    order = [away, {k: v[:1] for k, v in seen.items()}, away, away,
             {k: v[1:] for k, v in seen.items()}, away]
    cams = {k: np.concatenate([c[k] for c in order]) for k in seen}
    g, gc, r, out = gpu_forward(scene, cams, capacity=1 << 18, tight_rect=tileset != "rect",
                                tile_spans=tileset == "spans")
    P_or = oracle.project(scene, cams, tileset)
    vis = (P_or["tiles"] > 0).sum(axis=1)
    assert list(vis > 0) == [False, True, False, False, True, False], vis
    L_or = oracle.bin_sort(P_or, cams)
    L_g = lists_to_numpy(out["lists"])
    assert L_g["count"] == L_or["count"] > 0
    np.testing.assert_array_equal(L_g["keys"], L_or["keys"])
    np.testing.assert_array_equal(L_g["vals"], L_or["vals"])
    np.testing.assert_array_equal(L_g["ranges"], L_or["ranges"])
    tiles = (96 // 16) * (64 // 16)
    rg = L_g["ranges"].reshape(6, tiles, 2)
    assert (rg[[0, 2, 3, 5], :, 0] == rg[[0, 2, 3, 5], :, 1]).all()


def _bits_for(count):
    return max(int(count) - 1, 0).bit_length()


@pytest.mark.parametrize("ld", [65_536, 131_072])
def test_lists_bit_exact_when_tile_and_id_words_do_not_pack(ld):
    """One 4096x4096 view (65,536 tiles, 16 tile bits).  With ld = 65,536 a
    Gaussian id (16 bits) and a tile index fit one word but a tile count
    (17 bits) does not, so the tile sort moves packed words while the depth
    sort's values carry ids only; with ld = 131,072 neither packs and keys
    and ids move side by side.  Lists and keys are bit-exact against the
    oracle either way."""
    require_gpu()
    say(f"lists, unpacked words, ld {ld}")
    scene = scenes.make_scene(5_000, 43, -1.0, 1.0, -4.0, 0.5, 0, ld=ld)
    cams = scenes.axis_camera(4096, 4096, 4.0)
    max_tiles = 256 * 256
    idbits = _bits_for(ld)
    packed_tiles = idbits + _bits_for(max_tiles) <= 32
    packed_counts = idbits + _bits_for(max_tiles + 1) <= 32
    assert (packed_tiles, packed_counts) == ((True, False) if ld == 65_536 else (False, False))
    g, gc, r, out = gpu_forward(scene, cams, capacity=1 << 20)
    P_or = oracle.project(scene, cams)
    L_or = oracle.bin_sort(P_or, cams)
    L_g = lists_to_numpy(out["lists"])
    assert L_g["count"] == L_or["count"] > 0
    np.testing.assert_array_equal(L_g["keys"], L_or["keys"])
    np.testing.assert_array_equal(L_g["vals"], L_or["vals"])
    np.testing.assert_array_equal(L_g["ranges"], L_or["ranges"])
