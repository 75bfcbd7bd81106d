"""Temporal and keyframe terms (Sec. III-B) on the GPU against the oracle:
the temporal term fused into the delta backward, densification statistics
from the render backward, the keyframe L1 term, low-opacity culling (bit
exact) and plane gathers (bit exact)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2512_20943_amd import gs, scenes
from paper_2512_20943_amd.raster import Rasterizer, frame_of
from tests.gpu_helpers import assert_grad_close, gpu_forward, require_gpu

pytestmark = pytest.mark.gpu


def _oracle_image_grad(img_or, seed):
    rng = np.random.default_rng(seed)
    target = rng.uniform(0, 1, size=img_or["image"].shape)
    _, gI = oracle.l1(img_or["image"], target)
    gI[np.broadcast_to(img_or["near_threshold"][:, None], gI.shape)] = 0.0
    return gI


def test_temporal_term_fused_into_delta_gradient():
    require_gpu()
    full = scenes.make_scene(300_000, 0, -3.0, 3.0, -4.0, 0.5, 3)
    n = 2000
    sc = scenes.subset(full, n)
    gw = gh = scenes.grid_side(n)
    d = scenes.make_delta(n, gw, gh, 7)
    mask = scenes.prune_mask(d, n, 0.3)
    cams = scenes.arc_cameras(1, 5.0, 64, 64)
    lam_t = 1e-3
    frame = oracle.apply(sc, d, mask, gw, gh)
    P_or, L_or, img_or = oracle.forward(frame, cams)
    gI = _oracle_image_grad(img_or, 8)
    _, gr_or = oracle.backward(frame, cams, P_or, L_or, gI)
    t_loss, t_grad = oracle.temporal_l1(d, n, lam_t)
    want = oracle.apply_bwd(sc, mask, gw, gh, gr_or) + t_grad

    ctx = gs.default_context()
    anchor = gs.Gaussians.from_scene(sc)
    fr = frame_of(anchor)
    dt = torch.from_numpy(d).cuda()
    mt = torch.from_numpy(mask).cuda()
    gs.gs_apply_frame_update(ctx, anchor, dt, mt, gw, gh, fr)
    r = Rasterizer(capacity=1 << 16)
    gc = gs.Cameras(cams)
    out = r.forward(fr, gc)
    grad = gs.Gaussians.zeros_like(fr)
    dd = torch.full((8, gh, gw), float("nan"), device="cuda")
    tl = torch.zeros(1, dtype=torch.float64, device="cuda")
    ws = r.bwd_workspace(gc.V, fr.ld, "cuda")
    gs.gs_render_bwd(ctx, fr, out["proj"], out["lists"], gc, (0.0, 0.0, 0.0), out["final_T"],
                     out["n_contrib"], torch.from_numpy(gI.astype(np.float32)).cuda(), grad, ws,
                     upd=(anchor.quat, mt, gw, gh), dL_ddelta=dd, temporal=(lam_t, dt, tl))
    torch.cuda.synchronize()
    got = dd.cpu().numpy()
    assert np.all(got.reshape(8, -1)[:, n:] == 0)
    assert abs(tl.item() - t_loss) <= 1e-6 * t_loss
    assert_grad_close(got, want, "delta images with the temporal term")


def test_densify_stats_match_oracle():
    require_gpu()
    scene = scenes.make_scene(20_000, 2, -3.0, 3.0, -4.0, 0.5, 3)
    cams = scenes.arc_cameras(4, 5.0, 200, 150)
    g, gc, r, out = gpu_forward(scene, cams)
    P_or, L_or, img_or = oracle.forward(scene, cams)
    gI = _oracle_image_grad(img_or, 3)
    g2d_or, _ = oracle.backward(scene, cams, P_or, L_or, gI)
    acc_or, cnt_or = oracle.densify_stats(P_or["flags"], g2d_or)
    n = scene["n"]
    grad = gs.Gaussians.zeros_like(g)
    acc = torch.zeros(g.ld, device="cuda")
    cnt = torch.zeros(g.ld, dtype=torch.int32, device="cuda")
    ws = r.bwd_workspace(gc.V, g.ld, "cuda")
    dimg = torch.from_numpy(gI.astype(np.float32)).cuda()
    ctx = gs.default_context()
    for _ in range(2):   # statistics accumulate over iterations
        gs.gs_render_bwd(ctx, g, out["proj"], out["lists"], gc, (0.0, 0.0, 0.0), out["final_T"],
                         out["n_contrib"], dimg, grad, ws, densify=(acc, cnt))
    torch.cuda.synchronize()
    c = cnt.cpu().numpy()[:n]
    np.testing.assert_array_equal(c, 2 * cnt_or)
    assert cnt_or.sum() > 0
    assert_grad_close(acc.cpu().numpy()[:n], 2 * acc_or, "accumulated |dL/d mean2d|")


def test_keyframe_temporal_l1_matches_oracle():
    require_gpu()
    g = scenes.rng(4)
    x = g.normal(0, 1, (14, 1000)).astype(np.float32)
    prev = x + g.normal(0, 0.1, x.shape).astype(np.float32)
    prev[:, ::7] = x[:, ::7]          # unchanged entries: sign 0
    base = g.normal(0, 1, x.shape).astype(np.float32)
    loss_or, gr_or = oracle.keyframe_temporal_l1(x, prev, 937, 1e-3)
    ctx = gs.default_context()
    gt = torch.from_numpy(base).cuda()
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    gs.gs_keyframe_temporal_l1(ctx, torch.from_numpy(x).cuda(), torch.from_numpy(prev).cuda(),
                               937, 1e-3, gt, loss)
    torch.cuda.synchronize()
    np.testing.assert_allclose(gt.cpu().numpy(), base + gr_or.astype(np.float32), rtol=0,
                               atol=1e-7)
    assert abs(loss.item() - loss_or) <= 1e-6 * loss_or


@pytest.mark.parametrize("n,thr", [(0, 0.005), (1, 0.005), (1023, 0.005), (1025, 0.5),
                                   (300_000, 0.005), (2_000_000, 0.02), (5000, 0.999),
                                   (5000, 1e-6)])
def test_cull_low_opacity_bit_exact(n, thr):
    require_gpu()
    g = scenes.rng(n + 17)
    logit = g.normal(-4.0, 2.0, max(n, 1) + 64).astype(np.float32)
    want = oracle.low_opacity_keep(logit, n, thr)
    ctx = gs.default_context()
    lt = torch.from_numpy(logit).cuda()
    idx = torch.full((max(n, 1),), -1, dtype=torch.int32, device="cuda")
    m = gs.gs_cull_low_opacity(ctx, lt, n, thr, idx)
    assert m == len(want)
    np.testing.assert_array_equal(idx.cpu().numpy()[:m], want)


def test_cull_then_gather_compacts_a_gaussian_set():
    require_gpu()
    sc = scenes.make_scene(50_000, 6, -3.0, 3.0, -4.0, 0.5, 3)
    g = gs.Gaussians.from_scene(sc)
    ctx = gs.default_context()
    idx = torch.empty(g.n, dtype=torch.int32, device="cuda")
    m = gs.gs_cull_low_opacity(ctx, g.opacity, g.n, 0.3, idx)
    want = oracle.low_opacity_keep(sc["opacity"], sc["n"], 0.3)
    assert m == len(want) and 0 < m < g.n
    ld2 = scenes.round_up(m)
    for name in ("mean", "log_scale", "quat", "sh"):
        src = getattr(g, name)
        src2 = src.reshape(-1, g.ld)
        dst = torch.full((src2.shape[0], ld2), float("nan"), device="cuda")
        gs.gs_gather_planes(ctx, src2, idx, m, dst)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(dst.cpu().numpy()[:, :m],
                                      sc[name].reshape(-1, sc["ld"])[:, want])
