"""The allocation-free fused L1 forward (gs_render_fwd_l1_noalloc) against
gs_render_fwd_l1 with a caller workspace, through the C ABI: same kernels,
so every output is bit-identical.  Two calls in a row, the second smaller,
exercise the shared fixed scratch array that keeps the first call's
partials."""
import numpy as np
import pytest
import torch

from paper_2512_20943_amd import gs, scenes
from paper_2512_20943_amd.raster import Rasterizer
from tests.gpu_helpers import require_gpu

pytestmark = pytest.mark.gpu


def _case(n, n_views, W, H, seed):
    scene = scenes.make_scene(n, seed, -3.0, 3.0, -4.0, 0.5, 3)
    cams = gs.Cameras(scenes.arc_cameras(n_views, 5.0, W, H))
    g = gs.Gaussians.from_scene(scene)
    r = Rasterizer(capacity=1 << 20, tight_rect=True, tile_spans=True)
    proj = r.project(g, cams, own_buffers=True)
    lists = r.bin_sort(proj, cams, own_buffers=True)
    rng = np.random.default_rng(seed + 100)
    target = torch.from_numpy(rng.uniform(0, 1, (n_views, 3, H, W)).astype(np.float32)).cuda()
    return cams, proj, lists, target


def _run(fn, ctx, cams, proj, lists, target, ws=None):
    V, _, H, W = target.shape
    out = dict(image=torch.full_like(target, -7.0),
               final_T=torch.full((V, H, W), -7.0, device="cuda"),
               n_contrib=torch.full((V, H, W), -7, dtype=torch.int32, device="cuda"),
               grad=torch.full_like(target, -7.0),
               loss=torch.zeros(1, dtype=torch.float64, device="cuda"))
    args = (ctx, proj, lists, cams, (0.1, 0.2, 0.3), target, out["image"], out["final_T"],
            out["n_contrib"], out["grad"], out["loss"])
    if ws is None:
        fn(*args)
    else:
        fn(*args, ws)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def test_noalloc_fused_l1_forward_matches_workspace_call():
    require_gpu()
    ctx = gs.default_context()
    # first call: 6 views of 400x300 (25 x 19 tiles each); second: 2 views of
    # 200x150, fewer tiles, so stale partials of the first call sit beyond
    # the second call's range
    for n, V, W, H, seed in ((30_000, 6, 400, 300, 1), (8_000, 2, 200, 150, 2)):
        print(f"noalloc fused L1: n={n} views={V} {W}x{H}", flush=True)
        cams, proj, lists, target = _case(n, V, W, H, seed)
        assert lists.count > 0
        got = _run(gs.gs_render_fwd_l1_noalloc, ctx, cams, proj, lists, target)
        ws = torch.empty(gs.render_fwd_l1_workspace_size(V, W, H), dtype=torch.uint8,
                         device="cuda")
        ref = _run(gs.gs_render_fwd_l1, ctx, cams, proj, lists, target, ws)
        for k in ("image", "final_T", "n_contrib", "grad", "loss"):
            np.testing.assert_array_equal(got[k], ref[k], err_msg=k)
        assert ref["loss"][0] > 0
        assert (ref["n_contrib"] >= 0).all()


def test_noalloc_rejects_more_tiles_than_the_scratch_holds():
    require_gpu()
    ctx = gs.default_context()
    # 65 views of 1024x1024 = 65 * 4096 tiles > 2^18; the check comes before
    # anything is launched, so the buffers are never read
    V, W, H = 65, 1024, 1024
    cams = gs.Cameras(scenes.arc_cameras(V, 5.0, W, H))
    assert cams.n_segments() > gs.GS_NOALLOC_MAX_TILES
    proj = gs.Projected.empty(V, 64, 64)
    lists = gs.TileLists(64, cams.n_segments())
    t = torch.zeros(1, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    n_c = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(gs.GsError) as ei:
        gs.gs_render_fwd_l1_noalloc(ctx, proj, lists, cams, (0, 0, 0), t, None, t, n_c, t, loss)
    assert ei.value.code == gs.GS_ERR_INVALID_ARG
    assert "scratch" in str(ei.value)
