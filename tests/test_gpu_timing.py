"""Stage timing (gs_set_timing, gs_set_timing_mask): with every stage on, each
stage a forward + backward runs reports launches and a positive time; with a
mask, only the named stages are bracketed and the rest report nothing; the
images are the same whichever stages are timed."""
import numpy as np
import pytest
import torch

from paper_2512_20943_amd import gs, scenes
from paper_2512_20943_amd.raster import Rasterizer
from tests.gpu_helpers import require_gpu

pytestmark = pytest.mark.gpu


def test_timing_mask_brackets_only_the_named_stages():
    require_gpu()
    print("timing mask, 5k x 2 views 96x64", flush=True)
    scene = scenes.make_scene(5_000, 1, -3.0, 3.0, -4.0, 0.5, 3)
    cams = scenes.arc_cameras(2, 5.0, 96, 64)
    g = gs.Gaussians.from_scene(scene)
    gc = gs.Cameras(cams)
    ctx = gs.Context(torch.cuda.current_device())
    r = Rasterizer(ctx=ctx, capacity=1 << 18)
    dimg = torch.from_numpy(
        np.random.default_rng(2).uniform(-1, 1, (2, 3, 64, 96)).astype(np.float32)).cuda()

    def run():
        out = r.forward(g, gc)
        grad = gs.Gaussians.zeros_like(g)
        r.backward(g, gc, out, dimg, grad)
        torch.cuda.synchronize()
        return out["image"].clone(), grad.planes()[0].clone()

    base = run()
    ctx.set_timing(True)
    ctx.collect_timing()
    full = run()
    t_all = ctx.collect_timing()
    ran = {k for k, (ms, n) in t_all.items() if n > 0}
    assert {"project", "depth_sort", "segment_sort", "render_fwd", "render_bwd"} <= ran, ran
    assert all(t_all[k][0] >= 0 for k in ran)
    assert t_all["render_fwd"][0] > 0 and t_all["render_bwd"][0] > 0

    ctx.set_timing_stages(["render_fwd", "render_bwd"])
    masked = run()
    t_m = ctx.collect_timing()
    assert {k for k, (ms, n) in t_m.items() if n > 0} == {"render_fwd", "render_bwd"}
    assert t_m["render_fwd"][1] == t_all["render_fwd"][1]
    assert t_m["render_bwd"][1] == t_all["render_bwd"][1]

    ctx.set_timing_stages([])
    off = run()
    assert all(n == 0 for _, n in ctx.collect_timing().values())
    with pytest.raises(ValueError):
        ctx.set_timing_stages(["no_such_stage"])
    ctx.set_timing(False)
    for a, b in zip(base, full):
        assert torch.equal(a, b)
    for res in (masked, off):
        for a, b in zip(base, res):
            assert torch.equal(a, b)
