"""Usage-frequency counts from the forward render and the pruning-level sweep
(Sec. III-C, Alg. 1) on the GPU, against the oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_2512_20943_amd import gs, prune, scenes
from tests.gpu_helpers import gpu_forward, require_gpu

pytestmark = pytest.mark.gpu


def _gpu_usage(scene, cams):
    g = gs.Gaussians.from_scene(scene)
    gc = gs.Cameras(cams)
    from paper_2512_20943_amd.raster import Rasterizer
    r = Rasterizer(capacity=1 << 20)
    u = torch.zeros(g.ld, dtype=torch.int32, device="cuda")
    r.forward(g, gc, usage=u)
    torch.cuda.synchronize()
    return u.cpu().numpy().view(np.uint32)[: scene["n"]].astype(np.int64)


@pytest.mark.parametrize("which", ["plain_10k", "frame_20k_4v"])
def test_usage_counts_match_oracle(which):
    require_gpu()
    if which == "plain_10k":
        scene, cams, _ = scenes.workload_plain_10k(0)
    else:
        scene = scenes.make_scene(20_000, 1, -3.0, 3.0, -4.0, 0.5, 3)
        cams = scenes.arc_cameras(4, 5.0, 200, 150)
    got = _gpu_usage(scene, cams)
    _, _, img = oracle.forward(scene, cams)
    ref, slack = img["usage"], img["near_involved"]
    assert ref.sum() > 0
    diff = np.abs(got - ref)
    assert np.all(diff <= slack), f"{int((diff > slack).sum())} Gaussians differ beyond the near-threshold slack"
    exact = slack == 0
    np.testing.assert_array_equal(got[exact], ref[exact])


def test_pruning_sweep_matches_oracle():
    """Sweep of 11 usage-pruned levels of a frame: usage, PSNR against the
    frame's reference views (renders of a jittered copy, each side its own)
    and sizes against the oracle, and the level the sweep selects equals the
    oracle's Alg. 1 on the oracle's own quality/size table."""
    require_gpu()
    n = 20_000
    scene = scenes.make_scene(n, 5, -3.0, 3.0, -4.0, 0.5, 2)
    target_scene = scenes.jitter_means(scene, 0.01, 1005)
    gw = gh = scenes.grid_side(n)
    d = scenes.make_delta(n, gw, gh, 6, 0.02, 0.02, 0.3)
    cams = scenes.arc_cameras(2, 5.0, 160, 120)
    anchor = gs.Gaussians.from_scene(scene)
    gc = gs.Cameras(cams)
    from paper_2512_20943_amd.raster import Rasterizer
    ref_gpu = Rasterizer(capacity=1 << 20).forward(gs.Gaussians.from_scene(target_scene),
                                                    gc)["image"].clone()
    sweep = prune.PruningSweep(anchor, torch.from_numpy(d).cuda(), gw, gh, gc)
    budget = 30.0 * 0.5 * n * prune.BYTES_PER_UPDATE
    res = sweep.run(ref_gpu, beta=2.0, bandwidth=budget, rate=30.0)
    # oracle: its own usage, ranking rule, renders, reference and Alg. 1
    full = oracle.apply(scene, d, np.ones((gh, gw), np.uint8), gw, gh)
    _, _, fimg = oracle.forward(full, cams)
    usage = fimg["usage"]
    assert np.all(np.abs(res["usage"] - usage) <= fimg["near_involved"])
    _, _, ref_or = oracle.forward(target_scene, cams)
    psnr, sizes = [], []
    for lv in res["levels"]:
        m = oracle.usage_keep_mask(usage, n, gw, gh, lv)
        _, _, img = oracle.forward(oracle.apply(scene, d, m, gw, gh), cams)
        psnr.append(oracle.psnr(img["image"], ref_or["image"]))
        sizes.append(int(m.sum()) * prune.BYTES_PER_UPDATE)
    np.testing.assert_array_equal(res["size"], sizes)
    # PSNR of FP32 renders vs FP64 renders
    np.testing.assert_allclose(res["psnr"], psnr, atol=0.02)
    space = list(zip(psnr, sizes))
    assert res["selected"] == oracle.select_level(space, 2.0, budget, 30.0)
