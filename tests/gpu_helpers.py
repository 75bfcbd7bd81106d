"""Conversions between the HIP path's device buffers and the oracle's arrays,
and the tolerance checks the parity tests share."""
import numpy as np
import torch

from paper_2512_20943_amd import gs
from paper_2512_20943_amd.raster import Rasterizer

IMG_ATOL = 1e-4          # images and final transmittance, FP32 vs FP64
GRAD_REL = 1e-3          # parameter gradients, per-tensor relative L2
MEAN2D_ATOL = 1e-3       # screen means, px
REL = 1e-4               # conic, colour, opacity (relative, floor 1e-6)


def require_gpu():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    gs.load()


def projected_to_oracle(p: gs.Projected):
    n = p.n
    s = p.splat[:, :n].cpu().numpy().astype(np.float64)
    return dict(
        V=p.V, n=n, mean2d=s[..., 0:2], conic=s[..., 2:5], alpha_hat=s[..., 5], rgb=s[..., 6:9],
        depth=s[..., 9], detq=s[..., 10],
        rect=p.rect[:, :n].cpu().numpy(), tiles=p.tiles_touched[:, :n].cpu().numpy(),
        depth_bits=p.depth_bits[:, :n].cpu().numpy().view(np.uint32),
        flags=p.flags[:, :n].cpu().numpy())


def lists_to_numpy(L: gs.TileLists):
    M = L.count
    out = dict(count=M, vals=L.vals[:M].cpu().numpy().view(np.uint32),
               ranges=L.ranges[:L.n_segments].cpu().numpy().view(np.uint32))
    if L.keys is not None:
        out["keys"] = L.keys[:M].cpu().numpy().view(np.uint64)
    return out


def gpu_forward(scene, cams_np, bg=(0.0, 0.0, 0.0), with_keys=True, capacity=1 << 16,
                emission_bases=False, tight_rect=False, tile_spans=False):
    g = gs.Gaussians.from_scene(scene)
    cams = gs.Cameras(cams_np)
    r = Rasterizer(capacity=capacity, with_keys=with_keys, emission_bases=emission_bases,
                   tight_rect=tight_rect, tile_spans=tile_spans)
    out = r.forward(g, cams, bg)
    torch.cuda.synchronize()
    return g, cams, r, out


def assert_close_rel(got, ref, rel=REL, floor=1e-6, what=""):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    bad = np.abs(got - ref) > rel * np.abs(ref) + floor
    assert not bad.any(), (f"{what}: {bad.sum()} of {bad.size} outside rel {rel}; worst "
                           f"{np.abs(got - ref)[bad].max():.3e}")


def assert_grad_close(got, ref, what=""):
    got = np.asarray(got, np.float64).ravel()
    ref = np.asarray(ref, np.float64).ravel()
    nrm = np.linalg.norm(ref)
    if nrm == 0.0:
        assert np.abs(got).max() == 0.0, what
        return
    rel = np.linalg.norm(got - ref) / nrm
    assert rel <= GRAD_REL, f"{what}: relative L2 error {rel:.3e} > {GRAD_REL}"
    rms = nrm / np.sqrt(ref.size)
    bad = np.abs(got - ref) > GRAD_REL * np.abs(ref) + GRAD_REL * rms
    assert not bad.any(), (f"{what}: {bad.sum()} of {bad.size} elements outside tolerance; "
                           f"worst {np.abs(got - ref)[bad].max():.3e} (rms {rms:.3e})")
