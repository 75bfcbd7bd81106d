"""Conversions between the HIP path's device buffers and the oracle's arrays,
and the tolerance checks the parity tests share."""
import sys

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
        flags=p.flags[:, :n].cpu().numpy(),
        words=p.splat[:, :n].cpu().numpy().view(np.uint32).reshape(p.V, n, 16))


def span_rows(P):
    """Per-row tile columns (V, n, 4, 2) of span-mode records, absolute
    [first, end), empty rows (0, 0), from either side's projection: the
    oracle stores them as they are, the HIP record packs them relative to
    the rectangle's first column in word 15 (flag in bit 31 of word 13)."""
    if "spans" in P:
        sp = np.asarray(P["spans"], np.int64).copy()
        spanned = (np.asarray(P["flags"]) & 64) > 0
    else:
        w = P["words"]
        spanned = (w[..., 13] >> 31).astype(bool)
        x0 = P["rect"][..., 0].astype(np.int64)
        m = w[..., 15].astype(np.int64)
        sp = np.zeros(m.shape + (4, 2), np.int64)
        for r in range(4):
            a = (m >> (8 * r)) & 15
            b = (m >> (8 * r + 4)) & 15
            sp[..., r, 0] = np.where(b > a, x0 + a, 0)
            sp[..., r, 1] = np.where(b > a, x0 + b, 0)
    sp[~spanned] = 0
    return spanned, sp


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


# At a pixel whose skip/stop decision the oracle reports within the FP32
# error bound of its threshold, the two sides may composite one entry more or
# less; that entry's share of the pixel is bounded by (1/255 or alpha) * T,
# at most a few 1e-3.
NEAR_ATOL = 5e-3

# Cap on the fraction of a workload's pixels that the oracle reports near a
# threshold (those are held to NEAR_ATOL instead of IMG_ATOL).  The set is
# the oracle's alone -- it does not depend on the GPU -- so each cap sits just
# above the fraction the oracle reports for that workload and seed (in
# parentheses).  It grows with the depth complexity: every entry a pixel
# evaluates is one more chance to land within the margin of 1/255.
NEAR_FRAC_CAP = {
    "many_views_1100": 0.0015,   # 200 Gaussians, 1100 views of 16x16 (0.089 %)
    "plain_10k": 0.0025,         # seeds 0, 1 (0.201 %, 0.183 %)
    "frame_20k_4v": 0.0015,      # 20k of the frame distribution, 4 views 200x150 (0.089-0.103 %)
    "tiny": 0.0,                 # 500 Gaussians, 1x1 / 17x33 / 16x16 (0 %)
    "single_and_huge": 0.0,      # two hand-placed Gaussians, 96x80 (0 %)
    "frame_300k_view0": 0.015,   # 300k frame, view 0 at 1352x1014 (1.345 %)
    "large_2m_view0": 0.014,     # 2M scene, view 0 at 1920x1080 (1.253 %)
    "served_small": 0.010,       # 20k sequence, requests at 64x48..200x150 (0.10-0.98 %)
    "served_4k_2m": 0.014,       # 2M sequence, one 3840x2160 request (1.293 %)
}


def _near_checks(diff, near, max_frac, label):
    frac = float(near.mean()) if near.size else 0.0
    print(f"  [{label}] near-threshold pixels: {int(near.sum())} of {near.size} "
          f"({frac:.4%}, cap {max_frac:.4%})", flush=True)
    sys.stdout.flush()
    assert diff[near].max(initial=0.0) <= NEAR_ATOL, \
        "near-threshold pixel off by more than one entry"
    assert frac <= max_frac, f"{frac:.4%} pixels near a threshold (cap {max_frac:.4%})"


def compare_images(img_gpu, img_or, label, max_frac=None):
    """Images and final_T within IMG_ATOL and n_contrib equal away from the
    oracle's near-threshold pixels; those are held to NEAR_ATOL and their
    fraction to ``max_frac`` (default: the workload's NEAR_FRAC_CAP)."""
    if max_frac is None:
        max_frac = NEAR_FRAC_CAP[label]
    near = img_or["near_threshold"]
    keep = ~near
    im_g = img_gpu["image"].cpu().numpy()
    T_g = img_gpu["final_T"].cpu().numpy()
    n_g = img_gpu["n_contrib"].cpu().numpy()
    diff = np.abs(im_g - img_or["image"]).max(axis=1)
    err = diff[keep]
    assert err.max(initial=0.0) <= IMG_ATOL, f"image error {err.max():.3e}"
    errT = np.abs(T_g - img_or["final_T"])
    assert errT[keep].max(initial=0.0) <= IMG_ATOL, f"final_T error {errT[keep].max():.3e}"
    np.testing.assert_array_equal(n_g[keep], img_or["n_contrib"][keep])
    assert errT[near].max(initial=0.0) <= NEAR_ATOL
    _near_checks(diff, near, max_frac, label)
    return float(err.max(initial=0.0)), int(near.sum())


def compare_image_only(image, ref_image, near, label, max_frac=None):
    """A (3, H, W) image without its final_T and n_contrib (served requests):
    IMG_ATOL away from the near-threshold pixels, NEAR_ATOL and the fraction
    cap there."""
    if max_frac is None:
        max_frac = NEAR_FRAC_CAP[label]
    diff = np.abs(np.asarray(image, np.float64) - ref_image).max(axis=0)
    keep = ~near
    err = diff[keep].max(initial=0.0)
    assert err <= IMG_ATOL, f"[{label}] image error {err:.3e}"
    _near_checks(diff, near, max_frac, label)
    return float(err)
