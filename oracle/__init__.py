"""FP64 CPU oracle of the per-frame Gaussian-splatting rasterizer.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product path
(``paper_2512_20943_amd``) never imports it, and it never imports the product
package: the two share only the seeded input generators.

The arithmetic lives in ``gs_oracle.c`` (plain C99, FP64, ``-ffp-contract=off``,
OpenMP over tiles / Gaussians).  This module builds it with gcc and marshals
numpy arrays.  Each wrapper names the step of the forward / backward it
implements; the steps follow the paper's frame model (Eq. (2), (5), (12):
frame = anchor + accumulated delta; Eq. (3): one texel per Gaussian; Eq. (1):
L1 term) and the splatting rasterizer the paper cites in Sec. II, written out
from EWA splatting, real spherical harmonics and alpha compositing.

Scene dict (planar FP32, stride ``ld`` >= n):
    n, deg, ld, mean (3,ld), log_scale (3,ld), quat (4,ld) [w,x,y,z],
    opacity (ld,) logit, sh (K,3,ld) with K = (deg+1)^2.
Camera dict: R (V,3,3) f64 world->camera, t (V,3), f (V,4) = fx,fy,cx,cy,
    wh (V,2) int32 = width,height.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gs_oracle.c")
_LIB = os.path.join(_HERE, "libgs_oracle.so")
_lib = None

TILE = 16


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no FP contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = ctypes.CDLL(_LIB)
        _lib.or_count_instances.restype = ctypes.c_int64
        _lib.or_l1.restype = ctypes.c_double
        _lib.or_forward_loss.restype = ctypes.c_double
    return _lib


def _p(a):
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"], "oracle arrays must be C-contiguous"
    return a.ctypes.data_as(ctypes.c_void_p)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _cam_arrays(cams):
    R = _f64(np.asarray(cams["R"]).reshape(-1, 9))
    t = _f64(np.asarray(cams["t"]).reshape(-1, 3))
    f = _f64(np.asarray(cams["f"]).reshape(-1, 4))
    wh = np.ascontiguousarray(np.asarray(cams["wh"]).reshape(-1, 2), dtype=np.int32)
    return R, t, f, wh, R.shape[0]


def tiles_xy(w: int, h: int):
    return (w + TILE - 1) // TILE, (h + TILE - 1) // TILE


def segment_bases(cams):
    """First segment id of each view: views are laid out one after another,
    each with TX*TY tiles in row-major tile order."""
    wh = np.asarray(cams["wh"]).reshape(-1, 2)
    counts = [tiles_xy(int(w), int(h)) for w, h in wh]
    per = np.array([tx * ty for tx, ty in counts], dtype=np.int64)
    base = np.concatenate([[0], np.cumsum(per)[:-1]]).astype(np.int64)
    txv = np.array([tx for tx, _ in counts], dtype=np.int32)
    return base, txv, int(per.sum())


# --------------------------------------------------------------------------
# forward steps
# --------------------------------------------------------------------------

def apply(scene, delta, mask, gw, gh):
    """Step 1 (Eq. (2)/(5)/(12)): frame = anchor (+) masked delta texels.
    Returns a new scene dict whose mean/quat/opacity planes are the applied
    FP32 values; log_scale and sh are the anchor's."""
    lib = _load()
    n, ld = scene["n"], scene["ld"]
    mean_o = np.zeros_like(_f32(scene["mean"]))
    quat_o = np.zeros_like(_f32(scene["quat"]))
    opac_o = np.zeros_like(_f32(scene["opacity"]))
    d = _f32(delta).reshape(8, gh * gw)
    m = np.ascontiguousarray(mask, dtype=np.uint8).reshape(-1)
    lib.or_apply(ctypes.c_int(n), ctypes.c_int(ld), _p(_f32(scene["mean"])), _p(_f32(scene["quat"])),
                 _p(_f32(scene["opacity"])), _p(d), _p(m), ctypes.c_int(gw), ctypes.c_int(gh),
                 _p(mean_o), _p(quat_o), _p(opac_o))
    out = dict(scene)
    out.update(mean=mean_o, quat=quat_o, opacity=opac_o)
    return out


TILESETS = {"rect": 0, "tight": 1, "spans": 2}
SPAN_ROWS = 4
F_SPANS = 64


def project(scene, cams, tileset="rect"):
    """Steps 2-6: per (view, Gaussian) screen mean, conic, colour, opacity,
    depth, radius, tile rectangle and flags, all in FP64.  ``tileset``
    selects step 5b: "rect" keeps the step-5 rectangle, "tight" cuts it to
    the alpha >= 1/255 ellipse's bounding box, "spans" also keeps per-row
    column spans on small rectangles (``spans`` (V, n, 4, 2) absolute
    [first, end) columns, flag bit F_SPANS)."""
    lib = _load()
    n, ld, deg = scene["n"], scene["ld"], scene["deg"]
    R, t, f, wh, V = _cam_arrays(cams)
    out = dict(
        mean2d=np.zeros((V, n, 2)), conic=np.zeros((V, n, 3)), rgb=np.zeros((V, n, 3)),
        alpha_hat=np.zeros((V, n)), depth=np.zeros((V, n)),
        depth_bits=np.zeros((V, n), np.uint32), rect=np.zeros((V, n, 4), np.int32),
        tiles=np.zeros((V, n), np.int32), radius=np.zeros((V, n), np.int32),
        flags=np.zeros((V, n), np.uint8))
    lib.or_project(ctypes.c_int(n), ctypes.c_int(ld), ctypes.c_int(deg), _p(_f32(scene["mean"])),
                   _p(_f32(scene["log_scale"])), _p(_f32(scene["quat"])),
                   _p(_f32(scene["opacity"])), _p(_f32(scene["sh"])), ctypes.c_int(V), _p(R),
                   _p(t), _p(f), _p(wh), _p(out["mean2d"]), _p(out["conic"]), _p(out["rgb"]),
                   _p(out["alpha_hat"]), _p(out["depth"]), _p(out["depth_bits"]),
                   _p(out["rect"]), _p(out["tiles"]), _p(out["radius"]), _p(out["flags"]))
    out["spans"] = np.zeros((V, n, SPAN_ROWS, 2), np.int32)
    mode = TILESETS[tileset]
    if mode > 0:
        lib.or_tile_sets(ctypes.c_int(V), ctypes.c_int(n), _p(wh), _p(out["mean2d"]),
                         _p(out["conic"]), _p(out["alpha_hat"]), ctypes.c_int(mode),
                         _p(out["rect"]), _p(out["tiles"]), _p(out["spans"]), _p(out["flags"]))
    out["n"] = n
    out["V"] = V
    out["tileset"] = tileset
    return out


def bin_sort(proj, cams, depth_bits=None, rect=None, tiles=None):
    """Step 7: instances (Gaussian, tile) ordered by (segment, FP32 depth,
    Gaussian id); keys = (segment << 32) | depth bits.  Tile sets come from
    the projection (rectangles, or per-row spans where flagged).  The binning
    inputs may be overridden (to replay another implementation's
    rectangles; overriding uses plain rectangles)."""
    lib = _load()
    V, n = proj["V"], proj["n"]
    db = np.ascontiguousarray(proj["depth_bits"] if depth_bits is None else depth_bits,
                              dtype=np.uint32)
    rc = np.ascontiguousarray(proj["rect"] if rect is None else rect, dtype=np.int32)
    tl = np.ascontiguousarray(proj["tiles"] if tiles is None else tiles, dtype=np.int32)
    replay = rect is not None or tiles is not None
    spans = None if replay or "spans" not in proj else np.ascontiguousarray(proj["spans"],
                                                                          dtype=np.int32)
    flags = None if spans is None else np.ascontiguousarray(proj["flags"], dtype=np.uint8)
    base, txv, nseg = segment_bases(cams)
    M = int(lib.or_count_instances(ctypes.c_int(V), ctypes.c_int(n), _p(tl)))
    keys = np.zeros(max(M, 1), np.uint64)
    vals = np.zeros(max(M, 1), np.uint32)
    ranges = np.zeros((nseg, 2), np.uint32)
    lib.or_bin_sort(ctypes.c_int(V), ctypes.c_int(n), _p(db), _p(rc), _p(tl), _p(spans),
                    _p(flags), _p(base), _p(txv), ctypes.c_int64(nseg), _p(keys), _p(vals),
                    _p(ranges))
    return dict(keys=keys[:M], vals=vals[:M], ranges=ranges, count=M, seg_base=base,
                n_segments=nseg)


def render_fwd(proj, lists, cams, bg=None):
    """Step 8: per-pixel front-to-back compositing over each tile's list.
    Returns image (V,3,H,W), final_T (V,H,W), n_contrib (V,H,W),
    near_threshold (V,H,W) marking pixels where a decision sits within a
    small relative margin of a threshold, usage (n,) = number of (view,
    pixel) pairs compositing each Gaussian (the usage frequency the paper
    prunes by, Sec. III-C), and near_involved (n,) = near-threshold pixels
    whose list holds each Gaussian."""
    lib = _load()
    V, n = proj["V"], proj["n"]
    R, t, f, wh, _ = _cam_arrays(cams)
    W, H = int(wh[0, 0]), int(wh[0, 1])
    assert (wh[:, 0] == W).all() and (wh[:, 1] == H).all(), "views must share W, H"
    bgv = _f64(np.zeros((V, 3)) if bg is None else np.broadcast_to(np.asarray(bg, np.float64), (V, 3)))
    image = np.zeros((V, 3, H, W))
    T = np.zeros((V, H, W))
    nc = np.zeros((V, H, W), np.int32)
    near = np.zeros((V, H, W), np.uint8)
    usage = np.zeros(max(n, 1), np.int64)
    near_inv = np.zeros(max(n, 1), np.int64)
    vals = np.ascontiguousarray(lists["vals"], dtype=np.uint32)
    if vals.size == 0:
        vals = np.zeros(1, np.uint32)
    lib.or_render_fwd(ctypes.c_int(V), ctypes.c_int(n), _p(_f64(proj["mean2d"])),
                      _p(_f64(proj["conic"])), _p(_f64(proj["rgb"])), _p(_f64(proj["alpha_hat"])),
                      _p(np.ascontiguousarray(lists["seg_base"], np.int64)), _p(wh), _p(vals),
                      _p(np.ascontiguousarray(lists["ranges"], np.uint32)), _p(bgv), _p(image),
                      _p(T), _p(nc), _p(near), _p(usage), _p(near_inv))
    return dict(image=image, final_T=T, n_contrib=nc, near_threshold=near.astype(bool),
                usage=usage[:n], near_involved=near_inv[:n])


def render_brute(proj, cams, view=0, bg=None):
    """Plain definition of one view's image: every pixel composites all
    visible Gaussians whose tile set holds its tile, ordered by (FP32 depth,
    id), with no binning or sorting machinery."""
    lib = _load()
    n = proj["n"]
    R, t, f, wh, _ = _cam_arrays(cams)
    W, H = int(wh[view, 0]), int(wh[view, 1])
    bgv = _f64(np.zeros(3) if bg is None else bg)
    image = np.zeros((3, H, W))
    T = np.zeros((H, W))
    nc = np.zeros((H, W), np.int32)
    lib.or_render_brute(ctypes.c_int(n), _p(_f64(proj["mean2d"][view])),
                        _p(_f64(proj["conic"][view])), _p(_f64(proj["rgb"][view])),
                        _p(_f64(proj["alpha_hat"][view])),
                        _p(np.ascontiguousarray(proj["depth_bits"][view], np.uint32)),
                        _p(np.ascontiguousarray(proj["rect"][view], np.int32)),
                        _p(np.ascontiguousarray(proj["tiles"][view], np.int32)),
                        _p(np.ascontiguousarray(proj["spans"][view], np.int32)
                           if "spans" in proj else None),
                        _p(np.ascontiguousarray(proj["flags"][view], np.uint8)), ctypes.c_int(W),
                        ctypes.c_int(H), _p(bgv), _p(image), _p(T), _p(nc))
    return dict(image=image, final_T=T, n_contrib=nc)


def l1(image, target):
    """Step 9 (Eq. (1), L1 term): mean |I - I*| and sign(I - I*)/count."""
    lib = _load()
    img = _f64(image).reshape(-1)
    tgt = _f64(target).reshape(-1)
    grad = np.zeros_like(img)
    loss = lib.or_l1(ctypes.c_int64(img.size), _p(img), _p(tgt), _p(grad))
    return float(loss), grad.reshape(np.shape(image))


def l1_dssim(image, target, lam=0.2, with_map=False):
    """Eq. (1): (1 - lambda) L1 + lambda (1 - SSIM) over (V, 3, H, W) images
    (11x11 Gaussian window, sigma 1.5, zero padding, C1 = 0.01^2,
    C2 = 0.03^2) and its gradient w.r.t. the image."""
    lib = _load()
    lib.or_l1_dssim.restype = ctypes.c_double
    img = _f64(image)
    tgt = _f64(target)
    H, W = img.shape[-2], img.shape[-1]
    planes = int(img.size // (H * W))
    grad = np.zeros_like(img)
    smap = np.zeros_like(img) if with_map else None
    loss = lib.or_l1_dssim(ctypes.c_int(planes), ctypes.c_int(H), ctypes.c_int(W), _p(img),
                           _p(tgt), ctypes.c_double(lam), _p(grad), _p(smap))
    return (float(loss), grad, smap) if with_map else (float(loss), grad)


def ssim_window():
    lib = _load()
    w = np.zeros(11)
    lib.or_ssim_window(_p(w))
    return w


# --------------------------------------------------------------------------
# backward steps
# --------------------------------------------------------------------------

def render_bwd(proj, lists, cams, dL_dimage, bg=None):
    """Backward of step 8: per (view, Gaussian) gradients (V, n, 9) w.r.t.
    mean2d (0,1), conic A,B,C (2,3,4), opacity alpha_hat (5), rgb (6,7,8)."""
    lib = _load()
    V, n = proj["V"], proj["n"]
    R, t, f, wh, _ = _cam_arrays(cams)
    bgv = _f64(np.zeros((V, 3)) if bg is None else np.broadcast_to(np.asarray(bg, np.float64), (V, 3)))
    g2d = np.zeros((V, n, 9))
    vals = np.ascontiguousarray(lists["vals"], dtype=np.uint32)
    if vals.size == 0:
        vals = np.zeros(1, np.uint32)
    lib.or_render_bwd(ctypes.c_int(V), ctypes.c_int(n), _p(_f64(proj["mean2d"])),
                      _p(_f64(proj["conic"])), _p(_f64(proj["rgb"])), _p(_f64(proj["alpha_hat"])),
                      _p(np.ascontiguousarray(lists["seg_base"], np.int64)), _p(wh), _p(vals),
                      _p(np.ascontiguousarray(lists["ranges"], np.uint32)), _p(bgv),
                      _p(_f64(dL_dimage)), _p(g2d))
    return g2d


def project_bwd(scene, cams, g2d):
    """Backward of steps 2-6: parameter gradients summed over views."""
    lib = _load()
    n, ld, deg = scene["n"], scene["ld"], scene["deg"]
    K = (deg + 1) ** 2
    R, t, f, wh, V = _cam_arrays(cams)
    out = dict(mean=np.zeros((3, ld)), log_scale=np.zeros((3, ld)), quat=np.zeros((4, ld)),
               opacity=np.zeros(ld), sh=np.zeros((K, 3, ld)))
    lib.or_project_bwd(ctypes.c_int(n), ctypes.c_int(ld), ctypes.c_int(deg),
                       _p(_f32(scene["mean"])), _p(_f32(scene["log_scale"])),
                       _p(_f32(scene["quat"])), _p(_f32(scene["opacity"])), _p(_f32(scene["sh"])),
                       ctypes.c_int(V), _p(R), _p(t), _p(f), _p(wh), _p(_f64(g2d)),
                       _p(out["mean"]), _p(out["log_scale"]), _p(out["quat"]), _p(out["opacity"]),
                       _p(out["sh"]))
    return out


def apply_bwd(anchor, mask, gw, gh, grads):
    """Backward of step 1 to the (8, gh, gw) delta images."""
    lib = _load()
    n, ld = anchor["n"], anchor["ld"]
    out = np.zeros((8, gh, gw))
    m = np.ascontiguousarray(mask, dtype=np.uint8).reshape(-1)
    lib.or_apply_bwd(ctypes.c_int(n), ctypes.c_int(ld), _p(_f32(anchor["quat"])), _p(m),
                     ctypes.c_int(gw), ctypes.c_int(gh), _p(_f64(grads["mean"])),
                     _p(_f64(grads["quat"])), _p(_f64(grads["opacity"])), _p(out))
    return out


def adam(theta, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """Adam (Kingma & Ba 2015, Alg. 1), bias-corrected; returns new copies."""
    lib = _load()
    th = _f64(theta).reshape(-1).copy()
    mm = _f64(m).reshape(-1).copy()
    vv = _f64(v).reshape(-1).copy()
    g = _f64(grad).reshape(-1)
    lib.or_adam(ctypes.c_int64(th.size), _p(th), _p(g), _p(mm), _p(vv), ctypes.c_int(t),
                ctypes.c_double(lr), ctypes.c_double(beta1), ctypes.c_double(beta2),
                ctypes.c_double(eps))
    shp = np.shape(theta)
    return th.reshape(shp), mm.reshape(shp), vv.reshape(shp)


# --------------------------------------------------------------------------
# temporal and keyframe terms (Sec. III-B), plain definitions in FP64
# --------------------------------------------------------------------------

# The delta images hold the update itself: translation, the rotation
# quaternion dq applied as dq (x) q, and the opacity-logit increment.  "No
# motion" is therefore (0, 0, 0, 1, 0, 0, 0, 0), and the temporal term
# measures the distance of every delta from it.
IDENTITY_UPDATE = np.array([0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 0.0])


def temporal_l1(delta, n, weight):
    """Eq. (6)/(7): weight * sum over texels i < n and the 8 channels of
    |delta - identity update|, and its gradient weight * sign(.) (sign(0) = 0;
    padding texels i >= n carry neither loss nor gradient)."""
    d = _f64(delta).reshape(8, -1)
    r = d[:, :n] - IDENTITY_UPDATE[:, None]
    loss = weight * np.abs(r).sum()
    grad = np.zeros_like(d)
    grad[:, :n] = weight * np.sign(r)
    return float(loss), grad.reshape(np.shape(delta))


def keyframe_temporal_l1(x, x_prev, bound, weight):
    """Eq. (9) with the weight of Eq. (10): weight * sum over parameter rows
    and the first ``bound`` columns (the Gaussians carried over from the
    previous frame) of |x - x_prev|; gradient w.r.t. x."""
    a = _f64(x)
    b = _f64(x_prev)
    r = a[..., :bound] - b[..., :bound]
    grad = np.zeros_like(a)
    grad[..., :bound] = weight * np.sign(r)
    return float(weight * np.abs(r).sum()), grad


def densify_stats(flags, g2d):
    """Densification statistics for keyframe reconstruction (Sec. III-B): per
    Gaussian, the sum over the views where it is visible (flag 32) of the
    Euclidean norm of dL/d(screen mean) in pixels, and that view count."""
    vis = (np.asarray(flags) & 32) != 0
    g = np.asarray(g2d, np.float64)
    norm = np.sqrt(g[..., 0] ** 2 + g[..., 1] ** 2)
    return (np.where(vis, norm, 0.0).sum(axis=0), vis.sum(axis=0).astype(np.int64))


def low_opacity_keep(opacity_logit, n, min_opacity):
    """Indices (ascending) of the Gaussians i < n kept by low-opacity culling:
    sigmoid(logit) >= min_opacity, decided as logit >= log(m / (1 - m)) in
    FP64 from the FP32 logit."""
    x = np.asarray(opacity_logit, np.float32)[:n].astype(np.float64)
    t = np.log(min_opacity / (1.0 - min_opacity))
    return np.nonzero(x >= t)[0].astype(np.int64)


# --------------------------------------------------------------------------
# residual bookkeeping and quantised delta planes (Sec. III-C, Eq. (11)/(12))
# --------------------------------------------------------------------------
#
# Stored planes are FP32, and each step below is one IEEE operation per
# element (subtract, add, divide, multiply), so it is computed here in FP32:
# that fixes the rounding the transmitted and reconstructed planes carry.

def residual_delta(D_t, Dp_prev, mask, n):
    """Eq. (11): the update sent for frame t is the pruning mask applied to
    the residual between the true accumulated delta D_t and the accumulated
    delta already sent, D'_(t-1).  Returns d'_t (8, gh, gw) FP32 (zero at
    pruned and padding texels) and the per-channel max |d'_t| over i < n."""
    D = np.asarray(D_t, np.float32).reshape(8, -1)
    P = np.asarray(Dp_prev, np.float32).reshape(8, -1)
    m = np.asarray(mask, np.uint8).reshape(-1)
    d = np.zeros_like(D)
    keep = np.zeros(D.shape[1], bool)
    keep[:n] = m[:n] != 0
    d[:, keep] = D[:, keep] - P[:, keep]
    absmax = np.abs(d[:, :n]).max(axis=1) if n > 0 else np.zeros(8, np.float32)
    return d.reshape(np.shape(D_t)), absmax.astype(np.float32)


def quantize_delta(d, absmax, bits):
    """Symmetric per-channel quantisation of an update to signed ``bits``-bit
    codes: scale = absmax / (2^(bits-1) - 1) (0 when absmax is 0), code =
    round-half-even(d / scale) clamped to +-(2^(bits-1) - 1) (0 when the scale
    is 0).  Zero updates stay exactly zero."""
    qmax = np.float32(2 ** (bits - 1) - 1)
    a = np.asarray(absmax, np.float32)
    scale = np.where(a > 0, a / qmax, np.float32(0)).astype(np.float32)
    x = np.asarray(d, np.float32).reshape(8, -1)
    with np.errstate(divide="ignore", invalid="ignore"):
        q = np.where(scale[:, None] > 0, np.rint(x / scale[:, None]), np.float32(0))
    q = np.clip(q, -qmax, qmax).astype(np.int16 if bits == 16 else np.int8)
    return q.reshape(np.shape(d)), scale


def dequantize_delta(q, scale):
    s = np.asarray(scale, np.float32)
    x = np.asarray(q).reshape(8, -1).astype(np.float32)
    return (x * s[:, None]).astype(np.float32).reshape(np.shape(q))


def accumulate_sent(Dp_prev, d_sent):
    """Eq. (12): D'_t = D'_(t-1) + d'_t (FP32)."""
    return (np.asarray(Dp_prev, np.float32) + np.asarray(d_sent, np.float32)).astype(np.float32)


# --------------------------------------------------------------------------
# usage-frequency pruning and pruning-level selection (Sec. III-C, Alg. 1)
# --------------------------------------------------------------------------

def usage_keep_mask(usage, n, gw, gh, level):
    """p(.) of Sec. III-C: keep every update except those of the
    floor(level * n) least used Gaussians (usage = composited (view, pixel)
    pairs); among equal usage the lower id is dropped first.  Returns the
    (gh, gw) uint8 mask, 1 = keep, padding texels 0.  level * n is taken
    within 1e-9 of an integer as that integer (levels are decimal steps)."""
    drop = int(np.floor(level * n + 1e-9))
    ranked = sorted(range(n), key=lambda i: (int(usage[i]), i))
    m = np.zeros(gh * gw, np.uint8)
    m[:n] = 1
    for i in ranked[:drop]:
        m[i] = 0
    return m.reshape(gh, gw)


def select_level(space, beta, bandwidth, rate):
    """Alg. 1: ``space`` lists (quality, size) per pruning level, least
    pruned first.  Walk the levels from the second on, comparing each
    quality drop (quality of the level minus that of the level before) with
    the drop before it, the first comparison being the second level's drop
    with itself; the first level whose drop exceeds beta times the previous
    drop is the cliff, and the levels before it are the candidates.  The
    result is the first candidate (least pruned) whose size is at most
    B / R; if none is, the cliff level.
    Readings where the algorithm is silent: a previous drop of exactly 0
    makes a level a cliff when its own drop is negative (a loss after a
    lossless step); with no cliff and no fitting candidate the most pruned
    level is returned."""
    budget = bandwidth / rate
    candidates = [0]
    cliff = None
    previous = space[1][0] - space[0][0] if len(space) > 1 else 0.0
    for i in range(1, len(space)):
        drop = space[i][0] - space[i - 1][0]
        if previous == 0.0:
            is_cliff = drop < 0.0
        else:
            is_cliff = drop / previous > beta
        if is_cliff:
            cliff = i
            break
        candidates.append(i)
        previous = drop
    for i in candidates:
        if space[i][1] <= budget:
            return i
    return cliff if cliff is not None else len(space) - 1


def psnr(image, reference):
    """Mean over views of the PSNR (data range 1) of (V, 3, H, W) images."""
    a = np.asarray(image, np.float64)
    b = np.asarray(reference, np.float64)
    mse = ((a - b) ** 2).reshape(a.shape[0], -1).mean(axis=1)
    return float(np.mean(-10.0 * np.log10(mse)))


# --------------------------------------------------------------------------
# compositions used by tests
# --------------------------------------------------------------------------

def forward(scene, cams, bg=None, tileset="rect"):
    """Steps 2-8 for a scene: projection, lists and images."""
    proj = project(scene, cams, tileset)
    lists = bin_sort(proj, cams)
    img = render_fwd(proj, lists, cams, bg)
    return proj, lists, img


def backward(scene, cams, proj, lists, dL_dimage, bg=None):
    """Analytic gradient of the forward: returns (g2d, parameter grads)."""
    g2d = render_bwd(proj, lists, cams, dL_dimage, bg)
    return g2d, project_bwd(scene, cams, g2d)


def forward_loss(scene, cams, target, bg=None, overrides=None):
    """Whole forward to the L1 loss in FP64 and a structure signature.
    ``overrides`` maps plane names to FP64 arrays used instead of the FP32
    planes (finite-difference steps are not rounded)."""
    lib = _load()
    n, ld, deg = scene["n"], scene["ld"], scene["deg"]
    R, t, f, wh, V = _cam_arrays(cams)
    ov = overrides or {}
    bgv = _f64(np.zeros((V, 3)) if bg is None else np.broadcast_to(np.asarray(bg, np.float64), (V, 3)))
    sig = ctypes.c_uint64(0)
    get = lambda k: _f64(ov[k]) if k in ov else None  # noqa: E731
    loss = lib.or_forward_loss(
        ctypes.c_int(n), ctypes.c_int(ld), ctypes.c_int(deg), _p(_f32(scene["mean"])),
        _p(_f32(scene["log_scale"])), _p(_f32(scene["quat"])), _p(_f32(scene["opacity"])),
        _p(_f32(scene["sh"])), _p(get("mean")), _p(get("log_scale")), _p(get("quat")),
        _p(get("opacity")), _p(get("sh")), ctypes.c_int(V), _p(R), _p(t), _p(f), _p(wh), _p(bgv),
        _p(_f64(target)), ctypes.byref(sig))
    return float(loss), int(sig.value)


def quat_to_rot(q):
    lib = _load()
    R = np.zeros(9)
    lib.or_quat_to_rot(_p(_f64(q)), _p(R))
    return R.reshape(3, 3)


def quat_mul(a, b):
    lib = _load()
    out = np.zeros(4)
    lib.or_quat_mul(_p(_f64(a)), _p(_f64(b)), _p(out))
    return out


def sh_basis(deg, d):
    lib = _load()
    Y = np.zeros(16)
    lib.or_sh_basis(ctypes.c_int(deg), _p(_f64(d)), _p(Y))
    return Y[: (deg + 1) ** 2]
