"""Seeded synthetic inputs: Gaussian scenes, cameras, frame deltas, masks.

This module is the only code shared by the HIP path and the FP64 oracle.  It
draws random numbers and lays them out; it holds none of the rasterizer's
arithmetic.  Every generator uses numpy's PCG64 with an explicit seed.

The paper's workload (multi-view captures of a moving performer, Sec. IV-A)
is not available; these scenes stand in for it with the shapes stated in
each function: Gaussian counts, SH degree, mean box, log-scale and opacity
distributions, camera rings, image sizes, and 548x548 delta images with one
texel per Gaussian (Eq. (3)).

Layouts (all planar FP32 with a plane stride ``ld`` rounded up to 64):
    scene: dict(n, deg, ld, mean (3,ld), log_scale (3,ld), quat (4,ld) w,x,y,z,
                opacity (ld,) logit, sh (K,3,ld)), K = (deg+1)^2
    cams:  dict(R (V,3,3) f64 world->camera, t (V,3) f64,
                f (V,4) f64 = fx, fy, cx, cy, wh (V,2) int32)
    delta: (8, gh, gw) FP32 channels dx, dy, dz, dqw, dqx, dqy, dqz, do
    mask:  (gh, gw) uint8, 1 = keep the texel's update
"""
from __future__ import annotations

import math

import numpy as np

# Degree-0 real SH basis value 1/(2 sqrt(pi)); the generator stores the DC
# coefficient so that the DC colour (basis value x coefficient + 0.5) is the
# drawn colour.
_Y00 = 0.28209479177387814


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def round_up(x: int, m: int = 64) -> int:
    return (x + m - 1) // m * m


def make_scene(n: int, seed: int, mean_lo: float = -1.0, mean_hi: float = 1.0,
               log_scale_mu: float = -4.0, log_scale_sd: float = 0.5, sh_degree: int = 0,
               sh_rest_sd: float = 0.1, opacity_sd: float = 1.0, ld: int | None = None) -> dict:
    """n Gaussians: means U[lo,hi]^3, log-scales N(mu, sd) per axis, unit
    quaternions (normalised 4-D normal draws), opacity logits N(0, sd), DC
    colour U[0,1] per channel, higher SH coefficients N(0, sh_rest_sd)."""
    g = rng(seed)
    ld = round_up(max(n, 1)) if ld is None else ld
    K = (sh_degree + 1) ** 2
    mean = np.zeros((3, ld), np.float32)
    log_scale = np.zeros((3, ld), np.float32)
    quat = np.zeros((4, ld), np.float32)
    opacity = np.zeros(ld, np.float32)
    sh = np.zeros((K, 3, ld), np.float32)
    mean[:, :n] = g.uniform(mean_lo, mean_hi, size=(3, n))
    log_scale[:, :n] = g.normal(log_scale_mu, log_scale_sd, size=(3, n))
    q = g.normal(size=(4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    quat[:, :n] = q
    quat[0, n:] = 1.0
    opacity[:n] = g.normal(0.0, opacity_sd, size=n)
    colour = g.uniform(0.0, 1.0, size=(3, n))
    sh[0, :, :n] = (colour - 0.5) / _Y00
    if K > 1:
        sh[1:, :, :n] = g.normal(0.0, sh_rest_sd, size=(K - 1, 3, n))
    return dict(n=n, deg=sh_degree, ld=ld, mean=mean, log_scale=log_scale, quat=quat,
                opacity=opacity, sh=sh)


def jitter_means(scene: dict, sd: float, seed: int) -> dict:
    """Copy of the scene with means + N(0, sd) (the 'perturbed copy' that
    renders the training targets)."""
    g = rng(seed)
    out = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in scene.items()}
    n = scene["n"]
    out["mean"][:, :n] += g.normal(0.0, sd, size=(3, n)).astype(np.float32)
    return out


def subset(scene: dict, n: int) -> dict:
    """First n Gaussians of a scene, re-strided."""
    ld = round_up(n)
    out = dict(n=n, deg=scene["deg"], ld=ld)
    for k in ("mean", "log_scale", "quat", "opacity", "sh"):
        a = scene[k]
        b = np.zeros(a.shape[:-1] + (ld,), np.float32)
        b[..., :n] = a[..., :n]
        out[k] = b
    out["quat"][0, n:] = 1.0
    return out


# ----------------------------------------------------------------------------
# cameras
# ----------------------------------------------------------------------------

def focal_for_fov(width: int, fov_x_deg: float = 60.0) -> float:
    return (width / 2.0) / math.tan(math.radians(fov_x_deg) / 2.0)


def look_at(eye, target, up, width: int, height: int, fov_x_deg: float = 60.0):
    """World->camera rotation and translation of a pinhole camera at ``eye``
    looking at ``target`` (OpenCV frame: x right, y down, z forward)."""
    eye = np.asarray(eye, np.float64)
    target = np.asarray(target, np.float64)
    up = np.asarray(up, np.float64)
    zc = target - eye
    zc /= np.linalg.norm(zc)
    xc = np.cross(zc, up)
    xc /= np.linalg.norm(xc)
    yc = np.cross(zc, xc)
    R = np.stack([xc, yc, zc])
    t = -R @ eye
    f = focal_for_fov(width, fov_x_deg)
    return R, t, np.array([f, f, width / 2.0, height / 2.0]), (width, height)


def stack_cams(items) -> dict:
    R = np.stack([it[0] for it in items]).astype(np.float64)
    t = np.stack([it[1] for it in items]).astype(np.float64)
    f = np.stack([it[2] for it in items]).astype(np.float64)
    wh = np.array([it[3] for it in items], np.int32)
    return dict(R=R, t=t, f=f, wh=wh)


def axis_camera(width: int, height: int, distance: float = 4.0, fov_x_deg: float = 60.0) -> dict:
    """Camera at distance ``distance`` on the -z axis looking at the origin
    with R = I: t = (0, 0, distance)."""
    f = focal_for_fov(width, fov_x_deg)
    return stack_cams([(np.eye(3), np.array([0.0, 0.0, distance]),
                        np.array([f, f, width / 2.0, height / 2.0]), (width, height))])


def arc_cameras(n_views: int, radius: float, width: int, height: int,
                azimuth_deg: float = 120.0, fov_x_deg: float = 60.0) -> dict:
    """n_views cameras evenly spaced on a horizontal arc of ``azimuth_deg``
    degrees at ``radius``, all looking at the origin, world up +y."""
    half = math.radians(azimuth_deg) / 2.0
    angs = np.linspace(-half, half, n_views) if n_views > 1 else np.array([0.0])
    items = []
    for a in angs:
        eye = radius * np.array([math.sin(a), 0.0, -math.cos(a)])
        items.append(look_at(eye, [0.0, 0.0, 0.0], [0.0, 1.0, 0.0], width, height, fov_x_deg))
    return stack_cams(items)


def sphere_camera(g: np.random.Generator, r_lo: float, r_hi: float, width: int, height: int,
                  fov_x_deg: float = 60.0):
    """Random viewpoint: direction uniform on the sphere, radius U[r_lo, r_hi],
    looking at the origin; world up +y, switched to +z near the poles."""
    d = g.normal(size=3)
    d /= np.linalg.norm(d)
    r = g.uniform(r_lo, r_hi)
    up = [0.0, 1.0, 0.0] if abs(d[1]) <= 0.99 else [0.0, 0.0, 1.0]
    return look_at(r * d, [0.0, 0.0, 0.0], up, width, height, fov_x_deg)


# ----------------------------------------------------------------------------
# frame updates (delta images and pruning masks)
# ----------------------------------------------------------------------------

def grid_side(n: int) -> int:
    """Smallest square texel grid holding n Gaussians (548 for 300,000)."""
    return int(math.ceil(math.sqrt(n)))


def make_delta(n: int, gw: int, gh: int, seed: int, mean_sd: float = 0.005,
               quat_sd: float = 0.005, opacity_sd: float = 0.01) -> np.ndarray:
    """(8, gh, gw) delta images: translation N(0, mean_sd), quaternion delta
    (1,0,0,0) + N(0, quat_sd), opacity-logit delta N(0, opacity_sd).  Padding
    texels hold the identity update."""
    g = rng(seed)
    d = np.zeros((8, gh * gw), np.float32)
    d[3, :] = 1.0
    z = g.standard_normal(size=(8, n), dtype=np.float32)
    d[0:3, :n] = z[0:3] * np.float32(mean_sd)
    d[3:7, :n] += z[3:7] * np.float32(quat_sd)
    d[7, :n] = z[7] * np.float32(opacity_sd)
    return d.reshape(8, gh, gw)


def prune_mask(delta: np.ndarray, n: int, level: float) -> np.ndarray:
    """Keep-mask that drops floor(level * n) updates with the smallest
    magnitude |(d_mu, d_q - identity, d_o)|_2 (ties: lower id dropped first);
    padding texels are 0."""
    _, gh, gw = delta.shape
    flat = delta.reshape(8, -1)[:, :n].astype(np.float64)
    dev = flat.copy()
    dev[3] -= 1.0
    mag = np.sqrt((dev ** 2).sum(axis=0))
    order = np.argsort(mag, kind="stable")  # equal magnitudes: lower id first
    drop = order[: int(math.floor(level * n))]
    m = np.zeros(gh * gw, np.uint8)
    m[:n] = 1
    m[drop] = 0
    return m.reshape(gh, gw)


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------

def workload_plain_10k(seed: int = 0):
    """10,000 Gaussians, means U[-1,1]^3, log-scales N(-4, 0.5), SH degree 0;
    one 128x128 camera at distance 4 with a 60-degree FOV; the target is the
    render of the same scene with means jittered by N(0, 0.01)."""
    scene = make_scene(10_000, seed, -1.0, 1.0, -4.0, 0.5, 0)
    cams = axis_camera(128, 128, 4.0)
    target_scene = jitter_means(scene, 0.01, seed + 1000)
    return scene, cams, target_scene


def workload_frame_300k(seed: int = 0, n: int = 300_000, n_views: int = 20,
                        width: int = 1352, height: int = 1014):
    """300,000 Gaussians, means U[-3,3]^3, SH degree 3 (DC colour U[0,1], rest
    N(0, 0.1)); n_views cameras on a 120-degree arc at radius 5."""
    scene = make_scene(n, seed, -3.0, 3.0, -4.0, 0.5, 3)
    cams = arc_cameras(n_views, 5.0, width, height)
    target_scene = jitter_means(scene, 0.01, seed + 1000)
    return scene, cams, target_scene


def workload_large_2m(seed: int = 0, n: int = 2_000_000, n_views: int = 8,
                      width: int = 1920, height: int = 1080):
    """2,000,000 Gaussians, means U[-6,6]^3, log-scales N(-4.5, 0.7), SH
    degree 3; 8 cameras on the same arc at radius 5 (inside the cloud)."""
    scene = make_scene(n, seed, -6.0, 6.0, -4.5, 0.7, 3)
    cams = arc_cameras(n_views, 5.0, width, height)
    target_scene = jitter_means(scene, 0.01, seed + 1000)
    return scene, cams, target_scene


def image_pair(n_views: int, height: int, width: int, seed: int, noise: float = 0.05):
    """Render-like (V, 3, H, W) FP32 image in [0, 1] (a few random low-frequency
    cosines per channel plus a few flat rectangles) and a target that differs
    by N(0, noise) and, in one rectangle, by a constant shift."""
    g = rng(seed)
    yy, xx = np.meshgrid(np.arange(height, dtype=np.float64), np.arange(width, dtype=np.float64),
                         indexing="ij")
    img = np.empty((n_views, 3, height, width), np.float64)
    for v in range(n_views):
        for c in range(3):
            f = 0.5 * np.ones_like(xx)
            for _ in range(4):
                kx, ky = g.uniform(0.0, 0.08, 2)
                f += g.uniform(0.05, 0.2) * np.cos(kx * xx + ky * yy + g.uniform(0, 2 * np.pi))
            img[v, c] = f
        for _ in range(3):
            x0, y0 = int(g.integers(0, width)), int(g.integers(0, height))
            img[v, :, y0:y0 + height // 6, x0:x0 + width // 6] = g.uniform(0, 1, (3, 1, 1))
    img = np.clip(img, 0.0, 1.0)
    tgt = img + g.normal(0.0, noise, img.shape)
    x0, y0 = int(g.integers(0, width)), int(g.integers(0, height))
    tgt[:, :, y0:y0 + height // 5, x0:x0 + width // 5] += 0.1
    return img.astype(np.float32), np.clip(tgt, 0.0, 1.0).astype(np.float32)
