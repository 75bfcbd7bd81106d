"""Pins of the oracle's tile rectangles (forward step 5) and of the narrower
tile sets of step 5b (opacity-aware rectangles, per-row spans), against
hand-derived values and brute force.  CPU only.

Step 5b may drop a tile from a Gaussian's set only where no pixel of that
tile reaches alpha >= 1/255, because compositing skips every such pair: the
brute-force checks below evaluate alpha at every pixel of the rectangle and
require each pixel at or above 1/255 to lie in a kept tile, require every
kept span end to come within the stated slack of the widened ellipse, and
require the images to be identical under all three tile sets.
"""
import json
import math
import os

import numpy as np
import pytest

from paper_2512_20943_amd import scenes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "tile_rectangles.json")


def _camera(W, H, f=64.0, z=4.0):
    return dict(R=np.eye(3)[None].copy(), t=np.array([[0.0, 0.0, z]]),
                f=np.array([[f, f, W / 2.0, H / 2.0]]), wh=np.array([[W, H]], np.int32))


def _one(sigma, X, logit):
    ld = 64
    s = dict(n=1, deg=0, ld=ld, mean=np.zeros((3, ld), np.float32),
             log_scale=np.zeros((3, ld), np.float32), quat=np.zeros((4, ld), np.float32),
             opacity=np.zeros(ld, np.float32), sh=np.zeros((1, 3, ld), np.float32))
    s["quat"][0, :] = 1.0
    s["mean"][0, 0] = X
    s["log_scale"][:, 0] = math.log(sigma)
    s["opacity"][0] = logit
    return s


def test_golden_rectangles(oracle_mod):
    gold = json.load(open(GOLDEN))
    for case in gold["cases"]:
        sc = _one(case["sigma"], case["X"], case["logit"])
        P = oracle_mod.project(sc, _camera(case["W"], case["H"]))
        assert int(P["radius"][0, 0]) == case["radius"], case["name"]
        assert list(P["rect"][0, 0]) == case["rect"], case["name"]
        assert int(P["tiles"][0, 0]) == case["tiles"], case["name"]


def test_golden_opacity_aware_rectangles(oracle_mod):
    gold = json.load(open(GOLDEN))
    for case in gold["tight"]:
        sc = _one(case["sigma"], case["X"], case["logit"])
        cam = _camera(case["W"], case["H"])
        full = oracle_mod.project(sc, cam)
        assert list(full["rect"][0, 0]) == case["rect_full"], case["name"]
        for mode in ("tight", "spans"):
            P = oracle_mod.project(sc, cam, mode)
            assert list(P["rect"][0, 0]) == case["rect"], (case["name"], mode)
            assert int(P["tiles"][0, 0]) == case["tiles"], (case["name"], mode)


def _workloads():
    """Small scenes with the distributions of the benchmark frames: many
    faint and many anisotropic Gaussians, ragged image sizes."""
    a = scenes.make_scene(1500, 41, -3.0, 3.0, -4.0, 0.5, 1)
    b = scenes.make_scene(400, 42, -1.0, 1.0, -2.8, 0.8, 0)
    b["opacity"][:400] = np.random.default_rng(5).normal(-2.0, 2.5, 400).astype(np.float32)
    return [(a, scenes.arc_cameras(3, 5.0, 120, 90)), (b, scenes.arc_cameras(2, 3.0, 72, 56))]


def _alpha_pixels(P, v, i, W, H):
    """Every pixel (x, y) of Gaussian i's step-5 rectangle in view v, with its
    FP64 alpha before the 0.99 cap (alpha_hat exp(power))."""
    x0, y0, x1, y1 = P["rect"][v, i]
    xs = np.arange(16 * x0, min(16 * x1, W))
    ys = np.arange(16 * y0, min(16 * y1, H))
    X, Y = np.meshgrid(xs, ys)
    dx = P["mean2d"][v, i, 0] - X
    dy = P["mean2d"][v, i, 1] - Y
    A, B, C = P["conic"][v, i]
    power = -0.5 * (A * dx * dx + C * dy * dy) - B * dx * dy
    return X, Y, P["alpha_hat"][v, i] * np.exp(power)


def _members(P, v, i):
    """The set of (tx, ty) tiles in record (v, i)'s tile set."""
    if P["tiles"][v, i] <= 0:
        return set()
    x0, y0, x1, y1 = P["rect"][v, i]
    out = set()
    for ty in range(y0, y1):
        if P["flags"][v, i] & oracle_flag_spans():
            a, b = P["spans"][v, i, ty - y0]
        else:
            a, b = x0, x1
        out.update((tx, ty) for tx in range(a, b))
    return out


def oracle_flag_spans():
    import oracle
    return oracle.F_SPANS


@pytest.mark.parametrize("mode", ["tight", "spans"])
def test_every_pixel_reaching_1_over_255_is_in_a_kept_tile(oracle_mod, mode):
    for sc, cams in _workloads():
        full = oracle_mod.project(sc, cams)
        P = oracle_mod.project(sc, cams, mode)
        checked = 0
        for v in range(full["V"]):
            W, H = (int(x) for x in cams["wh"][v])
            for i in range(sc["n"]):
                if full["tiles"][v, i] <= 0:
                    assert P["tiles"][v, i] == 0
                    continue
                kept = _members(P, v, i)
                assert kept <= _members(full, v, i)
                assert len(kept) == P["tiles"][v, i]
                X, Y, a = _alpha_pixels(full, v, i, W, H)
                hit = a >= 1.0 / 255.0
                need = {(int(x) // 16, int(y) // 16) for x, y in zip(X[hit], Y[hit])}
                assert need <= kept, (v, i, sorted(need - kept))
                checked += int(hit.sum())
        assert checked > 10_000


def _box_min_q(A, B, C, x0, x1, y0, y1):
    """Minimum of q(d) = A dx^2 + 2 B dx dy + C dy^2 over the box of offsets
    [x0, x1] x [y0, y1] (q is convex: 0 if the box holds the origin, else the
    smallest of its four edge minima, each a clipped 1-D quadratic)."""
    if x0 <= 0.0 <= x1 and y0 <= 0.0 <= y1:
        return 0.0
    best = math.inf
    for (ax, ay, bx, by) in ((x0, y0, x1, y0), (x0, y1, x1, y1), (x0, y0, x0, y1),
                             (x1, y0, x1, y1)):
        ux, uy = bx - ax, by - ay
        a = A * ux * ux + 2 * B * ux * uy + C * uy * uy
        b = A * ax * ux + B * (ax * uy + ay * ux) + C * ay * uy
        t = min(1.0, max(0.0, -b / a)) if a > 0 else 0.0
        ex, ey = ax + t * ux, ay + t * uy
        best = min(best, A * ex * ex + 2 * B * ex * ey + C * ey * ey)
    return best


def test_span_ends_meet_the_widened_ellipse(oracle_mod):
    """Tightness: the first and last column kept in each row of a spanned
    record come within the slack of the ellipse q <= thr over the row's band
    (pixel-centre columns, band y +- 0.5 px), so spans drop every tile they
    can; rows left empty miss it."""
    spanned_rows = 0
    for sc, cams in _workloads():
        P = oracle_mod.project(sc, cams, "spans")
        for v in range(P["V"]):
            for i in np.flatnonzero(P["flags"][v] & oracle_flag_spans()):
                px, py = P["mean2d"][v, i]
                A, B, C = P["conic"][v, i]
                qm = 2.0 * (math.log(255.0) + math.log(P["alpha_hat"][v, i]))
                thr = qm + 2e-4 * abs(qm) + 1e-3
                x0, y0, x1, y1 = P["rect"][v, i]
                for ty in range(y0, y1):
                    a, b = P["spans"][v, i, ty - y0]
                    band = (16.0 * ty - 0.5 - py, 16.0 * ty + 15.5 - py)
                    eps = 1.1e-3
                    for tx in range(x0, x1):
                        q = _box_min_q(A, B, C, 16.0 * tx - px - eps, 16.0 * tx + 15 - px + eps,
                                       band[0] - eps, band[1] + eps)
                        inside = a <= tx < b
                        if tx in (a, b - 1) and inside:
                            assert q <= thr * (1 + 1e-9), (v, i, ty, tx, q, thr)
                        if not inside:
                            # a dropped tile is beyond the ellipse by the slack
                            qd = _box_min_q(A, B, C, 16.0 * tx - px + 0.9e-3,
                                            16.0 * tx + 15 - px - 0.9e-3, band[0] + 0.9e-3,
                                            band[1] - 0.9e-3)
                            assert qd > thr * (1 - 1e-9), (v, i, ty, tx, qd, thr)
                    spanned_rows += 1
    assert spanned_rows > 500


def test_images_identical_under_every_tile_set(oracle_mod):
    """Tile sets change the lists, never the compositing: images and final T
    are bit-identical, and the last composited Gaussian of every pixel is the
    same one (n_contrib counts positions in lists of different lengths)."""
    for sc, cams in _workloads():
        res = {m: oracle_mod.forward(sc, cams, tileset=m) for m in ("rect", "tight", "spans")}
        _, L0, I0 = res["rect"]
        assert res["spans"][1]["count"] < res["tight"][1]["count"] < L0["count"]
        for m in ("tight", "spans"):
            P, L, I = res[m]
            np.testing.assert_array_equal(I["image"], I0["image"])
            np.testing.assert_array_equal(I["final_T"], I0["final_T"])
            np.testing.assert_array_equal(I["usage"], I0["usage"])
            for v in range(P["V"]):
                W, H = (int(x) for x in cams["wh"][v])
                TX = (W + 15) // 16
                last = []
                for LL, II in ((L0, I0), (L, I)):
                    nc = II["n_contrib"][v]
                    yy, xx = np.mgrid[0:H, 0:W]
                    seg = LL["seg_base"][v] + (yy // 16) * TX + (xx // 16)
                    start = LL["ranges"][seg, 0].astype(np.int64)
                    pos = np.clip(start + nc - 1, 0, None)
                    last.append(np.where(nc > 0, LL["vals"][pos].astype(np.int64), -1))
                np.testing.assert_array_equal(last[0], last[1])


def test_span_lists_equal_brute_enumeration_and_brute_render(oracle_mod):
    sc, cams = _workloads()[0]
    P = oracle_mod.project(sc, cams, "spans")
    L = oracle_mod.bin_sort(P, cams)
    base, txv, nseg = oracle_mod.segment_bases(cams)
    inst = []
    for v in range(P["V"]):
        for i in range(sc["n"]):
            for (tx, ty) in _members(P, v, i):
                inst.append((int(base[v] + ty * txv[v] + tx), int(P["depth_bits"][v, i]), i))
    inst.sort()
    assert L["count"] == len(inst) == int(P["tiles"].sum())
    np.testing.assert_array_equal(L["keys"], [(s << 32) | d for s, d, _ in inst])
    np.testing.assert_array_equal(L["vals"], [i for _, _, i in inst])
    img = oracle_mod.render_fwd(P, L, cams)
    for v in range(P["V"]):
        bf = oracle_mod.render_brute(P, cams, v)
        np.testing.assert_array_equal(bf["image"], img["image"][v])
        np.testing.assert_array_equal(bf["n_contrib"], img["n_contrib"][v])
