"""Pins of the oracle's temporal/keyframe terms (Sec. III-B, Eq. (6), (7),
(9)), densification statistics, low-opacity culling, and the residual
bookkeeping and quantisation of sent updates (Sec. III-C, Eq. (11), (12))
against closed forms, invariants and library routines."""
import numpy as np
from scipy.special import expit

import oracle
from paper_2512_20943_amd import scenes


def _identity(gw, gh):
    d = np.zeros((8, gh, gw), np.float32)
    d[3] = 1.0
    return d


def test_temporal_identity_is_zero():
    loss, g = oracle.temporal_l1(_identity(5, 4), 17, 1e-3)
    assert loss == 0.0 and not g.any()


def test_temporal_single_texel_closed_form():
    d = _identity(4, 4)
    d[3, 1, 2] = 0.75          # quaternion w of texel 6: |0.75 - 1| = 0.25
    d[0, 0, 1] = -0.5          # translation x of texel 1
    d[7, 3, 3] = 9.0           # texel 15 is padding for n = 15
    loss, g = oracle.temporal_l1(d, 15, 0.1)
    assert abs(loss - 0.1 * (0.25 + 0.5)) < 1e-15
    assert g[3, 1, 2] == -0.1 and g[0, 0, 1] == -0.1
    assert g[7, 3, 3] == 0.0
    assert np.count_nonzero(g) == 2


def test_temporal_gradient_matches_differences():
    d = scenes.make_delta(50, 8, 7, 3).astype(np.float64)
    loss, g = oracle.temporal_l1(d, 50, 2e-3)
    h = 1e-7
    for (c, y, x) in [(0, 0, 3), (3, 2, 1), (5, 6, 1), (7, 4, 4)]:
        e = d.copy()
        e[c, y, x] += h
        fd = (oracle.temporal_l1(e, 50, 2e-3)[0] - loss) / h
        assert abs(fd - g[c, y, x]) < 1e-6


def test_keyframe_temporal_closed_form():
    x = np.arange(12, dtype=np.float32).reshape(3, 4)
    p = x.copy()
    p[0, 1] += 2.0
    p[2, 0] -= 0.5
    p[1, 3] += 7.0             # column 3 is beyond the bound
    loss, g = oracle.keyframe_temporal_l1(x, p, 3, 0.5)
    assert loss == 0.5 * (2.0 + 0.5)
    assert g[0, 1] == -0.5 and g[2, 0] == 0.5 and g[1, 3] == 0.0


def test_densify_stats_hand_built():
    flags = np.array([[32, 0, 32], [32, 32, 0]], np.uint8)      # 2 views, 3 Gaussians
    g2d = np.zeros((2, 3, 9))
    g2d[0, 0, :2] = (3.0, 4.0)
    g2d[1, 0, :2] = (-6.0, 8.0)
    g2d[0, 1, :2] = (1.0, 1.0)   # invisible in view 0: not counted
    g2d[1, 1, :2] = (0.0, -2.0)
    g2d[1, 2, :2] = (5.0, 5.0)   # invisible in view 1
    acc, cnt = oracle.densify_stats(flags, g2d)
    np.testing.assert_allclose(acc, [15.0, 2.0, 0.0])
    np.testing.assert_array_equal(cnt, [2, 1, 1])


def test_low_opacity_keep_matches_sigmoid():
    g = scenes.rng(5)
    x = g.normal(-4.0, 2.0, 4000).astype(np.float32)
    keep = oracle.low_opacity_keep(x, 3900, 0.005)
    s = expit(x[:3900].astype(np.float64))
    far = np.abs(s - 0.005) > 1e-12
    want = np.nonzero(s >= 0.005)[0]
    got_mask = np.zeros(3900, bool)
    got_mask[keep] = True
    np.testing.assert_array_equal(got_mask[far], (s >= 0.005)[far])
    assert np.all(np.diff(keep) > 0)
    assert abs(len(keep) - len(want)) <= int((~far).sum())


def test_residual_full_mask_tracks_truth():
    n, gw, gh = 30, 6, 6
    D = scenes.make_delta(n, gw, gh, 1)
    P = _identity(gw, gh)
    d, amax = oracle.residual_delta(D, P, np.ones((gh, gw), np.uint8), n)
    P2 = oracle.accumulate_sent(P, d)
    # every kept texel is reconstructed to within one FP32 rounding of D
    r = np.abs(P2.reshape(8, -1)[:, :n] - D.reshape(8, -1)[:, :n])
    assert np.all(r <= np.spacing(np.abs(D.reshape(8, -1)[:, :n])))
    np.testing.assert_array_equal(d.reshape(8, -1)[:, n:], 0.0)
    np.testing.assert_array_equal(amax, np.abs(d.reshape(8, -1)[:, :n]).max(axis=1))


def test_residual_pruned_motion_is_sent_later():
    """A texel pruned at frame 1 and kept at frame 2 receives the motion of
    both frames at frame 2 (no drift from pruning)."""
    n, gw, gh = 16, 4, 4
    P0 = _identity(gw, gh)
    D1 = P0.copy()
    D1[0] += 0.25              # frame-1 motion: +0.25 on x for every texel
    D2 = D1.copy()
    D2[0] += 0.125             # frame-2 motion: a further +0.125
    m1 = np.ones((gh, gw), np.uint8)
    m1[1, 2] = 0               # texel 6 pruned at frame 1
    d1, _ = oracle.residual_delta(D1, P0, m1, n)
    P1 = oracle.accumulate_sent(P0, d1)
    assert d1[0, 1, 2] == 0.0 and P1[0, 1, 2] == 0.0
    d2, _ = oracle.residual_delta(D2, P1, np.ones((gh, gw), np.uint8), n)
    P2 = oracle.accumulate_sent(P1, d2)
    assert d2[0, 1, 2] == 0.375 and d2[0, 0, 0] == 0.125
    np.testing.assert_array_equal(P2, D2)


def test_residual_zero_mask_sends_nothing():
    n, gw, gh = 20, 5, 4
    D = scenes.make_delta(n, gw, gh, 2)
    P = _identity(gw, gh)
    d, amax = oracle.residual_delta(D, P, np.zeros((gh, gw), np.uint8), n)
    assert not d.any() and not amax.any()


def test_quantize_error_bound_and_symmetry():
    g = scenes.rng(9)
    for bits in (8, 16):
        d = g.normal(0, 0.01, (8, 7, 9)).astype(np.float32)
        d[:, 0, 0] = 0.0
        d[5] = 0.0                                  # an all-zero channel
        amax = np.abs(d.reshape(8, -1)).max(axis=1)
        q, s = oracle.quantize_delta(d, amax, bits)
        qmax = 2 ** (bits - 1) - 1
        assert q.dtype == (np.int16 if bits == 16 else np.int8)
        assert np.all(np.abs(q.astype(np.int64)) <= qmax)
        x = oracle.dequantize_delta(q, s)
        err = np.abs(x.astype(np.float64) - d)
        bound = (s.astype(np.float64) * (0.5 + 1e-6))[:, None, None] + 1e-12
        assert np.all(err <= bound)
        assert not q[:, 0, 0].any() and not x[:, 0, 0].any()
        assert s[5] == 0.0 and not q[5].any()
        # the largest magnitude of each channel reaches the end of the code range
        flat = np.abs(q.reshape(8, -1).astype(np.int64)).max(axis=1)
        assert np.all(flat[amax > 0] == qmax)
        q2, _ = oracle.quantize_delta(-d, amax, bits)
        np.testing.assert_array_equal(q2, -q)
