"""Residual bookkeeping of sent updates and their quantised planes (Sec.
III-C, Eq. (11), (12)) on the GPU against the oracle, bit exact: the sent
update, its per-channel range, the codes and scales, the server's and the
client's running sums, and the frame the client applies."""
import numpy as np
import pytest
import torch

import oracle
from paper_2512_20943_amd import gs, scenes
from paper_2512_20943_amd.raster import frame_of
from tests.gpu_helpers import require_gpu

pytestmark = pytest.mark.gpu


def _identity(gw, gh):
    d = np.zeros((8, gh, gw), np.float32)
    d[3] = 1.0
    return d


def _sequence(n, gw, gh, frames, seed):
    """True accumulated deltas D_1..D_T of a synthetic motion sequence."""
    D = [_identity(gw, gh)]
    for t in range(frames):
        step = scenes.make_delta(n, gw, gh, seed + t) - _identity(gw, gh)
        D.append((D[-1] + step).astype(np.float32))
    return D[1:]


@pytest.mark.parametrize("n,bits", [(1, 8), (2000, 8), (2000, 16), (70_001, 16)])
def test_sent_updates_bit_exact(n, bits):
    require_gpu()
    gw = gh = scenes.grid_side(n)
    sc = scenes.make_scene(n, 1, -3, 3, -4, 0.5, 0)
    anchor = gs.Gaussians.from_scene(sc)
    ctx = gs.default_context()
    Ds = _sequence(n, gw, gh, 3, 40 + n)
    P_srv = torch.from_numpy(_identity(gw, gh)).cuda()
    P_cli = P_srv.clone()
    P_or = _identity(gw, gh)
    frame = frame_of(anchor)
    qdt = torch.int8 if bits == 8 else torch.int16
    for t, D in enumerate(Ds):
        mask = scenes.prune_mask(D, n, (0.5, 0.0, 0.3)[t])
        d_or, amax_or = oracle.residual_delta(D, P_or, mask, n)
        q_or, s_or = oracle.quantize_delta(d_or, amax_or, bits)
        P_or = oracle.accumulate_sent(P_or, oracle.dequantize_delta(q_or, s_or))
        f_or = oracle.apply(sc, P_or, np.ones((gh, gw), np.uint8), gw, gh)

        d = torch.full((8, gh, gw), float("nan"), device="cuda")
        amax = torch.zeros(8, device="cuda")
        gs.gs_residual_delta(ctx, torch.from_numpy(D).cuda(), P_srv, torch.from_numpy(mask).cuda(),
                             n, gw, gh, d, amax)
        q = torch.full((8, gh, gw), 99, dtype=qdt, device="cuda")
        s = torch.full((8,), float("nan"), device="cuda")
        gs.gs_quantize_delta(ctx, d, amax, bits, n, gw, gh, q, s, P_srv)
        gs.gs_apply_quantized_update(ctx, anchor, q, bits, s, P_cli, gw, gh, frame)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(d.cpu().numpy(), d_or)
        np.testing.assert_array_equal(amax.cpu().numpy(), amax_or)
        np.testing.assert_array_equal(q.cpu().numpy(), q_or)
        np.testing.assert_array_equal(s.cpu().numpy(), s_or)
        Pn = P_srv.cpu().numpy().reshape(8, -1)[:, :n]
        np.testing.assert_array_equal(Pn, P_or.reshape(8, -1)[:, :n])
        np.testing.assert_array_equal(P_cli.cpu().numpy().reshape(8, -1)[:, :n], Pn)
        for k, tt in (("mean", frame.mean), ("quat", frame.quat), ("opacity", frame.opacity)):
            np.testing.assert_array_equal(tt.cpu().numpy()[..., :n], f_or[k][..., :n])


def test_pruned_motion_reaches_the_client_later():
    require_gpu()
    n, gw, gh = 16, 4, 4
    ctx = gs.default_context()
    P0 = _identity(gw, gh)
    D1 = P0.copy()
    D1[0] += 0.25
    D2 = D1.copy()
    D2[0] += 0.125
    m1 = np.ones((gh, gw), np.uint8)
    m1[1, 2] = 0
    P = torch.from_numpy(P0).cuda()
    for D, m in ((D1, m1), (D2, np.ones((gh, gw), np.uint8))):
        d = torch.empty(8, gh, gw, device="cuda")
        amax = torch.zeros(8, device="cuda")
        gs.gs_residual_delta(ctx, torch.from_numpy(D).cuda(), P, torch.from_numpy(m).cuda(), n,
                             gw, gh, d, amax)
        q = torch.empty(8, gh, gw, dtype=torch.int16, device="cuda")
        s = torch.empty(8, device="cuda")
        gs.gs_quantize_delta(ctx, d, amax, 16, n, gw, gh, q, s, P)
    torch.cuda.synchronize()
    # the frame-1 quantisation error is corrected by the frame-2 residual, so
    # every texel ends within half a frame-2 code step (plus FP32 rounding)
    got = P.cpu().numpy()
    assert abs(got[0, 1, 2] - 0.375) <= 0.375 / 32767
    assert np.all(np.abs(got[0] - 0.375) <= 0.375 / 32767)
