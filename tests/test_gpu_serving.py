"""Serving path on the GPU: every request's image is the same alone, in a
mixed batch, through the continuous-batching server and through the plain
one-request-per-launch renderer; a served image matches the oracle."""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2512_20943_amd import gs, scenes, serve
from tests.gpu_helpers import compare_image_only, require_gpu

pytestmark = pytest.mark.gpu

SMALL_RES = ((64, 48), (128, 96), (200, 150))


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def seq():
    require_gpu()
    anchor = scenes.make_scene(20_000, 11, -3.0, 3.0, -4.0, 0.5, 3)
    return serve.ResidentSequence(anchor, 6, seed=3), anchor


def test_request_alone_equals_request_in_mixed_batch(seq):
    s, _ = seq
    reqs = serve.make_trace(12, 1000.0, None, 4, s.n_frames, 5, resolutions=SMALL_RES)
    w = serve.BatchWorker(s)
    _, mixed = w.render(reqs)
    mixed = [m.clone() for m in mixed]
    plain = serve.PlainRenderer(s)
    for r, m in zip(reqs, mixed):
        _, alone = w.render([r])
        assert torch.equal(alone[0], m), f"request {r.rid} differs alone vs mixed"
        assert torch.equal(plain.render(r), m), f"request {r.rid} differs plain vs batched"


def test_served_image_matches_oracle(seq):
    s, anchor = seq
    reqs = serve.make_trace(3, 1000.0, None, 4, s.n_frames, 6, resolutions=SMALL_RES)
    w = serve.BatchWorker(s)
    _, imgs = w.render(reqs)
    for r, im in zip(reqs, imgs):
        d, m = s.frame_inputs(r.frame)
        frame = oracle.apply(anchor, d, m, s.gw, s.gh)
        cams = scenes.stack_cams([r.cam])
        _, _, ref = oracle.forward(frame, cams)
        compare_image_only(im.cpu().numpy(), ref["image"][0], ref["near_threshold"][0],
                           "served_small")


def test_continuous_batching_server_results_match_plain(seq):
    s, _ = seq
    trace = serve.make_trace(None, 400.0, 0.25, 64, s.n_frames, 7, resolutions=SMALL_RES)
    assert len(trace) > 20
    server = serve.Server(s, budget_bytes=8 << 30, max_batch=16, keep_images=True)
    server.run(trace)
    assert all(np.isfinite(r.t_done) for r in trace)
    assert max(server.batches) > 1, "no request was batched with another"
    plain = serve.PlainRenderer(s)
    for r in trace:
        assert torch.equal(r.image, plain.render(r)), f"request {r.rid}"
    st = serve.summarize(trace)
    say(f"  served {st}")


def test_tiny_hbm_budget_serialises_but_completes(seq):
    s, _ = seq
    trace = serve.make_trace(None, 300.0, 0.1, 8, s.n_frames, 8, resolutions=SMALL_RES)
    one = max(serve.request_bytes(r, s.anchor.ld, 600.0) for r in trace)
    server = serve.Server(s, budget_bytes=int(one * 1.2), max_batch=16)
    server.run(trace)
    assert all(np.isfinite(r.t_done) for r in trace)
    assert max(server.batches) <= 2


def test_serving_4k_requests_on_the_2m_scene():
    """Two 3840x2160 requests on a two-frame sequence of the 2M-Gaussian
    anchor: the batched launch equals the plain renderer bit for bit, and one
    served image matches the oracle."""
    require_gpu()
    anchor = scenes.make_scene(2_000_000, 0, -6.0, 6.0, -4.5, 0.7, 3)
    s = serve.ResidentSequence(anchor, 2, seed=5)
    g = scenes.rng(41)
    reqs = [serve.Request(k, k, scenes.sphere_camera(g, 4.0, 6.0, 3840, 2160), 0.0)
            for k in range(2)]
    w = serve.BatchWorker(s)
    _, imgs = w.render(reqs)
    imgs = [m.clone() for m in imgs]
    plain = serve.PlainRenderer(s)
    for r, m in zip(reqs, imgs):
        assert torch.equal(plain.render(r), m), f"request {r.rid} differs plain vs batched"
    d, m = s.frame_inputs(reqs[0].frame)
    frame = oracle.apply(anchor, d, m, s.gw, s.gh)
    _, _, ref = oracle.forward(frame, scenes.stack_cams([reqs[0].cam]))
    err = compare_image_only(imgs[0].cpu().numpy(), ref["image"][0], ref["near_threshold"][0],
                             "served_4k_2m")
    say(f"  4K request 0: max image error {err:.2e}")


def test_native_server_images_equal_the_plain_renderer(seq):
    """The native server's images, batched and in its plain mode, are the
    plain Python-driven renderer's bit for bit; requests share batches."""
    s, _ = seq
    trace = serve.make_trace(None, 400.0, 0.25, 64, s.n_frames, 17, resolutions=SMALL_RES)
    assert len(trace) > 20
    srv = serve.NativeServer(s, budget_bytes=8 << 30, max_batch=16)
    plain = serve.PlainRenderer(s)
    for mode in (False, True):
        tr = [serve.Request(r.rid, r.frame, r.cam, r.arrival, r.viewer) for r in trace]
        srv.run(tr, plain=mode, keep_images=True)
        assert all(np.isfinite(r.t_done) and r.t_done >= r.t_start >= 0.0 for r in tr)
        st = srv.stats()
        say(f"  native {'plain' if mode else 'batched'}: {serve.summarize(tr)} {st}")
        for r in tr:
            assert torch.equal(r.image, plain.render(r)), f"request {r.rid} (plain={mode})"
    srv.close()


def test_native_server_batches_a_burst_and_respects_the_budget(seq):
    s, _ = seq
    burst = serve.make_trace(24, 1e6, None, 8, s.n_frames, 18, resolutions=SMALL_RES)
    srv = serve.NativeServer(s, budget_bytes=8 << 30, max_batch=16, inline_singletons=False)
    srv.run(burst)
    st = srv.stats()
    assert st["max_batch"] > 1 and st["inline_requests"] == 0
    assert all(np.isfinite(r.t_done) for r in burst)
    one = max(serve.request_bytes(r, s.anchor.ld, 600.0) for r in burst)
    tight = serve.NativeServer(s, budget_bytes=int(one * 1.2), max_batch=16)
    tr = serve.make_trace(24, 1e6, None, 8, s.n_frames, 19, resolutions=SMALL_RES)
    tight.run(tr)
    assert tight.stats()["max_batch"] <= 2
    assert all(np.isfinite(r.t_done) for r in tr)
    srv.close()
    tight.close()


def test_native_server_rejects_bad_requests(seq):
    s, _ = seq
    srv = serve.NativeServer(s, budget_bytes=8 << 30)
    tr = serve.make_trace(3, 1000.0, None, 4, s.n_frames, 20, resolutions=SMALL_RES)
    bad = [serve.Request(r.rid, r.frame, r.cam, r.arrival) for r in tr]
    bad[1].frame = s.n_frames
    with pytest.raises(gs.GsError):
        srv.run(bad)
    late = [serve.Request(r.rid, r.frame, r.cam, r.arrival) for r in tr]
    late[0].arrival, late[2].arrival = late[2].arrival, late[0].arrival
    with pytest.raises(gs.GsError):
        srv.run(late)
    srv.close()
