"""Forward-state ownership in the Rasterizer (host logic, no GPU): the C calls
are replaced by stand-ins that only record which buffers they were given."""
import types

import pytest
import torch

from paper_2512_20943_amd import gs, raster


class FakeLists:
    def __init__(self, capacity, nseg, with_keys, device, gv=0):
        self.capacity, self.n_segments, self.gv = capacity, nseg, gv
        self.count = 0


@pytest.fixture()
def fake_gs(monkeypatch):
    calls = []

    def project(ctx, g, cams, proj, stream=None):
        calls.append(("project", id(proj)))

    def bin_sort(ctx, proj, cams, lists, ws, stream=None):
        lists.count = 7
        calls.append(("bin_sort", id(proj), id(lists)))
        return 7

    def render_fwd(ctx, proj, lists, cams, bg, image, final_T, n_contrib, stream=None,
                   usage=None):
        calls.append(("render_fwd", id(proj), id(lists)))

    def render_bwd(ctx, g, proj, lists, cams, bg, final_T, n_contrib, dimg, grad, ws, upd,
                   dd, stream=None, temporal=None):
        calls.append(("render_bwd", id(proj), id(lists)))

    monkeypatch.setattr(gs, "gs_project", project)
    monkeypatch.setattr(gs, "gs_bin_sort", bin_sort)
    monkeypatch.setattr(gs, "gs_render_fwd", render_fwd)
    monkeypatch.setattr(gs, "gs_render_bwd", render_bwd)
    monkeypatch.setattr(gs, "TileLists", FakeLists)
    monkeypatch.setattr(gs, "bin_sort_workspace_size", lambda *a: 256)
    monkeypatch.setattr(gs, "render_bwd_workspace_size", lambda *a: 256)
    return calls


def _inputs():
    g = types.SimpleNamespace(n=10, ld=64, mean=torch.zeros(3, 64))
    cams = types.SimpleNamespace(V=2, wh=[(32, 16), (32, 16)], n_segments=lambda: 4)
    return g, cams


def test_second_plain_forward_makes_the_first_state_stale(fake_gs):
    g, cams = _inputs()
    r = raster.Rasterizer(ctx=object())
    s1 = r.forward(g, cams)
    s2 = r.forward(g, cams)
    assert s1["proj"] is s2["proj"] and s1["lists"] is s2["lists"]  # shared buffers
    with pytest.raises(RuntimeError, match="stale"):
        r.backward(g, cams, s1, torch.zeros(1), None)
    r.backward(g, cams, s2, torch.zeros(1), None)
    assert fake_gs[-1] == ("render_bwd", id(s2["proj"]), id(s2["lists"]))
    # project or bin_sort alone also reuse the shared buffers
    r.project(g, cams)
    with pytest.raises(RuntimeError, match="stale"):
        r.backward(g, cams, s2, torch.zeros(1), None)


def test_own_buffer_states_never_alias_and_stay_valid(fake_gs):
    g, cams = _inputs()
    r = raster.Rasterizer(ctx=object())
    a = r.forward(g, cams, own_buffers=True)
    b = r.forward(g, cams, own_buffers=True)
    shared = r.forward(g, cams)
    assert a["proj"] is not b["proj"] and a["lists"] is not b["lists"]
    assert shared["proj"] is not a["proj"] and shared["lists"] is not a["lists"]
    # every own-buffer state can still be differentiated, in any order
    for st in (b, a):
        r.backward(g, cams, st, torch.zeros(1), None)
        assert fake_gs[-1] == ("render_bwd", id(st["proj"]), id(st["lists"]))
    r.backward(g, cams, shared, torch.zeros(1), None)
