"""The peak-rate probes do the work they report: the copy probe copies, the
atomic probes add exactly the counts they claim, every probe returns a
positive duration, and short buffers or unknown kinds are refused."""
import pytest
import torch

from paper_2512_20943_amd import gs
from tests.gpu_helpers import require_gpu

pytestmark = pytest.mark.gpu

THREADS = 4096 * 256


def test_copy_probe_copies_and_reports_bytes():
    require_gpu()
    ctx = gs.default_context()
    n = 1 << 20
    buf = torch.empty(2 * n, dtype=torch.float32, device="cuda")
    buf[:n] = torch.arange(n, dtype=torch.float32, device="cuda")
    buf[n:] = -1.0
    ms, work = gs.gs_peak_run(ctx, "copy", buf)
    torch.cuda.synchronize()
    assert ms > 0 and work == 2 * 4 * n
    assert torch.equal(buf[n:], buf[:n])


@pytest.mark.parametrize("kind,iters,addrs", [("atomic_spread", 3, THREADS),
                                              ("atomic_same", 2, 64)])
def test_atomic_probes_add_exact_counts(kind, iters, addrs):
    require_gpu()
    ctx = gs.default_context()
    buf = torch.zeros(gs.peak_min_bytes(kind) // 4, dtype=torch.float32, device="cuda")
    ms, work = gs.gs_peak_run(ctx, kind, buf, iters)
    torch.cuda.synchronize()
    assert ms > 0 and work == THREADS * iters
    expect = float(THREADS // addrs * iters)
    assert torch.all(buf[:addrs] == expect)


@pytest.mark.parametrize("kind,iters", [("read", 1), ("lds", 2), ("fma", 8), ("exp", 8)])
def test_compute_probes_run(kind, iters):
    require_gpu()
    ctx = gs.default_context()
    nbytes = gs.peak_min_bytes(kind) + (1 << 20 if kind == "read" else 0)
    buf = torch.zeros(nbytes // 4, dtype=torch.float32, device="cuda")
    ms, work = gs.gs_peak_run(ctx, kind, buf, iters)
    torch.cuda.synchronize()
    assert ms > 0 and work > 0


def test_probe_arguments_are_checked():
    require_gpu()
    ctx = gs.default_context()
    small = torch.zeros(16, dtype=torch.float32, device="cuda")
    with pytest.raises(gs.GsError):
        gs.gs_peak_run(ctx, "fma", small, 1)
    with pytest.raises(gs.GsError):
        gs.gs_peak_run(ctx, "lds", torch.zeros(gs.peak_min_bytes("lds") // 4, device="cuda"), 0)
    buf = torch.zeros(1 << 20, dtype=torch.float32, device="cuda")
    st = ctx.lib.gs_peak_run(ctx.handle, 99, gs._ptr(buf), 4 << 20, 1, None, None, None)
    assert st == gs.GS_ERR_INVALID_ARG
