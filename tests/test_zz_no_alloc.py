"""sar_rda_execute_noalloc: the whole RDA with the library's static
workspace instead of a caller's buffer, for callers that cannot allocate.
Its images must equal sar_rda_execute's bit for bit (same kernels, same
order), call after call on the shared array -- here a 4096^2 hyperbolic
scene (the largest workspace the array holds) followed by smaller scenes --
and under graph capture, where an allocation would fail."""
import numpy as np
import pytest

import paper_2604_03585_amd as sar
from paper_2604_03585_amd import _lib
from gpu_util import host, torch_cuda
from sarsim import config

pytestmark = pytest.mark.gpu


def _raw(torch, na, nr, seed):
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    return torch.randn((na, nr), dtype=torch.complex64, device="cuda", generator=g)


def _both(torch, plan, raw):
    ref = torch.empty(plan.image_shape(), dtype=torch.complex64, device="cuda")
    got = torch.full(plan.image_shape(), float("nan"), dtype=torch.complex64, device="cuda")
    work = torch.empty(((plan.workspace_bytes + 7) // 8,), dtype=torch.complex64, device="cuda")
    s = torch.cuda.current_stream()
    sar.sar_rda_execute(plan.handle, raw, ref, work, s)
    sar.sar_rda_execute_noalloc(plan.handle, raw, got, s)
    return host(ref), host(got)


CASES = [  # (config, overrides, precision, schedule): largest first, then smaller
    ("c2", {}, "fp32", "fused"),
    ("c2", {}, "fp32", "turn_free"),
    ("c1", dict(Na=1024, Nr=512), "fp32", "turn_free"),
    ("c1", {}, "fp32", "fused"),
    ("c2", dict(Na=2048, Nr=1024, range_len=256, range_tbp=100.0), "fp32_halfstore", "fused"),
    ("c2", dict(Na=1024, Nr=1024, range_len=256, range_tbp=100.0), "fp32", "unfused"),
    ("c1", {}, "split_fp16", "fused"),
]


def test_noalloc_equals_execute_call_after_call():
    torch = torch_cuda()
    for i, (name, over, prec, sched) in enumerate(CASES):
        cfg = config(name, **over)
        print(f"case {i}: {name} {cfg['Na']}x{cfg['Nr']} {prec} {sched}", flush=True)
        with sar.Plan(cfg, precision=prec, schedule=sched) as p:
            assert p.workspace_bytes <= _lib.SAR_NOALLOC_WORKSPACE_BYTES
            raw = _raw(torch, cfg["Na"], cfg["Nr"], 100 + i)
            ref, got = _both(torch, p, raw)
        assert np.isfinite(ref).all()
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), (name, prec, sched)


def test_noalloc_rejects_a_plan_beyond_the_static_workspace():
    torch = torch_cuda()
    cfg = config("c1", Na=4096, Nr=8192, range_len=1024, range_tbp=512.0, az_len=512,
                 az_tbp=256.0)
    with sar.Plan(cfg) as p:
        assert p.workspace_bytes > _lib.SAR_NOALLOC_WORKSPACE_BYTES
        raw = torch.zeros((cfg["Na"], cfg["Nr"]), dtype=torch.complex64, device="cuda")
        img = torch.empty(p.image_shape(), dtype=torch.complex64, device="cuda")
        with pytest.raises(sar.SarError) as e:
            sar.sar_rda_execute_noalloc(p.handle, raw, img)
        assert e.value.status == _lib.SAR_ERR_BAD_SIZE
        assert "static workspace" in sar.sar_last_error()
        torch.cuda.synchronize()


def test_noalloc_under_graph_capture():
    """Captured into a graph and replayed several times, with eager work of
    the program's own between the replays: every replay equals the eager
    result."""
    torch = torch_cuda()
    cfg = config("c2", Na=1024, Nr=2048, range_len=256, range_tbp=100.0)
    with sar.Plan(cfg) as p:
        raw = _raw(torch, cfg["Na"], cfg["Nr"], 7)
        eager_ref, eager = _both(torch, p, raw)
        assert np.array_equal(eager, eager_ref)
        img = torch.empty(p.image_shape(), dtype=torch.complex64, device="cuda")
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            sar.sar_rda_execute_noalloc(p.handle, raw, img, s)      # warm-up outside the capture
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            sar.sar_rda_execute_noalloc(p.handle, raw, img, s)
        other = _raw(torch, cfg["Na"], cfg["Nr"], 8)
        for r in range(3):
            img.fill_(float("nan"))
            g.replay()
            got = host(img)
            assert np.array_equal(got.view(np.uint32), eager.view(np.uint32)), r
            # eager work on the same static workspace between replays
            tmp = torch.empty_like(img)
            sar.sar_rda_execute_noalloc(p.handle, other, tmp)
            torch.cuda.synchronize()
