"""sar_rda_execute captured into a HIP graph by the caller (torch's graph
capture on a side stream): every replay, with eager work and
synchronisations in between, reproduces the eager result bit for bit.  The
library records kernel launches only (no memset or copy nodes)."""
import numpy as np
import pytest

import paper_2604_03585_amd as sar
from gpu_util import dev, torch_cuda
from sarsim import config, simulate

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", ["c1", "c2"])
@pytest.mark.parametrize("transpose_back", [0, 1])
def test_captured_rda_replays_match_eager(name, transpose_back):
    torch = torch_cuda()
    cfg = config(name)
    raw = dev(simulate(cfg).raw)
    with sar.Plan(cfg, transpose_back=transpose_back) as p:
        shape = p.image_shape()
        eager = torch.empty(shape, dtype=torch.complex64, device="cuda")
        work = torch.empty(cfg["Na"] * cfg["Nr"], dtype=torch.complex64, device="cuda")
        p.execute(raw, eager, work)
        torch.cuda.synchronize()
        img = torch.empty_like(eager)
        work2 = torch.empty_like(work)
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            p.execute(raw, img, work2, stream=s)    # warm-up outside the capture
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            sar.sar_rda_execute(p.handle, raw, img, work2, s)
        for rep in range(3):
            img.fill_(float("nan"))                 # eager work between replays
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(img.view(torch.int64), eager.view(torch.int64)), rep
        del g


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_captured_half_storage_replays_match_eager(name):
    """The half-storage schedule (four kernels, FP16 workspace with exponent
    arrays) captured by the caller: every replay equals the eager result."""
    torch = torch_cuda()
    cfg = config(name)
    raw = dev(simulate(cfg).raw)
    with sar.Plan(cfg, precision="fp32_halfstore") as p:
        words = (p.workspace_bytes + 7) // 8
        eager = torch.empty(p.image_shape(), dtype=torch.complex64, device="cuda")
        work = torch.empty(words, dtype=torch.complex64, device="cuda")
        p.execute(raw, eager, work)
        torch.cuda.synchronize()
        img = torch.empty_like(eager)
        work2 = torch.empty_like(work)
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            p.execute(raw, img, work2, stream=s)
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            sar.sar_rda_execute(p.handle, raw, img, work2, s)
        for rep in range(3):
            img.fill_(float("nan"))
            work2.fill_(float("nan"))              # stale exponents must not leak into a replay
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(img.view(torch.int64), eager.view(torch.int64)), rep
        del g
