"""The server on the device: scenes of mixed sizes and precisions, submitted
with Poisson arrivals so that they overlap on several streams under a tight
HBM budget, give exactly the image each gives alone (same plan, same
kernels: bit-identical), and the budget is never exceeded."""
import numpy as np
import pytest

import paper_2604_03585_amd as sar
from gpu_util import dev, host, rel_l2, torch_cuda
from oracle import oracle as O
from paper_2604_03585_amd.server import GpuExecutor, Server, footprint_bytes, replay


def copy_out(res):
    """on_result: bring the image to the host, give its arena block back."""
    img = res.image.cpu().numpy()
    res.release()
    res.image = img
from sarsim import config, lfm_scene, poisson_arrivals, simulate


pytestmark = pytest.mark.gpu


def pool():
    cfgs = [lfm_scene(nr, na, 5, seed, f"s{na}x{nr}")
            for nr, na, seed in [(256, 256, 11), (1024, 512, 12), (512, 2048, 13),
                                 (2048, 1024, 14), (4096, 256, 15)]]
    cfgs.append(config("c2", Nr=1024, Na=2048, range_len=256, range_tbp=100.0, n_targets=2,
                       seed=16))
    return cfgs


@pytest.mark.parametrize("slots", [1, 4])
def test_served_equals_alone(slots):
    torch = torch_cuda()
    cfgs = pool()
    scenes = [simulate(c) for c in cfgs]
    raws = [dev(s.raw) for s in scenes]
    precs = ["fp32", "split_fp16", "fp32_halfstore"]
    alone = {}
    for i, c in enumerate(cfgs):
        for p in precs:
            with sar.Plan(c, precision=p) as plan:
                alone[(i, p)] = host(plan.execute(raws[i]))
    torch.cuda.synchronize()
    # 60 requests, Poisson at ~5 kHz: several on the device at once
    _, which = poisson_arrivals(seed=21, n=60, rate_hz=5000.0, pool_size=len(cfgs))
    arrivals = np.cumsum(np.random.default_rng(21).exponential(1 / 5000.0, size=60))
    arrivals[:8] = 0.0                      # a burst first: requests must overlap
    reqs = [(cfgs[w], raws[w], precs[k % 3]) for k, w in enumerate(which)]
    budget = 2 * max(footprint_bytes(c) for c in cfgs)
    ex = GpuExecutor(slots, budget)
    srv = Server(budget, slots=slots, executor=ex, on_result=copy_out)
    try:
        results, errors, wall = replay(srv, reqs, arrivals)
    finally:
        srv.close()
    assert not errors
    assert srv.max_used <= budget and srv.used_bytes == 0
    print(f"slots {slots}: max concurrent {srv.max_concurrent}, wall {wall * 1e3:.1f} ms")
    if slots > 1:
        assert srv.max_concurrent > 1
    for r, (c, raw, p), w in zip(results, reqs, which):
        assert np.array_equal(r.image, alone[(int(w), p)]), (r.id, c["name"], p)
    ex.close()


def test_served_fp32_matches_oracle():
    cfgs = pool()[:3]
    scenes = [simulate(c) for c in cfgs]
    raws = [dev(s.raw) for s in scenes]
    srv = Server(1 << 30, slots=3)
    try:
        futs = [srv.submit(c, r) for c, r in zip(cfgs, raws)]
        res = [f.result(60) for f in futs]
    finally:
        srv.close()
    for c, s, r in zip(cfgs, scenes, res):
        ref = O.rda(s.raw, c)
        assert rel_l2(host(r.image).T, ref) <= 1e-5
        r.release()
    assert srv.used_bytes == 0
    srv.executor.close()


def test_submit_orders_copy_after_client_stream():
    """A client fills raw asynchronously on its own stream (a delay, then a
    non-blocking copy from pinned host memory) and submits at once: the
    request's staging copy must wait for that work, so the served image is
    the image of the scene, not of the buffer's earlier contents."""
    torch = torch_cuda()
    cfg = pool()[3]
    sc = simulate(cfg)
    with sar.Plan(cfg) as plan:
        want = host(plan.execute(dev(sc.raw)))
    pinned = torch.from_numpy(sc.raw).pin_memory()
    raw = torch.zeros(pinned.shape, dtype=torch.complex64, device="cuda")
    torch.cuda.synchronize()
    producer = torch.cuda.Stream()
    srv = Server(1 << 30, slots=2)
    try:
        with torch.cuda.stream(producer):
            if hasattr(torch.cuda, "_sleep"):
                torch.cuda._sleep(20_000_000)       # ~10 ms of device time first
            raw.copy_(pinned, non_blocking=True)
            fut = srv.submit(cfg, raw)
        res = fut.result(60)
        got = host(res.image)
        res.release()
    finally:
        srv.close()
    assert np.array_equal(got, want)
    srv.executor.close()
