"""The batched and served workloads at their full sizes, in the launch
configuration the benchmark times.

Batched: the 64 uneven LFM scenes (Nr 1024..16384 x Na 512..8192, 1640 Mpx)
run as one batch replayed from a hipGraph on a stream.  Every scene must be
bit-identical to its own single-scene run, every point target must focus on
its seeded cell, and two sampled scenes (the smallest and the largest) must
match the FP64 oracle within 1e-5 relative L2.

Served: requests drawn from the full pool of 32 scenes (1024^2 .. 8192 x
16384) under a 64 GiB budget with four slots; every result must be
bit-identical to the scene run alone.
"""
import numpy as np
import pytest

import paper_2604_03585_amd as sar
from gpu_util import rel_l2, torch_cuda
from oracle import oracle as O
from oracle import quality as Q
from paper_2604_03585_amd.server import GpuExecutor, Server, replay
from sarsim import batch_configs, serve_pool_configs, simulate, simulate_many

pytestmark = pytest.mark.gpu

GiB = 1 << 30


def upload_all(torch, cfgs):
    raws = [None] * len(cfgs)
    targets = [None] * len(cfgs)

    def up(i, sc):
        raws[i] = torch.from_numpy(sc.raw).cuda()
        targets[i] = sc.targets

    simulate_many(cfgs, workers=8, consume=up)
    torch.cuda.synchronize()
    return raws, targets


def test_c4_full_batch():
    torch = torch_cuda()
    cfgs = batch_configs()
    assert len(cfgs) == 64
    raws, targets = upload_all(torch, cfgs)
    params = [sar.make_params(c) for c in cfgs]
    s = torch.cuda.Stream()
    b = sar.sar_batch_plan(params, s)
    try:
        imgs = [torch.empty((c["Nr"], c["Na"]), dtype=torch.complex64, device="cuda")
                for c in cfgs]
        work = torch.empty(sar.sar_batch_workspace_bytes(b) // 8 + 1, dtype=torch.complex64,
                           device="cuda")
        for _ in range(2):                        # capture, then a replay
            sar.sar_batch_execute(b, raws, imgs, work, s)
        s.synchronize()
        for i, c in enumerate(cfgs):
            with sar.Plan(c) as p:
                one = torch.empty((c["Nr"], c["Na"]), dtype=torch.complex64, device="cuda")
                p.execute(raws[i], one, work)
                torch.cuda.synchronize()
            assert torch.equal(one.view(torch.int64), imgs[i].view(torch.int64)), c["name"]
            for t in targets[i]:
                m, n = t["m"], t["n"]
                m0, n0 = max(0, m - 8), max(0, n - 8)
                win = imgs[i][n0:n + 9, m0:m + 9].cpu().numpy().T      # image is [Nr][Na]
                pm, pn = Q.peak_cell(win, m - m0, n - n0)
                assert (pm + m0, pn + n0) == (m, n), (c["name"], t)
        px = [c["Na"] * c["Nr"] for c in cfgs]
        for i in (int(np.argmin(px)), int(np.argmax(px))):
            sc = simulate(cfgs[i])
            ref = O.rda(sc.raw, cfgs[i])
            err = rel_l2(imgs[i].cpu().numpy().T, ref)
            print(f"{cfgs[i]['name']}: rel L2 vs oracle {err:.3e}")
            assert err <= 1e-5
    finally:
        torch.cuda.synchronize()
        sar.sar_batch_destroy(b)


def test_c5_full_pool_served_equals_alone():
    torch = torch_cuda()
    cfgs = serve_pool_configs()
    raws, _ = upload_all(torch, cfgs)
    alone = []
    for c, r in zip(cfgs, raws):
        with sar.Plan(c) as p:
            alone.append(p.execute(r))
    torch.cuda.synchronize()
    rng = np.random.default_rng(55)
    which = rng.integers(0, len(cfgs), size=48)
    arrivals = np.cumsum(rng.exponential(1 / 2000.0, size=48))
    arrivals[:8] = 0.0                      # a burst first: requests must overlap
    mismatched = []

    def check(res):
        # res.id counts submissions from 0 in submission order
        w = int(which[res.id])
        if not torch.equal(res.image.view(torch.int64), alone[w].view(torch.int64)):
            mismatched.append(res.id)
        res.release()

    ex = GpuExecutor(4, 64 * GiB)
    srv = Server(64 * GiB, slots=4, executor=ex, on_result=check)
    try:
        results, errors, _ = replay(srv, [(cfgs[w], raws[w], "fp32") for w in which], arrivals)
    finally:
        srv.close()
        ex.close()
    assert not errors and len(results) == 48
    assert srv.max_concurrent > 1
    assert not mismatched, mismatched
