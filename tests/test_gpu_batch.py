"""Batched execution of scenes of uneven size (one launch per stage and line
length for all scenes, corner turns of all scenes in one launch, hipGraph
replay on a non-null stream).

Every scene of a batch must come out bit-identical to its own single-scene
sar_rda_execute (the batched launches run the same per-line code), in graph
mode, in direct mode (null stream) and on repeated replays; a subset of the
batched workload is also held to the oracle bar (1e-5 relative L2).
"""
import numpy as np
import pytest

import paper_2604_03585_amd as sar
from gpu_util import dev, host, rel_l2, torch_cuda
from oracle import oracle as O
from oracle import quality as Q
from sarsim import batch_configs, config, lfm_scene, simulate

pytestmark = pytest.mark.gpu


def small_batch():
    """Uneven small scenes: LFM of several sizes (two of them in split FP16 /
    split BF16, batched with their own launches), one with transpose_back,
    one hyperbolic and one unfused (both run outside the batched launches)."""
    cfgs = [c for c in batch_configs(seed=4, n=64, nr_choices=(256, 512, 1024),
                                     na_choices=(256, 512))][:6]
    hyp = config("c2", Nr=512, Na=2048, range_len=256, range_tbp=100.0, n_targets=1, seed=9)
    opts = [dict() for _ in cfgs]
    opts[1] = dict(precision="split_fp16")
    opts[4] = dict(precision="split_bf16")
    return cfgs, opts + [dict(), dict(schedule="unfused"), dict(transpose_back=1)], hyp


def run_batch(cfgs, opts, scenes, stream, reps=1):
    torch = torch_cuda()
    params = [sar.make_params(c, **o) for c, o in zip(cfgs, opts)]
    b = sar.sar_batch_plan(params, stream)
    try:
        raws = [dev(s.raw) for s in scenes]
        imgs = [torch.empty(s.raw.shape[::-1] if not o.get("transpose_back") else s.raw.shape,
                            dtype=torch.complex64, device="cuda") for s, o in zip(scenes, opts)]
        work = torch.empty(sar.sar_batch_workspace_bytes(b) // 8 + 1, dtype=torch.complex64,
                           device="cuda")
        outs = []
        for _ in range(reps):
            for im in imgs:
                im.zero_()
            sar.sar_batch_execute(b, raws, imgs, work, stream)
            outs.append([host(im) for im in imgs])
        return outs
    finally:
        torch.cuda.synchronize()
        sar.sar_batch_destroy(b)


def single(cfg, opt, raw):
    with sar.Plan(cfg, **opt) as p:
        return host(p.execute(dev(raw)))


@pytest.mark.parametrize("graph", [True, False])
def test_batch_matches_single_scene_runs(graph):
    torch = torch_cuda()
    cfgs, opts, hyp = small_batch()
    cfgs = cfgs + [hyp, cfgs[0], cfgs[1]]
    scenes = [simulate(c) for c in cfgs]
    stream = torch.cuda.Stream() if graph else 0
    with torch.cuda.stream(stream) if graph else torch.cuda.stream(torch.cuda.current_stream()):
        outs = run_batch(cfgs, opts, scenes, stream, reps=3)
    for rep in outs:
        for i, (c, o, s) in enumerate(zip(cfgs, opts, scenes)):
            ref = single(c, o, s.raw)
            assert np.array_equal(rep[i].view(np.uint32), ref.view(np.uint32)), (i, c["name"], o)


@pytest.mark.parametrize("graph", [True, False])
def test_batch_long_lines_and_large_scenes(graph):
    """Lines of 8192 and 16384 points in shared launches (scenes below 2^22
    pixels) next to a scene of 2^22 pixels, which runs its own launches after
    them; every image bit-identical to its single-scene run."""
    torch = torch_cuda()
    cfgs = [lfm_scene(16384, 128, 1, 11, "r16k"), lfm_scene(128, 16384, 1, 12, "a16k"),
            lfm_scene(8192, 256, 1, 13, "r8k"), lfm_scene(2048, 2048, 2, 14, "big"),
            lfm_scene(256, 8192, 1, 15, "a8k")]
    opts = [dict() for _ in cfgs]
    scenes = [simulate(c) for c in cfgs]
    stream = torch.cuda.Stream() if graph else 0
    with torch.cuda.stream(stream) if graph else torch.cuda.stream(torch.cuda.current_stream()):
        outs = run_batch(cfgs, opts, scenes, stream, reps=2)
    for rep in outs:
        for i, (c, o, s) in enumerate(zip(cfgs, opts, scenes)):
            ref = single(c, o, s.raw)
            assert np.array_equal(rep[i].view(np.uint32), ref.view(np.uint32)), (i, c["name"])


def test_batch_against_oracle():
    torch = torch_cuda()
    cfgs = batch_configs(seed=4, n=64, nr_choices=(1024, 2048), na_choices=(512, 1024))[:4]
    scenes = [simulate(c) for c in cfgs]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        out = run_batch(cfgs, [dict()] * len(cfgs), scenes, stream)[0]
    for c, s, img in zip(cfgs, scenes, out):
        ref = O.rda(s.raw, c)
        assert rel_l2(img.T, ref) <= 1e-5, c["name"]
        for t in s.targets:
            assert Q.peak_cell(img.T, t["m"], t["n"]) == (t["m"], t["n"])


def test_batch_buffer_rules():
    """Shared raw inputs are allowed; images overlapping each other or another
    scene's raw input are rejected before anything is launched."""
    torch = torch_cuda()
    cfgs = batch_configs(seed=4, n=64, nr_choices=(256,), na_choices=(256,))[:2]
    params = [sar.make_params(c) for c in cfgs]
    b = sar.sar_batch_plan(params, None)
    try:
        px = 256 * 256
        raw = dev(simulate(cfgs[0]).raw)
        pool = torch.empty(4 * px, dtype=torch.complex64, device="cuda")
        img0, img1 = pool[:px], pool[px:2 * px]
        work = torch.empty(sar.sar_batch_workspace_bytes(b) // 8 + 1, dtype=torch.complex64,
                           device="cuda")
        # the same raw for both scenes: fine, and both images equal
        sar.sar_batch_execute(b, [raw, raw], [img0, img1], work, 0)
        torch.cuda.synchronize()
        assert torch.equal(img0.view(torch.int64), img1.view(torch.int64))
        with pytest.raises(sar.SarError) as e:
            sar.sar_batch_execute(b, [raw, raw], [img0, pool[px // 2:px // 2 + px]], work, 0)
        assert e.value.status == sar._lib.SAR_ERR_ALIAS
        with pytest.raises(sar.SarError) as e:
            sar.sar_batch_execute(b, [raw, img0], [img0, img1], work, 0)   # image 0 = raw 1
        assert e.value.status == sar._lib.SAR_ERR_ALIAS
    finally:
        torch.cuda.synchronize()
        sar.sar_batch_destroy(b)
