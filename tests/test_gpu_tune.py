"""The autotuner on the device: sar_autotune writes a cache the next plans
use, and every kernel variant it can choose gives the oracle's result
(variants differ in scheduling only: relative L2 <= 1e-5 against the FP64
oracle, <= 1e-6 against the default variant; batched = single-scene
bit-identical when both use the same twiddle scheme)."""
import json

import numpy as np
import pytest

import paper_2604_03585_amd as sar
from gpu_util import dev, host, rel_l2, torch_cuda
from oracle import oracle as O
from paper_2604_03585_amd import _lib
from sarsim import batch_configs, config, simulate

pytestmark = pytest.mark.gpu

KINDS = ["fused", "fwd", "inv", "rcmc", "batch_fused", "turn", "strip"]


def arch():
    torch = torch_cuda()
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def write_cache(path, entries):
    a = arch()
    with open(path, "w") as f:
        for kind, n, prec, v in entries:
            f.write(json.dumps({"arch": a, "kind": kind, "n": n, "prec": prec, "variant": v}) + "\n")
    sar.sar_tune_load(str(path))


@pytest.fixture(autouse=True)
def clear_table():
    yield
    sar.sar_tune_load(None)


_oracle = {}


def scene(name, **over):
    key = (name, tuple(sorted(over.items())))
    if key not in _oracle:
        cfg = config(name, **over)
        sc = simulate(cfg)
        _oracle[key] = (cfg, sc, O.rda(sc.raw, cfg))
    return _oracle[key]


def run(cfg, raw, **opts):
    with sar.Plan(cfg, **opts) as p:
        return host(p.execute(dev(raw))).T


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_autotune_writes_cache_and_plans_use_it(tmp_path, name):
    cfg, sc, ref = scene(name)
    path = tmp_path / "tune.jsonl"
    sar.sar_autotune(sar.make_params(cfg), str(path))
    # split precisions are tuned under their own keys (prec 1) in the same file
    sar.sar_autotune(sar.make_params(cfg, precision="split_fp16"), str(path))
    split = [json.loads(l) for l in path.read_text().splitlines() if json.loads(l)["prec"] == 1]
    assert split and all(e["variant"] in (0, 2) for e in split), split
    path.write_text("".join(l + "\n" for l in path.read_text().splitlines()
                            if json.loads(l)["prec"] == 0))
    sar.sar_tune_load(str(path))
    lines = [json.loads(l) for l in path.read_text().splitlines()]
    kinds = {(e["kind"], e["n"]) for e in lines}
    if cfg["az_model"] == "lfm":
        want = {("fused", cfg["Nr"]), ("fused", cfg["Na"]), ("batch_fused", cfg["Nr"]),
                ("batch_fused", cfg["Na"]), ("turn", cfg["Nr"])}
    else:
        want = {("fused", cfg["Nr"]), ("fwd", cfg["Na"]), ("rcmc", cfg["Na"]), ("turn", cfg["Nr"])}
    assert kinds == want
    for e in lines:
        assert e["arch"] == arch()
        assert e["us_best"] <= e["us_default"]
        assert sar.sar_tune_variant(KINDS.index(e["kind"]), e["n"], 0) == e["variant"]
        print(e)
    # tuning again merges (same keys replaced, not duplicated)
    sar.sar_autotune(sar.make_params(cfg), str(path))
    assert len(path.read_text().splitlines()) == len(lines)
    img = run(cfg, sc.raw)
    assert rel_l2(img, ref) <= 1e-5


@pytest.mark.parametrize("rcmc_variant", [0, 1, 2, 3, 4, 5])
def test_hyperbolic_variants_match_oracle(tmp_path, rcmc_variant):
    cfg, sc, ref = scene("c2")
    base = run(cfg, sc.raw)
    tw = rcmc_variant & 1
    write_cache(tmp_path / "t.jsonl", [("fused", cfg["Nr"], 0, tw), ("fwd", cfg["Na"], 0, tw),
                                       ("rcmc", cfg["Na"], 0, rcmc_variant)])
    assert sar.sar_tune_variant(_lib.TUNE_RCMC, cfg["Na"], 0) == rcmc_variant
    img = run(cfg, sc.raw)
    e_ref, e_base = rel_l2(img, ref), rel_l2(img, base)
    print(f"RCMC variant {rcmc_variant}: vs oracle {e_ref:.3e}, vs default {e_base:.3e}")
    assert e_ref <= 1e-5 and e_base <= 1e-6


@pytest.mark.parametrize("rcmc_variant", [4, 5])
def test_wide_rcmc_8192_matches_oracle(tmp_path, rcmc_variant):
    """The wide two-row RCMC kernel (two line slots' threads per row pair)
    on 8192-point azimuth lines, with product and table twiddles."""
    cfg, sc, ref = scene("c2", Na=8192, Nr=1024, range_len=256, range_tbp=100.0, n_targets=2)
    base = run(cfg, sc.raw)
    tw = rcmc_variant & 1
    write_cache(tmp_path / "t.jsonl", [("fused", cfg["Nr"], 0, tw), ("fwd", cfg["Na"], 0, tw),
                                       ("rcmc", cfg["Na"], 0, rcmc_variant)])
    assert sar.sar_tune_variant(_lib.TUNE_RCMC, cfg["Na"], 0) == rcmc_variant
    img = run(cfg, sc.raw)
    e_ref, e_base = rel_l2(img, ref), rel_l2(img, base)
    print(f"RCMC variant {rcmc_variant}, Na 8192: vs oracle {e_ref:.3e}, vs default {e_base:.3e}")
    assert e_ref <= 1e-5 and e_base <= 1e-6


@pytest.mark.parametrize("prec,tol", [("split_fp16", 1e-5), ("split_bf16", 3e-4)])
def test_split_one_row_rcmc_matches_oracle(tmp_path, prec, tol):
    """The one-row RCMC kernel in the split precisions (the only non-default
    variant the tuner may pick for them)."""
    cfg, sc, ref = scene("c2", Na=4096, Nr=1024, range_len=256, range_tbp=100.0, n_targets=3)
    p = {"split_fp16": 1, "split_bf16": 2}[prec]
    write_cache(tmp_path / "t.jsonl", [("rcmc", cfg["Na"], p, 2)])
    assert sar.sar_tune_variant(_lib.TUNE_RCMC, cfg["Na"], p) == 2
    img = run(cfg, sc.raw, precision=prec)
    err = rel_l2(img, ref)
    print(f"{prec} one-row RCMC: vs oracle {err:.3e}")
    assert err <= tol
    for t in sc.targets:
        sub = np.abs(img[t["m"] - 8:t["m"] + 9, t["n"] - 8:t["n"] + 9])
        assert np.unravel_index(int(np.argmax(sub)), sub.shape) == (8, 8)


@pytest.mark.parametrize("schedule", ["fused", "unfused"])
def test_lfm_table_twiddles_match_oracle(tmp_path, schedule):
    cfg, sc, ref = scene("c1")
    base = run(cfg, sc.raw, schedule=schedule)
    n = cfg["Nr"]
    write_cache(tmp_path / "t.jsonl", [(k, n, 0, 1) for k in ("fused", "fwd", "inv")])
    img = run(cfg, sc.raw, schedule=schedule)
    assert rel_l2(img, ref) <= 1e-5 and rel_l2(img, base) <= 1e-6


@pytest.mark.parametrize("variant", [0, 1, 4, 5, 8, 9, 12, 13])
def test_batch_variants_bit_identical_to_single(tmp_path, variant):
    torch = torch_cuda()
    cfgs = batch_configs(seed=4, n=64, nr_choices=(256, 512, 1024), na_choices=(256, 512))[:5]
    sizes = sorted({c["Nr"] for c in cfgs} | {c["Na"] for c in cfgs})
    write_cache(tmp_path / "t.jsonl", [("fused", n, 0, variant & 1) for n in sizes] +
                [("batch_fused", n, 0, variant) for n in sizes])
    scenes = [simulate(c) for c in cfgs]
    params = [sar.make_params(c) for c in cfgs]
    stream = torch.cuda.Stream()
    b = sar.sar_batch_plan(params, stream)
    try:
        raws = [dev(s.raw) for s in scenes]
        imgs = [torch.empty(s.raw.shape[::-1], dtype=torch.complex64, device="cuda")
                for s in scenes]
        work = torch.empty(sar.sar_batch_workspace_bytes(b) // 8 + 1, dtype=torch.complex64,
                           device="cuda")
        for _ in range(2):
            sar.sar_batch_execute(b, raws, imgs, work, stream)
        stream.synchronize()
        for c, s, img in zip(cfgs, scenes, imgs):
            single = run(c, s.raw)
            assert np.array_equal(host(img).T, single)
    finally:
        sar.sar_batch_destroy(b)


def _lfm_plan_cfg(n):
    return dict(Nr=n, Na=64, range_len=max(2, n // 4), range_tbp=max(1.0, n / 8.0),
                az_model="lfm", az_len=32, az_tbp=8.0, lam=0.0, v=0.0, r_near=0.0,
                rcmc_taps=0, rcmc_beta=2.5)


@pytest.mark.parametrize("n", [64, 512, 4096, 16384])
@pytest.mark.parametrize("inverse", [0, 1])
def test_split_layout_line_fft_bit_identical(tmp_path, n, inverse):
    """Forward / inverse variants 2 and 3 exchange real and imaginary parts
    through two LDS float arrays; the butterflies are the same, so each is
    bit-identical to variant 0 / 1, and within FP32 rounding of the oracle."""
    from gpu_util import empty, rand_c64
    rng = np.random.Generator(np.random.PCG64(900 + n + inverse))
    lines = 2 * max(1, 256 // (n // 16)) + 3
    x = rand_c64(rng, (lines, n))
    kind = "inv" if inverse else "fwd"
    outs = {}
    for v in (0, 1, 2, 3):
        write_cache(tmp_path / f"v{v}.jsonl", [(kind, n, 0, v)])
        assert sar.sar_tune_variant(KINDS.index(kind), n, 0) == v
        with sar.Plan(_lfm_plan_cfg(n)) as p:
            out = empty((lines, n))
            sar.sar_fft_lines(p.handle, 0, inverse, dev(x), out, lines)
            outs[v] = host(out)
    assert np.array_equal(outs[2].view(np.uint32), outs[0].view(np.uint32))
    assert np.array_equal(outs[3].view(np.uint32), outs[1].view(np.uint32))
    ref = np.stack([O.fft(r, inverse=bool(inverse)) for r in x])
    assert rel_l2(outs[2], ref) < 2e-6


@pytest.mark.parametrize("rows, cols", [(4096, 4096), (256, 4096), (2048, 512), (64, 128)])
@pytest.mark.parametrize("variant", [0, 1, 2])
def test_corner_turn_grids_bit_exact(tmp_path, rows, cols, variant):
    """Every corner-turn grid the tuner can choose (five or four workgroups
    per CU, or one per tile) moves every sample to its transposed place."""
    torch = torch_cuda()
    write_cache(tmp_path / "t.jsonl", [("turn", cols, 0, variant)])
    cfg = config("c1", Nr=cols, Na=rows, range_len=min(64, cols // 2), range_tbp=16.0,
                 az_len=min(64, rows // 2), az_tbp=16.0)
    rng = np.random.Generator(np.random.PCG64(900 + rows + cols + variant))
    x = (rng.standard_normal((rows, cols)) + 1j * rng.standard_normal((rows, cols))).astype(np.complex64)
    out = torch.empty((cols, rows), dtype=torch.complex64, device="cuda")
    with sar.Plan(cfg) as p:
        sar.sar_corner_turn(p.handle, dev(x), out, rows, cols)
        got = host(out)
    assert np.array_equal(got.view(np.uint32), np.ascontiguousarray(x.T).view(np.uint32))


@pytest.mark.parametrize("name, na", [("c1", 4096), ("c2", 4096), ("c1", 1024), ("c1", 256)])
def test_strip_widths_bit_identical(tmp_path, name, na):
    """Half-width turn-free strips give the default width's image bit for
    bit (LFM and hyperbolic; 4096-point lines in strips of two, 1024- and
    256-point lines in strips of eight)."""
    if name == "c1":
        cfg = config("c1", Nr=512, Na=na, range_len=64, range_tbp=32.0, az_len=min(64, na // 2),
                     az_tbp=min(32.0, na / 4), n_targets=1, spacing=4)
        sc = simulate(cfg)
    else:
        cfg, sc, _ = scene("c2")
    base = np.ascontiguousarray(run(cfg, sc.raw, schedule="turn_free"))
    write_cache(tmp_path / "t.jsonl", [("strip", cfg["Na"], 0, 1)])
    assert sar.sar_tune_variant(_lib.TUNE_STRIP, cfg["Na"], 0) == 1
    half = np.ascontiguousarray(run(cfg, sc.raw, schedule="turn_free"))
    assert np.array_equal(half.view(np.uint32), base.view(np.uint32))


def test_autotune_turn_free_tunes_strips(tmp_path):
    """A turn-free plan has no corner turn: the tuner times its strip widths
    instead, and the plan built afterwards uses the winner."""
    cfg, sc, ref = scene("c2")
    path = tmp_path / "tune.jsonl"
    sar.sar_autotune(sar.make_params(cfg, schedule="turn_free"), str(path))
    lines = [json.loads(l) for l in path.read_text().splitlines()]
    kinds = {(e["kind"], e["n"]) for e in lines}
    assert ("strip", cfg["Na"]) in kinds and not any(k == "turn" for k, _ in kinds), kinds
    sar.sar_tune_load(str(path))
    img = run(cfg, sc.raw, schedule="turn_free")
    assert rel_l2(img, ref) <= 1e-5


@pytest.mark.parametrize("n", [256, 1024, 4096, 8192])
@pytest.mark.parametrize("kind", ["fused", "fwd", "inv"])
@pytest.mark.parametrize("tab", [0, 1])
def test_double_lines_per_workgroup_bit_identical(tmp_path, n, kind, tab):
    """Twice the default lines per workgroup (variant bit 2) runs the same
    per-line transforms: bit-identical to the default grouping.  The forward
    and inverse cases use a line count that leaves the last workgroup partly
    empty; the fused one runs over the plan's 64 lines."""
    torch = torch_cuda()
    lines = 64 if kind == "fused" else 3 * 2 * max(1, 256 // (n // 16)) + 1
    cfg = config("c1", Nr=n, Na=64, range_len=max(2, n // 8), range_tbp=max(1.0, n / 16),
                 az_len=16, az_tbp=8.0)
    rng = np.random.Generator(np.random.PCG64(1000 + n + tab))
    x = dev((rng.standard_normal((lines, n)) + 1j * rng.standard_normal((lines, n)))
            .astype(np.complex64))
    outs = []
    for v in (tab, tab | 4):
        write_cache(tmp_path / f"t{v}.jsonl", [(kind, n, 0, v)])
        assert sar.sar_tune_variant(KINDS.index(kind), n, 0) == v
        out = torch.empty((lines, n), dtype=torch.complex64, device="cuda")
        with sar.Plan(cfg) as p:
            if kind == "fused":
                sar.sar_range_compress(p.handle, x, out)
            else:
                sar.sar_fft_lines(p.handle, 0, int(kind == "inv"), x, out, lines)
            outs.append(host(out))
    assert np.array_equal(outs[0].view(np.uint32), outs[1].view(np.uint32))
