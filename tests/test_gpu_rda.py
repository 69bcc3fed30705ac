"""End-to-end parity of the HIP Range Doppler Algorithm with the FP64 oracle.

Acceptance (FP32): relative L2 <= 1e-5 against the oracle image, peak cells
equal to the oracle's and to the seeded cells, |dPSLR|, |dISLR| <= 0.1 dB,
|dSNR| <= 0.05 dB; fused vs unfused FP32 within 1e-6.
"""
import numpy as np
import pytest

import paper_2604_03585_amd as sar
from gpu_util import dev, empty, host, rel_l2
from oracle import oracle as O
from oracle import quality as Q
from sarsim import config, simulate

pytestmark = pytest.mark.gpu

TOL_RDA = 1e-5


def guard_half(cfg):
    return (16, 32) if cfg["Nr"] <= 256 else (64, 64)


_cache = {}


def scene_and_oracle(name, **over):
    key = (name, tuple(sorted(over.items())))
    if key not in _cache:
        cfg = config(name, **over)
        sc = simulate(cfg)
        _cache[key] = (cfg, sc, O.rda(sc.raw, cfg))
    return _cache[key]


def run_gpu(cfg, raw, schedule="fused", transpose_back=0):
    with sar.Plan(cfg, schedule=schedule, transpose_back=transpose_back) as p:
        img = p.execute(dev(raw))
        out = host(img)
    return out if transpose_back else out.T


@pytest.mark.parametrize("name", ["c1", "c2"])
@pytest.mark.parametrize("schedule", ["fused", "unfused", "turn_free"])
def test_rda_parity(name, schedule):
    cfg, sc, ref = scene_and_oracle(name)
    img = run_gpu(cfg, sc.raw, schedule)
    err = rel_l2(img, ref)
    print(f"{name} {schedule}: rel L2 {err:.3e}  max abs {Q.max_abs(img, ref):.3e}")
    assert err <= TOL_RDA
    guard, half = guard_half(cfg)
    rg = Q.point_target_report(img, sc.targets, guard, half)
    ro = Q.point_target_report(ref, sc.targets, guard, half)
    for t, a, b in zip(sc.targets, rg, ro):
        assert a["peak"] == b["peak"] == (t["m"], t["n"])
        for key in ("pslr_range", "islr_range", "pslr_azimuth", "islr_azimuth"):
            assert abs(a[key] - b[key]) <= 0.1, key
        assert abs(a["snr_db"] - b["snr_db"]) <= 0.05


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_fused_matches_unfused(name):
    cfg, sc, _ = scene_and_oracle(name)
    a = run_gpu(cfg, sc.raw, "fused")
    b = run_gpu(cfg, sc.raw, "unfused")
    assert rel_l2(a, b) < 1e-6


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_transpose_back(name):
    cfg, sc, ref = scene_and_oracle(name)
    img = run_gpu(cfg, sc.raw, "fused", transpose_back=1)
    assert rel_l2(img, ref) <= TOL_RDA


def test_repeat_runs_bit_identical():
    cfg, sc, _ = scene_and_oracle("c2")
    with sar.Plan(cfg) as p:
        raw = dev(sc.raw)
        a = host(p.execute(raw))
        for _ in range(3):
            b = host(p.execute(raw))
            assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


@pytest.mark.parametrize("nr, na", [(64, 64), (16384, 64), (64, 16384), (512, 2048)])
def test_extreme_shapes(nr, na):
    """Smallest and largest line lengths on both axes (LFM geometry)."""
    cfg = config("c1", Nr=nr, Na=na, range_len=min(64, nr // 2), range_tbp=min(32, nr // 4),
                 az_len=min(64, na // 2), az_tbp=min(32, na // 4), n_targets=1, spacing=4)
    sc = simulate(cfg)
    ref = O.rda(sc.raw, cfg)
    img = run_gpu(cfg, sc.raw)
    assert rel_l2(img, ref) <= TOL_RDA
    t = sc.targets[0]
    assert Q.peak_cell(img, t["m"], t["n"]) == (t["m"], t["n"])


@pytest.mark.parametrize("nr, na", [(16384, 64), (64, 16384), (256, 8192)])
@pytest.mark.parametrize("schedule", ["fused", "unfused"])
def test_extreme_shapes_hyperbolic(nr, na, schedule):
    """Longest azimuth lines through RCMC (16384 points: the two-row kernel at
    its largest line, 1024 threads per line) and longest range lines, in the
    hyperbolic geometry."""
    lr = min(512, nr // 2)
    cfg = config("c2", Nr=nr, Na=na, range_len=lr, range_tbp=min(200.0, lr / 2.0),
                 n_targets=1, spacing=8, exposure=min(1024, na // 2))
    sc = simulate(cfg)
    ref = O.rda(sc.raw, cfg)
    img = run_gpu(cfg, sc.raw, schedule)
    err = rel_l2(img, ref)
    print(f"hyperbolic {nr}x{na} {schedule}: rel L2 {err:.3e}")
    assert err <= TOL_RDA
    t = sc.targets[0]
    assert Q.peak_cell(img, t["m"], t["n"]) == Q.peak_cell(ref, t["m"], t["n"])


def test_noise_only_scene():
    """A scene with no targets (the image is compressed noise only)."""
    cfg, sc, ref = scene_and_oracle("c1", n_targets=0)
    img = run_gpu(cfg, sc.raw)
    assert rel_l2(img, ref) <= TOL_RDA


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_turn_free_bit_identical_to_fused(name):
    """The turn-free schedule reads strips of azimuth lines straight from the
    range output instead of turning it; the butterflies are the same, so the
    image equals the fused schedule's bit for bit."""
    cfg, sc, _ = scene_and_oracle(name)
    a = np.ascontiguousarray(run_gpu(cfg, sc.raw, "fused"))
    b = np.ascontiguousarray(run_gpu(cfg, sc.raw, "turn_free"))
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


@pytest.mark.parametrize("nr, na, model", [(64, 64, "c1"), (4096, 64, "c1"), (64, 4096, "c1"),
                                           (128, 2048, "c1"), (1024, 512, "c1"),
                                           (512, 4096, "c2"), (1024, 1024, "c2"),
                                           (256, 2048, "c2")])
def test_turn_free_shapes(nr, na, model):
    """Every strip width (16 lines up to 1024 points, 8 at 2048, 4 at 4096)
    and the narrowest scenes, LFM and hyperbolic, against the oracle and bit
    for bit against the fused schedule."""
    if model == "c1":
        cfg = config("c1", Nr=nr, Na=na, range_len=min(64, nr // 2), range_tbp=min(32, nr // 4),
                     az_len=min(64, na // 2), az_tbp=min(32, na // 4), n_targets=1, spacing=4)
    else:
        lr = min(512, nr // 2)
        cfg = config("c2", Nr=nr, Na=na, range_len=lr, range_tbp=min(200.0, lr / 2.0),
                     n_targets=1, spacing=8, exposure=min(1024, na // 2))
    sc = simulate(cfg)
    ref = O.rda(sc.raw, cfg)
    img = run_gpu(cfg, sc.raw, "turn_free")
    err = rel_l2(img, ref)
    print(f"turn-free {model} {nr}x{na}: rel L2 {err:.3e}")
    assert err <= TOL_RDA
    fused = np.ascontiguousarray(run_gpu(cfg, sc.raw, "fused"))
    assert np.array_equal(np.ascontiguousarray(img).view(np.uint32), fused.view(np.uint32))
