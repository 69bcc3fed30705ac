"""Split-precision variant: radix-16 butterflies as DFT matmuls on MFMA with
hi+lo FP16 or BF16 operands and FP32 accumulation (twiddles, filters, RCMC
and phases stay in FP32, tables from FP64).

Every line is scaled by a power of two of its own before its values are
split (its largest component lands in [2^14, 2^15)), so FP16 neither
overflows nor loses its lo parts to subnormals whatever the input's scale:
scaling the input by 2^k scales the output by exactly 2^k.

Stated accuracy (checked here against the FP64 oracle):
  split FP16: each operand keeps 22 significand bits (11 + 11), so a line
  FFT stays within 2e-6 and the whole RDA within 1e-5 relative L2, the
  FP32 acceptance bar;
  split BF16: 16 significand bits (8 + 8), error ~2^-16 per pass: line FFT
  within 1e-4, RDA within 3e-4 relative L2.
Peak cells must equal the oracle's in both.
"""
import numpy as np
import pytest

import paper_2604_03585_amd as sar
from gpu_util import dev, empty, host, rand_c64, rel_l2
from oracle import oracle as O
from oracle import quality as Q
from sarsim import config, simulate

pytestmark = pytest.mark.gpu

PRECS = ["split_fp16", "split_bf16"]
TOL_FFT = {"split_fp16": 2e-6, "split_bf16": 1e-4}
TOL_RDA = {"split_fp16": 1e-5, "split_bf16": 3e-4}
SIZES = [64, 256, 512, 4096, 8192, 16384]


def lfm_cfg(nr, na):
    return dict(Nr=nr, Na=na, range_len=max(2, nr // 4), range_tbp=max(1.0, nr / 8.0),
                az_model="lfm", az_len=max(2, na // 4), az_tbp=max(1.0, na / 8.0),
                lam=0.0, v=0.0, r_near=0.0, rcmc_taps=0, rcmc_beta=2.5)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("inverse", [0, 1])
def test_split_line_fft(prec, n, inverse):
    rng = np.random.Generator(np.random.PCG64(700 + n + inverse))
    lines = 2 * max(1, 256 // (n // 16)) + 3
    x = rand_c64(rng, (lines, n))
    with sar.Plan(lfm_cfg(n, 64), precision=prec) as p:
        out = empty((lines, n))
        sar.sar_fft_lines(p.handle, 0, inverse, dev(x), out, lines)
        got = host(out)
    ref = np.stack([O.fft(r, inverse=bool(inverse)) for r in x])
    err = rel_l2(got, ref)
    print(f"{prec} N={n} inv={inverse}: rel L2 {err:.3e}")
    assert err < TOL_FFT[prec]


_cache = {}


def scene(name):
    if name not in _cache:
        cfg = config(name)
        sc = simulate(cfg)
        _cache[name] = (cfg, sc, O.rda(sc.raw, cfg))
    return _cache[name]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("name", ["c1", "c2"])
@pytest.mark.parametrize("schedule", ["fused", "unfused"])
def test_split_rda(prec, name, schedule):
    cfg, sc, ref = scene(name)
    with sar.Plan(cfg, precision=prec, schedule=schedule) as p:
        img = host(p.execute(dev(sc.raw))).T
    err = rel_l2(img, ref)
    guard, half = (16, 32) if cfg["Nr"] <= 256 else (64, 64)
    rg = Q.point_target_report(img, sc.targets, guard, half)
    ro = Q.point_target_report(ref, sc.targets, guard, half)
    d = {k: max(abs(a[k] - b[k]) for a, b in zip(rg, ro))
         for k in ("snr_db", "pslr_range", "islr_range", "pslr_azimuth", "islr_azimuth")}
    print(f"{prec} {name} {schedule}: rel L2 {err:.3e} max abs {Q.max_abs(img, ref):.3e} "
          + " ".join(f"d{k}={v:.4f}" for k, v in d.items()))
    assert err <= TOL_RDA[prec]
    for t, a, b in zip(sc.targets, rg, ro):
        assert a["peak"] == b["peak"] == (t["m"], t["n"])


SCALES = [-20, -12, 12, 16, 20]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("k", SCALES)
def test_split_line_fft_scaled(prec, k):
    """Line FFTs of inputs scaled by 2^k: within the same bar as unit-scale
    inputs against the scaled oracle, and exactly 2^k times the unit-scale
    output (the per-line exponent absorbs the scale)."""
    n = 4096
    rng = np.random.Generator(np.random.PCG64(770 + k))
    x = rand_c64(rng, (5, n))
    x[2] *= 1e-3                                    # lines of different scales
    x[3, 17] = 300.0 + 200.0j                       # a spike over the noise
    xs = (x * np.float32(2.0 ** k)).astype(np.complex64)
    with sar.Plan(lfm_cfg(n, 64), precision=prec) as p:
        out1, outk = empty((5, n)), empty((5, n))
        sar.sar_fft_lines(p.handle, 0, 0, dev(x), out1, 5)
        sar.sar_fft_lines(p.handle, 0, 0, dev(xs), outk, 5)
        g1, gk = host(out1), host(outk)
    assert np.array_equal(gk, (g1 * np.float32(2.0 ** k)).astype(np.complex64))
    ref = np.stack([O.fft(r) for r in x.astype(np.complex128)]) * 2.0 ** k
    for i in range(5):
        assert rel_l2(gk[i], ref[i]) < TOL_FFT[prec], i


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("k", [-12, 12, 16])
def test_split_rda_scaled(prec, k):
    """The c2 scene with its raw data scaled by 2^k (-12: a weak scene whose
    lo parts would go subnormal; +12, +16: ADC-count-like magnitudes whose
    range-compressed peaks exceed FP16's 65504 without the per-line scale):
    within the unit-scale bar against the equally scaled oracle, peaks at the
    seeded cells, and exactly 2^k times the unit-scale image."""
    cfg, sc, ref = scene("c2")
    raw_k = (sc.raw * np.float32(2.0 ** k)).astype(np.complex64)
    with sar.Plan(cfg, precision=prec) as p:
        img1 = host(p.execute(dev(sc.raw)))
        imgk = host(p.execute(dev(raw_k)))
    assert np.array_equal(imgk, (img1 * np.float32(2.0 ** k)).astype(np.complex64))
    img = imgk.T
    err = rel_l2(img, ref * 2.0 ** k)
    print(f"{prec} c2 x 2^{k}: rel L2 {err:.3e}")
    assert err <= TOL_RDA[prec]
    for t in sc.targets:
        sub = np.abs(img[t["m"] - 8:t["m"] + 9, t["n"] - 8:t["n"] + 9])
        assert np.unravel_index(int(np.argmax(sub)), sub.shape) == (8, 8)
