"""Each HIP kernel through the C ABI against the matching oracle stage.

Tolerances: FP32 kernels vs the FP64 oracle, relative L2 per case.  One FFT
of length N in FP32 has an error of order u * sqrt(log2 N) (u = 6e-8), so
1e-6 bounds a line FFT, a line compression and one azimuth stage; data
movement (corner turn) must be bit-exact.
"""
import math

import numpy as np
import pytest

import paper_2604_03585_amd as sar
from gpu_util import dev, empty, host, rand_c64, rel_l2
from oracle import oracle as O
from sarsim import config

pytestmark = pytest.mark.gpu

SIZES = [64, 128, 256, 512, 1024, 2048, 4096, 8192, 16384]
TOL_STAGE = 1e-6


def lfm_cfg(nr, na, lr=None, la=None):
    lr = lr or max(2, nr // 4)
    la = la or max(2, na // 4)
    return dict(Nr=nr, Na=na, range_len=lr, range_tbp=lr / 2.0, az_model="lfm",
                az_len=la, az_tbp=la / 2.0, lam=0.0, v=0.0, r_near=0.0,
                rcmc_taps=0, rcmc_beta=2.5)


def lines_for(n):
    """A ragged line count: several workgroups plus a partial one."""
    per_wg = max(1, 256 // (n // 16))
    return 2 * per_wg + 3


@pytest.fixture(scope="module")
def plans():
    made = {}

    def get(cfg, schedule="fused"):
        key = (tuple(sorted(cfg.items())), schedule)
        if key not in made:
            made[key] = sar.Plan(cfg, schedule=schedule)
        return made[key]
    yield get
    import torch
    torch.cuda.synchronize()
    for p in made.values():
        p.close()


def test_tables_match_oracle(plans):
    for cfg in (config("c1"), lfm_cfg(4096, 1024, 512, 128), lfm_cfg(16384, 64, 2048, 8)):
        p = plans(cfg)
        Hr = sar.sar_plan_get_table(p.handle, 0)
        ref = O.matched_filter(cfg["Nr"], cfg["range_len"], cfg["range_tbp"], +1) / cfg["Nr"]
        assert rel_l2(Hr, ref) < 2e-7
        Ha = sar.sar_plan_get_table(p.handle, 1)
        ref = O.matched_filter(cfg["Na"], cfg["az_len"], cfg["az_tbp"], -1) / cfg["Na"]
        assert rel_l2(Ha, ref) < 2e-7
    c2 = config("c2")
    p = plans(c2)
    st = sar.sar_plan_get_table(p.handle, 2)
    rt = sar.sar_plan_get_table(p.handle, 3)
    k = np.arange(c2["Na"])
    f = np.where(k < c2["Na"] // 2, k, k - c2["Na"]) / c2["Na"]
    D = np.sqrt(1.0 - (c2["lam"] * f / (2 * c2["v"])) ** 2)
    assert np.max(np.abs(st - (1.0 / D - 1.0))) < 1e-15
    assert np.max(np.abs(rt / (2.0 * D / c2["lam"]) - 1.0)) < 1e-15


def test_rcmc_weight_table_matches_oracle(plans):
    """The plan's piecewise-quadratic weights reproduce the exact Kaiser-sinc
    weights of the oracle to < 1e-7 everywhere on [0, 1) (fit error 2.2e-8
    plus the FP32 rounding of the coefficients)."""
    p = plans(config("c2"))
    tab = sar.sar_plan_get_table(p.handle, 4).astype(np.float64)
    nb = sar._lib.RCMC_INTERVALS
    c = tab.reshape(nb, 8, 3)
    worst = 0.0
    for x in np.concatenate([np.linspace(0, 1, 4001, endpoint=False), [1 - 1e-9, 0.5, 1e-7]]):
        b = min(int(x * nb), nb - 1)
        u = x * nb - b
        w = c[b, :, 0] + u * (c[b, :, 1] + u * c[b, :, 2])
        worst = max(worst, float(np.max(np.abs(w - O.rcmc_weights(x, 2.5, 8)))))
    print(f"RCMC weight table: max error {worst:.3e}")
    assert worst < 1e-7, worst


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("inverse", [0, 1])
def test_line_fft(n, inverse, plans):
    rng = np.random.Generator(np.random.PCG64(100 + n + inverse))
    lines = lines_for(n)
    x = rand_c64(rng, (lines, n))
    p = plans(lfm_cfg(n, 64))
    out = empty((lines, n))
    sar.sar_fft_lines(p.handle, 0, inverse, dev(x), out, lines)
    got = host(out)
    ref = np.stack([O.fft(r, inverse=bool(inverse)) for r in x])
    assert rel_l2(got, ref) < TOL_STAGE


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("schedule", ["fused", "unfused"])
def test_range_compress(n, schedule, plans):
    rng = np.random.Generator(np.random.PCG64(200 + n))
    na = 64
    cfg = lfm_cfg(n, na)
    x = rand_c64(rng, (na, n))
    p = plans(cfg, schedule)
    out = empty((na, n))
    sar.sar_range_compress(p.handle, dev(x), out)
    ref = O.compress_rows(x, O.matched_filter(n, cfg["range_len"], cfg["range_tbp"], +1))
    assert rel_l2(host(out), ref) < TOL_STAGE


def test_range_compress_in_place_and_line_count(plans):
    """in == out is allowed; a line count that is not a multiple of the lines
    per workgroup leaves nothing out."""
    rng = np.random.Generator(np.random.PCG64(7))
    cfg = lfm_cfg(256, 128)
    x = rand_c64(rng, (128, 256))
    p = plans(cfg)
    buf = dev(x)
    sar.sar_range_compress(p.handle, buf, buf)
    ref = O.compress_rows(x, O.matched_filter(256, cfg["range_len"], cfg["range_tbp"], +1))
    assert rel_l2(host(buf), ref) < TOL_STAGE


@pytest.mark.parametrize("shape", [(64, 64), (256, 4096), (4096, 256), (100, 37), (1, 5),
                                   (130, 200), (2048, 2048)])
def test_corner_turn_bit_exact(shape):
    rng = np.random.Generator(np.random.PCG64(300 + shape[0]))
    x = rand_c64(rng, shape)
    out = empty((shape[1], shape[0]))
    sar.sar_corner_turn(0, dev(x), out, shape[0], shape[1])
    got = host(out)
    assert np.array_equal(got.view(np.uint32), np.ascontiguousarray(x.T).view(np.uint32))


@pytest.mark.parametrize("na", [64, 1024, 4096, 16384])
@pytest.mark.parametrize("schedule", ["fused", "unfused"])
def test_azimuth_lfm(na, schedule, plans):
    rng = np.random.Generator(np.random.PCG64(400 + na))
    nr = 64
    cfg = lfm_cfg(nr, na)
    x = rand_c64(rng, (nr, na))
    p = plans(cfg, schedule)
    out = empty((nr, na))
    sar.sar_azimuth_compress(p.handle, dev(x), out)
    ref = O.compress_rows(x, O.matched_filter(na, cfg["az_len"], cfg["az_tbp"], -1))
    assert rel_l2(host(out), ref) < TOL_STAGE


def hyper_cfg(nr, na, taps=8):
    lr = min(512, nr // 2)
    return config("c2", Nr=nr, Na=na, rcmc_taps=taps, range_len=lr,
                  range_tbp=min(200.0, lr / 2.0))


@pytest.mark.parametrize("nr, na", [(64, 64), (256, 512), (512, 4096), (4096, 4096)])
@pytest.mark.parametrize("schedule", ["fused", "unfused"])
def test_azimuth_fft_and_rcmc(nr, na, schedule, plans):
    rng = np.random.Generator(np.random.PCG64(500 + nr + na))
    cfg = hyper_cfg(nr, na)
    x = rand_c64(rng, (nr, na))
    p = plans(cfg, schedule)
    A = empty((nr, na))
    sar.sar_azimuth_fft(p.handle, dev(x), A)
    A_h = host(A)
    A_ref = O.fft_rows(x)
    assert rel_l2(A_h, A_ref) < TOL_STAGE
    out = empty((nr, na))
    sar.sar_rcmc_azimuth(p.handle, A, out)
    ref = O.rcmc_azimuth(A_h, cfg["lam"], cfg["v"], cfg["r_near"], 8, cfg["rcmc_beta"])
    assert rel_l2(host(out), ref) < TOL_STAGE


def test_rcmc_disabled(plans):
    rng = np.random.Generator(np.random.PCG64(600))
    cfg = hyper_cfg(128, 256, taps=0)
    A = rand_c64(rng, (128, 256))
    p = plans(cfg)
    out = empty((128, 256))
    sar.sar_rcmc_azimuth(p.handle, dev(A), out)
    ref = O.rcmc_azimuth(A, cfg["lam"], cfg["v"], cfg["r_near"], 0, cfg["rcmc_beta"])
    assert rel_l2(host(out), ref) < TOL_STAGE


def test_rcmc_edge_rows(plans):
    """Rows near both scene edges read taps outside [0, Nr), which count 0."""
    cfg = hyper_cfg(64, 4096)
    A = np.zeros((64, 4096), np.complex64)
    A[0, :] = 1.0
    A[63, :] = 1.0 + 1.0j
    p = plans(cfg)
    out = empty((64, 4096))
    sar.sar_rcmc_azimuth(p.handle, dev(A), out)
    ref = O.rcmc_azimuth(A, cfg["lam"], cfg["v"], cfg["r_near"], 8, cfg["rcmc_beta"])
    assert rel_l2(host(out), ref) < TOL_STAGE


def test_execute_rejects_aliasing(plans):
    cfg = config("c1")
    p = plans(cfg)
    buf = empty((3, 256, 256))
    with pytest.raises(sar.SarError) as ei:
        sar.sar_rda_execute(p.handle, buf[0], buf[0], buf[1])
    assert ei.value.status == sar._lib.SAR_ERR_ALIAS
    with pytest.raises(sar.SarError):
        sar.sar_corner_turn(p.handle, buf[0], buf[0], 256, 256)


def test_time_next_launch_brackets_one_kernel():
    """The armed events record the next launch only: a corner turn of 128 MiB
    timed by its own dispatch takes between the time of moving its bytes at
    16 TB/s and 10 ms, and the launch after it leaves the events alone."""
    import torch
    rng = np.random.Generator(np.random.PCG64(31))
    x = dev(rand_c64(rng, (4096, 4096)))
    out = empty((4096, 4096))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s = torch.cuda.current_stream()
    e0.record(s)
    e1.record(s)
    torch.cuda.synchronize()
    sar.sar_time_next_launch(e0, e1)
    sar.sar_corner_turn(0, x, out, 4096, 4096)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    assert 2 * 4096 * 4096 * 8 / 16e12 * 1e3 < ms < 10.0, ms
    sar.sar_corner_turn(0, out, x, 4096, 4096)      # not armed: events unchanged
    torch.cuda.synchronize()
    assert e0.elapsed_time(e1) == ms
    print(f"corner turn 4096^2 by its own dispatch: {ms * 1e3:.1f} us")
