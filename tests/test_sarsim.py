"""Seeded scene generator: determinism, placement rules, noise level (CPU)."""
import numpy as np

from sarsim import batch_configs, config, serve_pool_configs, simulate


def test_deterministic_per_seed():
    a = simulate(config("c1"))
    b = simulate(config("c1"))
    assert np.array_equal(a.raw.view(np.uint8), b.raw.view(np.uint8))
    assert a.targets == b.targets
    c = simulate(config("c1", seed=99))
    assert not np.array_equal(a.raw, c.raw)


def test_target_placement_rules():
    cfg = config("c1")
    sc = simulate(cfg)
    La, Lr = cfg["az_len"], cfg["range_len"]
    cells = [(t["m"], t["n"]) for t in sc.targets]
    assert len(cells) == cfg["n_targets"]
    for m, n in cells:
        assert La // 2 <= m <= cfg["Na"] - La // 2
        assert Lr // 2 <= n <= cfg["Nr"] - Lr // 2
    for i in range(len(cells)):
        for j in range(i):
            assert abs(cells[i][0] - cells[j][0]) >= 16
            assert abs(cells[i][1] - cells[j][1]) >= 16


def test_noise_variance():
    cfg = config("c1", Na=512, Nr=512, n_targets=0)
    sc = simulate(cfg)
    v = np.mean(np.abs(sc.raw.astype(np.complex128)) ** 2)
    assert abs(v / cfg["sigma2"] - 1.0) < 0.01
    assert abs(np.mean(sc.raw.real ** 2) / np.mean(sc.raw.imag ** 2) - 1.0) < 0.02


def test_hyperbolic_echo_migrates():
    """The echo centre follows R(m) - r_near: at the aperture edge the range
    chirp has moved by the expected migration (<= 8 cells at near range)."""
    cfg = config("c2", Na=2048, Nr=1024)
    sc = simulate(cfg, noise=False, targets=[(1000, 400)])
    R0 = cfg["r_near"] + 400
    mig = np.sqrt(R0 ** 2 + (cfg["v"] * 512) ** 2) - R0
    assert 7.0 < mig <= 8.0
    row_c = np.abs(sc.raw[1000])
    row_e = np.abs(sc.raw[1000 - 512])
    # support [n_k + delay - L/2, n_k + delay + L/2) -> first nonzero column
    first_c = int(np.nonzero(row_c)[0][0])
    first_e = int(np.nonzero(row_e)[0][0])
    assert first_c == 400 - 256
    assert first_e - first_c == int(np.ceil(mig))
    assert np.count_nonzero(sc.raw[:1000 - 512]) == 0
    assert np.count_nonzero(sc.raw[1000 + 512:]) == 0


def test_batch_and_pool_configs():
    b = batch_configs()
    assert len(b) == 64
    for c in b:
        assert c["Nr"] in (1024, 2048, 4096, 8192, 16384)
        assert c["Na"] in (512, 1024, 2048, 4096, 8192)
        assert 3 <= c["n_targets"] <= 9
        assert c["range_len"] == c["Nr"] // 8 and c["az_len"] == c["Na"] // 8
    assert batch_configs() == b
    p = serve_pool_configs()
    assert len(p) == 32 and all(c["n_targets"] == 5 for c in p)
