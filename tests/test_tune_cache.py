"""Host logic of the autotuner's cache: parsing, architecture filtering,
rejection of out-of-range variants, clearing (no GPU needed: the
architecture is passed explicitly)."""
import pytest

import paper_2604_03585_amd as sar
from paper_2604_03585_amd import _lib

CACHE = """\
{"arch":"gfx950","kind":"fused","n":4096,"prec":0,"variant":1,"us_default":64.1,"us_best":61.0}
{"arch":"gfx950","kind":"rcmc","n":4096,"prec":0,"variant":3,"us_default":93.0,"us_best":90.0}
{"arch":"gfx950","kind":"batch_fused","n":1024,"prec":0,"variant":13}
{"arch":"gfx950","kind":"inv","n":512,"prec":1,"variant":0}
{"arch":"gfx942","kind":"fwd","n":4096,"prec":0,"variant":1}
{"arch":"gfx950","kind":"fused","n":2048,"prec":0,"variant":2}
{"arch":"gfx950","kind":"batch_fused","n":2048,"prec":0,"variant":2}
{"arch":"gfx950","kind":"fused","n":3000,"prec":0,"variant":1}
{"arch":"gfx950","kind":"fused","n":256,"prec":7,"variant":1}
{"arch":"gfx950","kind":"nonsense","n":256,"prec":0,"variant":1}
{"arch":"gfx950","kind":"inv","n":1024,"prec":0,"variant":3}
{"arch":"gfx950","kind":"fwd","n":1024,"prec":0,"variant":4}
{"arch":"gfx950","kind":"rcmc","n":2048,"prec":1,"variant":2}
{"arch":"gfx950","kind":"rcmc","n":1024,"prec":2,"variant":4}
{"arch":"gfx950","kind":"batch_fused","n":1024,"prec":1,"variant":4}
{"arch":"gfx950","kind":"fused","n":1024,"prec":2,"variant":1}
not json at all
{"arch":"gfx950","kind":"fwd","n":256,"prec":0}
{"arch":"gfx950","kind":"turn","n":4096,"prec":0,"variant":2}
{"arch":"gfx950","kind":"turn","n":2048,"prec":0,"variant":3}
{"arch":"gfx950","kind":"turn","n":1024,"prec":1,"variant":1}
{"arch":"gfx950","kind":"strip","n":4096,"prec":0,"variant":1}
{"arch":"gfx950","kind":"strip","n":2048,"prec":0,"variant":2}
"""


@pytest.fixture
def cache(tmp_path):
    p = tmp_path / "tune.jsonl"
    p.write_text(CACHE)
    yield str(p)
    sar.sar_tune_load(None)


def test_cache_entries_for_this_arch(cache):
    sar.sar_tune_load(cache, "gfx950")
    v = sar.sar_tune_variant
    assert v(_lib.TUNE_FUSED, 4096, 0) == 1
    assert v(_lib.TUNE_RCMC, 4096, 0) == 3
    assert v(_lib.TUNE_BATCH_FUSED, 1024, 0) == 13
    assert v(_lib.TUNE_INV, 512, 1) == 0
    # other architectures, other keys: untuned
    assert v(_lib.TUNE_FWD, 4096, 0) == 0
    assert v(_lib.TUNE_FUSED, 4096, 1) == 0
    assert v(99, 4096, 0) == -1


def test_invalid_lines_are_ignored(cache):
    sar.sar_tune_load(cache, "gfx950")
    v = sar.sar_tune_variant
    assert v(_lib.TUNE_FUSED, 2048, 0) == 0          # variant 2 is not a fused-kernel variant
    assert v(_lib.TUNE_BATCH_FUSED, 2048, 0) == 0    # bit 1 is not a batch variant
    assert v(_lib.TUNE_FUSED, 3000, 0) == 0          # not a power of two
    assert v(_lib.TUNE_FUSED, 256, 7) == 0           # unknown precision
    assert v(_lib.TUNE_FWD, 256, 0) == 0             # no variant field
    assert v(_lib.TUNE_INV, 1024, 0) == 3            # split layout + table twiddles
    assert v(_lib.TUNE_FWD, 1024, 0) == 4            # twice the lines per workgroup
    # split precisions: default kernels and the one-row RCMC kernel only
    assert v(_lib.TUNE_RCMC, 2048, 1) == 2
    assert v(_lib.TUNE_RCMC, 1024, 2) == 0           # the wide RCMC kernel is FP32 only
    assert v(_lib.TUNE_BATCH_FUSED, 1024, 1) == 0    # no persistent split grids
    assert v(_lib.TUNE_FUSED, 1024, 2) == 0          # table twiddles are FP32 only
    # corner-turn grids (0..2) and strip widths (0, 1), keyed as FP32
    assert v(_lib.TUNE_TURN, 4096, 0) == 2
    assert v(_lib.TUNE_TURN, 2048, 0) == 0           # no fourth grid
    assert v(_lib.TUNE_TURN, 1024, 1) == 0           # not keyed by a split precision
    assert v(_lib.TUNE_STRIP, 4096, 0) == 1
    assert v(_lib.TUNE_STRIP, 2048, 0) == 0          # half width is the only other width


def test_other_arch_and_clear(cache):
    sar.sar_tune_load(cache, "gfx942")
    assert sar.sar_tune_variant(_lib.TUNE_FWD, 4096, 0) == 1
    assert sar.sar_tune_variant(_lib.TUNE_FUSED, 4096, 0) == 0
    sar.sar_tune_load(None)
    assert sar.sar_tune_variant(_lib.TUNE_FWD, 4096, 0) == 0


def test_unreadable_cache(tmp_path):
    with pytest.raises(sar.SarError) as e:
        sar.sar_tune_load(str(tmp_path / "missing.jsonl"), "gfx950")
    assert e.value.status == _lib.SAR_ERR_BAD_PARAM
