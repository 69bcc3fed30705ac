"""The C-ABI library loads, exports every declared symbol, and rejects bad
arguments on the host before any HIP call (CPU only)."""
import ctypes

import pytest

import paper_2604_03585_amd as sar
from paper_2604_03585_amd import _lib
from sarsim import config


def test_every_declared_symbol_is_exported():
    names = _lib.header_functions()
    assert len(names) >= 18
    missing = [n for n in names if not hasattr(_lib.library(), n)]
    assert not missing, missing


def test_params_struct_layout():
    # int32 struct_size..range_len (16 B), then doubles at 8-byte alignment
    assert ctypes.sizeof(_lib.sar_params) == 96
    assert _lib.sar_params.range_tbp.offset == 16
    assert _lib.sar_params.lambda_.offset == 40
    assert _lib.sar_params.rcmc_beta.offset == 72


def _status(params):
    with pytest.raises(sar.SarError) as ei:
        sar.sar_plan(params, stream=0)
    assert sar.sar_last_error()
    return ei.value.status


@pytest.mark.parametrize("change, status", [
    (dict(Nr=100), _lib.SAR_ERR_BAD_SIZE),
    (dict(Na=32), _lib.SAR_ERR_BAD_SIZE),
    (dict(Nr=32768), _lib.SAR_ERR_BAD_SIZE),
    (dict(range_len=0), _lib.SAR_ERR_BAD_SIZE),
    (dict(range_len=257), _lib.SAR_ERR_BAD_SIZE),
    (dict(az_len=300), _lib.SAR_ERR_BAD_SIZE),
    (dict(az_model=7), _lib.SAR_ERR_BAD_PARAM),
    (dict(range_tbp=float("nan")), _lib.SAR_ERR_BAD_PARAM),
])
def test_plan_rejects_bad_lfm_params(change, status):
    assert _status(sar.make_params(config("c1", **change))) == status


@pytest.mark.parametrize("change, status", [
    (dict(lam=0.0), _lib.SAR_ERR_BAD_PARAM),
    (dict(v=-1.0), _lib.SAR_ERR_BAD_PARAM),
    (dict(lam=10.0, v=1.0), _lib.SAR_ERR_BAD_PARAM),
    (dict(rcmc_taps=4), _lib.SAR_ERR_BAD_PARAM),
    (dict(rcmc_beta=-1.0), _lib.SAR_ERR_BAD_PARAM),
    (dict(r_near=float("inf")), _lib.SAR_ERR_BAD_PARAM),
])
def test_plan_rejects_bad_hyperbolic_params(change, status):
    assert _status(sar.make_params(config("c2", **change))) == status


def test_plan_rejects_bad_enums_and_struct_size():
    p = sar.make_params(config("c1"))
    p.struct_size = 80
    assert _status(p) == _lib.SAR_ERR_BAD_PARAM
    assert _status(sar.make_params(config("c1"), schedule=5)) == _lib.SAR_ERR_BAD_PARAM
    assert _status(sar.make_params(config("c1"), transpose_back=2)) == _lib.SAR_ERR_BAD_PARAM
    assert _status(sar.make_params(config("c1"), precision=9)) == _lib.SAR_ERR_BAD_PARAM


@pytest.mark.parametrize("scene, kw", [
    ("c1", dict(schedule="unfused")),
    ("c1", dict(transpose_back=1)),
    ("c2", dict(schedule="unfused")),
    ("c2", dict(rcmc_taps=0)),
    ("c2", dict(lam=3.2, v=1.0)),        # stretch 0.67: the 8-row RCMC window cannot hold it
])
def test_half_storage_rejects_what_it_does_not_implement(scene, kw):
    plan_kw = {k: kw.pop(k) for k in ("schedule", "transpose_back") if k in kw}
    p = sar.make_params(config(scene, **kw), precision="fp32_halfstore", **plan_kw)
    assert _status(p) == _lib.SAR_ERR_UNSUPPORTED


def test_half_storage_bad_enums_stay_bad_param():
    p = sar.make_params(config("c1"), precision="fp32_halfstore", schedule=5)
    assert _status(p) == _lib.SAR_ERR_BAD_PARAM


def test_null_arguments():
    h = ctypes.c_void_p()
    assert _lib._sar_plan(None, None, ctypes.byref(h)) == _lib.SAR_ERR_NULL
    p = sar.make_params(config("c1"))
    assert _lib._sar_plan(ctypes.byref(p), None, None) == _lib.SAR_ERR_NULL
    assert _lib._sar_range_compress(None, 16, 32, None) == _lib.SAR_ERR_NULL
    assert _lib._sar_rda_execute(None, 16, 32, 48, None) == _lib.SAR_ERR_NULL
    assert _lib._sar_batch_plan(None, 1, None, ctypes.byref(h)) == _lib.SAR_ERR_NULL
    assert _lib._sar_batch_execute(None, None, None, None, None) == _lib.SAR_ERR_NULL
    assert "NULL" in sar.sar_last_error()


def test_corner_turn_host_validation():
    # plan may be NULL; bad sizes and overlap are rejected before any launch
    assert _lib._sar_corner_turn(None, 0, 256, 4, 4, None) == _lib.SAR_ERR_NULL
    assert _lib._sar_corner_turn(None, 16, 4096, 0, 4, None) == _lib.SAR_ERR_BAD_SIZE
    assert _lib._sar_corner_turn(None, 16, 4096, 1 << 21, 4, None) == _lib.SAR_ERR_BAD_SIZE
    assert _lib._sar_corner_turn(None, 4096, 4096 + 64, 16, 16, None) == _lib.SAR_ERR_ALIAS
    assert _lib._sar_corner_turn(None, 4100, 8192, 16, 16, None) == _lib.SAR_ERR_BAD_PARAM


def test_no_cpu_fallback_in_product_path():
    """No file of the product package imports or loads the oracle."""
    import os
    import re
    pkg = os.path.dirname(sar.__file__)
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".hpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"(import|from)\s+oracle|liboracle|orc_", text), f


def test_noalloc_workspace_size_matches_header():
    import os
    import re
    hdr = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                            "include", "sar_rda.h")).read()
    m = re.search(r"#define SAR_NOALLOC_WORKSPACE_BYTES \(\(size_t\)(\d+) << (\d+)\)", hdr)
    assert m and int(m.group(1)) << int(m.group(2)) == _lib.SAR_NOALLOC_WORKSPACE_BYTES


def test_noalloc_rejects_null_plan():
    with pytest.raises(sar.SarError) as e:
        sar.sar_rda_execute_noalloc(None, 16, 16, 0)
    assert e.value.status == _lib.SAR_ERR_NULL


def test_time_next_launches_checks_its_arguments():
    with pytest.raises(sar.SarError) as e:
        sar.sar_time_next_launch(16, None)
    assert e.value.status == _lib.SAR_ERR_NULL
    with pytest.raises(sar.SarError) as e:
        sar.sar_time_next_launches([16] * 17, [32] * 17)
    assert e.value.status == _lib.SAR_ERR_BAD_SIZE
    sar.sar_time_next_launch(None, None)     # disarm: always fine, no GPU call
    sar.sar_time_next_launches([], [])


@pytest.mark.parametrize("change", [dict(precision=1), dict(precision=3), dict(transpose_back=1),
                                    dict(Na=8192)])
def test_turn_free_limits_are_unsupported(change):
    cfg = config("c1", **({"Na": change["Na"], "az_len": 64} if "Na" in change else {}))
    p = sar.make_params(cfg, schedule="turn_free")
    for k, v in change.items():
        if k != "Na":
            setattr(p, k, v)
    assert _status(p) == _lib.SAR_ERR_UNSUPPORTED
