"""ctypes binding of libsar_rda.so (include/sar_rda.h).

Argument marshalling only: every step of the Range Doppler Algorithm runs in
the library's HIP kernels.  Device pointers may be given as torch CUDA tensors
or integers; streams as torch.cuda.Stream, integers or None (= torch's current
stream).  A non-OK status raises SarError carrying sar_last_error().

There is no fallback: if the shared library is missing or cannot be loaded,
importing this module raises ImportError.
"""
from __future__ import annotations

import ctypes
import os
import re

_HERE = os.path.dirname(os.path.abspath(__file__))
# SAR_RDA_LIB selects another build of the same library (same ABI).
LIB_PATH = os.environ.get("SAR_RDA_LIB") or os.path.join(_HERE, "libsar_rda.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "sar_rda.h")

# torch is imported first: ROCm builds of PyTorch carry their own HIP runtime
# (soname libamdhip64.so.7), and loading it before this library makes the
# library bind to that same runtime instead of a second copy from /opt/rocm,
# which could not open the GPU next to torch's.
import torch  # noqa: E402,F401

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python paper_2604_03585_amd/build.py` "
                      "(the HIP library has no CPU fallback)")
try:
    _L = ctypes.CDLL(LIB_PATH)
except OSError as e:  # pragma: no cover - depends on the ROCm runtime
    raise ImportError(f"cannot load {LIB_PATH}: {e}") from e

# ---------------------------------------------------------------- constants
SAR_OK = 0
SAR_ERR_NULL = 1
SAR_ERR_BAD_SIZE = 2
SAR_ERR_BAD_PARAM = 3
SAR_ERR_ALIAS = 4
SAR_ERR_NO_MEMORY = 5
SAR_ERR_HIP = 6
SAR_ERR_UNSUPPORTED = 7
STATUS_NAMES = {0: "SAR_OK", 1: "SAR_ERR_NULL", 2: "SAR_ERR_BAD_SIZE", 3: "SAR_ERR_BAD_PARAM",
                4: "SAR_ERR_ALIAS", 5: "SAR_ERR_NO_MEMORY", 6: "SAR_ERR_HIP",
                7: "SAR_ERR_UNSUPPORTED"}

SAR_AZ_LFM, SAR_AZ_HYPERBOLIC = 0, 1
SAR_FP32, SAR_SPLIT_FP16, SAR_SPLIT_BF16, SAR_FP32_HALF_STORAGE = 0, 1, 2, 3
SAR_FUSED, SAR_UNFUSED, SAR_TURN_FREE = 0, 1, 2

TABLE_HR, TABLE_HA, TABLE_STRETCH, TABLE_RATE, TABLE_RCMC = 0, 1, 2, 3, 4
RCMC_INTERVALS = 128
RCMC_PER_INTERVAL = 24          # 8 taps x 3 quadratic coefficients


class sar_params(ctypes.Structure):
    """Mirror of the C struct (same field order, natural alignment)."""
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("Nr", ctypes.c_int32), ("Na", ctypes.c_int32),
        ("range_len", ctypes.c_int32),
        ("range_tbp", ctypes.c_double),
        ("az_model", ctypes.c_int32),
        ("az_len", ctypes.c_int32),
        ("az_tbp", ctypes.c_double),
        ("lambda_", ctypes.c_double), ("v", ctypes.c_double), ("r_near", ctypes.c_double),
        ("rcmc_taps", ctypes.c_int32),
        ("rcmc_beta", ctypes.c_double),
        ("precision", ctypes.c_int32), ("schedule", ctypes.c_int32),
        ("transpose_back", ctypes.c_int32),
    ]


class SarError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        self.status = status
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {message}")


_vp = ctypes.c_void_p
_st = ctypes.c_int
_PP = ctypes.POINTER(sar_params)


def _fn(name, args, res=_st):
    f = getattr(_L, name)
    f.argtypes = args
    f.restype = res
    return f


_sar_plan = _fn("sar_plan", [_PP, _vp, ctypes.POINTER(_vp)])
_sar_plan_destroy = _fn("sar_plan_destroy", [_vp], None)
_sar_workspace_bytes = _fn("sar_workspace_bytes", [_vp], ctypes.c_size_t)
_sar_range_compress = _fn("sar_range_compress", [_vp, _vp, _vp, _vp])
_sar_corner_turn = _fn("sar_corner_turn", [_vp, _vp, _vp, ctypes.c_int32, ctypes.c_int32, _vp])
_sar_azimuth_compress = _fn("sar_azimuth_compress", [_vp, _vp, _vp, _vp, _vp])
_sar_rda_execute = _fn("sar_rda_execute", [_vp, _vp, _vp, _vp, _vp])
_sar_rda_execute_noalloc = _fn("sar_rda_execute_noalloc", [_vp, _vp, _vp, _vp])
_sar_time_next_launches = _fn("sar_time_next_launches",
                             [ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.c_int32])
_sar_fft_lines = _fn("sar_fft_lines", [_vp, ctypes.c_int32, ctypes.c_int32, _vp, _vp,
                                       ctypes.c_int32, _vp])
_sar_azimuth_fft = _fn("sar_azimuth_fft", [_vp, _vp, _vp, _vp])
_sar_rcmc_azimuth = _fn("sar_rcmc_azimuth", [_vp, _vp, _vp, _vp])
_sar_plan_get_table = _fn("sar_plan_get_table", [_vp, ctypes.c_int32, _vp, ctypes.c_size_t])
_sar_batch_plan = _fn("sar_batch_plan", [_PP, ctypes.c_int32, _vp, ctypes.POINTER(_vp)])
_sar_batch_workspace_bytes = _fn("sar_batch_workspace_bytes", [_vp], ctypes.c_size_t)
_sar_batch_execute = _fn("sar_batch_execute", [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                                               _vp, _vp])
_sar_batch_destroy = _fn("sar_batch_destroy", [_vp], None)
_sar_autotune = _fn("sar_autotune", [_PP, ctypes.c_char_p])
_sar_tune_load = _fn("sar_tune_load", [ctypes.c_char_p, ctypes.c_char_p])
_sar_tune_variant = _fn("sar_tune_variant", [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32],
                        ctypes.c_int32)
_sar_last_error = _fn("sar_last_error", [], ctypes.c_char_p)
_sar_version = _fn("sar_version", [], ctypes.c_char_p)


def library():
    """The loaded ctypes library (for symbol checks)."""
    return _L


def header_functions() -> list[str]:
    """Names of the functions include/sar_rda.h declares."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sar_[a-z_0-9]+)\s*\(", text)))


# ------------------------------------------------------------ marshalling
def _ptr(x) -> int | None:
    if x is None:
        return None
    if hasattr(x, "data_ptr"):
        return int(x.data_ptr())
    return int(x)


def _stream(s) -> int | None:
    if s is None:
        import torch
        return int(torch.cuda.current_stream().cuda_stream)
    if hasattr(s, "cuda_stream"):
        return int(s.cuda_stream)
    return int(s)


def _check(status: int, where: str):
    if status != SAR_OK:
        raise SarError(status, where, (_sar_last_error() or b"").decode())


def sar_last_error() -> str:
    return (_sar_last_error() or b"").decode()


def sar_version() -> str:
    return (_sar_version() or b"").decode()


_AZ = {"lfm": SAR_AZ_LFM, "hyperbolic": SAR_AZ_HYPERBOLIC}
_PREC = {"fp32": SAR_FP32, "split_fp16": SAR_SPLIT_FP16, "split_bf16": SAR_SPLIT_BF16,
         "fp32_halfstore": SAR_FP32_HALF_STORAGE}
_SCHED = {"fused": SAR_FUSED, "unfused": SAR_UNFUSED, "turn_free": SAR_TURN_FREE}


def make_params(cfg: dict, precision="fp32", schedule="fused", transpose_back=0) -> sar_params:
    """sar_params from a scene dictionary (keys Nr, Na, range_len, range_tbp,
    az_model, az_len, az_tbp, lam, v, r_near, rcmc_taps, rcmc_beta)."""
    p = sar_params()
    p.struct_size = ctypes.sizeof(sar_params)
    p.Nr, p.Na = int(cfg["Nr"]), int(cfg["Na"])
    p.range_len, p.range_tbp = int(cfg["range_len"]), float(cfg["range_tbp"])
    am = cfg["az_model"]
    p.az_model = _AZ[am] if isinstance(am, str) else int(am)
    p.az_len, p.az_tbp = int(cfg.get("az_len", 0)), float(cfg.get("az_tbp", 0.0))
    p.lambda_, p.v, p.r_near = float(cfg.get("lam", 0.0)), float(cfg.get("v", 0.0)), \
        float(cfg.get("r_near", 0.0))
    p.rcmc_taps, p.rcmc_beta = int(cfg.get("rcmc_taps", 0)), float(cfg.get("rcmc_beta", 2.5))
    p.precision = _PREC[precision] if isinstance(precision, str) else int(precision)
    p.schedule = _SCHED[schedule] if isinstance(schedule, str) else int(schedule)
    p.transpose_back = int(transpose_back)
    return p


# ------------------------------------------------------------ entry points
_plan_sizes: dict[int, tuple[int, int]] = {}


def sar_plan(params: sar_params, stream=None) -> int:
    h = _vp()
    _check(_sar_plan(ctypes.byref(params), _stream(stream), ctypes.byref(h)), "sar_plan")
    _plan_sizes[int(h.value)] = (params.Nr, params.Na)
    return int(h.value)


def sar_plan_destroy(plan: int) -> None:
    _plan_sizes.pop(plan, None)
    _sar_plan_destroy(plan)


def sar_workspace_bytes(plan: int) -> int:
    return int(_sar_workspace_bytes(plan))


def sar_range_compress(plan, in_dev, out_dev, stream=None):
    _check(_sar_range_compress(plan, _ptr(in_dev), _ptr(out_dev), _stream(stream)),
           "sar_range_compress")


def sar_corner_turn(plan, in_dev, out_dev, rows: int, cols: int, stream=None):
    _check(_sar_corner_turn(plan, _ptr(in_dev), _ptr(out_dev), rows, cols, _stream(stream)),
           "sar_corner_turn")


def sar_azimuth_compress(plan, in_dev, out_dev, work_dev=None, stream=None):
    _check(_sar_azimuth_compress(plan, _ptr(in_dev), _ptr(out_dev), _ptr(work_dev),
                                 _stream(stream)), "sar_azimuth_compress")


def sar_rda_execute(plan, raw_dev, img_dev, work_dev, stream=None):
    _check(_sar_rda_execute(plan, _ptr(raw_dev), _ptr(img_dev), _ptr(work_dev),
                            _stream(stream)), "sar_rda_execute")


def sar_time_next_launches(starts, stops):
    """Arm pairs of events for the next len(starts) kernel launches on this
    thread (torch.cuda.Event with timing, or raw hipEvent_t handles; empty
    lists disarm).  A torch event whose handle does not exist yet is created
    by recording it once on the current stream."""
    def handle(e):
        if hasattr(e, "cuda_event"):
            if not e.cuda_event:
                import torch
                e.record(torch.cuda.current_stream())
            return int(e.cuda_event)
        return int(e) if e is not None else None
    if len(starts) != len(stops):
        raise ValueError("starts and stops differ in length")
    n = len(starts)
    a = (_vp * max(n, 1))(*[handle(e) for e in starts])
    b = (_vp * max(n, 1))(*[handle(e) for e in stops])
    _check(_sar_time_next_launches(a, b, n), "sar_time_next_launches")


def sar_time_next_launch(start_event, stop_event):
    """sar_time_next_launches for one launch (None, None disarms)."""
    if start_event is None and stop_event is None:
        sar_time_next_launches([], [])
    else:
        sar_time_next_launches([start_event], [stop_event])


def sar_rda_execute_noalloc(plan, raw_dev, img_dev, stream=None):
    _check(_sar_rda_execute_noalloc(plan, _ptr(raw_dev), _ptr(img_dev), _stream(stream)),
           "sar_rda_execute_noalloc")


# sar_rda_execute_noalloc's static workspace (bytes per GPU)
SAR_NOALLOC_WORKSPACE_BYTES = 128 << 20


def sar_fft_lines(plan, axis: int, inverse: int, in_dev, out_dev, lines: int, stream=None):
    _check(_sar_fft_lines(plan, axis, inverse, _ptr(in_dev), _ptr(out_dev), lines,
                          _stream(stream)), "sar_fft_lines")


def sar_azimuth_fft(plan, in_dev, out_dev, stream=None):
    _check(_sar_azimuth_fft(plan, _ptr(in_dev), _ptr(out_dev), _stream(stream)),
           "sar_azimuth_fft")


def sar_rcmc_azimuth(plan, A_dev, out_dev, stream=None):
    _check(_sar_rcmc_azimuth(plan, _ptr(A_dev), _ptr(out_dev), _stream(stream)),
           "sar_rcmc_azimuth")


def sar_plan_get_table(plan, which: int):
    """A plan table as a numpy array (complex64 filters, float64 tables)."""
    import numpy as np
    nr, na = _plan_sizes[plan]
    if which == TABLE_HR:
        out = np.empty(nr, np.complex64)
    elif which == TABLE_HA:
        out = np.empty(na, np.complex64)
    elif which == TABLE_RCMC:
        out = np.empty(RCMC_PER_INTERVAL * RCMC_INTERVALS, np.float32)
    else:
        out = np.empty(na, np.float64)
    _check(_sar_plan_get_table(plan, which, out.ctypes.data, out.nbytes), "sar_plan_get_table")
    return out


def sar_batch_plan(params_list, stream=None) -> int:
    arr = (sar_params * len(params_list))(*params_list)
    h = _vp()
    _check(_sar_batch_plan(arr, len(params_list), _stream(stream), ctypes.byref(h)),
           "sar_batch_plan")
    return int(h.value)


def sar_batch_workspace_bytes(batch: int) -> int:
    return int(_sar_batch_workspace_bytes(batch))


def sar_batch_execute(batch, raws, imgs, work_dev, stream=None):
    n = len(raws)
    r = (_vp * n)(*[_ptr(x) for x in raws])
    i = (_vp * n)(*[_ptr(x) for x in imgs])
    _check(_sar_batch_execute(batch, r, i, _ptr(work_dev), _stream(stream)), "sar_batch_execute")


def sar_batch_destroy(batch: int) -> None:
    _sar_batch_destroy(batch)


def sar_autotune(params: sar_params, cache_path: str | None = None):
    _check(_sar_autotune(ctypes.byref(params), cache_path.encode() if cache_path else None),
           "sar_autotune")


TUNE_FUSED, TUNE_FWD, TUNE_INV, TUNE_RCMC, TUNE_BATCH_FUSED, TUNE_TURN, TUNE_STRIP = range(7)


def sar_tune_load(path: str | None, arch: str | None = None):
    _check(_sar_tune_load(path.encode() if path else None, arch.encode() if arch else None),
           "sar_tune_load")


def sar_tune_variant(kind: int, n: int, precision: int = 0) -> int:
    return int(_sar_tune_variant(kind, n, precision))
