"""MI355X-native kernel-fused SAR Range Doppler Algorithm.

The computation lives in libsar_rda.so (hand-written HIP for gfx950) behind
the C ABI of include/sar_rda.h; this package is its thin binding.  PyTorch
provides device memory and streams only.
"""
from __future__ import annotations

from . import _lib
from ._lib import (SarError, make_params, sar_params, sar_plan, sar_plan_destroy,
                   sar_workspace_bytes, sar_range_compress, sar_corner_turn,
                   sar_azimuth_compress, sar_rda_execute, sar_rda_execute_noalloc,
                   sar_time_next_launch, sar_time_next_launches,
                   sar_fft_lines, sar_azimuth_fft,
                   sar_rcmc_azimuth, sar_plan_get_table, sar_batch_plan,
                   sar_batch_workspace_bytes, sar_batch_execute, sar_batch_destroy,
                   sar_autotune, sar_tune_load, sar_tune_variant, sar_last_error,
                   sar_version)

__all__ = ["Plan", "SarError", "make_params", "sar_params", "sar_plan", "sar_plan_destroy",
           "sar_workspace_bytes", "sar_range_compress", "sar_corner_turn",
           "sar_azimuth_compress", "sar_rda_execute", "sar_rda_execute_noalloc",
           "sar_time_next_launch", "sar_time_next_launches",
           "sar_fft_lines", "sar_azimuth_fft",
           "sar_rcmc_azimuth", "sar_plan_get_table", "sar_batch_plan",
           "sar_batch_workspace_bytes", "sar_batch_execute", "sar_batch_destroy",
           "sar_autotune", "sar_tune_load", "sar_tune_variant", "sar_last_error",
           "sar_version"]


class Plan:
    """An immutable RDA plan for one scene geometry.

    ``cfg`` holds the processing keys of a scene dictionary (Nr, Na,
    range_len, range_tbp, az_model, az_len, az_tbp, lam, v, r_near,
    rcmc_taps, rcmc_beta).  The plan's tables are built on ``stream``.
    """

    def __init__(self, cfg: dict, precision="fp32", schedule="fused", transpose_back=0,
                 stream=None):
        self.params = make_params(cfg, precision, schedule, transpose_back)
        self.Nr, self.Na = self.params.Nr, self.params.Na
        self.transpose_back = int(transpose_back)
        self.handle = sar_plan(self.params, stream)

    @property
    def workspace_bytes(self) -> int:
        return sar_workspace_bytes(self.handle)

    def image_shape(self):
        return (self.Na, self.Nr) if self.transpose_back else (self.Nr, self.Na)

    def execute(self, raw, out=None, work=None, stream=None):
        """raw: complex64 CUDA tensor (Na, Nr) -> image tensor ((Nr, Na), or
        (Na, Nr) with transpose_back).  Asynchronous on ``stream`` (default:
        the current stream).  ``out`` and ``work`` are checked for device,
        dtype, contiguity and size; temporaries are allocated on ``stream``."""
        import torch
        if raw.dtype != torch.complex64 or not raw.is_cuda or not raw.is_contiguous():
            raise ValueError("raw must be a contiguous complex64 CUDA tensor")
        if tuple(raw.shape) != (self.Na, self.Nr):
            raise ValueError(f"raw has shape {tuple(raw.shape)}, plan wants {(self.Na, self.Nr)}")
        if out is not None:
            if (out.dtype != torch.complex64 or out.device != raw.device
                    or not out.is_contiguous() or tuple(out.shape) != self.image_shape()):
                raise ValueError(f"out must be a contiguous complex64 tensor of shape "
                                 f"{self.image_shape()} on {raw.device}")
        if work is not None:
            if (work.device != raw.device or not work.is_contiguous()
                    or work.numel() * work.element_size() < self.workspace_bytes):
                raise ValueError(f"work must be a contiguous tensor of at least "
                                 f"{self.workspace_bytes} bytes on {raw.device}")
        if stream is None:
            s = torch.cuda.current_stream(raw.device)
        elif isinstance(stream, torch.cuda.Stream):
            s = stream
        else:   # a raw hipStream_t handle
            s = torch.cuda.ExternalStream(int(stream), device=raw.device)
        with torch.cuda.stream(s):
            # allocated on `s`: the caching allocator will not hand these
            # blocks to other streams while the kernels below may use them
            if out is None:
                out = torch.empty(self.image_shape(), dtype=torch.complex64, device=raw.device)
            tmp = None
            if work is None:
                tmp = work = torch.empty(((self.workspace_bytes + 7) // 8,),
                                         dtype=torch.complex64, device=raw.device)
            sar_rda_execute(self.handle, raw, out, work, s)
            del tmp
        return out

    def close(self):
        if getattr(self, "handle", None):
            sar_plan_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        import torch
        torch.cuda.synchronize()
        self.close()
