"""Helpers for the GPU tests: numpy <-> device tensors (torch is used for
device memory only; every computation goes through libsar_rda.so)."""
import numpy as np


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        import pytest
        pytest.skip("no GPU")
    return torch


def dev(a):
    torch = torch_cuda()
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex64)).cuda()


def empty(shape):
    torch = torch_cuda()
    return torch.empty(shape, dtype=torch.complex64, device="cuda")


def host(t):
    torch = torch_cuda()
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel_l2(a, ref):
    a = np.asarray(a, np.complex128)
    ref = np.asarray(ref, np.complex128)
    return float(np.linalg.norm((a - ref).ravel()) / np.linalg.norm(ref.ravel()))


def rand_c64(rng, shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex64)
