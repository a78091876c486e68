"""Helpers of the GPU tests: device selection and host/device transfer."""
import numpy as np
import pytest


def torch_cuda():
    """torch with a visible HIP device.  The gpu-marked tests run on a GPU
    host; a missing device there is a failure, not a reason to skip."""
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no HIP device visible to torch (gpu-marked tests need one)")
    return torch


def dev(a, dtype):
    torch = torch_cuda()
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def host(t):
    return t.detach().to("cpu").double().numpy()


def rel_fro(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))
