"""Helpers for the GPU parity tests (device transfers, error measures)."""
import numpy as np
import torch

DEV = torch.device('cuda')


def dev(a, dtype=torch.complex128):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV).to(dtype)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.complex128)


def rel_err(a, ref):
    """max |a - ref| / max |ref| (elementwise, in the max norm)."""
    return float(np.abs(np.asarray(a) - ref).max() / np.abs(ref).max())


def divisors(n):
    return [d for d in range(1, n + 1) if n % d == 0]
