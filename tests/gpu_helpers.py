"""Helpers shared by the GPU tests: moving TT cores between NumPy and the
device, and the parity measures (stable difference norm from the oracle)."""
import sys

import numpy as np


def to_dev(cores):
    import torch
    return [torch.tensor(np.ascontiguousarray(c), dtype=torch.float64, device="cuda") for c in cores]


def to_host(cores):
    return [c.detach().cpu().numpy().astype(np.float64) for c in cores]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_tensor_diff(x, a, b):
    """||A - B|| / ||X|| with the oracle's formal-difference norm."""
    from oracle import tt
    return tt.diff_norm(a, b) / tt.norm(x)
