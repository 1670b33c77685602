"""Helpers of the GPU tests (test infrastructure)."""
import os
import sys

import numpy as np


def say(*a):
    """Name the case before each GPU step, flushed, so a failure is located."""
    print("[gpu-case]", *a, file=sys.stderr, flush=True)


def oracle_threads():
    return max(1, min(16, os.cpu_count() or 1))


def device_tensor(arr):
    import torch
    a = np.ascontiguousarray(arr)
    t = torch.from_numpy(a.view(np.int64) if a.dtype == np.uint64 else a.view(np.int32))
    t = t.to("cuda")
    return t.view(torch.uint64) if a.dtype == np.uint64 else t.view(torch.uint32)
