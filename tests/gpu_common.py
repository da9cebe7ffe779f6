"""Helpers shared by the GPU parity tests (oracle on the host, HIP path through the C ABI)."""
import functools
import sys

import numpy as np
import torch

from oracle import geometry, operator as op
from paper_2004_13904_amd import workloads as W


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def announce(*parts):
    print("[case]", *parts, flush=True)
    sys.stdout.flush()


def ogeom(s):
    return geometry.Geometry(**s)


@functools.lru_cache(maxsize=8)
def otable(name):
    return op.kernel_table(ogeom(W.SURVEYS[name]))


def to_dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def to_host(t):
    torch.cuda.synchronize()
    return t.detach().double().cpu().numpy()
