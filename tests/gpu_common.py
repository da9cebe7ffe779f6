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


def agree(a, b, tol):
    """Parity bar of an operator result a against the oracle's b: relative l2 error and the worst
    element, relative to the largest reference element, both within tol (an error confined to a
    few entries, such as a crop edge or a ragged tail, fails the second)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    assert np.isfinite(a).all()
    e = rel(a, b)
    m = float(np.abs(a - b).max() / np.abs(b).max())
    assert e <= tol and m <= tol, (e, m, tol)
    return e, m


def same(a, b):
    """Batched against single-vector results: bit-identical in FP64 (same kernels); in FP32 the
    batched column passes add the layer terms in another order, so agreement is to rounding
    (a few units of 2^-24 on the norm)."""
    assert a.dtype == b.dtype and a.shape == b.shape
    if a.dtype == torch.float64:
        assert torch.equal(a, b)
    else:
        e = rel(to_host(a), to_host(b))
        assert e <= 2e-6, e


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
