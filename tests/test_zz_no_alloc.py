"""The allocation-free block product: ff_apply_block_noalloc through the C ABI against
apply_G_block on the same inputs (same kernels, intermediates in the library's fixed array)."""
import ctypes as C

import numpy as np
import pytest
import torch

from gpu_common import announce, rel, to_host
from paper_2004_13904_amd import _lib as L
from paper_2004_13904_amd import workloads as W
from paper_2004_13904_amd.operator import Operator

pytestmark = pytest.mark.gpu


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _both(lib, A, transpose, X, w_pre=None, w_post=None):
    """Y by apply_G_block and by ff_apply_block_noalloc (columns of X: k vectors)."""
    rin, rout = (A.m, A.n) if transpose else (A.n, A.m)
    k = X.shape[0]
    Y0 = torch.full((k, rout), float("nan"), dtype=X.dtype, device="cuda")
    Y1 = torch.full((k, rout), float("nan"), dtype=X.dtype, device="cuda")
    wp = w_pre.data_ptr() if w_pre is not None else None
    wq = w_post.data_ptr() if w_post is not None else None
    L.check("apply_G_block", lib.apply_G_block(A.h, transpose, k, X.data_ptr(), rin, Y0.data_ptr(), rout, wp, wq,
                                               _stream()))
    L.check("ff_apply_block_noalloc", lib.ff_apply_block_noalloc(A.h, transpose, k, X.data_ptr(), rin,
                                                                 Y1.data_ptr(), rout, wp, wq, _stream()))
    torch.cuda.synchronize()
    return Y0, Y1


def _agree(Y0, Y1):
    a, b = to_host(Y1), to_host(Y0)
    assert np.isfinite(a).all()
    scale = np.abs(b).max()
    assert np.abs(a - b).max() <= 1e-6 * scale, np.abs(a - b).max() / scale
    assert rel(a, b) <= 1e-6


def test_noalloc_block_matches_apply_G_block_twice():
    lib = L.load()
    g = torch.Generator(device="cuda").manual_seed(11)
    # first call: the n = 1e6 magnetic survey, 20 vectors (several launches through the array)
    s = W.SURVEYS["magnetic_1m"]
    A = Operator(s, torch.float32)
    announce("noalloc", "magnetic_1m G", "k=20")
    X = torch.rand((20, A.n), generator=g, device="cuda")
    wpre = torch.rand(A.n, generator=g, device="cuda") + 0.5
    wpost = torch.rand(A.m, generator=g, device="cuda") + 0.5
    Y0, Y1 = _both(lib, A, 0, X, wpre, wpost)
    _agree(Y0, Y1)
    announce("noalloc", "magnetic_1m G^T", "k=9")
    D = torch.randn((9, A.m), generator=g, device="cuda")
    Y0, Y1 = _both(lib, A, 1, D)
    _agree(Y0, Y1)
    A.close()
    # second call: a smaller input, a padded gravity survey in double precision, 3 vectors; the
    # array keeps the first call's contents, which must not leak into this result
    s2 = W.survey(9, 7, 3, 20.0, 20.0, 20.0, pad=(2, 1, 0, 3))
    B = Operator(s2, torch.float64)
    announce("noalloc", "padded 9x7x3 FP64", "k=3")
    X2 = torch.rand((3, B.n), generator=g, device="cuda", dtype=torch.float64)
    Y0, Y1 = _both(lib, B, 0, X2)
    assert torch.equal(Y0, Y1)
    D2 = torch.randn((3, B.m), generator=g, device="cuda", dtype=torch.float64)
    Y0, Y1 = _both(lib, B, 1, D2)
    assert torch.equal(Y0, Y1)
    # an empty block does nothing
    assert lib.ff_apply_block_noalloc(B.h, 0, 0, X2.data_ptr(), B.n, Y1.data_ptr(), B.m, None, None, _stream()) == 0
    B.close()


def test_noalloc_rejects_vectors_larger_than_the_array():
    # 300 x 300 stations, 60 layers: one vector's row intermediates (60 x 512 x 304 complex64,
    # about 75 MB) exceed the 64 MiB array; the call fails before any launch
    lib = L.load()
    s = W.survey(300, 300, 60, 10.0, 10.0, 10.0)
    A = Operator(s, torch.float32)
    announce("noalloc", "300x300x60 oversize")
    x = torch.zeros((1, A.n), device="cuda")
    y = torch.full((1, A.m), 7.0, device="cuda")
    rc = lib.ff_apply_block_noalloc(A.h, 0, 1, x.data_ptr(), A.n, y.data_ptr(), A.m, None, None, _stream())
    assert rc == L.FF_ENOMEM
    assert b"exceed the fixed scratch array" in lib.ff_last_error()
    torch.cuda.synchronize()
    assert bool((y == 7.0).all())
    A.close()
