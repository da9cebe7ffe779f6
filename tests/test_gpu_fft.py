"""The device FFT of the operator's passes, stand-alone (ff_fft_1d), against numpy's FFT as a
test-only reference: every length from 8 to 2048 (one-wavefront and multi-wavefront transforms)
in each of the three stage plans (radix-8 stages with the radix-4 or radix-2 stage last or first,
and radix-4 stages), both directions, FP32 and FP64, and the round trip."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2004_13904_amd import _lib as L

pytestmark = pytest.mark.gpu
SIZES = [8, 16, 32, 64, 128, 256, 512, 1024, 2048]


def device_fft(x, inverse, plan=0):
    n = x.shape[-1]
    out = torch.empty_like(x)
    tw = torch.empty(n, dtype=x.dtype, device=x.device)
    dt = L.FF_F32 if x.dtype == torch.complex64 else L.FF_F64
    L.call("ff_fft_1d", n, dt, int(inverse), int(plan), x.shape[0], C.c_void_p(x.data_ptr()), C.c_void_p(out.data_ptr()),
           C.c_void_p(tw.data_ptr()), C.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
@pytest.mark.parametrize("inverse", [0, 1])
@pytest.mark.parametrize("plan", [0, 1, 2])
def test_fft_matches_numpy(n, dtype, inverse, plan):
    rng = np.random.default_rng(n + 7 * inverse)
    xh = rng.standard_normal((5, n)) + 1j * rng.standard_normal((5, n))
    ref = np.fft.fft(xh, axis=1) if not inverse else n * np.fft.ifft(xh, axis=1)
    y = device_fft(torch.tensor(xh, dtype=dtype, device="cuda"), inverse, plan).cpu().numpy()
    err = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    # a radix-8 FFT's rounding error grows like log n; FP32 against the FP64 reference
    tol = (4e-16 if dtype == torch.complex128 else 2e-7) * max(1.0, np.log2(n))
    assert err <= tol, (n, dtype, inverse, err)


@pytest.mark.parametrize("n", [8, 64, 512, 2048])
@pytest.mark.parametrize("plan", [0, 2])
def test_fft_round_trip_and_impulses(n, plan):
    x = torch.randn(3, n, dtype=torch.complex128, device="cuda")
    back = device_fft(device_fft(x, 0, plan), 1, plan) / n
    assert torch.allclose(back, x, rtol=0, atol=1e-13 * np.log2(n))
    # an impulse at position k transforms to exp(-2 pi i j k / n)
    e = torch.zeros(3, n, dtype=torch.complex128, device="cuda")
    ks = [0, 1, n - 1]
    for r, k in enumerate(ks):
        e[r, k] = 1.0
    y = device_fft(e, 0, plan).cpu().numpy()
    j = np.arange(n)
    for r, k in enumerate(ks):
        # the phase reduced modulo n first: exp of the unreduced 2 pi j k / n would lose ~1e-13
        assert np.abs(y[r] - np.exp(-2j * np.pi * ((j * k) % n) / n)).max() <= 1e-14 * np.log2(n)
