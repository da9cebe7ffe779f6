"""Parity of the HIP operator (C ABI) with the CPU oracle, per the bars:
FP64 operators within 1e-12 relative l2 of the dense / direct-sum definition, FP32 within 1e-5.
"""
import numpy as np
import pytest
import torch

from gpu_common import agree, announce, ogeom, otable, rel, same, to_dev, to_host
from oracle import geometry, operator as op
from paper_2004_13904_amd import workloads as W
from paper_2004_13904_amd import _lib as L
from paper_2004_13904_amd.operator import Operator

pytestmark = pytest.mark.gpu

F64, F32 = torch.float64, torch.float32
TOL = {F64: 1e-12, F32: 1e-5}


def survey(**kw):
    s = W.survey(kw.pop("sx"), kw.pop("sy"), kw.pop("nz"), kw.pop("dx"), kw.pop("dy"), kw.pop("dz"),
                 kernel=kw.pop("kernel", "gravity"), incl=kw.pop("incl", 90.0),
                 decl=kw.pop("decl", 0.0), pad=kw.pop("pad", (0, 0, 0, 0)))
    assert not kw
    return s


SMALL = {
    "tiny": W.SURVEYS["tiny"],
    "padded_ragged": survey(sx=9, sy=7, nz=3, dx=20, dy=25, dz=15, pad=(2, 1, 0, 3)),
    "mag45": survey(sx=8, sy=6, nz=3, dx=20, dy=20, dz=20, kernel="magnetic", incl=45, decl=45),
    "mag_padded": survey(sx=7, sy=9, nz=2, dx=20, dy=20, dz=30, kernel="magnetic", incl=60, decl=-20,
                         pad=(1, 2, 3, 1)),
    "wide_tail": survey(sx=37, sy=11, nz=5, dx=20, dy=20, dz=10, pad=(3, 0, 2, 2)),
    "mag_many_layers": survey(sx=23, sy=19, nz=33, dx=25, dy=25, dz=12, kernel="magnetic", incl=70,
                              decl=10),
}


@pytest.mark.parametrize("name", list(SMALL))
@pytest.mark.parametrize("dtype", [F64, F32])
def test_small_against_dense_G(name, dtype):
    s = SMALL[name]
    announce("dense", name, dtype)
    g = ogeom(s)
    G = op.dense_G(g)
    rng = np.random.default_rng(0)
    x = rng.random(g.n)
    d = rng.standard_normal(g.m)
    A = Operator(s, dtype)
    dG = to_host(A.G(to_dev(x, dtype)))
    xT = to_host(A.GT(to_dev(d, dtype)))
    agree(dG, G @ x, TOL[dtype])
    agree(xT, G.T @ d, TOL[dtype])
    A.close()


def test_tiny_fp64_adjoint_identity():
    s = W.SURVEYS["tiny"]
    A = Operator(s, F64)
    x = W.uniform_model(s, 0)
    d = W.gaussian_data(s, 1)
    Gx = to_host(A.G(to_dev(x, F64)))
    GTd = to_host(A.GT(to_dev(d, F64)))
    assert abs(Gx @ d - x @ GTd) <= 1e-13 * np.linalg.norm(Gx) * np.linalg.norm(d)


@pytest.mark.parametrize("name", ["tiny", "mag_padded", "gravity_l4", "magnetic_1m"])
def test_kernel_table_matches_oracle(name):
    s = SMALL.get(name) or W.SURVEYS[name]
    announce("table", name)
    A = Operator(s, F64)
    t = to_host(A.kernel_table())
    ref = otable(name) if name in W.SURVEYS else op.kernel_table(ogeom(s))
    assert t.shape == ref.shape
    # entries agree to the rounding of the 8-corner sums (far entries cancel; bounded by the
    # largest entry of the table)
    assert np.abs(t - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("nfft", [(32, 32), (64, 32), (32, 128)])
def test_embedding_size_invariance(nfft):
    s = W.SURVEYS["tiny"]
    x = W.uniform_model(s, 0)
    A = Operator(s, F64, nfft=nfft)
    B = Operator(s, F64)
    assert A.nfft == nfft and B.nfft == (32, 32)
    a = to_host(A.G(to_dev(x, F64)))
    b = to_host(B.G(to_dev(x, F64)))
    agree(a, b, 1e-13)


@pytest.mark.parametrize("nfft", [(1024, 32), (32, 1024), (2048, 32), (32, 2048)])
@pytest.mark.parametrize("name", ["tiny", "mag_padded"])
@pytest.mark.parametrize("dtype", [F64, F32])
def test_large_embeddings_against_dense_G(nfft, name, dtype):
    # rows and columns of 1024 and 2048 points: transforms that span several wavefronts, one row
    # or column per block; one vector and a block of three (the per-vector column kernels over
    # the batch) against the dense definition
    s = SMALL[name]
    announce("embedding", name, nfft, dtype)
    g = ogeom(s)
    G = op.dense_G(g)
    rng = np.random.default_rng(7)
    X = rng.random((3, g.n))
    D = rng.standard_normal((3, g.m))
    A = Operator(s, dtype, nfft=nfft)
    assert A.nfft == nfft
    agree(to_host(A.G(to_dev(X[0], dtype))), G @ X[0], TOL[dtype])
    agree(to_host(A.GT(to_dev(D[0], dtype))), G.T @ D[0], TOL[dtype])
    Y = to_host(A.G_block(to_dev(X, dtype)))
    Z = to_host(A.G_block(to_dev(D, dtype), transpose=True))
    for i in range(3):
        agree(Y[i], G @ X[i], TOL[dtype])
        agree(Z[i], G.T @ D[i], TOL[dtype])
    A.close()


def test_too_small_embedding_is_rejected():
    with pytest.raises(L.FastFocusError) as e:
        Operator(W.SURVEYS["tiny"], F64, nfft=(16, 32))
    assert e.value.code == -2


@pytest.mark.parametrize("name", ["gravity_l4", "gravity_diff", "gravity_rsvd", "magnetic_1m"])
def test_full_size_fp32_against_direct_sums(name):
    s = W.SURVEYS[name]
    announce("full", name)
    g = ogeom(s)
    T = otable(name)
    x = W.uniform_model(s, 0)
    d = W.gaussian_data(s, 1)
    A = Operator(s, F32)
    dG = to_host(A.G(to_dev(x, F32)))
    xT = to_host(A.GT(to_dev(d, F32)))
    ref_d = op.apply_G(g, x, T)
    ref_x = op.apply_GT(g, d, T)
    agree(dG, ref_d, 1e-5)
    agree(xT, ref_x, 1e-5)
    # the embedding size, the spectra and both FFT directions are exercised by the adjoint
    assert abs(dG @ d - x @ xT) <= 1e-5 * np.linalg.norm(dG) * np.linalg.norm(d)


@pytest.mark.parametrize("dtype", [F64, F32])
def test_weighted_operator(dtype):
    s = SMALL["padded_ragged"]
    g = ogeom(s)
    G = op.dense_G(g)
    rng = np.random.default_rng(2)
    x, d = rng.random(g.n), rng.standard_normal(g.m)
    wn, wm = 0.5 + rng.random(g.n), 0.5 + rng.random(g.m)
    A = Operator(s, dtype)
    out = to_host(A.G(to_dev(x, dtype), w_pre=to_dev(wn, dtype), w_post=to_dev(wm, dtype)))
    agree(out, wm * (G @ (wn * x)), TOL[dtype])
    out = to_host(A.GT(to_dev(d, dtype), w_pre=to_dev(wm, dtype), w_post=to_dev(wn, dtype)))
    agree(out, wn * (G.T @ (wm * d)), TOL[dtype])


@pytest.mark.parametrize("dtype", [F64, F32])
@pytest.mark.parametrize("k", [1, 5, 16, 21])
def test_block_apply_equals_vector_loop(dtype, k):
    s = SMALL["wide_tail"]
    g = ogeom(s)
    G = op.dense_G(g)
    rng = np.random.default_rng(k)
    X = rng.standard_normal((k, g.n))
    Y = rng.standard_normal((k, g.m))
    A = Operator(s, dtype)
    GX = A.G_block(to_dev(X, dtype))
    GTY = A.G_block(to_dev(Y, dtype), transpose=True)
    for c in range(k):
        # FP64 blocks run the single-vector kernels (bit-identical); FP32 blocks the batched
        # column passes, whose layer sums are taken in another order
        same(GX[c], A.G(to_dev(X[c], dtype)))
        same(GTY[c], A.GT(to_dev(Y[c], dtype)))
    agree(to_host(GX), X @ G.T, TOL[dtype])
    agree(to_host(GTY), Y @ G, TOL[dtype])


@pytest.mark.parametrize("k", [2, 6])
def test_batched_full_size_equals_vector_loop(k):
    # the batched column passes (4 vectors per block) at the n = 1e6 magnetic survey
    s = W.SURVEYS["magnetic_1m"]
    A = Operator(s, F32)
    g = torch.Generator(device="cuda").manual_seed(k)
    X = torch.rand(k, A.n, device="cuda", generator=g)
    D = torch.randn(k, A.m, device="cuda", generator=g)
    GX = A.G_block(X)
    GTD = A.G_block(D, transpose=True)
    for c in range(k):
        same(GX[c], A.G(X[c].contiguous()))
        same(GTD[c], A.GT(D[c].contiguous()))


def test_rsvd_block_product_full_size_sampled_columns():
    # the RSVD block product as the benchmark times it: gravity 200 x 150 x 12 (n = 360000),
    # k = 3750 FP32 vectors in one call each way; the first, a middle and the last column against
    # the oracle's direct sums
    s = W.SURVEYS["gravity_rsvd"]
    announce("block full size", "gravity_rsvd", 3750)
    g = ogeom(s)
    T = op.kernel_table(g)
    A = Operator(s, F32)
    k = 3750
    gen = torch.Generator(device="cuda").manual_seed(3)
    X = torch.randn(k, A.n, device="cuda", generator=gen)
    D = torch.randn(k, A.m, device="cuda", generator=gen)
    Y = A.G_block(X)
    Z = A.G_block(D, transpose=True)
    for c in (0, 1877, k - 1):
        agree(to_host(Y[c]), op.apply_G(g, to_host(X[c]), T), 1e-5)
        agree(to_host(Z[c]), op.apply_GT(g, to_host(D[c]), T), 1e-5)
    del X, D, Y, Z
    A.close()
    torch.cuda.empty_cache()


def test_empty_block_apply():
    # k = 0 vectors: empty results, nothing launched; through the C ABI with valid pointers too
    A = Operator(SMALL["wide_tail"], F32)
    assert tuple(A.G_block(torch.empty(0, A.n, device="cuda")).shape) == (0, A.m)
    assert tuple(A.G_block(torch.empty(0, A.m, device="cuda"), transpose=True).shape) == (0, A.n)
    x = torch.zeros(A.n, device="cuda")
    y = torch.full((A.m,), 3.0, device="cuda")
    L.call("apply_G_block", A.h, 0, 0, x.data_ptr(), A.n, y.data_ptr(), A.m, None, None, None)
    torch.cuda.synchronize()
    assert bool((y == 3.0).all())
    A.close()


def test_zero_and_impulse_inputs():
    s = SMALL["mag45"]
    g = ogeom(s)
    G = op.dense_G(g)
    A = Operator(s, F64)
    z = to_host(A.G(torch.zeros(g.n, dtype=F64, device="cuda")))
    assert np.all(z == 0)
    # G^T e_s is row s of G; G e_c is column c
    for st in (0, g.m - 1, 13):
        e = np.zeros(g.m)
        e[st] = 1.0
        agree(to_host(A.GT(to_dev(e, F64))), G[st], 1e-12)
    for c in (0, g.n - 1, 77):
        e = np.zeros(g.n)
        e[c] = 1.0
        agree(to_host(A.G(to_dev(e, F64))), G[:, c], 1e-12)


def test_deterministic_repeats():
    s = W.SURVEYS["gravity_l4"]
    A = Operator(s, F32)
    x = to_dev(W.uniform_model(s, 0), F32)
    ref = A.G(x)
    for _ in range(10):
        assert torch.equal(A.G(x), ref)


def test_wrong_tensor_arguments_raise():
    A = Operator(W.SURVEYS["tiny"], F32)
    with pytest.raises(L.FastFocusError):
        A.G(torch.zeros(10, dtype=F32, device="cuda"))
    with pytest.raises(L.FastFocusError):
        A.G(torch.zeros(A.n, dtype=F64, device="cuda"))


@pytest.mark.parametrize("name,dtype", [("mag_padded", F64), ("wide_tail", F32)])
def test_spectra_checkpoint_round_trip(tmp_path, name, dtype):
    s = SMALL[name]
    A = Operator(s, dtype)
    path = tmp_path / "op.ffs"
    A.save(str(path))
    B = Operator.load(str(path))
    assert B.dtype == dtype and B.nfft == A.nfft and (B.m, B.n) == (A.m, A.n)
    for k in ("sx", "sy", "nz", "dx", "dy", "kernel", "pad_xl", "pad_xr", "pad_yl", "pad_yr"):
        assert B.survey[k] == A.survey[k], k
    assert tuple(B.survey["z_edges"]) == tuple(A.survey["z_edges"])
    rng = np.random.default_rng(3)
    x = to_dev(rng.standard_normal(A.n), dtype)
    d = to_dev(rng.standard_normal(A.m), dtype)
    assert torch.equal(B.G(x), A.G(x))
    assert torch.equal(B.GT(d), A.GT(d))
    # a flipped spectra byte and a truncated file are refused
    raw = bytearray(path.read_bytes())
    bad = tmp_path / "bad.ffs"
    raw[len(raw) // 2] ^= 0x40
    bad.write_bytes(bytes(raw))
    with pytest.raises(L.FastFocusError):
        Operator.load(str(bad))
    bad.write_bytes(path.read_bytes()[:-100])
    with pytest.raises(L.FastFocusError):
        Operator.load(str(bad))


def _full_size_check(s, seed):
    # FP32 G and G^T at full size against the oracle's direct sums over the Toeplitz blocks
    g = ogeom(s)
    T = op.kernel_table(g)
    rng = np.random.default_rng(seed)
    x = rng.random(g.n)
    d = rng.standard_normal(g.m)
    A = Operator(s, F32)
    agree(to_host(A.G(to_dev(x, F32))), op.apply_G(g, x, T), 1e-5)
    agree(to_host(A.GT(to_dev(d, F32))), op.apply_GT(g, d, T), 1e-5)


@pytest.mark.parametrize("nz", [20, 239])
def test_table3_geometry_padded_many_layers(nz):
    # Table 3's field geometry: 62 x 62 stations, 5 padding cells per side, up to 239 thin
    # layers (n = 1238976); non-zero extraction offsets and a long layer loop
    announce("table3", nz)
    _full_size_check(W.table3_survey(nz), nz)


@pytest.mark.parametrize("ell,kernel", [(4, "gravity"), (7, "gravity"), (5, "magnetic"), (7, "magnetic")])
def test_padded_size_ladder(ell, kernel):
    # the padded ladder of Sec. 3.2 / Table 2 (pad = round(0.05 s) cells per side)
    announce("ladder", ell, kernel)
    _full_size_check(W.ladder_survey(ell, kernel), ell)


@pytest.mark.parametrize("ell,kernel", [(11, "magnetic"), (12, "gravity")])
def test_high_resolution_ladder(ell, kernel):
    # the high-resolution sizes of Sec. 3.3.3 (n = 998250 and 1296000, unpadded): 1024-point rows
    announce("ladder", ell, kernel)
    s = W.ladder_survey(ell, kernel, pad_fraction=0.0)
    assert W.sizes(s)[4] == {11: 998250, 12: 1296000}[ell]
    _full_size_check(s, ell)
