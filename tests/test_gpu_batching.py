"""Uneven multi-survey batch in one HIP graph, and the launch autotuner."""
import json
import os

import numpy as np
import pytest
import torch

from gpu_common import agree, announce, ogeom, otable, rel, to_dev, to_host
from oracle import operator as op
from paper_2004_13904_amd import workloads as W
from paper_2004_13904_amd.autotune import autotune, candidates, fft_plans
from paper_2004_13904_amd.operator import Operator, SurveyBatch

pytestmark = pytest.mark.gpu
F32 = torch.float32


def test_uneven_surveys_in_one_graph():
    surveys = W.uneven_surveys()
    B = SurveyBatch(surveys, F32)
    g = torch.Generator(device="cuda").manual_seed(0)
    xs = [torch.rand(o.n, device="cuda", generator=g) for o in B.ops]
    ds = [torch.randn(o.m, device="cuda", generator=g) for o in B.ops]
    B.bind(xs, ds)
    assert B.grouped_launches          # all eight fit the grouped kernels (FP32, <= 512 x 512)
    # the grouped launches without the graph
    B.apply()
    torch.cuda.synchronize()
    for o, x, d, a, b in zip(B.ops, xs, ds, B.gx, B.gtd):
        assert torch.equal(a, o.G(x))
        assert torch.equal(b, o.GT(d))
    for rep in range(3):
        # new inputs between replays, eager work in between, every replay checked
        for x, d in zip(xs, ds):
            x.uniform_(generator=g)
            d.normal_(generator=g)
        B.replay()
        torch.cuda.synchronize()
        for o, x, d, a, b in zip(B.ops, xs, ds, B.gx, B.gtd):
            assert torch.equal(a, o.G(x))
            assert torch.equal(b, o.GT(d))
    # and every survey against the oracle's direct sums (relative l2 and worst element)
    for i in range(len(surveys)):
        gi = ogeom(surveys[i])
        T = op.kernel_table(gi)
        agree(to_host(B.gx[i]), op.apply_G(gi, to_host(xs[i]), T), 1e-5)
        agree(to_host(B.gtd[i]), op.apply_GT(gi, to_host(ds[i]), T), 1e-5)


def test_grouped_plan_partial_products_and_fallback():
    # G only for some surveys, G^T only for others; a layer-group tuning of 2; and an FP64 batch,
    # which the grouped kernels do not take (per-survey launches instead)
    surveys = W.uneven_surveys()[:4]
    ops = [Operator(s, F32) for s in surveys]
    ops[1].set_tuning(lg_G=2, lg_GT=2)
    g = torch.Generator(device="cuda").manual_seed(1)
    xs = [torch.rand(o.n, device="cuda", generator=g) for o in ops]
    ds = [torch.randn(o.m, device="cuda", generator=g) for o in ops]
    gx = [torch.full((o.m,), -1.0, device="cuda") for o in ops]
    gtd = [torch.full((o.n,), -1.0, device="cuda") for o in ops]
    import ctypes as C
    from paper_2004_13904_amd import _lib as L
    arr = C.c_void_p * 4
    use_g, use_t = [True, True, False, True], [True, False, True, True]
    plan = C.c_void_p()
    L.call("ff_multi_create", 4, arr(*[o.h.value for o in ops]),
           arr(*[x.data_ptr() if u else None for x, u in zip(xs, use_g)]),
           arr(*[y.data_ptr() if u else None for y, u in zip(gx, use_g)]),
           arr(*[d.data_ptr() if u else None for d, u in zip(ds, use_t)]),
           arr(*[y.data_ptr() if u else None for y, u in zip(gtd, use_t)]), C.byref(plan))
    L.call("ff_multi_apply", plan, C.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    for o, x, d, a, b, ug, ut in zip(ops, xs, ds, gx, gtd, use_g, use_t):
        if ug:
            assert torch.equal(a, o.G(x))
        else:
            assert bool((a == -1.0).all())
        if ut:
            assert torch.equal(b, o.GT(d))
        else:
            assert bool((b == -1.0).all())
    L.call("ff_multi_free", plan)
    # the same handle twice is refused
    with pytest.raises(L.FastFocusError):
        L.call("ff_multi_create", 2, arr(ops[0].h.value, ops[0].h.value), arr(xs[0].data_ptr(), xs[0].data_ptr()),
               arr(gx[0].data_ptr(), gx[0].data_ptr()), None, None, C.byref(plan))
    B = SurveyBatch(surveys, torch.float64)
    xs64 = [x.double() for x in xs]
    ds64 = [d.double() for d in ds]
    B.bind(xs64, ds64)
    assert not B.grouped_launches
    B.replay()
    torch.cuda.synchronize()
    for o, x, d, a, b in zip(B.ops, xs64, ds64, B.gx, B.gtd):
        assert torch.equal(a, o.G(x))
        assert torch.equal(b, o.GT(d))


def test_autotune_picks_valid_tuning_and_keeps_results(tmp_path):
    s = W.SURVEYS["gravity_l4"]
    A = Operator(s, F32)
    x = to_dev(W.uniform_model(s, 0), F32)
    d = to_dev(W.gaussian_data(s, 1), F32)
    cache = str(tmp_path / "tune.json")
    choice = autotune(A, x, d, cache=cache, reps=5)
    assert 1 <= choice["lg_G"] <= A.nz and 1 <= choice["lg_GT"] <= A.nz
    assert choice["row_tile"] in (0, 1, 2, 3, 4)
    assert choice["fft_plan_x"] in fft_plans(A.nfft[0]) and choice["fft_plan_y"] in fft_plans(A.nfft[1])
    assert os.path.exists(cache)
    with open(cache) as f:
        assert list(json.load(f)) == [f"NX{A.nfft[0]}:NY{A.nfft[1]}:nz{A.nz}:k1:{A.dtype}"]
    # the chosen tuning against the oracle's direct sums
    g = ogeom(s)
    agree(to_host(A.G(x)), op.apply_G(g, to_host(x), otable("gravity_l4")), 1e-5)
    agree(to_host(A.GT(d)), op.apply_GT(g, to_host(d), otable("gravity_l4")), 1e-5)
    B = Operator(s, F32)
    assert autotune(B, x, d, cache=cache) == choice     # cache hit
    assert B.tuning == choice


# embeddings 32 x 32 (pruned transforms), 128 x 128 (pruned, three plans on both axes) and
# 64 x 64 (unpruned: the data rows and model rows reach past the half of the embedding; plans 0
# and 2 only, 64 being a power of 8)
CANDIDATE_SURVEYS = {
    "tiny": W.SURVEYS["tiny"],
    "s40x33": W.survey(40, 33, 5, 20, 20, 20, kernel="magnetic", incl=60.0, decl=-20.0),
    "padded64": W.survey(20, 20, 4, 20, 20, 20, pad=(14, 0, 14, 0)),
}


@pytest.mark.parametrize("name", list(CANDIDATE_SURVEYS))
def test_every_tuning_candidate_matches_oracle(name):
    # every value the autotuner may try, one key at a time from the default tuning, and every
    # pair of row and column stage plans, for single and block products (5 vectors: the batched
    # column passes), against the oracle's direct sums at the FP32 bar
    s = CANDIDATE_SURVEYS[name]
    A = Operator(s, F32)
    g = ogeom(s)
    T = op.kernel_table(g)
    rng = np.random.default_rng(12)
    X = rng.random((5, g.n))
    D = rng.standard_normal((5, g.m))
    GX = np.stack([op.apply_G(g, v, T) for v in X])
    GTD = np.stack([op.apply_GT(g, v, T) for v in D])
    Xd, Dd = to_dev(X, F32), to_dev(D, F32)
    base = A.tuning
    cand = candidates(A, batched=True)
    configs = [dict(base, **{k: v}) for k, vals in cand.items() for v in vals]
    configs += [dict(base, fft_plan_x=px, fft_plan_y=py) for px in cand["fft_plan_x"] for py in cand["fft_plan_y"]]
    if name == "tiny":
        assert cand["fft_plan_x"] == cand["fft_plan_y"] == [0, 1, 2]
    if name == "padded64":
        assert A.nfft == (64, 64) and cand["fft_plan_y"] == [0, 2]
    for cfg in configs:
        A.set_tuning(**cfg)
        announce("tuning candidate", name, cfg)
        agree(to_host(A.G(Xd[0])), GX[0], 1e-5)
        agree(to_host(A.GT(Dd[0])), GTD[0], 1e-5)
        agree(to_host(A.G_block(Xd)), GX, 1e-5)
        agree(to_host(A.G_block(Dd, transpose=True)), GTD, 1e-5)


def test_tuning_variants_keep_results():
    s = W.SURVEYS["gravity_l4"]
    A = Operator(s, F32)
    g = torch.Generator(device="cuda").manual_seed(4)
    X = torch.rand(6, A.n, device="cuda", generator=g)
    D = torch.randn(6, A.m, device="cuda", generator=g)
    ref_g, ref_t = A.G_block(X).clone(), A.G_block(D, transpose=True).clone()
    base = A.tuning
    assert base["batch"] == A.batch_max >= 16 and base["col_batched"] == 2
    # the row tile changes only which block runs a row transform: bit-identical
    for tile in (1, 2, 3, 4, 0):
        A.set_tuning(row_tile=tile)
        assert torch.equal(A.G_block(X), ref_g)
        assert torch.equal(A.G_block(D, transpose=True), ref_t)
    # batch schedule and per-vector column blocks: the same sums in another order
    for kw in ({"batch": 1}, {"batch": 4}, {"batch": 5}, {"batch": A.batch_max, "col_batched": 0},
               {"col_batched": 1}, {"batch": 5, "col_batched": 1}, {"batch": 5, "col_batched": 2}):
        A.set_tuning(**kw)
        assert rel(to_host(A.G_block(X)), to_host(ref_g)) <= 2e-6
        assert rel(to_host(A.G_block(D, transpose=True)), to_host(ref_t)) <= 2e-6
    from paper_2004_13904_amd import _lib as L
    for bad in ({"row_tile": 5}, {"batch": 0}, {"batch": A.batch_max + 1}, {"col_batched": 3}, {"rsvd_qr": 3},
                {"lg_G": 0}, {"lg_GT": A.nz + 1}, {"gkb_onesided": 3}, {"gkb_onesided": -1}):
        with pytest.raises(L.FastFocusError):
            A.set_tuning(**bad)
    A.set_tuning(**base)
    assert A.tuning == base


@pytest.mark.parametrize("name", ["magnetic_1m", "padded_heavy", "many_layers", "tiny", "gravity_l4"])
def test_pair_plan_equals_separate_calls(name):
    # the grouped plan of one survey with both products, its column pass shared by G x and G^T d
    # (forced with pair_fused = 2 where the default would not pick it): equal bit for bit to
    # apply_G / apply_GT, and within the bars of the oracle.  The geometries cover the pruned
    # transforms (rows in the first half of the embedding) and the unpruned ones (heavy padding:
    # ny > NY/2), several columns per wave (NY < 512), fewer layers than wave groups (tiny), more
    # layers than fit one wave group's pipeline (many_layers) and the packed DC/Nyquist slot.
    import ctypes as C
    from paper_2004_13904_amd import _lib as L
    s = {"magnetic_1m": W.SURVEYS["magnetic_1m"], "tiny": W.SURVEYS["tiny"],
         "gravity_l4": W.SURVEYS["gravity_l4"],
         "padded_heavy": W.survey(20, 14, 5, 20.0, 20.0, 20.0, kernel="magnetic", incl=60.0, decl=-20.0,
                                  pad=(30, 25, 31, 24)),
         "many_layers": W.survey(23, 19, 33, 25.0, 25.0, 12.0, kernel="magnetic", incl=70.0, decl=10.0)}[name]
    A = Operator(s, F32)
    A.set_tuning(pair_fused=2)
    g = torch.Generator(device="cuda").manual_seed(21)
    x = torch.rand(A.n, device="cuda", generator=g)
    d = torch.randn(A.m, device="cuda", generator=g)
    gx = torch.full((A.m,), float("nan"), device="cuda")
    gtd = torch.full((A.n,), float("nan"), device="cuda")
    arr = C.c_void_p * 1
    plan = C.c_void_p()
    L.call("ff_multi_create", 1, arr(A.h.value), arr(x.data_ptr()), arr(gx.data_ptr()), arr(d.data_ptr()),
           arr(gtd.data_ptr()), C.byref(plan))
    for _ in range(2):
        L.call("ff_multi_apply", plan, C.c_void_p(torch.cuda.current_stream().cuda_stream))
        torch.cuda.synchronize()
        assert torch.equal(gx, A.G(x))
        assert torch.equal(gtd, A.GT(d))
    L.load().ff_multi_free(plan)
    gi = ogeom(s)
    T = op.kernel_table(gi)
    agree(to_host(gx), op.apply_G(gi, to_host(x), T), 1e-5)
    agree(to_host(gtd), op.apply_GT(gi, to_host(d), T), 1e-5)
    A.close()
