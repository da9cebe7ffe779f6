"""Uneven multi-survey batch in one HIP graph, and the launch autotuner."""
import os

import numpy as np
import pytest
import torch

from gpu_common import ogeom, otable, rel, to_dev, to_host
from oracle import operator as op
from paper_2004_13904_amd import workloads as W
from paper_2004_13904_amd.autotune import autotune
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
    # and against the oracle for the smallest and a mid-size survey
    for i in (0, 4):
        gi = ogeom(surveys[i])
        T = op.kernel_table(gi)
        assert rel(to_host(B.gx[i]), op.apply_G(gi, to_host(xs[i]), T)) <= 1e-5
        assert rel(to_host(B.gtd[i]), op.apply_GT(gi, to_host(ds[i]), T)) <= 1e-5


def test_autotune_picks_valid_tuning_and_keeps_results(tmp_path):
    s = W.SURVEYS["gravity_l4"]
    A = Operator(s, F32)
    x = to_dev(W.uniform_model(s, 0), F32)
    d = to_dev(W.gaussian_data(s, 1), F32)
    ref_g, ref_t = A.G(x).clone(), A.GT(d).clone()
    cache = str(tmp_path / "tune.json")
    choice = autotune(A, x, d, cache=cache)
    assert 1 <= choice["lg_G"] <= A.nz and 1 <= choice["lg_GT"] <= A.nz
    assert os.path.exists(cache)
    # the tuning changes only the summation order of the layer groups
    assert rel(to_host(A.G(x)), to_host(ref_g)) <= 1e-6
    assert rel(to_host(A.GT(d)), to_host(ref_t)) <= 1e-6
    B = Operator(s, F32)
    assert autotune(B, x, d, cache=cache) == choice     # cache hit
    assert B.tuning == choice
