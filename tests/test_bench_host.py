"""Host-side checks of bench.py's contract and byte models (no GPU needed)."""
import types

import bench


def test_more_than_one_gpu_is_refused(capsys):
    # the bench measures one GPU; --gpus N > 1 exits with a message instead of running
    assert bench.main(["--gpus", "2"]) == 2
    assert "one GPU" in capsys.readouterr().err


def _fake_operator(survey, nfft, lg_G=1):
    # the fields the byte models read, for a survey of the named workloads
    nx = survey["sx"] + survey.get("pad_xl", 0) + survey.get("pad_xr", 0)
    ny = survey["sy"] + survey.get("pad_yl", 0) + survey.get("pad_yr", 0)
    return types.SimpleNamespace(survey=survey, nfft=nfft, ny=ny, n=nx * ny * survey["nz"],
                                 m=survey["sx"] * survey["sy"], tuning={"lg_G": lg_G, "lg_GT": lg_G})


def test_pass_model_of_the_headline_pair():
    # the magnetic n = 1e6 survey in a 512 x 512 embedding: the method's bytes of one product are
    # 4n + 4m + the spectra (20 layers x 512 x 257 complex64) = 25.25 MB, and the pair's column
    # pass moves the model rows' intermediate twice, the data rows' twice and the spectra once
    from paper_2004_13904_amd import workloads as W
    A = _fake_operator(W.SURVEYS["magnetic_1m"], (512, 512))
    S = 20 * 257 * 512 * 8
    assert 4 * A.n + 4 * A.m + S == 25_253_440
    pm = bench.pass_model_bytes(A)
    X1 = 20 * 200 * 256 * 8
    D1 = 200 * 256 * 8
    assert pm["pair.cols"] == 2 * X1 + 2 * D1 + S
    assert pm["pair.rows"] == pm["pair.irows"] == 4 * A.n + 4 * A.m + X1 + D1
