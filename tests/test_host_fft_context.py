"""The bench's host rendering of the paper's method (scipy FFTs on the BCCB embedding, reading R3
of the circulant placement) agrees with the oracle's direct sums: an independent host check of the
embedding, cropping and adjoint placement, with and without padding."""
import numpy as np
import pytest

import bench
from oracle import geometry, operator as op
from paper_2004_13904_amd import workloads as W


@pytest.mark.parametrize("s", [W.SURVEYS["tiny"],
                               W.survey(9, 7, 3, 25, 25, 25, kernel="magnetic", incl=45, decl=45, pad=(2, 1, 0, 3))])
def test_host_fft_pair_matches_direct_sums(s):
    g = geometry.Geometry(**s)
    T = op.kernel_table(g)
    x = W.uniform_model(s, 0)
    d = W.gaussian_data(s, 1)
    rd, rx = op.apply_G(g, x, T), op.apply_GT(g, d, T)
    NX = 1 << int(np.ceil(np.log2(g.sx + g.nx - 1)))
    NY = 1 << int(np.ceil(np.log2(g.sy + g.ny - 1)))
    out = bench.host_fft_pairs(g, T, x, d, rd, rx, (NX, 2 * NY))     # a larger embedding is exact too
    assert out["rel_err_vs_oracle"]["G"] < 1e-13 and out["rel_err_vs_oracle"]["GT"] < 1e-13
    assert out["value"] > 0
