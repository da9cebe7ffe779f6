"""Host-side checks of the seeded workloads: the ladder structure stand-in and the noise levels."""
import numpy as np
import pytest

from paper_2004_13904_amd import workloads as W


def _body_volume():
    v = sum((x1 - x0) * (y1 - y0) * (z1 - z0) for x0, x1, y0, y1, z0, z1, _ in W.LADDER_BOXES)
    x0, x1, y0, y1, z0, z1, _ = W.LADDER_DIKE
    return v + (x1 - x0) * (y1 - y0) * (z1 - z0)


@pytest.mark.parametrize("ell", [4, 5, 7, 12])
def test_ladder_structure_volume_converges(ell):
    """The rasterized bodies fill their metric volume up to cell-size effects that shrink with l."""
    s = W.ladder_survey(ell, pad_fraction=0.0)
    m = W.ladder_structure(s, "gravity")
    cell = s["dx"] * s["dy"] * (s["z_edges"][1] - s["z_edges"][0])
    vol = (m > 0).sum() * cell
    assert abs(vol / _body_volume() - 1.0) < 0.6 / ell


@pytest.mark.parametrize("ell", [4, 6])
def test_ladder_structure_padding_and_values(ell):
    """Padding cells stay empty, the interior equals the unpadded structure, and the magnetic
    values are 0.06 (dike, wells) and 0.04 (boxes)."""
    s0 = W.ladder_survey(ell, pad_fraction=0.0)
    s1 = W.ladder_survey(ell, pad_fraction=0.05)
    nx0, ny0, nz, _, _ = W.sizes(s0)
    nx1, ny1, _, _, _ = W.sizes(s1)
    for kind in ("gravity", "magnetic"):
        a = W.ladder_structure(s0, kind).reshape(nz, ny0, nx0)
        b = W.ladder_structure(s1, kind).reshape(nz, ny1, nx1)
        px, py = s1["pad_xl"], s1["pad_yl"]
        assert px > 0 and py > 0
        assert np.array_equal(b[:, py:py + ny0, px:px + nx0], a)
        assert np.count_nonzero(b) == np.count_nonzero(a)
    mag = W.ladder_structure(s0, "magnetic")
    assert set(np.unique(mag)) == {0.0, 0.04, 0.06}
    grav = W.ladder_structure(s0, "gravity")
    assert np.array_equal(grav > 0, mag > 0)


def test_ladder_dike_dips_45_degrees():
    """The dike's x-extent moves by one metre per metre of depth: on l = 8 (dx = 10 m, dz = 25 m)
    its first occupied column moves by 2.5 cells per layer on average."""
    s = W.ladder_survey(8, pad_fraction=0.0)
    nx, ny, nz, _, _ = W.sizes(s)
    m = W.ladder_structure(s, "gravity").reshape(nz, ny, nx)
    x0, x1, y0, y1, z0, z1, _ = W.LADDER_DIKE
    q = int((y0 + y1) / 2 / s["dy"])
    firsts = []
    for r in range(nz):
        zc = 0.5 * (s["z_edges"][r] + s["z_edges"][r + 1])
        if z0 <= zc < z1:
            cols = np.nonzero(m[r, q, int(900 / s["dx"]):])[0]
            firsts.append(cols[0])
    slope = np.polyfit(np.arange(len(firsts)), firsts, 1)[0]
    assert len(firsts) == 12 and abs(slope - 2.5) < 0.1


def test_snr_and_tau_table():
    """eq. (SNR) on a constructed case, and the tau2 table covers l = 4 .. 12 with tau2 < tau1."""
    d = np.full(100, 3.0)
    eta = np.full(100, 0.3)
    assert abs(W.snr_db(d, eta) - 20.0) < 1e-12
    assert sorted(W.LADDER_TAU2) == list(range(4, 13))
    assert all(0 < g < W.LADDER_TAU1 and 0 < mg < W.LADDER_TAU1 for g, mg in W.LADDER_TAU2.values())
