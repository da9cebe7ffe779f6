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


def _pow2_at_least(v):
    p = 1
    while p < v:
        p *= 2
    return p


def test_named_surveys_sizes_and_embeddings():
    """Stations m, cells n and the smallest power-of-two embedding N >= s + n - 1 per axis."""
    want = {"tiny": (256, 1024, (32, 32)), "gravity_l4": (6000, 60000, (256, 128)),
            "magnetic_1m": (50000, 1000000, (512, 512)), "gravity_rsvd": (30000, 360000, (512, 512)),
            "gravity_diff": (16384, 262144, (256, 256))}
    assert sorted(W.SURVEYS) == sorted(want)
    for name, (m, n, emb) in want.items():
        s = W.SURVEYS[name]
        nx, ny, nz, mm, nn = W.sizes(s)
        assert (mm, nn) == (m, n)
        assert (_pow2_at_least(s["sx"] + nx - 1), _pow2_at_least(s["sy"] + ny - 1)) == emb
    assert W.SURVEYS["magnetic_1m"]["kernel"] == "magnetic"


def test_uneven_surveys_span_the_embedding_sizes():
    """Eight gravity surveys of 20 m cubes whose embeddings run from 64 x 64 to 512 x 256."""
    embs = []
    for s in W.uneven_surveys():
        nx, ny, _, _, _ = W.sizes(s)
        assert s["dx"] == s["dy"] == 20.0 and s["kernel"] == "gravity"
        embs.append((_pow2_at_least(s["sx"] + nx - 1), _pow2_at_least(s["sy"] + ny - 1)))
    assert len(embs) == 8 and embs[0] == (64, 64) and embs[-1] == (512, 256)
    assert len(set(embs)) >= 5


def test_block_models_in_metres():
    """The gravity_l4 blocks (20 m cells, 40 m layers) cover x [500, 800), y [400, 700),
    z [40, 160) and x [1200, 1500), y [500, 900), z [80, 240) at 1 g/cc."""
    s = W.SURVEYS["gravity_l4"]
    nx, ny, nz, _, _ = W.sizes(s)
    m = W.block_model(s, W.GRAVITY_L4_BLOCKS).reshape(nz, ny, nx)
    ze = np.asarray(s["z_edges"])
    boxes = [(500, 800, 400, 700, 40, 160), (1200, 1500, 500, 900, 80, 240)]
    xc = (np.arange(nx) + 0.5) * s["dx"]
    yc = (np.arange(ny) + 0.5) * s["dy"]
    zc = 0.5 * (ze[:-1] + ze[1:])
    Z, Y, X = np.meshgrid(zc, yc, xc, indexing="ij")
    inside = np.zeros_like(m, dtype=bool)
    for x0, x1, y0, y1, z0, z1 in boxes:
        inside |= (X >= x0) & (X < x1) & (Y >= y0) & (Y < y1) & (Z >= z0) & (Z < z1)
    assert np.array_equal(m > 0, inside) and set(np.unique(m)) == {0.0, 1.0}


def test_magnetic_1m_cube_and_dike():
    """A 10-cell cube of 0.1 SI at 60-260 m depth and a 3-cell-thick dike, 100 cells along
    strike, in layers 2-15, moving one column per 20 m layer (45 degrees on 20 m cubes)."""
    s = W.SURVEYS["magnetic_1m"]
    nx, ny, nz, _, _ = W.sizes(s)
    m = W.block_model(s, W.MAGNETIC_1M_BLOCKS).reshape(nz, ny, nx)
    cube = W.MAGNETIC_1M_BLOCKS[0]
    p0, p1, q0, q1, r0, r1, v = cube
    assert (p1 - p0, q1 - q0, r1 - r0, v) == (10, 10, 10, 0.1)
    assert (s["z_edges"][r0], s["z_edges"][r1]) == (60.0, 260.0)
    assert np.all(m[r0:r1, q0:q1, p0:p1] == 0.1)
    dike = W.MAGNETIC_1M_BLOCKS[1:]
    assert [b[4] for b in dike] == list(range(2, 16))
    for (a0, a1, b0, b1, r, _, val), nxt in zip(dike, dike[1:] + [None]):
        assert (a1 - a0, b1 - b0, val) == (3, 100, 0.1)
        if nxt is not None:
            assert nxt[0] == a0 + 1
    # the cube (columns 60-69) and the dike (columns 152 and beyond) do not overlap
    assert np.count_nonzero(m) == 10 * 10 * 10 + 14 * 3 * 100
