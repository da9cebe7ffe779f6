"""Seeded synthetic workloads shared by the tests, the benchmark and the checks.

This module holds geometry *parameters*, synthetic models and random draws, plus the noise
model and the SNR of the paper's experiments; it contains none of the method's arithmetic (no
kernel integrals, no operator, no solver).  Both the CPU
oracle and the HIP path build their own geometry objects from the plain dicts here.

Survey geometries follow the paper's setting (Sec. 2.1, Fig. 1): stations at the
centres of the surface cells, uniform prisms, z positive downward from the station
plane.  Sizes and models:

* ``tiny``       16 x 16 stations, 50 m cells, 4 layers of 50 m (m = 256, n = 1024),
                 gravity; m ~ U[0,1) seed 0, d ~ N(0,1) seed 1.
* ``gravity_l4`` 100 x 60 stations, 20 m cells, 10 layers of 40 m (m = 6000,
                 n = 60000), gravity; two 1 g/cc blocks, 1 % noise.  The paper's
                 smallest ladder grid (l = 4) with 10 layers.
* ``magnetic_1m`` 250 x 200 stations, 20 m cubes, 20 layers (m = 50000, n = 1e6),
                 TFA kernel, I = D = 45 deg, F = 50000 nT; 0.1 SI cube and
                 45-degree dipping dike, 2 % noise.
* ``gravity_rsvd`` 200 x 150 stations, 20 m cubes, 12 layers (m = 30000,
                 n = 360000), gravity; blocks of k = 3750 Gaussian vectors.
* ``gravity_diff`` 128 x 128 stations, 20 m cubes, 16 layers (m = 16384,
                 n = 262144), gravity; batch of 4 random block models.
* ``uneven_surveys`` eight gravity surveys from 32 x 32 x 6 to 180 x 120 x 16.
* ``table3_survey(nz)`` the field-data geometry of Table 3: 62 x 62 stations at 100 m, 5
                 padding cells on every side (72 x 72 prisms per layer), nz equal layers
                 down to 2000 m (nz = 20 .. 239, n up to 1238976); TFA kernel with an
                 assumed field (I = 75 deg, D = 5 deg, F = 50000 nT: the paper prints none
                 and its data set is not available).
* ``ladder_survey(l)`` the size ladder of Sec. 3.2 / Table 2: l (25, 15, 2) stations and
                 layers over 2000 x 1200 x 400 m, padded by round(0.05 s) cells per side
                 (round half away from zero).
* ``ladder_structure(s, kind)`` a stand-in for the volume structure of Sec. 3.2 on any ladder
                 grid: three boxes, an elongated well, a very small well and a dike dipping at
                 45 degrees over six 50 m depth bands, fixed in metres so that every l sees the
                 same bodies; density 1 for gravity; susceptibility 0.06 (dike and wells) and
                 0.04 (boxes) for magnetic data.  ``LADDER_TAU2`` holds the paper's noise
                 levels tau2 per l (tau1 = 0.02).

The paper's own synthetic structure exists only in its figures and its field data
set is not available; the models here stand in for them.
"""
from __future__ import annotations

import numpy as np


def survey(sx, sy, nz, dx, dy, dz, kernel="gravity", incl=90.0, decl=0.0, field=50000.0,
           pad=(0, 0, 0, 0)):
    return dict(sx=sx, sy=sy, nz=nz, dx=float(dx), dy=float(dy),
                z_edges=tuple(float(dz) * k for k in range(nz + 1)), kernel=kernel,
                incl_deg=float(incl), decl_deg=float(decl), field_nT=float(field),
                pad_xl=pad[0], pad_xr=pad[1], pad_yl=pad[2], pad_yr=pad[3])


SURVEYS = {
    "tiny": survey(16, 16, 4, 50, 50, 50),
    "gravity_l4": survey(100, 60, 10, 20, 20, 40),
    "magnetic_1m": survey(250, 200, 20, 20, 20, 20, kernel="magnetic", incl=45.0, decl=45.0),
    "gravity_rsvd": survey(200, 150, 12, 20, 20, 20),
    "gravity_diff": survey(128, 128, 16, 20, 20, 20),
}


def table3_survey(nz, incl=75.0, decl=5.0):
    return dict(sx=62, sy=62, nz=nz, dx=100.0, dy=100.0,
                z_edges=tuple(2000.0 * k / nz for k in range(nz + 1)), kernel="magnetic",
                incl_deg=float(incl), decl_deg=float(decl), field_nT=50000.0,
                pad_xl=5, pad_xr=5, pad_yl=5, pad_yr=5)


TABLE3_NZ = (20, 40, 59, 80, 100, 119, 160, 200, 239)


def _round_half_away(v):
    return int(np.floor(abs(v) + 0.5)) * (1 if v >= 0 else -1)


def ladder_survey(ell, kernel="gravity", pad_fraction=0.05, incl=45.0, decl=45.0):
    sx, sy, nz = 25 * ell, 15 * ell, 2 * ell
    px, py = _round_half_away(pad_fraction * sx), _round_half_away(pad_fraction * sy)
    return survey(sx, sy, nz, 2000.0 / sx, 1200.0 / sy, 400.0 / nz, kernel=kernel, incl=incl, decl=decl,
                  pad=(px, px, py, py))


# tau2 of eq. (noisydata) per ladder size l, gravity and magnetic, with tau1 = 0.02 (the table of
# problem dimensions in Sec. 3.2; chosen there to give an SNR of about 24 dB for the paper's structure)
LADDER_TAU1 = 0.02
LADDER_TAU2 = {4: (0.0138, 0.0081), 5: (0.0147, 0.0083), 6: (0.0133, 0.0074), 7: (0.0133, 0.0070),
               8: (0.0133, 0.0071), 9: (0.0133, 0.0069), 10: (0.0132, 0.0070), 11: (0.0135, 0.0075),
               12: (0.0135, 0.0075)}

# Bodies of the ladder structure in metres over the 2000 x 1200 x 400 m station domain (x along the
# sx stations, y along sy, z down).  Boxes: (x0, x1, y0, y1, z0, z1, susceptibility); the dike's top
# x-range [x0, x1) moves by +1 m per metre of depth between z0 and z1.
LADDER_BOXES = [(250.0, 600.0, 250.0, 550.0, 50.0, 150.0, 0.04),
                (1300.0, 1700.0, 650.0, 1000.0, 100.0, 250.0, 0.04),
                (700.0, 1000.0, 800.0, 1000.0, 25.0, 100.0, 0.04),
                (400.0, 475.0, 700.0, 1100.0, 50.0, 300.0, 0.06),      # elongated well
                (1750.0, 1800.0, 250.0, 300.0, 25.0, 75.0, 0.06)]      # very small well
LADDER_DIKE = (1000.0, 1100.0, 200.0, 550.0, 50.0, 350.0, 0.06)


def ladder_structure(s, kind="gravity"):
    """Model vector (layer, row, column) of the ladder structure on survey s: a cell takes a body's
    value when its centre lies inside the body (half-open extents); gravity uses 1 for every body.
    Padding cells lie outside the station domain and stay 0."""
    nx, ny, nz, _, _ = sizes(s)
    xc = (np.arange(nx) - s["pad_xl"] + 0.5) * s["dx"]
    yc = (np.arange(ny) - s["pad_yl"] + 0.5) * s["dy"]
    ze = np.asarray(s["z_edges"])
    zc = 0.5 * (ze[:-1] + ze[1:])
    Z, Y, X = np.meshgrid(zc, yc, xc, indexing="ij")
    out = np.zeros((nz, ny, nx))
    for x0, x1, y0, y1, z0, z1, v in LADDER_BOXES:
        inside = (X >= x0) & (X < x1) & (Y >= y0) & (Y < y1) & (Z >= z0) & (Z < z1)
        out[inside] = 1.0 if kind == "gravity" else v
    x0, x1, y0, y1, z0, z1, v = LADDER_DIKE
    shift = Z - z0
    inside = (X >= x0 + shift) & (X < x1 + shift) & (Y >= y0) & (Y < y1) & (Z >= z0) & (Z < z1)
    out[inside] = 1.0 if kind == "gravity" else v
    return out.reshape(-1)


def snr_db(d_exact, eta):
    """eq. (SNR): 20 log10(||d_exact|| / ||d_obs - d_exact||)."""
    return float(20.0 * np.log10(np.linalg.norm(d_exact) / np.linalg.norm(eta)))


UNEVEN = [(32, 32, 6), (48, 48, 8), (64, 48, 8), (80, 64, 10), (100, 60, 10),
          (128, 96, 12), (160, 100, 14), (180, 120, 16)]


def uneven_surveys():
    return [survey(sx, sy, nz, 20, 20, 20) for sx, sy, nz in UNEVEN]


def sizes(s):
    nx = s["sx"] + s["pad_xl"] + s["pad_xr"]
    ny = s["sy"] + s["pad_yl"] + s["pad_yr"]
    return nx, ny, s["nz"], s["sx"] * s["sy"], nx * ny * s["nz"]


def rng(seed):
    return np.random.default_rng(seed)


def uniform_model(s, seed=0):
    """m ~ U[0, 1) over the model vector (layer, row, column), float64."""
    n = sizes(s)[4]
    return rng(seed).random(n)


def gaussian_data(s, seed=1):
    """d ~ N(0, 1) over the data vector (row, column), float64."""
    m = sizes(s)[3]
    return rng(seed).standard_normal(m)


def gaussian_matrix(rows, cols, seed):
    """rows x cols standard normal matrix (float64, C order)."""
    return rng(seed).standard_normal((rows, cols))


def block_model(s, blocks):
    """Model vector with value v in each cell box (p0, p1, q0, q1, r0, r1, v), half-open."""
    nx, ny, nz, _, _ = sizes(s)
    x = np.zeros((nz, ny, nx))
    for p0, p1, q0, q1, r0, r1, v in blocks:
        x[r0:r1, q0:q1, p0:p1] = v
    return x.reshape(-1)


# gravity_l4: blocks at x in [500, 800), y in [400, 700), z in [40, 160) and
# x in [1200, 1500), y in [500, 900), z in [80, 240) (20 m cells, 40 m layers)
GRAVITY_L4_BLOCKS = [(25, 40, 20, 35, 1, 4, 1.0), (60, 75, 25, 45, 2, 6, 1.0)]


def dike_cells(p0, width, q0, q1, r0, r1):
    """A 45-degree dipping dike on a grid with dx = dz: shifts one column per layer."""
    return [(p0 + r, p0 + r + width, q0, q1, r, r + 1, 0.1) for r in range(r0, r1)]


MAGNETIC_1M_BLOCKS = [(60, 70, 80, 90, 3, 13, 0.1)] + dike_cells(150, 3, 50, 150, 2, 16)


def gravity_diff_models(s, batch=4, seed=5):
    """batch random block models with 1-3 cell-aligned blocks, density U[0.5, 1]."""
    nx, ny, nz, _, _ = sizes(s)
    g = rng(seed)
    out = []
    for _ in range(batch):
        blocks = []
        for _ in range(int(g.integers(1, 4))):
            w, h, t = (int(g.integers(4, 24)), int(g.integers(4, 24)), int(g.integers(2, 6)))
            p0 = int(g.integers(0, nx - w)); q0 = int(g.integers(0, ny - h))
            r0 = int(g.integers(0, nz - t))
            blocks.append((p0, p0 + w, q0, q0 + h, r0, r0 + t, float(g.uniform(0.5, 1.0))))
        out.append(block_model(s, blocks))
    return np.stack(out)


def noise(d_exact, tau1, tau2, seed):
    """Noise vector and its standard deviations per eq. (noisydata) of the paper:
    eta_i = (tau1 |d_i| + tau2 ||d||_inf) e_i, e ~ N(0, 1).  Returns (eta, sigma)."""
    d_exact = np.asarray(d_exact, dtype=np.float64)
    sigma = tau1 * np.abs(d_exact) + tau2 * np.abs(d_exact).max()
    e = rng(seed).standard_normal(d_exact.shape[0])
    return sigma * e, sigma
