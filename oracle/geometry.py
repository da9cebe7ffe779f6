"""Survey / volume bookkeeping (oracle; test infrastructure only).

Sec. 2.1 and Fig. 1 of the paper: stations s_ij on the surface at the centres of the
unpadded surface cells, prisms c_pqr on a uniform grid with optional padding cells
(no stations over them), m = s_x s_y data and n = n_x n_y n_z unknowns.

Vector layouts (the paper does not fix the order in which its 2-D arrays become vectors;
this reading is fixed for the whole project): the model vector is ordered (layer r, row q,
column p) with p fastest, the data vector (row j, column i) with i fastest.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class Geometry:
    sx: int
    sy: int
    nz: int
    dx: float
    dy: float
    z_edges: tuple            # nz + 1 depths, z_edges[0] = 0 is the station plane
    kernel: str = "gravity"   # "gravity" (g_z, mGal per g/cc) or "magnetic" (TFA, nT per SI)
    pad_xl: int = 0
    pad_xr: int = 0
    pad_yl: int = 0
    pad_yr: int = 0
    incl_deg: float = 90.0
    decl_deg: float = 0.0
    field_nT: float = 50000.0

    def __post_init__(self):
        if len(self.z_edges) != self.nz + 1:
            raise ValueError("z_edges needs nz + 1 entries")
        if self.z_edges[0] != 0.0 or any(b <= a for a, b in zip(self.z_edges, self.z_edges[1:])):
            raise ValueError("z_edges must start at 0 and increase")
        if self.kernel not in ("gravity", "magnetic"):
            raise ValueError("kernel must be 'gravity' or 'magnetic'")

    @property
    def nx(self):
        return self.sx + self.pad_xl + self.pad_xr

    @property
    def ny(self):
        return self.sy + self.pad_yl + self.pad_yr

    @property
    def m(self):
        return self.sx * self.sy

    @property
    def n(self):
        return self.nx * self.ny * self.nz

    def station_xy(self, i, j):
        """Station (i, j) sits at the centre of surface cell (i + p_xL, j + p_yL)."""
        return ((np.asarray(i) + self.pad_xl + 0.5) * self.dx,
                (np.asarray(j) + self.pad_yl + 0.5) * self.dy)

    def cell_bounds(self, p, q, r):
        """Absolute bounds (x1, x2, y1, y2, z1, z2) of prism (p, q, r)."""
        p, q, r = np.asarray(p), np.asarray(q), np.asarray(r)
        ze = np.asarray(self.z_edges, dtype=np.float64)
        return (p * self.dx, (p + 1) * self.dx, q * self.dy, (q + 1) * self.dy, ze[r], ze[r + 1])

    def layer_mid_depths(self):
        ze = np.asarray(self.z_edges, dtype=np.float64)
        return 0.5 * (ze[1:] + ze[:-1])


def uniform_geometry(sx, sy, nz, dx, dy, dz, kernel="gravity", pad=(0, 0, 0, 0), **mag):
    """Geometry with nz equal layers of thickness dz."""
    return Geometry(sx=sx, sy=sy, nz=nz, dx=float(dx), dy=float(dy),
                    z_edges=tuple(float(dz) * k for k in range(nz + 1)), kernel=kernel,
                    pad_xl=pad[0], pad_xr=pad[1], pad_yl=pad[2], pad_yr=pad[3], **mag)


def matlab_round(v):
    """Round half away from zero (MATLAB's round), which the padding rule uses."""
    return int(math.floor(abs(v) + 0.5)) * (1 if v >= 0 else -1)


def padding_cells(s, pad_fraction):
    """Cells added on each side: p_L = p_R = round(pad * s) (Sec. 3.2, Table 2)."""
    return matlab_round(pad_fraction * s)


def ladder_size(ell):
    """(s_x, s_y, n_z) = ell * (25, 15, 2) and the cell sizes of the 2000 x 1200 x 400 m
    domain (Sec. 3.2)."""
    sx, sy, nz = 25 * ell, 15 * ell, 2 * ell
    return (sx, sy, nz), (2000.0 / sx, 1200.0 / sy, 400.0 / nz)


def ladder_counts(ell, pad_fraction=0.05):
    """m, n and padded n of Table 2 for scale factor ell."""
    (sx, sy, nz), _ = ladder_size(ell)
    m = sx * sy
    n = m * nz
    nxp = sx + 2 * padding_cells(sx, pad_fraction)
    nyp = sy + 2 * padding_cells(sy, pad_fraction)
    return m, n, nxp * nyp * nz


def subspace_sizes(m, s, cap=5000):
    """t = floor(m / s) limited by 5000, and the oversampled t_p = floor(1.05 t)
    (Secs. 2.3 and 3.1)."""
    t = min(m // s, cap)
    # floor(1.05 t) taken as the exact rational floor(21 t / 20), free of the binary
    # representation of 1.05.
    tp = (21 * t) // 20
    return t, tp
