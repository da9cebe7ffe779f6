"""The sensitivity matrix G and its products by definition (oracle; test infrastructure only).

eq. (blockG): G = [G^(1), ..., G^(nz)], one column block per depth layer, entry
G[(j, i), (r, q, p)] = kernel integral of prism c_pqr seen from station s_ij.
For stations on a uniform grid each G^(r) is BTTB (Sec. 2.1): the entry depends only
on the offsets u = i + p_xL - p and v = j + p_yL - q.  The oracle never uses the
fast method (circulant embedding + FFT of Appendix A).  It computes
* dense G entry by entry from absolute coordinates (tiny grids),
* rows / columns of G entry by entry (sampled checks at any size),
* the per-offset table t_r(u, v) and G x, G^T y by direct summation over the
  Toeplitz blocks of every G^(r) (one matrix product per block offset).
"""
from __future__ import annotations

import numpy as np

from . import prism
from .geometry import Geometry


def _kernel(geom: Geometry, x1, x2, y1, y2, z1, z2):
    if geom.kernel == "gravity":
        return prism.gravity_entry(x1, x2, y1, y2, z1, z2)
    return prism.magnetic_entry(x1, x2, y1, y2, z1, z2, geom.incl_deg, geom.decl_deg,
                                geom.field_nT)


def entries(geom: Geometry, i, j, p, q, r):
    """G[(j, i), (r, q, p)] for broadcastable index arrays, from absolute coordinates."""
    a, b = geom.station_xy(i, j)
    x1, x2, y1, y2, z1, z2 = geom.cell_bounds(p, q, r)
    return _kernel(geom, x1 - a, x2 - a, y1 - b, y2 - b, z1, z2)


def dense_G(geom: Geometry):
    """Full m x n matrix, entry by entry (use only for small grids)."""
    j, i = np.divmod(np.arange(geom.m), geom.sx)
    r, rem = np.divmod(np.arange(geom.n), geom.nx * geom.ny)
    q, p = np.divmod(rem, geom.nx)
    return entries(geom, i[:, None], j[:, None], p[None, :], q[None, :], r[None, :])


def rows(geom: Geometry, stations):
    """Rows of G (shape (len(stations), n)) for flat station indices, entry by entry."""
    stations = np.asarray(stations)
    j, i = np.divmod(stations, geom.sx)
    r, rem = np.divmod(np.arange(geom.n), geom.nx * geom.ny)
    q, p = np.divmod(rem, geom.nx)
    out = np.empty((len(stations), geom.n))
    for k in range(len(stations)):
        out[k] = entries(geom, i[k], j[k], p, q, r)
    return out


def cols(geom: Geometry, cells):
    """Columns of G (shape (m, len(cells))) for flat cell indices, entry by entry."""
    cells = np.asarray(cells)
    r, rem = np.divmod(cells, geom.nx * geom.ny)
    q, p = np.divmod(rem, geom.nx)
    j, i = np.divmod(np.arange(geom.m), geom.sx)
    out = np.empty((geom.m, len(cells)))
    for k in range(len(cells)):
        out[:, k] = entries(geom, i, j, p[k], q[k], r[k])
    return out


def offset_ranges(geom: Geometry):
    """Offset ranges u in [u0, u1], v in [v0, v1] met by G^(r) (inclusive)."""
    u0, u1 = geom.pad_xl - geom.nx + 1, geom.sx - 1 + geom.pad_xl
    v0, v1 = geom.pad_yl - geom.ny + 1, geom.sy - 1 + geom.pad_yl
    return u0, u1, v0, v1


def kernel_table(geom: Geometry):
    """t_r(u, v) for every layer and offset; array (nz, #v, #u) indexed [r, v - v0, u - u0].

    The prism at offset (u, v) spans x in [-(u + 1/2) dx, -(u - 1/2) dx] relative to the
    station, likewise in y.
    """
    u0, u1, v0, v1 = offset_ranges(geom)
    u = np.arange(u0, u1 + 1, dtype=np.float64)
    v = np.arange(v0, v1 + 1, dtype=np.float64)
    ze = np.asarray(geom.z_edges, dtype=np.float64)
    x1 = (-u - 0.5) * geom.dx
    x2 = (-u + 0.5) * geom.dx
    y1 = (-v - 0.5) * geom.dy
    y2 = (-v + 0.5) * geom.dy
    out = np.empty((geom.nz, len(v), len(u)))
    for r in range(geom.nz):
        out[r] = _kernel(geom, x1[None, :], x2[None, :], y1[:, None], y2[:, None], ze[r], ze[r + 1])
    return out


def _toeplitz_block(geom: Geometry, table_r, v):
    """The s_x x n_x Toeplitz block of G^(r) at row-block offset v: [i, p] -> t_r(i + p_xL - p, v)."""
    u0, _, v0, _ = offset_ranges(geom)
    i = np.arange(geom.sx)[:, None]
    p = np.arange(geom.nx)[None, :]
    return table_r[v - v0][i + geom.pad_xl - p - u0]


def _block_pairs(geom: Geometry, v):
    """Station rows j and model rows q = j + p_yL - v that meet at block offset v."""
    j = np.arange(geom.sy)
    q = j + geom.pad_yl - v
    ok = (q >= 0) & (q < geom.ny)
    return j[ok], q[ok]


def apply_G(geom: Geometry, x, table=None):
    """d = G x by direct summation:
    d[j, i] = sum_r sum_q sum_p t_r(i + p_xL - p, j + p_yL - q) x[r, q, p]."""
    table = kernel_table(geom) if table is None else table
    X = np.asarray(x, dtype=np.float64).reshape(geom.nz, geom.ny, geom.nx)
    D = np.zeros((geom.sy, geom.sx))
    _, _, v0, v1 = offset_ranges(geom)
    for r in range(geom.nz):
        for v in range(v0, v1 + 1):
            js, qs = _block_pairs(geom, v)
            if len(js):
                D[js] += X[r, qs] @ _toeplitz_block(geom, table[r], v).T
    return D.reshape(-1)


def apply_GT(geom: Geometry, d, table=None):
    """x = G^T d by direct summation:
    x[r, q, p] = sum_j sum_i t_r(i + p_xL - p, j + p_yL - q) d[j, i]."""
    table = kernel_table(geom) if table is None else table
    D = np.asarray(d, dtype=np.float64).reshape(geom.sy, geom.sx)
    X = np.zeros((geom.nz, geom.ny, geom.nx))
    _, _, v0, v1 = offset_ranges(geom)
    for r in range(geom.nz):
        for v in range(v0, v1 + 1):
            js, qs = _block_pairs(geom, v)
            if len(js):
                X[r, qs] += D[js] @ _toeplitz_block(geom, table[r], v)
    return X.reshape(-1)


def apply_G_cols(geom: Geometry, X, table=None):
    """G X for an n x k block, column by column (a block product is a loop over its columns, Sec. 2.5)."""
    X = np.asarray(X, dtype=np.float64)
    return np.stack([apply_G(geom, X[:, c], table) for c in range(X.shape[1])], axis=1)


def apply_GT_cols(geom: Geometry, Y, table=None):
    """G^T Y for an m x k block, column by column."""
    Y = np.asarray(Y, dtype=np.float64)
    return np.stack([apply_GT(geom, Y[:, c], table) for c in range(Y.shape[1])], axis=1)
