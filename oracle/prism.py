"""Closed-form right-rectangular-prism integrals (oracle; test infrastructure only).

The paper (Sec. 2.1) builds every entry of G from the integral of the gravity or
magnetic kernel over one prism c_pqr, citing Haaz / Li-Oldenburg for gravity and
Rao-Babu for the magnetic case, without printing the formulas.  This module writes
them out from the mathematics:

* Coordinates are *relative*: prism bounds minus the station position, with x and y
  horizontal and z positive downward.  A station on the surface therefore sees the
  top layer at z1 = 0.
* U(r0) = integral over the prism of 1/|r - r0| dV  (Newtonian potential of unit
  density, no gravitational constant).  psi_z = dU/dz0 is the downward attraction,
  T_ij = d^2 U / dx0_i dx0_j is the gravity-gradient tensor (derivatives taken
  with respect to the observation point).
* Corner sums carry mu = (-1)^(number of lower bounds used), i.e. +1 at the
  (x2, y2, z2) corner.

Boundary reading (the paper is silent): a station on the top face of a prism is
taken as the limit from above.  Every arctangent is the principal value of
atan(num/den); den = 0 gives (pi/2) sign(num), num = 0 gives 0.  The z*atan term of
psi_z vanishes at z = 0.  Horizontal coordinates x, y of a corner must be non-zero
for the tensor (stations sit at cell centres, so they always are in this method).
"""
from __future__ import annotations

import numpy as np

GAMMA_SI = 6.6743e-11       # m^3 kg^-1 s^-2 (CODATA 2018); the paper gives no value
GCC_TO_KGM3 = 1.0e3         # density contrast given in g/cc
MS2_TO_MGAL = 1.0e5         # 1 mGal = 1e-5 m/s^2
GRAV_SCALE = GAMMA_SI * GCC_TO_KGM3 * MS2_TO_MGAL   # mGal per (g/cc * m)


def _corners():
    """Yield (ix, iy, iz, mu) for the 8 prism corners; index 1 = upper bound."""
    for ix in (0, 1):
        for iy in (0, 1):
            for iz in (0, 1):
                mu = 1.0 if (3 - ix - iy - iz) % 2 == 0 else -1.0
                yield ix, iy, iz, mu


def _log_a_plus_R(a, R, rest2):
    """ln(a + R) with R = sqrt(a^2 + rest2), free of cancellation when a < 0."""
    a = np.asarray(a, dtype=np.float64)
    out = np.empty(np.broadcast(a, R, rest2).shape)
    a, R, rest2 = np.broadcast_arrays(a, R, rest2)
    pos = a >= 0
    out[pos] = np.log(a[pos] + R[pos])
    neg = ~pos
    out[neg] = np.log(rest2[neg]) - np.log(R[neg] - a[neg])
    return out


def _atan_pv(num, den):
    """Principal value atan(num/den) with the top-face limit rule for den = 0."""
    num, den = np.broadcast_arrays(np.asarray(num, float), np.asarray(den, float))
    out = np.zeros(num.shape)
    nz = den != 0
    out[nz] = np.arctan(num[nz] / den[nz])
    z = (~nz) & (num != 0)
    out[z] = 0.5 * np.pi * np.sign(num[z])
    return out


def _bounds(x1, x2, y1, y2, z1, z2):
    xs = (np.asarray(x1, float), np.asarray(x2, float))
    ys = (np.asarray(y1, float), np.asarray(y2, float))
    zs = (np.asarray(z1, float), np.asarray(z2, float))
    if np.any(zs[0] < 0) or np.any(zs[1] < zs[0]):
        raise ValueError("prism must lie at or below the station plane (0 <= z1 <= z2)")
    return xs, ys, zs


def psi_z(x1, x2, y1, y2, z1, z2):
    """Downward attraction dU/dz0 of a unit-density prism [m] (gravity kernel, Sec. 2.1).

    Antiderivative of z / r^3 over the box:
        F(x, y, z) = -[ x ln(y + R) + y ln(x + R) - z atan(x y / (z R)) ].
    Pinned by: the infinite-slab limit 2 pi h, Gauss-Legendre quadrature of z/r^3,
    the 1-D polar reduction for a station on the top face, exact additivity of
    adjacent prisms and the point-mass far field (tests/test_oracle_prism.py).
    """
    xs, ys, zs = _bounds(x1, x2, y1, y2, z1, z2)
    acc = 0.0
    for ix, iy, iz, mu in _corners():
        x, y, z = xs[ix], ys[iy], zs[iz]
        R = np.sqrt(x * x + y * y + z * z)
        t = x * _log_a_plus_R(y, R, x * x + z * z) + y * _log_a_plus_R(x, R, y * y + z * z)
        t = t - z * _atan_pv(x * y, z * R)
        acc = acc - mu * t
    return acc


def psi_x(x1, x2, y1, y2, z1, z2):
    """Horizontal attraction dU/dx0 (cyclic permutation of psi_z; used by the tests).

    Pinned by Gauss-Legendre quadrature of x / r^3.
    """
    xs, ys, zs = _bounds(x1, x2, y1, y2, z1, z2)
    acc = 0.0
    for ix, iy, iz, mu in _corners():
        x, y, z = xs[ix], ys[iy], zs[iz]
        R = np.sqrt(x * x + y * y + z * z)
        t = y * _log_a_plus_R(z, R, x * x + y * y) + z * _log_a_plus_R(y, R, x * x + z * z)
        t = t - x * _atan_pv(y * z, x * R)
        acc = acc - mu * t
    return acc


def psi_y(x1, x2, y1, y2, z1, z2):
    """Horizontal attraction dU/dy0 (cyclic permutation of psi_z; used by the tests)."""
    xs, ys, zs = _bounds(x1, x2, y1, y2, z1, z2)
    acc = 0.0
    for ix, iy, iz, mu in _corners():
        x, y, z = xs[ix], ys[iy], zs[iz]
        R = np.sqrt(x * x + y * y + z * z)
        t = z * _log_a_plus_R(x, R, y * y + z * z) + x * _log_a_plus_R(z, R, x * x + y * y)
        t = t - y * _atan_pv(z * x, y * R)
        acc = acc - mu * t
    return acc


def gradient_tensor(x1, x2, y1, y2, z1, z2):
    """Gravity-gradient tensor of a unit-density prism, dimensionless.

    Returns (Txx, Tyy, Tzz, Txy, Txz, Tyz) with T_ij = d^2 U / dx0_i dx0_j:
        T_xx = -sum mu atan(y z / (x R)),  T_yy = -sum mu atan(x z / (y R)),
        T_zz = -sum mu atan(x y / (z R)),
        T_xy = +sum mu ln(z + R),  T_xz = +sum mu ln(y + R),  T_yz = +sum mu ln(x + R).
    Pinned by: finite differences of psi_x, psi_y, psi_z (themselves pinned by
    quadrature), the Laplace trace, and the point-dipole far field.
    """
    xs, ys, zs = _bounds(x1, x2, y1, y2, z1, z2)
    if np.any(xs[0] == 0) or np.any(xs[1] == 0) or np.any(ys[0] == 0) or np.any(ys[1] == 0):
        raise ValueError("tensor corners need x != 0 and y != 0 (stations off vertical faces)")
    txx = tyy = tzz = txy = txz = tyz = 0.0
    for ix, iy, iz, mu in _corners():
        x, y, z = xs[ix], ys[iy], zs[iz]
        R = np.sqrt(x * x + y * y + z * z)
        txx = txx - mu * _atan_pv(y * z, x * R)
        tyy = tyy - mu * _atan_pv(x * z, y * R)
        tzz = tzz - mu * _atan_pv(x * y, z * R)
        txy = txy + mu * _log_a_plus_R(z, R, x * x + y * y)
        txz = txz + mu * _log_a_plus_R(y, R, x * x + z * z)
        tyz = tyz + mu * _log_a_plus_R(x, R, y * y + z * z)
    return txx, tyy, tzz, txy, txz, tyz


def field_direction(incl_deg, decl_deg):
    """Unit vector of the inducing field in (x = north, y = east, z = down)."""
    I = np.deg2rad(incl_deg)
    D = np.deg2rad(decl_deg)
    return np.array([np.cos(I) * np.cos(D), np.cos(I) * np.sin(D), np.sin(I)])


def gravity_entry(x1, x2, y1, y2, z1, z2):
    """Vertical gravity of a prism per unit density contrast [mGal per g/cc]."""
    return GRAV_SCALE * psi_z(x1, x2, y1, y2, z1, z2)


def magnetic_entry(x1, x2, y1, y2, z1, z2, incl_deg, decl_deg, field_nT):
    """Total-field anomaly of a prism per unit susceptibility [nT per SI].

    Induced magnetization only (no remanence, no self-demagnetization, as the paper
    assumes), parallel to the inducing field f.  With M = kappa F / mu0 the TFA is
        dT = (F / 4 pi) f^T T f,
    T the gradient tensor above (Poisson's relation); mu0 cancels.
    """
    f = field_direction(incl_deg, decl_deg)
    txx, tyy, tzz, txy, txz, tyz = gradient_tensor(x1, x2, y1, y2, z1, z2)
    q = (f[0] * f[0] * txx + f[1] * f[1] * tyy + f[2] * f[2] * tzz
         + 2.0 * (f[0] * f[1] * txy + f[0] * f[2] * txz + f[1] * f[2] * tyz))
    return field_nT / (4.0 * np.pi) * q
