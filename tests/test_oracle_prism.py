"""Pins of the oracle's prism integrals against mathematics independent of the closed forms."""
import math

import numpy as np
import pytest
from numpy.polynomial.legendre import leggauss
from scipy import integrate

from oracle import prism


def gauss3(bounds, f, npts=40):
    """Tensor Gauss-Legendre quadrature of f over a box (smooth integrands only)."""
    g, w = leggauss(npts)
    (x1, x2), (y1, y2), (z1, z2) = bounds
    X = 0.5 * (x1 + x2) + 0.5 * (x2 - x1) * g
    Y = 0.5 * (y1 + y2) + 0.5 * (y2 - y1) * g
    Z = 0.5 * (z1 + z2) + 0.5 * (z2 - z1) * g
    XX, YY, ZZ = np.meshgrid(X, Y, Z, indexing="ij")
    W = np.einsum("i,j,k->ijk", w, w, w) * (x2 - x1) * (y2 - y1) * (z2 - z1) / 8.0
    return float((W * f(XX, YY, ZZ)).sum())


BURIED = [
    (10.0, 60.0, -30.0, 20.0, 40.0, 90.0),
    (-75.0, -25.0, 15.0, 65.0, 30.0, 50.0),
    (-20.0, 20.0, -20.0, 20.0, 25.0, 45.0),
    (130.0, 150.0, -170.0, -150.0, 5.0, 25.0),
]


@pytest.mark.parametrize("b", BURIED)
def test_attraction_matches_quadrature(b):
    bx = ((b[0], b[1]), (b[2], b[3]), (b[4], b[5]))
    r3 = lambda x, y, z: (x * x + y * y + z * z) ** 1.5
    for fn, integrand in ((prism.psi_z, lambda x, y, z: z / r3(x, y, z)),
                          (prism.psi_x, lambda x, y, z: x / r3(x, y, z)),
                          (prism.psi_y, lambda x, y, z: y / r3(x, y, z))):
        ref = gauss3(bx, integrand)
        assert abs(fn(*b) - ref) <= 1e-10 * max(abs(ref), 1e-3), (fn.__name__, fn(*b), ref)


def test_infinite_slab_limit():
    h = 50.0
    W = 1e7
    val = prism.psi_z(-W, W, -W, W, 0.0, h)
    assert abs(val / (2 * math.pi * h) - 1.0) < 1e-4
    # a buried slab gives the same 2 pi h (Bouguer): independent of depth
    val2 = prism.psi_z(-W, W, -W, W, 300.0, 300.0 + h)
    assert abs(val2 / (2 * math.pi * h) - 1.0) < 1e-4


def test_top_face_centre_against_polar_reduction():
    # station at the centre of the top face of a square prism of half-width a, depth h:
    # integrating z/r^3 over z and then in polar coordinates over the 8 triangles of the
    # square leaves 8 * int_0^{pi/4} [a sec(t) - sqrt(a^2 sec(t)^2 + h^2) + h] dt
    for a, h in ((25.0, 50.0), (10.0, 40.0), (25.0, 5.0)):
        f = lambda t: a / math.cos(t) - math.sqrt((a / math.cos(t)) ** 2 + h * h) + h
        ref = 8.0 * integrate.quad(f, 0.0, math.pi / 4, epsabs=0, epsrel=1e-13)[0]
        assert abs(prism.psi_z(-a, a, -a, a, 0.0, h) - ref) <= 1e-12 * ref


def test_additivity_of_adjacent_prisms():
    rng = np.random.default_rng(7)
    for z0 in (0.0, 40.0):
        xs = np.array([-60.0, -10.0, 30.0])
        ys = np.array([-20.0, 25.0, 90.0])
        zs = np.array([z0, z0 + 30.0, z0 + 80.0])
        merged = prism.psi_z(xs[0], xs[2], ys[0], ys[2], zs[0], zs[2])
        parts = sum(prism.psi_z(xs[i], xs[i + 1], ys[j], ys[j + 1], zs[k], zs[k + 1])
                    for i in range(2) for j in range(2) for k in range(2))
        assert abs(parts - merged) <= 1e-13 * abs(merged)
        T_m = np.array(prism.gradient_tensor(xs[0], xs[2], ys[0], ys[2], zs[0], zs[2]))
        T_p = sum(np.array(prism.gradient_tensor(xs[i], xs[i + 1], ys[j], ys[j + 1], zs[k], zs[k + 1]))
                  for i in range(2) for j in range(2) for k in range(2))
        assert np.abs(T_p - T_m).max() <= 1e-12 * np.abs(T_m).max()
    del rng


def test_point_mass_far_field():
    a = 10.0
    for cx, cy, cz in ((800.0, 0.0, 30.0), (300.0, -250.0, 400.0), (0.0, 0.0, 800.0)):
        val = prism.psi_z(cx - a, cx + a, cy - a, cy + a, cz - a, cz + a)
        r = math.sqrt(cx * cx + cy * cy + cz * cz)
        ref = (2 * a) ** 3 * cz / r ** 3
        assert abs(val / ref - 1.0) < 1e-6


def test_gravity_mirror_symmetry():
    b = (10.0, 60.0, -30.0, 20.0, 0.0, 90.0)
    v = prism.psi_z(*b)
    assert abs(prism.psi_z(-b[1], -b[0], b[2], b[3], b[4], b[5]) - v) <= 1e-14 * abs(v)
    assert abs(prism.psi_z(b[0], b[1], -b[3], -b[2], b[4], b[5]) - v) <= 1e-14 * abs(v)


def _shift(b, dx=0.0, dy=0.0, dz=0.0):
    # moving the station by +d moves the prism by -d in relative coordinates
    return (b[0] - dx, b[1] - dx, b[2] - dy, b[3] - dy, b[4] - dz, b[5] - dz)


@pytest.mark.parametrize("b", BURIED + [(-25.0, 25.0, -25.0, 25.0, 0.0, 50.0),
                                        (35.0, 85.0, -45.0, 5.0, 0.0, 40.0)])
def test_tensor_is_derivative_of_attraction(b):
    h = 1e-2
    T = dict(zip(("xx", "yy", "zz", "xy", "xz", "yz"), prism.gradient_tensor(*b)))
    scale = max(abs(v) for v in T.values())

    def cd(fn, axis):
        kw_p = {axis: h}
        kw_m = {axis: -h}
        return (fn(*_shift(b, **kw_p)) - fn(*_shift(b, **kw_m))) / (2 * h)

    on_top = b[4] == 0.0
    if on_top:
        # one-sided (from above: station moves up = prism moves down in relative z)
        d_z = lambda fn: (-3 * fn(*b) + 4 * fn(*_shift(b, dz=-h)) - fn(*_shift(b, dz=-2 * h))) / (-2 * h)
    else:
        d_z = lambda fn: cd(fn, "dz")
    checks = {
        "xx": cd(prism.psi_x, "dx"), "xy": cd(prism.psi_x, "dy"), "xz": cd(prism.psi_z, "dx"),
        "yy": cd(prism.psi_y, "dy"), "yz": cd(prism.psi_z, "dy"), "zz": d_z(prism.psi_z),
    }
    for k, v in checks.items():
        assert abs(T[k] - v) <= 1e-7 * scale, (k, T[k], v)


def test_laplace_trace():
    for b in BURIED + [(-25.0, 25.0, -25.0, 25.0, 0.0, 50.0), (35.0, 85.0, -45.0, 5.0, 0.0, 40.0),
                       (-15.0, 5.0, -5.0, 15.0, 0.0, 20.0)]:
        T = prism.gradient_tensor(*b)
        assert abs(T[0] + T[1] + T[2]) <= 1e-12 * max(abs(t) for t in T)


def test_tensor_matches_quadrature_off_body():
    b = BURIED[0]
    bx = ((b[0], b[1]), (b[2], b[3]), (b[4], b[5]))
    T = prism.gradient_tensor(*b)

    def k(i, j):
        def f(x, y, z):
            c = (x, y, z)
            r2 = x * x + y * y + z * z
            return (3 * c[i] * c[j] - (r2 if i == j else 0.0)) / r2 ** 2.5
        return f
    idx = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]
    for t, (i, j) in zip(T, idx):
        ref = gauss3(bx, k(i, j))
        assert abs(t - ref) <= 1e-9 * max(abs(v) for v in T)


def test_tfa_dipole_far_field():
    a = 10.0
    F = 50000.0
    for inc, dec in ((45.0, 45.0), (60.0, -20.0), (90.0, 0.0)):
        f = prism.field_direction(inc, dec)
        for c in (np.array([800.0, 100.0, 300.0]), np.array([-400.0, 600.0, 50.0])):
            val = prism.magnetic_entry(c[0] - a, c[0] + a, c[1] - a, c[1] + a, c[2] - a, c[2] + a,
                                       inc, dec, F)
            r = np.linalg.norm(c)
            ref = F / (4 * math.pi) * (2 * a) ** 3 * (3 * (f @ c / r) ** 2 - 1) / r ** 3
            assert abs(val / ref - 1.0) < 1e-5


def test_tfa_vertical_field_positive_over_body():
    v = prism.magnetic_entry(-25.0, 25.0, -25.0, 25.0, 0.0, 50.0, 90.0, 0.0, 50000.0)
    T = prism.gradient_tensor(-25.0, 25.0, -25.0, 25.0, 0.0, 50.0)
    assert v > 0
    assert abs(v - 50000.0 / (4 * math.pi) * T[2]) <= 1e-12 * v


def test_tfa_declination_half_turn_is_point_reflection():
    b = (35.0, 85.0, -45.0, 5.0, 20.0, 40.0)
    refl = (-b[1], -b[0], -b[3], -b[2], b[4], b[5])
    v1 = prism.magnetic_entry(*b, 45.0, 30.0, 50000.0)
    v2 = prism.magnetic_entry(*refl, 45.0, 210.0, 50000.0)
    assert abs(v1 - v2) <= 1e-12 * abs(v1)


@pytest.mark.parametrize("dist,tol", [(800.0, 1e-6), (4990.0, 1e-4)])
def test_far_corner_cancellation_is_bounded(dist, tol):
    # The 8-corner sum of psi_z cancels terms of size r ln r down to V z / r^3, so a
    # shallow prism far away loses about log10(8 r^4 / (V z)) digits and a little more: ~7 at 800 m and
    # ~10 at 5 km for a 20 m cube 30 m deep.  The cube's point-mass limit is exact up
    # to (a/r)^4, far below these bounds, so it measures the loss directly.
    a = 10.0
    c = np.array([-dist, 10.0, 30.0])
    val = prism.psi_z(c[0] - a, c[0] + a, c[1] - a, c[1] + a, c[2] - a, c[2] + a)
    r = np.linalg.norm(c)
    ref = (2 * a) ** 3 * c[2] / r ** 3
    assert abs(val / ref - 1.0) < tol


# ---- unit scale of the gravity entries ---------------------------------------------------
# The entries are in mGal per g/cc.  Two values from outside the oracle fix the scale: the
# Bouguer slab constant 2 pi G rho h, which the textbooks print as 0.04193 mGal per metre of
# thickness per g/cc (to four digits, i.e. within 1.2e-4 relative), and Newton's law for a
# compact body far away, g = G M / r^2 with G = 6.674e-11 (four digits, 6e-5 relative).

def test_gravity_unit_scale_bouguer_slab():
    for h in (1.0, 50.0, 120.0):
        W = 1e7
        val = prism.gravity_entry(-W, W, -W, W, 0.0, h)
        assert abs(val / (0.04193 * h) - 1.0) < 2e-4, (h, val)
        # a factor of ten in any unit conversion or a lost 2 pi is far outside that
        assert abs(val / (0.04193 * h) - 1.0) < 1e-3


def test_gravity_unit_scale_point_mass():
    # a 20 m cube of 1 g/cc = 1000 kg/m^3 holds 8e6 kg; 1 m/s^2 = 1e5 mGal
    a = 10.0
    for c in ((0.0, 0.0, 3000.0), (2000.0, -1500.0, 800.0)):
        val = prism.gravity_entry(c[0] - a, c[0] + a, c[1] - a, c[1] + a, c[2] - a, c[2] + a)
        r = math.sqrt(c[0] ** 2 + c[1] ** 2 + c[2] ** 2)
        g_down = 6.674e-11 * 8.0e6 / r ** 2 * (c[2] / r) * 1e5
        assert abs(val / g_down - 1.0) < 2e-4, (c, val, g_down)


# ---- labelling of the field direction ----------------------------------------------------
# Axes are x = north, y = east, z = down, declination clockwise from north.  These checks do
# not use the oracle's field_direction: they state what the direction must do.

def test_zero_declination_is_even_in_the_east_offset():
    # D = 0 puts the field and the magnetization in the x-z plane: reflecting y -> -y maps the
    # problem onto itself, so the TFA of a prism equals that of its mirror image across y = 0
    for inc in (30.0, 60.0, 75.0):
        for b in ((35.0, 85.0, -45.0, 5.0, 20.0, 40.0), (-70.0, -10.0, 15.0, 55.0, 0.0, 30.0)):
            v = prism.magnetic_entry(*b, inc, 0.0, 50000.0)
            vm = prism.magnetic_entry(b[0], b[1], -b[3], -b[2], b[4], b[5], inc, 0.0, 50000.0)
            assert abs(v - vm) <= 1e-12 * abs(v), (inc, b)
            # and is not even in the north offset (the field has a north component)
            vx = prism.magnetic_entry(-b[1], -b[0], b[2], b[3], b[4], b[5], inc, 0.0, 50000.0)
            assert abs(v - vx) > 1e-3 * abs(v)


def test_east_declination_is_even_in_the_north_offset():
    for inc in (30.0, 60.0):
        b = (35.0, 85.0, -45.0, 5.0, 20.0, 40.0)
        v = prism.magnetic_entry(*b, inc, 90.0, 50000.0)
        vm = prism.magnetic_entry(-b[1], -b[0], b[2], b[3], b[4], b[5], inc, 90.0, 50000.0)
        assert abs(v - vm) <= 1e-12 * abs(v)
        vy = prism.magnetic_entry(b[0], b[1], -b[3], -b[2], b[4], b[5], inc, 90.0, 50000.0)
        assert abs(v - vy) > 1e-3 * abs(v)


@pytest.mark.parametrize("inc,dec,fhat", [
    (0.0, 0.0, (1.0, 0.0, 0.0)),       # horizontal field pointing north
    (0.0, 90.0, (0.0, 1.0, 0.0)),      # horizontal field pointing east
    (0.0, -90.0, (0.0, -1.0, 0.0)),    # west
    (90.0, 0.0, (0.0, 0.0, 1.0)),      # vertical, pointing down
    (30.0, 0.0, (math.sqrt(3) / 2, 0.0, 0.5)),   # northward, dipping down by 30 degrees
    (0.0, 45.0, (math.sqrt(0.5), math.sqrt(0.5), 0.0)),     # north-east (clockwise from north)
    (0.0, -45.0, (math.sqrt(0.5), -math.sqrt(0.5), 0.0)),   # north-west
    (-30.0, 180.0, (-math.sqrt(3) / 2, 0.0, -0.5)),        # southward, pointing up
])
def test_tfa_far_field_of_axis_dipoles(inc, dec, fhat):
    # far from a small cube the TFA is that of a point dipole of moment V kappa F f / mu0:
    #     dT = F / (4 pi) V (3 (f . r^)^2 - 1) / r^3,
    # with the direction f written out here for each (I, D)
    a = 10.0
    F = 50000.0
    f = np.array(fhat)
    for c in (np.array([800.0, 100.0, 300.0]), np.array([-400.0, 600.0, 50.0]), np.array([300.0, -700.0, 200.0])):
        val = prism.magnetic_entry(c[0] - a, c[0] + a, c[1] - a, c[1] + a, c[2] - a, c[2] + a, inc, dec, F)
        r = np.linalg.norm(c)
        ref = F / (4 * math.pi) * (2 * a) ** 3 * (3 * (f @ c / r) ** 2 - 1) / r ** 3
        assert abs(val / ref - 1.0) < 1e-5, (inc, dec, c, val, ref)
