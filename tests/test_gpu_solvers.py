"""Parity of the HIP projected solvers and IRLS step with the oracle's Algorithms 1 and 2."""
import math
import time

import numpy as np
import pytest
import torch

from galerkin import galerkin_defects, iterated_tikhonov, rsvd_galerkin_defects
from gpu_common import announce, ogeom, rel, to_dev, to_host
from oracle import irls as oirls, operator as op, philox, solvers as osol
from paper_2004_13904_amd import _lib as L
from paper_2004_13904_amd import solvers as S
from paper_2004_13904_amd import workloads as W
from paper_2004_13904_amd.operator import Operator

pytestmark = pytest.mark.gpu
F64, F32 = torch.float64, torch.float32


def problem(name="small", kernel="gravity", seed=0):
    if name == "small":
        s = W.survey(8, 8, 2, 25, 25, 25, kernel=kernel, incl=45.0, decl=45.0)
    else:
        s = W.survey(24, 20, 6, 20, 20, 20, kernel=kernel, incl=45.0, decl=45.0, pad=(1, 2, 0, 1))
    g = ogeom(s)
    G = op.dense_G(g)
    rng = np.random.default_rng(seed)
    wd = 1.0 / (0.05 + rng.random(g.m))
    winv = 0.5 + rng.random(g.n)
    Gt = wd[:, None] * G * winv[None, :]
    r = rng.standard_normal(g.m) * 3.0
    return s, g, G, wd, winv, Gt, r


def dense_ops(Gt):
    return (lambda x: Gt @ x), (lambda y: Gt.T @ y)


def check_alpha(mode, a, a0, s_t, c_t, dtype):
    """alpha parity.  Fixed and eq. (eq:alpha1) values are closed forms: compare directly.  The
    UPRE minimizer sits on a flat minimum whose location rounding moves by about sqrt(eps)
    relative, so compare what is unique: the oracle's UPRE value at the two parameters."""
    if mode == "upre":
        u0 = osol.upre(a0, s_t, c_t)
        u1 = osol.upre(a, s_t, c_t)
        assert u1 <= u0 + (1e-10 if dtype == F64 else 1e-6) * abs(u0)
        assert abs(a - a0) <= (1e-5 if dtype == F64 else 1e-3) * a0
    else:
        assert abs(a - a0) <= (1e-10 if dtype == F64 else 1e-5) * a0


@pytest.mark.parametrize("kernel", ["gravity", "magnetic"])
def test_gkb_full_space_is_tikhonov(kernel):
    s, g, G, wd, winv, Gt, r = problem(kernel=kernel)
    alpha = 0.3 * np.linalg.svd(Gt, compute_uv=False)[5]
    A = Operator(s, F64)
    y, a, sig = S.gkb_project(A, to_dev(r, F64), to_dev(wd, F64), to_dev(winv, F64), g.m, g.m,
                              "fixed", alpha)
    assert a == alpha
    ref = osol.tikhonov_z(Gt, r, alpha)
    assert rel(to_host(y), ref) <= 1e-9
    assert rel(to_host(sig), np.linalg.svd(Gt, compute_uv=False)) <= 1e-9


@pytest.mark.parametrize("mode", ["fixed", "upre", "alpha1"])
@pytest.mark.parametrize("dtype", [F64, F32])
def test_gkb_matches_oracle_algorithm(mode, dtype):
    s, g, G, wd, winv, Gt, r = problem("mid", kernel="magnetic", seed=1)
    t, tp = 40, 42
    announce("gkb", mode, dtype)
    y0, a0, s0, F = osol.gkb(*dense_ops(Gt), r, g.n, t, tp, mode, 2.0, return_factors=True)
    A = Operator(s, dtype)
    y, a, sig = S.gkb_project(A, to_dev(r, F64), to_dev(wd, F64), to_dev(winv, F64), t, tp, mode, 2.0)
    tol = 1e-9 if dtype == F64 else 2e-5
    assert rel(to_host(sig), s0) <= tol
    check_alpha(mode, a, a0, s0[:t], np.linalg.norm(r) * F["U"][0, :t], dtype)
    # y at the oracle's alpha is the algorithm's output; the alpha difference moves it
    # proportionally (dy/dalpha ~ y/alpha)
    ya = S.gkb_project(A, to_dev(r, F64), to_dev(wd, F64), to_dev(winv, F64), t, tp, "fixed", a0)[0]
    assert rel(to_host(ya), y0) <= (1e-8 if dtype == F64 else 1e-4)
    assert rel(to_host(y), y0) <= (1e-8 if dtype == F64 else 1e-4) + 2 * abs(a - a0) / a0


@pytest.mark.parametrize("solver", ["gkb", "rsvd", "gkb_lean"])
@pytest.mark.parametrize("t,tp", [(1, 1), (1, 2), (2, 2), (2, 3)])
@pytest.mark.parametrize("mode", ["fixed", "alpha1"])
def test_smallest_projected_sizes(solver, t, tp, mode):
    # the degenerate projected problems: one to three basis vectors (a 2 x 1 to 4 x 3 bidiagonal
    # for GKB, a 1 x 1 to 3 x 3 Gram matrix for RSVD), FP64 against the oracle's algorithms;
    # gkb_lean: GKB with the model-side basis rebuilt from its two-column ring (gkb_onesided = 2)
    s, g, G, wd, winv, Gt, r = problem("mid", kernel="gravity", seed=3)
    announce("smallest", solver, t, tp, mode)
    A = Operator(s, F64)
    if solver == "gkb_lean":
        A.set_tuning(gkb_onesided=2)
        solver = "gkb"
    args = (to_dev(r, F64), to_dev(wd, F64), to_dev(winv, F64), t, tp)
    if solver == "gkb":
        y0, a0, s0 = osol.gkb(*dense_ops(Gt), r, g.n, t, tp, mode, 2.0)
        y, a, sig = S.gkb_project(A, *args, mode, 2.0)
    else:
        omega = np.random.default_rng(5).standard_normal((tp, g.m))
        y0, a0, s0 = osol.rsvd(*dense_ops(Gt), r, g.n, t, tp, omega, mode, 2.0)
        y, a, sig = S.rsvd_project(A, *args, to_dev(omega, F64), mode, 2.0)
    assert rel(to_host(sig), s0) <= 1e-9
    assert abs(a - a0) <= 1e-10 * a0
    assert rel(to_host(y), y0) <= 1e-8


@pytest.mark.parametrize("kernel", ["gravity", "magnetic"])
def test_rsvd_full_space_is_tikhonov(kernel):
    s, g, G, wd, winv, Gt, r = problem(kernel=kernel)
    alpha = 0.3 * np.linalg.svd(Gt, compute_uv=False)[5]
    omega = np.random.default_rng(9).standard_normal((g.m, g.m))
    A = Operator(s, F64)
    y, a, sig = S.rsvd_project(A, to_dev(r, F64), to_dev(wd, F64), to_dev(winv, F64), g.m, g.m,
                               to_dev(omega, F64), "fixed", alpha)
    ref = osol.tikhonov_z(Gt, r, alpha)
    assert rel(to_host(y), ref) <= 1e-8
    assert rel(to_host(sig), np.linalg.svd(Gt, compute_uv=False)) <= 1e-8


@pytest.mark.parametrize("mode", ["fixed", "upre", "alpha1"])
@pytest.mark.parametrize("dtype", [F64, F32])
@pytest.mark.parametrize("qr", [0, 1, 2])
def test_rsvd_matches_oracle_algorithm(mode, dtype, qr):
    # qr 0: CholeskyQR2 first (then shifted CholeskyQR3, then Householder); 1: Householder QR
    # always; 2: shifted CholeskyQR3 first
    s, g, G, wd, winv, Gt, r = problem("mid", kernel="gravity", seed=2)
    t, tp = 60, 63
    announce("rsvd", mode, dtype, "qr", qr)
    omega = np.random.default_rng(4).standard_normal((tp, g.m))
    y0, a0, s0, F = osol.rsvd(*dense_ops(Gt), r, g.n, t, tp, omega, mode, 2.0, return_factors=True)
    A = Operator(s, dtype)
    A.set_tuning(rsvd_qr=qr)
    y, a, sig = S.rsvd_project(A, to_dev(r, F64), to_dev(wd, F64), to_dev(winv, F64), t, tp,
                               to_dev(omega, F64), mode, 2.0)
    tol = 1e-8 if dtype == F64 else 2e-5
    assert rel(to_host(sig)[:t], s0[:t]) <= tol
    c0 = F["U"].T @ (F["B"].T @ r)
    check_alpha(mode, a, a0, s0[:t], c0, dtype)
    ya = S.rsvd_project(A, to_dev(r, F64), to_dev(wd, F64), to_dev(winv, F64), t, tp,
                        to_dev(omega, F64), "fixed", a0)[0]
    assert rel(to_host(ya), y0) <= (1e-8 if dtype == F64 else 1e-4)
    assert rel(to_host(y), y0) <= (1e-8 if dtype == F64 else 1e-4) + 2 * abs(a - a0) / a0
    counts = A.qr_counts
    # three factorizations per call (one power iteration), two calls
    assert sum(counts.values()) == 6
    if qr == 1:
        assert counts["householder"] == 6
    elif qr == 2:
        assert counts["cholesky2"] == 0 and counts["cholesky3"] >= 1
    else:
        assert counts["cholesky2"] + counts["cholesky3"] >= 1


def test_rsvd_split_gram_with_remainder_rows():
    # n = 27 * 21 * 5 = 2835 rows: the tall Gram products are split into two row chunks of 1417
    # rows plus one remainder row; the result is the oracle's Algorithm 2
    s = W.survey(24, 20, 5, 20, 20, 20, kernel="magnetic", incl=45.0, decl=45.0, pad=(1, 2, 0, 1))
    g = ogeom(s)
    assert g.n == 2835
    rng = np.random.default_rng(5)
    wd = 1.0 / (0.05 + rng.random(g.m))
    winv = 0.5 + rng.random(g.n)
    Gt = wd[:, None] * op.dense_G(g) * winv[None, :]
    r = rng.standard_normal(g.m)
    t, tp = 40, 42
    omega = rng.standard_normal((tp, g.m))
    y0, a0, s0 = osol.rsvd(*dense_ops(Gt), r, g.n, t, tp, omega, "fixed", 1.5)
    A = Operator(s, F64)
    y, a, sig = S.rsvd_project(A, to_dev(r, F64), to_dev(wd, F64), to_dev(winv, F64), t, tp,
                               to_dev(omega, F64), "fixed", 1.5)
    assert rel(to_host(sig), s0) <= 1e-8
    assert rel(to_host(y), y0) <= 1e-8
    assert A.qr_counts["cholesky2"] + A.qr_counts["cholesky3"] == 3


@pytest.mark.parametrize("kernel", ["gravity", "magnetic"])
def test_gkb_single_precision_basis(kernel):
    # the bases stored in FP32 (every product and sum in FP64): the oracle's Algorithm 1 to the
    # level of the basis rounding
    s, g, G, wd, winv, Gt, r = problem("mid", kernel=kernel, seed=1)
    t, tp = 60, 63
    announce("gkb f32 basis", kernel)
    y0, a0, s0, F = osol.gkb(*dense_ops(Gt), r, g.n, t, tp, "fixed", 2.0, return_factors=True)
    A = Operator(s, F64)
    y, a, sig = S.gkb_project(A, to_dev(r, F64), to_dev(wd, F64), to_dev(winv, F64), t, tp, "fixed", 2.0,
                              basis="f32")
    assert rel(to_host(sig), s0) <= 1e-6
    assert rel(to_host(y), y0) <= 2e-5
    # half the basis memory
    assert S.workspace_bytes(A, "gkb", tp, basis="f32") < 0.75 * S.workspace_bytes(A, "gkb", tp)


@pytest.mark.parametrize("onesided", [1, 2])
@pytest.mark.parametrize("basis", ["f64", "f32"])
@pytest.mark.parametrize("kernel", ["gravity", "magnetic"])
def test_gkb_onesided_matches_oracle(onesided, basis, kernel):
    # gkb_onesided = 1: only the data-side basis H is reorthogonalized; = 2: besides, the model-side
    # basis is not stored but rebuilt in a second pass to form y.  Against the oracle's Algorithm 1
    # (both bases reorthogonalized by MGS): the same projected problem to rounding, at the bars of
    # the both-sided GPU solve; modes 1 and 2 share the first pass, so sigma and alpha agree bit for
    # bit and y to rounding; mode 2's workspace drops t_p - 2 columns of A.
    s, g, G, wd, winv, Gt, r = problem("mid", kernel=kernel, seed=1)
    t, tp = 60, 63
    announce("gkb onesided", onesided, basis, kernel)
    y0, a0, s0, F = osol.gkb(*dense_ops(Gt), r, g.n, t, tp, "upre", 2.0, return_factors=True)
    A = Operator(s, F64)
    args = (to_dev(r, F64), to_dev(wd, F64), to_dev(winv, F64), t, tp)
    ws0 = S.workspace_bytes(A, "gkb", tp, basis=basis)
    A.set_tuning(gkb_onesided=1)
    y1, a1, s1 = S.gkb_project(A, *args, "upre", basis=basis)
    A.set_tuning(gkb_onesided=onesided)
    y, a, sig = S.gkb_project(A, *args, "upre", basis=basis)
    ya = S.gkb_project(A, *args, "fixed", a0, basis=basis)[0]
    tol_s, tol_y = (1e-9, 1e-8) if basis == "f64" else (1e-6, 2e-5)
    assert rel(to_host(sig), s0) <= tol_s
    check_alpha("upre", a, a0, s0[:t], np.linalg.norm(r) * F["U"][0, :t], F64 if basis == "f64" else F32)
    assert rel(to_host(ya), y0) <= tol_y
    assert torch.equal(sig, s1) and a == a1
    assert rel(to_host(y), to_host(y1)) <= 1e-13
    if onesided == 2:
        lda = (g.n + 63) // 64 * 64
        per = 8 if basis == "f64" else 4
        assert S.workspace_bytes(A, "gkb", tp, basis=basis) <= ws0 - (tp - 2) * lda * per


@pytest.mark.parametrize("q", [0, 2])
def test_rsvd_power_iterations_and_device_omega(q):
    # Omega drawn on the device from a seed (Philox4x32-10) and q power iterations, against the
    # oracle's Algorithm 2 with the host rendering of the same generator; t_p < m, so the
    # result depends on Omega
    s, g, G, wd, winv, Gt, r = problem("mid", kernel="gravity", seed=2)
    t, tp = 60, 63
    seed = (1 << 40) + 17
    announce("rsvd device omega", q)
    omega = philox.gaussian(tp * g.m, seed).reshape(tp, g.m)
    y0, a0, s0 = osol.rsvd(*dense_ops(Gt), r, g.n, t, tp, omega, "fixed", 2.0, power_iters=q)
    A = Operator(s, F64)
    y, a, sig = S.rsvd_project(A, to_dev(r, F64), to_dev(wd, F64), to_dev(winv, F64), t, tp, None, "fixed", 2.0,
                               seed=seed, power_iters=q)
    assert rel(to_host(sig)[:t], s0[:t]) <= 1e-8
    assert rel(to_host(y), y0) <= 1e-8
    # another seed is another sketch
    y2 = S.rsvd_project(A, to_dev(r, F64), to_dev(wd, F64), to_dev(winv, F64), t, tp, None, "fixed", 2.0,
                        seed=seed + 1, power_iters=q)[0]
    assert rel(to_host(y2), y0) > 1e-6
    with pytest.raises(L.FastFocusError):
        S.rsvd_project(A, to_dev(r, F64), to_dev(wd, F64), to_dev(winv, F64), t, tp, None, "fixed", 2.0,
                       power_iters=9)


def test_irls_rsvd_with_device_omega_matches_oracle():
    # irls_step draws Omega from (seed, stream = k) when it is not given
    s = W.survey(16, 12, 5, 25, 25, 25)
    g = ogeom(s)
    G = op.dense_G(g)
    rng = np.random.default_rng(3)
    m_true = np.zeros(g.n)
    m_true[rng.choice(g.n, 20, replace=False)] = 1.0
    d_exact = G @ m_true
    eta, sd = W.noise(d_exact, 0.02, 0.002, 5)
    d_obs = d_exact + eta
    wd = 1.0 / sd
    t, tp, seed = 40, 42, 99
    A = Operator(s, F64)
    po = oirls.IrlsParams(solver="rsvd", t=t, tp=tp, lam=0.0, beta_depth=0.8, m_min=0.0, m_max=1.0)
    pg = S.IrlsParams(solver="rsvd", t=t, tp=tp, lam=0.0, beta_depth=0.8, m_min=0.0, m_max=1.0, seed=seed)
    om1 = philox.gaussian(tp * g.m, seed, stream=1).reshape(tp, g.m)
    m1o, a1o, c1o, _ = oirls.irls_step(g, po, 1, d_obs, wd, np.zeros(g.n), None, om1, G_dense=G)
    m1, a1, c1 = S.irls_step(A, pg, 1, to_dev(d_obs, F64), to_dev(wd, F64),
                             torch.zeros(g.n, dtype=F64, device="cuda"), None, None)
    assert abs(a1 - a1o) <= 1e-8 * a1o
    assert rel(to_host(m1), m1o) <= 1e-7
    assert abs(c1 - c1o) <= 1e-8 * c1o


@pytest.mark.parametrize("solver", ["gkb", "rsvd", "gkb_onesided"])
def test_irls_step_matches_oracle(solver):
    # gkb_onesided: GKB reorthogonalizing the data-side basis only, the model-side basis rebuilt
    # in a second pass (gkb_onesided = 2), against the oracle's Algorithm 1
    onesided = solver == "gkb_onesided"
    solver = "gkb" if onesided else solver
    s = W.survey(16, 12, 5, 25, 25, 25)
    g = ogeom(s)
    G = op.dense_G(g)
    rng = np.random.default_rng(3)
    m_true = np.zeros(g.n)
    m_true[rng.choice(g.n, 20, replace=False)] = 1.0
    d_exact = G @ m_true
    eta, sd = W.noise(d_exact, 0.02, 0.002, 5)
    d_obs = d_exact + eta
    wd = 1.0 / sd
    t, tp = 40, 42
    omega = rng.standard_normal((tp, g.m))
    A = Operator(s, F64)
    if onesided:
        A.set_tuning(gkb_onesided=2)
    po = oirls.IrlsParams(solver=solver, t=t, tp=tp, lam=0.0, beta_depth=0.8, m_min=0.0, m_max=1.0)
    pg = S.IrlsParams(solver=solver, t=t, tp=tp, lam=0.0, beta_depth=0.8, m_min=0.0, m_max=1.0)
    m1o, a1o, c1o, _ = oirls.irls_step(g, po, 1, d_obs, wd, np.zeros(g.n), None, omega, G_dense=G)
    m1, a1, c1 = S.irls_step(A, pg, 1, to_dev(d_obs, F64), to_dev(wd, F64),
                             torch.zeros(g.n, dtype=F64, device="cuda"), None,
                             to_dev(omega, F64) if solver == "rsvd" else None)
    assert abs(a1 - a1o) <= 1e-8 * a1o
    assert rel(to_host(m1), m1o) <= 1e-7
    assert abs(c1 - c1o) <= 1e-8 * c1o
    # second step: focusing weights from m1 - m0 and UPRE alpha
    m2o, a2o, c2o, _ = oirls.irls_step(g, po, 2, d_obs, wd, m1o, np.zeros(g.n), omega, G_dense=G)
    m2, a2, c2 = S.irls_step(A, pg, 2, to_dev(d_obs, F64), to_dev(wd, F64), to_dev(m1o, F64),
                             torch.zeros(g.n, dtype=F64, device="cuda"),
                             to_dev(omega, F64) if solver == "rsvd" else None)
    # UPRE alpha at k = 2: flat minimum (see check_alpha); the iterate follows alpha
    assert abs(a2 - a2o) <= 1e-5 * a2o
    assert rel(to_host(m2), m2o) <= 1e-6 + 2 * abs(a2 - a2o) / a2o
    assert abs(c2 - c2o) <= (1e-6 + 4 * abs(a2 - a2o) / a2o) * c2o


def c1_weighted_problem():
    """The timed IRLS configuration's first weighted problem, from the oracle: gravity 100 x 60
    stations, 10 layers (n = 60000), two 1 g/cc blocks, 1 % noise, W = W_z with beta = 0.8,
    r~ = W_d d_obs; products with G~ by the oracle's direct sums."""
    s = W.SURVEYS["gravity_l4"]
    g = ogeom(s)
    T = op.kernel_table(g)
    d_exact = op.apply_G(g, W.block_model(s, W.GRAVITY_L4_BLOCKS), T)
    eta, sd = W.noise(d_exact, 0.01, 0.001, 2)
    wd = 1.0 / sd
    winv = 1.0 / oirls.depth_weights(g, 0.8)
    r = wd * (d_exact + eta)
    Gt = lambda v: wd * op.apply_G(g, winv * v, T)
    GtT = lambda y: winv * op.apply_GT(g, wd * y, T)
    return s, g, wd, winv, r, Gt, GtT


def oracle_sigma1(Gt, GtT, r, iters=40):
    """Largest singular value of G~ by power iteration on G~^T G~ (the Rayleigh quotient settles
    to ~1e-13 within 40 steps on the problem above)."""
    v = GtT(r)
    v /= np.linalg.norm(v)
    for _ in range(iters):
        v = GtT(Gt(v))
        v /= np.linalg.norm(v)
    return float(np.linalg.norm(Gt(v)))


def test_gkb_full_size_properties():
    # GKB in the timed configuration (FP32 operator, FP64 solve, t = 750, t_p = 787).  The
    # oracle's Algorithm 1 takes minutes at this size, so the result is checked by what holds at
    # any size, with the oracle's direct sums: eq. (eq:alpha1) on the returned spectrum, sigma_1
    # by power iteration, and the Galerkin conditions of the projected Tikhonov solution at a
    # fixed alpha.
    announce("gkb full size", "gravity_l4", 750, 787)
    s, g, wd, winv, r, Gt, GtT = c1_weighted_problem()
    A = Operator(s, F32)
    t, tp = 750, 787
    args = (to_dev(r, F64), to_dev(wd, F64), to_dev(winv, F64), t, tp)
    _, a1, sig = S.gkb_project(A, *args, alpha_mode="alpha1")
    sig = to_host(sig)
    assert np.all(np.diff(sig) <= 0) and sig[-1] > 0
    assert abs(a1 - osol.alpha_one(g.n, g.m, sig)) <= 1e-12 * a1
    s1 = oracle_sigma1(Gt, GtT, r)
    assert abs(sig[0] - s1) <= 1e-5 * s1
    alpha = float(sig[t // 2])
    y, a, _ = S.gkb_project(A, *args, alpha_mode="fixed", alpha=alpha)
    assert a == alpha
    # exact GKB gives ~1e-16, FP32-sized errors in every product ~1e-8; a solution for alpha
    # 1 % off gives ~1e-2
    assert galerkin_defects(Gt, GtT, r, to_host(y), alpha).max() <= 2e-5
    A.close()


def test_rsvd_full_size_properties():
    # RSVD on the same problem (FP32 operator, FP64 solve, one power iteration, t = t_p = 787,
    # Omega passed in): eq. (eq:alpha1) on the returned spectrum, sigma_1 by power iteration,
    # and the Galerkin conditions over range(Q), which holds G~^T G~ G~^T Omega^T c for any c.
    announce("rsvd full size", "gravity_l4", 787, 787)
    s, g, wd, winv, r, Gt, GtT = c1_weighted_problem()
    A = Operator(s, F32)
    tp = 787
    omega = W.gaussian_matrix(tp, g.m, 11)
    args = (to_dev(r, F64), to_dev(wd, F64), to_dev(winv, F64), tp, tp, to_dev(omega, F64))
    _, a1, sig = S.rsvd_project(A, *args, alpha_mode="alpha1")
    sig = to_host(sig)
    assert np.all(np.diff(sig) <= 0) and sig[-1] > 0
    assert abs(a1 - osol.alpha_one(g.n, g.m, sig)) <= 1e-12 * a1
    s1 = oracle_sigma1(Gt, GtT, r)
    assert abs(sig[0] - s1) <= 1e-5 * s1
    alpha = float(sig[tp // 2])
    y, a, _ = S.rsvd_project(A, *args, alpha_mode="fixed", alpha=alpha)
    assert a == alpha
    # exact Algorithm 2 gives ~1e-16, FP32-sized errors in every product ~1e-8; alpha 1 % off
    # gives >= 3e-3
    assert rsvd_galerkin_defects(Gt, GtT, r, to_host(y), alpha, omega).max() <= 2e-5
    A.close()


def test_workspace_errors():
    s = W.survey(8, 8, 2, 25, 25, 25)
    A = Operator(s, F64)
    with pytest.raises(L.FastFocusError):
        S.workspace_bytes(A, "gkb", A.m + 1)
    r = torch.ones(A.m, dtype=F64, device="cuda")
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    y = torch.empty(A.n, dtype=F64, device="cuda")
    sig = torch.empty(4, dtype=F64, device="cuda")
    a = __import__("ctypes").c_double(1.0)
    lib = L.load()
    from paper_2004_13904_amd.operator import _ptr, _stream
    rc = lib.gkb_project(A.h, _ptr(r), _ptr(r), _ptr(torch.ones(A.n, dtype=F64, device="cuda")), 2, 4, 2, 1,
                         _ptr(y), __import__("ctypes").byref(a), _ptr(sig), _ptr(small), 16, _stream())
    assert rc == -4


@pytest.mark.parametrize("where", ["d_obs", "wd", "m_prev"])
def test_irls_step_rejects_non_finite_inputs(where):
    # a NaN in the data, the weights or the previous iterate is reported before the solve
    s = W.survey(8, 8, 2, 25, 25, 25)
    A = Operator(s, F64)
    d = torch.randn(A.m, dtype=F64, device="cuda")
    wd = torch.ones(A.m, dtype=F64, device="cuda")
    m0 = torch.zeros(A.n, dtype=F64, device="cuda")
    {"d_obs": d, "wd": wd, "m_prev": m0}[where][3] = float("nan")
    p = S.IrlsParams(solver="gkb", t=8, tp=9, lam=1.0)
    with pytest.raises(L.FastFocusError) as e:
        S.irls_step(A, p, 1, d, wd, m0)
    assert e.value.code == L.FF_EINVAL and "non-finite" in str(e.value)
    d[3] = 0.0 if where == "d_obs" else d[3]
    wd[3] = 1.0
    m0[3] = 0.0
    S.irls_step(A, p, 1, d, wd, m0)      # the same call with finite inputs succeeds


# ---- the n = 1e6 magnetic inversion (t = m/20 = 2500, t_p = 2625) -----------------------------

@pytest.fixture(scope="module")
def c2_problem():
    """The first IRLS step's weighted problem on the n = 1e6 magnetic survey: the cube + dike
    model, 2 % noise (tau1 = 0.02, tau2 = 0.002, seed 2), depth weighting beta = 1.4, W_L = I,
    r~ = W_d d_obs; products with G~ by the oracle's direct sums.  Also the largest singular
    value of G~ by Lanczos iteration on G~^T G~ over those products."""
    from scipy.sparse.linalg import LinearOperator, eigsh
    s = W.SURVEYS["magnetic_1m"]
    g = ogeom(s)
    T = op.kernel_table(g)
    m_true = W.block_model(s, W.MAGNETIC_1M_BLOCKS)
    d_exact = op.apply_G(g, m_true, T)
    eta, sd = W.noise(d_exact, 0.02, 0.002, 2)
    d_obs = d_exact + eta
    wd = 1.0 / sd
    winv = 1.0 / oirls.depth_weights(g, 1.4)
    r = wd * d_obs
    count = [0]
    t0 = time.perf_counter()

    def tick(what):
        # progress of the long host products (each about a second on many cores)
        count[0] += 1
        print(f"[c2 oracle] product {count[0]} ({what}) at {time.perf_counter() - t0:.1f} s", flush=True)

    def Gt(v):
        tick("G")
        return wd * op.apply_G(g, winv * v, T)

    def GtT(y):
        tick("G^T")
        return winv * op.apply_GT(g, wd * y, T)
    v0 = GtT(r)
    lo = LinearOperator((g.n, g.n), matvec=lambda v: GtT(Gt(np.asarray(v).ravel())), dtype=np.float64)
    lam = eigsh(lo, k=1, which="LA", v0=v0, tol=1e-8, ncv=20, maxiter=40, return_eigenvectors=False)
    return dict(s=s, g=g, T=T, d_obs=d_obs, wd=wd, winv=winv, r=r, Gt=Gt, GtT=GtT,
                sigma1=float(math.sqrt(lam[0])))


@pytest.mark.parametrize("basis", ["f64", "f32", "lean"])
def test_gkb_c2_full_size_properties(c2_problem, basis):
    # GKB at the metric's IRLS size (n = 1e6, t = 2500, t_p = 2625, FP32 operator; the n x t_p basis
    # in FP64, 21 GB, or FP32): eq. (eq:alpha1) on the returned spectrum, sigma_1 against the
    # oracle's Lanczos value, and the Galerkin conditions of the projected Tikhonov solution at a
    # fixed alpha, with the oracle's direct sums (size-dependent indexing of the 2.6e9-element
    # bases runs here)
    # "lean": FP64 bases with only the data-side basis reorthogonalized and the model-side basis
    # rebuilt in a second pass instead of stored (gkb_onesided = 2: a 1 GB workspace, not 22 GB)
    P = c2_problem
    g = P["g"]
    announce("gkb c2", basis, 2500, 2625)
    A = Operator(P["s"], F32)
    lean = basis == "lean"
    if lean:
        A.set_tuning(gkb_onesided=2)
        basis = "f64"
        assert S.workspace_bytes(A, "gkb", 2625) < 2e9
    t, tp = 2500, 2625
    args = (to_dev(P["r"], F64), to_dev(P["wd"], F64), to_dev(P["winv"], F64), t, tp)
    _, a1, sig = S.gkb_project(A, *args, alpha_mode="alpha1", basis=basis)
    sig = to_host(sig)
    assert np.all(np.diff(sig) <= 0) and sig[-1] > 0
    assert abs(a1 - osol.alpha_one(g.n, g.m, sig)) <= 1e-12 * a1
    assert abs(sig[0] - P["sigma1"]) <= 1e-5 * P["sigma1"], (sig[0], P["sigma1"])
    alpha = float(sig[t // 2])
    y, a, _ = S.gkb_project(A, *args, alpha_mode="fixed", alpha=alpha, basis=basis)
    assert a == alpha
    y = to_host(y)
    assert np.isfinite(y).all()
    assert galerkin_defects(P["Gt"], P["GtT"], P["r"], y, alpha, powers=2).max() <= 2e-5
    if lean:
        # against both bases reorthogonalized at the same alpha: the model-side basis keeps its
        # orthogonality to about 4e-8 through the FP32 operator, and y moves by about 2e-7
        A.set_tuning(gkb_onesided=0)
        y2 = to_host(S.gkb_project(A, *args, alpha_mode="fixed", alpha=alpha, basis="f64")[0])
        assert rel(y, y2) <= 1e-5, rel(y, y2)
    A.close()
    torch.cuda.empty_cache()


def test_irls_step_c2(c2_problem):
    # one IRLS step (k = 1, lambda = 1, GKB t = 2500, t_p = 2625, FP32 basis, alpha of
    # eq. (eq:alpha1)) at n = 1e6: the step equals clip(W^{-1} y) for the projected solve of the same
    # r~ (gkb_project), its scaled chi^2 equals eq. (scaledchi2) evaluated by the oracle on the
    # returned model, and the bounds hold
    P = c2_problem
    g = P["g"]
    announce("irls c2", 2500, 2625)
    A = Operator(P["s"], F32)
    p = S.IrlsParams(solver="gkb", t=2500, tp=2625, lam=1.0, eps2=1e-9, beta_depth=1.4, m_min=0.0,
                     m_max=0.1, basis="f32")
    d_obs = to_dev(P["d_obs"], F64)
    wd = to_dev(P["wd"], F64)
    m0 = torch.zeros(g.n, dtype=F64, device="cuda")
    m1, alpha, chi2 = S.irls_step(A, p, 1, d_obs, wd, m0)
    m1 = to_host(m1)
    assert np.isfinite(m1).all() and m1.min() >= 0.0 and m1.max() <= 0.1
    y, a1, _ = S.gkb_project(A, to_dev(P["r"], F64), wd, to_dev(P["winv"], F64), 2500, 2625,
                             alpha_mode="alpha1", basis="f32")
    # the same solve (the step's depth weights and r~ agree with the host's to rounding)
    assert abs(alpha - a1) <= 1e-9 * a1
    ref = np.clip(P["winv"] * to_host(y), 0.0, 0.1)
    assert np.abs(m1 - ref).max() <= 1e-6 * 0.1
    c_or = oirls.chi2_scaled(op.apply_G(g, m1, P["T"]), P["d_obs"], P["wd"])
    assert abs(chi2 - c_or) <= 1e-4 * c_or, (chi2, c_or)
    A.close()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("basis,onesided", [("f64", 0), ("f32", 0), ("f64", 1), ("f64", 2)])
def test_gkb_graph_replay_equals_launches(basis, onesided):
    # The GKB iteration loop captured into a graph at the first solve and replayed by the next
    # ones (gkb_graph = 1) gives the same y, sigma and alpha bit for bit as the same loop launched
    # kernel by kernel (gkb_graph = 0); the replays see new r~ and weights through the workspace.
    # Also with one-sided reorthogonalization (gkb_onesided = 1, 2; mode 2's second pass runs
    # launched after the replayed loop)
    s, g, G, wd, winv, Gt, r = problem("medium", "magnetic", seed=3)
    A = Operator(s, F32)
    A.set_tuning(gkb_onesided=onesided)
    t, tp = 40, 48
    ws = S._workspace(A, "gkb", tp, 0, None, basis)
    rng = np.random.default_rng(8)
    cases = [(r, wd, winv), (rng.standard_normal(g.m), 1.0 / (0.1 + rng.random(g.m)), 0.5 + rng.random(g.n))]
    for rr, ww, wi in cases + cases[::-1]:
        args = (to_dev(rr, F64), to_dev(ww, F64), to_dev(wi, F64), t, tp)
        out = {}
        for graph in (0, 1):
            A.set_tuning(gkb_graph=graph)
            y, a, sig = S.gkb_project(A, *args, alpha_mode="upre", ws=ws, basis=basis)
            torch.cuda.synchronize()
            out[graph] = (y.clone(), a, sig.clone())
        assert torch.equal(out[0][0], out[1][0])
        assert torch.equal(out[0][2], out[1][2])
        assert out[0][1] == out[1][1]
        # and the result is the oracle's Algorithm 1 within the FP32-operator bar
        Gt2 = ww[:, None] * G * wi[None, :]
        z, a_o, s_o = osol.gkb(lambda v: Gt2 @ v, lambda v: Gt2.T @ v, rr, g.n, t, tp, "upre")
        assert rel(to_host(out[1][2]), s_o) <= 1e-5
    # replays after a tuning change recapture (the key holds the tuning version)
    A.set_tuning(gkb_graph=1, lg_G=2)
    y2, _, _ = S.gkb_project(A, to_dev(r, F64), to_dev(wd, F64), to_dev(winv, F64), t, tp, alpha_mode="upre", ws=ws,
                             basis=basis)
    assert torch.isfinite(y2).all()
    A.close()


@pytest.mark.parametrize("mode", ["fixed", "upre", "alpha1"])
@pytest.mark.parametrize("qr,power", [(0, 1), (2, 1), (0, 0), (0, 2)])
def test_rsvd_single_precision_basis(mode, qr, power):
    # Algorithm 2 with the n x t_p matrices stored in FP32 (chunked FP64 Gram products and R^-1
    # products, FP64 projected problem) against the oracle's Algorithm 2 at the FP32-operator bar
    s, g, G, wd, winv, Gt, r = problem("mid", kernel="gravity", seed=2)
    t, tp = 60, 63
    announce("rsvd f32 basis", mode, "qr", qr, "power", power)
    omega = np.random.default_rng(4).standard_normal((tp, g.m))
    y0, a0, s0, F = osol.rsvd(*dense_ops(Gt), r, g.n, t, tp, omega, mode, 2.0, return_factors=True,
                              power_iters=power)
    A = Operator(s, F32)
    A.set_tuning(rsvd_qr=qr)
    args = (to_dev(r, F64), to_dev(wd, F64), to_dev(winv, F64), t, tp, to_dev(omega, F64))
    y, a, sig = S.rsvd_project(A, *args, mode, 2.0, power_iters=power, basis="f32")
    assert rel(to_host(sig)[:t], s0[:t]) <= 2e-5
    c0 = F["U"].T @ (F["B"].T @ r)
    check_alpha(mode, a, a0, s0[:t], c0, F32)
    ya = S.rsvd_project(A, *args, "fixed", a0, power_iters=power, basis="f32")[0]
    assert rel(to_host(ya), y0) <= 1e-4
    # the same problem with FP64 storage agrees to the FP32 storage's rounding
    yd = S.rsvd_project(A, *args, "fixed", a0, power_iters=power, basis="f64")[0]
    assert rel(to_host(ya), to_host(yd)) <= 1e-5



def test_rsvd_single_precision_basis_workspace_and_errors():
    # at the n = 1e6 magnetic survey with t_p = 2625 the FP32 storage keeps the workspace of
    # Algorithm 2 (and of the IRLS step around it) under 32 GB, against over 60 GB with the n x t_p
    # matrices in FP64; Householder QR (rsvd_qr = 1) needs FP64 storage, and an FP64 handle
    # rejects FP32 storage
    A = Operator(W.SURVEYS["magnetic_1m"], F32)
    tp = 2625
    b64 = S.workspace_bytes(A, "rsvd", tp, 1, "f64")
    b32 = S.workspace_bytes(A, "rsvd", tp, 1, "f32")
    i32 = S.workspace_bytes(A, "irls", tp, 1, "f32")
    announce("rsvd workspace", b64 / 1e9, b32 / 1e9, i32 / 1e9)
    assert b64 > 60e9 and b32 <= 32e9 and i32 <= 32e9
    assert b32 >= 8 * A.n * tp       # the two n x t_p FP32 matrices
    A.close()
    s, g, G, wd, winv, Gt, r = problem("mid", kernel="gravity", seed=2)
    A = Operator(s, F32)
    A.set_tuning(rsvd_qr=1)
    args = (to_dev(r, F64), to_dev(wd, F64), to_dev(winv, F64), 20, 21)
    with pytest.raises(L.FastFocusError) as e:
        S.rsvd_project(A, *args, None, "fixed", 2.0, basis="f32")
    assert e.value.code == L.FF_ENOTIMPL
    B = Operator(s, F64)
    with pytest.raises(L.FastFocusError) as e:
        S.rsvd_project(B, *args, None, "fixed", 2.0, basis="f32")
    assert e.value.code == L.FF_EDTYPE


def test_irls_rsvd_single_precision_basis_matches_oracle():
    # two IRLS steps with RSVD and FP32 storage of the n x t_p matrices against the oracle's steps
    s = W.survey(16, 12, 5, 25, 25, 25)
    g = ogeom(s)
    G = op.dense_G(g)
    rng = np.random.default_rng(3)
    m_true = np.zeros(g.n)
    m_true[rng.choice(g.n, 20, replace=False)] = 1.0
    d_exact = G @ m_true
    eta, sd = W.noise(d_exact, 0.02, 0.002, 5)
    d_obs = d_exact + eta
    wd = 1.0 / sd
    t, tp = 40, 42
    omega = rng.standard_normal((tp, g.m))
    A = Operator(s, F32)
    po = oirls.IrlsParams(solver="rsvd", t=t, tp=tp, lam=0.0, beta_depth=0.8, m_min=0.0, m_max=1.0)
    pg = S.IrlsParams(solver="rsvd", t=t, tp=tp, lam=0.0, beta_depth=0.8, m_min=0.0, m_max=1.0, basis="f32")
    m1o, a1o, c1o, _ = oirls.irls_step(g, po, 1, d_obs, wd, np.zeros(g.n), None, omega, G_dense=G)
    m1, a1, c1 = S.irls_step(A, pg, 1, to_dev(d_obs, F64), to_dev(wd, F64),
                             torch.zeros(g.n, dtype=F64, device="cuda"), None, to_dev(omega, F64))
    assert abs(a1 - a1o) <= 1e-5 * a1o
    assert rel(to_host(m1), m1o) <= 1e-4
    assert abs(c1 - c1o) <= 1e-4 * c1o
    m2o, a2o, c2o, _ = oirls.irls_step(g, po, 2, d_obs, wd, m1o, np.zeros(g.n), omega, G_dense=G)
    m2, a2, c2 = S.irls_step(A, pg, 2, to_dev(d_obs, F64), to_dev(wd, F64), to_dev(m1o, F64),
                             torch.zeros(g.n, dtype=F64, device="cuda"), to_dev(omega, F64))
    assert abs(a2 - a2o) <= 1e-3 * a2o
    assert rel(to_host(m2), m2o) <= 1e-4 + 2 * abs(a2 - a2o) / a2o
    assert abs(c2 - c2o) <= (1e-4 + 4 * abs(a2 - a2o) / a2o) * c2o


@pytest.mark.parametrize("solver", ["gkb", "rsvd"])
def test_irls_trajectory_matches_oracle(solver):
    # six free-running IRLS steps (Secs. 2.2-2.3, the paper's lambda = 1) on the FP64 operator
    # against the oracle's own loop from m^(0) = 0: every step's alpha, model and scaled chi^2.
    # Step 1 (eq. (eq:alpha1)) agrees to rounding; from step 2 on alpha is the UPRE minimizer, whose
    # flat minimum rounding moves by about 1e-7 relative, and each step feeds the next: the
    # trajectories stay within 2e-6 (measured: at most 5e-7 in alpha, 6e-8 in the model).
    s = W.survey(16, 12, 5, 25, 25, 25)
    g = ogeom(s)
    G = op.dense_G(g)
    rng = np.random.default_rng(3)
    m_true = np.zeros(g.n)
    m_true[rng.choice(g.n, 20, replace=False)] = 1.0
    d_exact = G @ m_true
    eta, sd = W.noise(d_exact, 0.02, 0.002, 5)
    d_obs = d_exact + eta
    wd = 1.0 / sd
    t, tp, K = 40, 42, 6
    omegas = {k: np.random.default_rng(100 + k).standard_normal((tp, g.m)) for k in range(1, K + 1)}
    po = oirls.IrlsParams(solver=solver, t=t, tp=tp, lam=1.0, beta_depth=0.8, m_min=0.0, m_max=1.0)
    pg = S.IrlsParams(solver=solver, t=t, tp=tp, lam=1.0, beta_depth=0.8, m_min=0.0, m_max=1.0)
    ref = []
    m_prev, m_prev2 = np.zeros(g.n), None
    for k in range(1, K + 1):
        m_new, a, c, _ = oirls.irls_step(g, po, k, d_obs, wd, m_prev, m_prev2, omegas[k], G_dense=G)
        ref.append((m_new, a, c))
        m_prev2, m_prev = m_prev, m_new
    got = []
    A = Operator(s, F64)
    S.irls(A, pg, to_dev(d_obs, F64), to_dev(wd, F64), k_max=K, stop_at_chi2=False,
           omega_fn=lambda k: to_dev(omegas[k], F64),
           callback=lambda k, m, a, c: got.append((to_host(m), a, c)))
    assert len(got) == K
    for k, ((mg, ag, cg), (mo, ao, co)) in enumerate(zip(got, ref), start=1):
        tol = 1e-11 if k == 1 else 2e-6
        announce("irls trajectory", solver, k, abs(ag - ao) / ao, rel(mg, mo), abs(cg - co) / co)
        assert abs(ag - ao) <= tol * ao
        assert rel(mg, mo) <= tol
        assert abs(cg - co) <= tol * co


@pytest.mark.parametrize("solver", ["gkb", "rsvd"])
def test_irls_trajectory_is_iterated_tikhonov(solver):
    # six chained IRLS steps of the device loop against a closed form (Secs. 2.2-2.3): with
    # lambda = 2 every focusing weight of eq. (WLdefn) is 1, with alpha fixed, the bounds inactive
    # and t = t_p = m each step adds the exact Tikhonov update of the current residual, so y = W m
    # follows iterated Tikhonov from y^(0) = 0 (tests/galerkin.py).  FP64 operator.
    s = W.survey(8, 8, 2, 25, 25, 25)
    g = ogeom(s)
    G = op.dense_G(g)
    rng = np.random.default_rng(4)
    d_obs = G @ rng.random(g.n) + 0.01 * rng.standard_normal(g.m)
    wd = 1.0 / (0.05 + rng.random(g.m))
    w = oirls.depth_weights(g, 0.8)
    Gt = wd[:, None] * G / w[None, :]
    alpha = 0.3 * np.linalg.svd(Gt, compute_uv=False)[5]
    K = 6
    ref = iterated_tikhonov(Gt, wd * d_obs, alpha, K)
    p = S.IrlsParams(solver=solver, t=g.m, tp=g.m, lam=2.0, beta_depth=0.8, m_min=-1e300, m_max=1e300,
                     alpha_fixed=alpha)
    got = []
    A = Operator(s, F64)
    S.irls(A, p, to_dev(d_obs, F64), to_dev(wd, F64), k_max=K, stop_at_chi2=False,
           omega_fn=lambda k: to_dev(np.random.default_rng(50 + k).standard_normal((g.m, g.m)), F64),
           callback=lambda k, m, a, c: got.append((to_host(m), a, c)))
    assert len(got) == K
    for k, (m_k, a, c) in enumerate(got, start=1):
        y = w * m_k
        r = wd * d_obs - Gt @ ref[k - 1]
        c_ref = (r @ r) / (g.m + math.sqrt(2.0 * g.m))
        announce("iterated tikhonov", solver, k, rel(y, ref[k - 1]), abs(c - c_ref) / c_ref)
        assert a == alpha
        assert rel(y, ref[k - 1]) <= 1e-10   # measured 2e-14
        assert abs(c - c_ref) <= 1e-10 * c_ref
