"""Pins of the oracle's GKB, RSVD and UPRE against dense linear algebra and statistics."""
import math

import numpy as np
import pytest

from galerkin import galerkin_defects, iterated_tikhonov, rsvd_galerkin_defects
from oracle import geometry, irls, operator as op, solvers


def small_problem(kernel="gravity", seed=0):
    g = geometry.uniform_geometry(8, 8, 2, 25.0, 25.0, 25.0, kernel=kernel, incl_deg=45.0,
                                  decl_deg=45.0)
    G = op.dense_G(g)
    rng = np.random.default_rng(seed)
    wd = 1.0 / (0.05 + rng.random(g.m))
    winv = 0.5 + rng.random(g.n)          # W^{-1}
    Gt = wd[:, None] * G * winv[None, :]
    r = rng.standard_normal(g.m) * 3.0
    return g, G, wd, winv, Gt, r


def ops(Gt):
    return (lambda x: Gt @ x), (lambda y: Gt.T @ y)


@pytest.mark.parametrize("kernel", ["gravity", "magnetic"])
def test_gkb_full_space_equals_tikhonov(kernel):
    g, G, wd, winv, Gt, r = small_problem(kernel)
    alpha = 0.3 * np.linalg.svd(Gt, compute_uv=False)[5]
    y, a, S = solvers.gkb(*ops(Gt), r, g.n, g.m, g.m, "fixed", alpha)
    ref = solvers.tikhonov_z(Gt, r, alpha)
    assert np.linalg.norm(y - ref) <= 1e-9 * np.linalg.norm(ref)


def test_gkb_factorization_relations():
    g, G, wd, winv, Gt, r = small_problem()
    tp = 30
    y, a, S, F = solvers.gkb(*ops(Gt), r, g.n, 20, tp, "fixed", 1.0, return_factors=True)
    A, H, B = F["A"], F["H"], F["B"]
    assert np.linalg.norm(Gt @ A - H @ B) <= 1e-12 * np.linalg.norm(B)
    assert np.abs(A.T @ A - np.eye(tp)).max() <= 1e-12
    assert np.abs(H.T @ H - np.eye(tp + 1)).max() <= 1e-12
    # B is lower bidiagonal: diagonal gamma_i, subdiagonal beta_{i+1}
    assert np.count_nonzero(np.triu(B, 1)) == 0 and np.count_nonzero(np.tril(B, -2)) == 0
    # leading singular values of the projected problem converge to those of G~
    s_true = np.linalg.svd(Gt, compute_uv=False)
    assert np.allclose(S[:3], s_true[:3], rtol=1e-10)


@pytest.mark.parametrize("kernel,q", [("gravity", 1), ("magnetic", 1), ("gravity", 0), ("magnetic", 2)])
def test_rsvd_full_space_equals_tikhonov(kernel, q):
    # with t_p = m the sketch spans the whole range of G~ for any number q of power iterations
    g, G, wd, winv, Gt, r = small_problem(kernel)
    alpha = 0.3 * np.linalg.svd(Gt, compute_uv=False)[5]
    omega = np.random.default_rng(9).standard_normal((g.m, g.m))
    y, a, S = solvers.rsvd(*ops(Gt), r, g.n, g.m, g.m, omega, "fixed", alpha, power_iters=q)
    ref = solvers.tikhonov_z(Gt, r, alpha)
    assert np.linalg.norm(y - ref) <= 1e-8 * np.linalg.norm(ref)
    assert np.allclose(S, np.linalg.svd(Gt, compute_uv=False), rtol=1e-8)


def test_rsvd_power_iteration_captures_dominant_space():
    g, G, wd, winv, Gt, r = small_problem()
    omega = np.random.default_rng(10).standard_normal((24, g.m))
    y, a, S, F = solvers.rsvd(*ops(Gt), r, g.n, 16, 24, omega, "fixed", 1.0, return_factors=True)
    s_true = np.linalg.svd(Gt, compute_uv=False)
    assert np.allclose(S[:4], s_true[:4], rtol=1e-4)
    Q = F["Q"]
    assert np.abs(Q.T @ Q - np.eye(24)).max() <= 1e-12


def test_rsvd_more_power_iterations_sharpen_the_spectrum():
    # a rank-deficient sketch: each power iteration raises the accuracy of the leading values
    g, G, wd, winv, Gt, r = small_problem()
    s_true = np.linalg.svd(Gt, compute_uv=False)
    omega = np.random.default_rng(11).standard_normal((12, g.m))
    err = []
    for q in (0, 1, 3):
        _, _, S = solvers.rsvd(*ops(Gt), r, g.n, 8, 12, omega, "fixed", 1.0, power_iters=q)
        err.append(np.abs(S[:6] - s_true[:6]).max() / s_true[0])
    assert err[0] > err[1] > err[2]


def test_upre_is_unbiased_for_predictive_risk():
    # For c = diag(s) xi + e with e ~ N(0, I): E[U(alpha)] equals E[||A(x_alpha - x)||^2]
    # exactly (Vogel's UPRE).  A dropped factor or a wrong sign breaks the equality.
    rng = np.random.default_rng(4)
    s = np.sort(rng.random(40) * 10)[::-1] + 1e-3
    xi = rng.standard_normal(40) / (1 + np.arange(40))
    for alpha in (0.05, 0.5, 3.0):
        phi = s * s / (s * s + alpha * alpha)
        U, P = [], []
        for _ in range(4000):
            c = s * xi + rng.standard_normal(40)
            U.append(solvers.upre(alpha, s, c))
            P.append(np.sum((phi * c - s * xi) ** 2))
        U, P = np.array(U), np.array(P)
        se = math.sqrt(np.var(U - P) / len(U))
        assert abs(U.mean() - P.mean()) < 5 * se


def test_upre_minimizer_against_brute_force():
    rng = np.random.default_rng(6)
    for trial in range(5):
        s = np.sort(np.exp(rng.uniform(-6, 2, 60)))[::-1]
        c = s * rng.standard_normal(60) * 3 + rng.standard_normal(60)
        a = solvers.upre_alpha(s, c)
        grid = np.exp(np.linspace(np.log(s[-1] * 1e-3), np.log(s[0]), 10000))
        brute = min(solvers.upre(g, s, c) for g in grid)
        assert solvers.upre(a, s, c) <= brute + 1e-9 * abs(brute)


def test_irls_step_matches_dense_closed_form():
    # One step with fixed alpha and a full projected space equals eq. (constantWL) with
    # m_apr -> m^(k-1), W = W_z W_L^(k), followed by the bound restriction.
    g = geometry.uniform_geometry(6, 5, 3, 30.0, 30.0, 30.0)
    G = op.dense_G(g)
    rng = np.random.default_rng(12)
    m_true = np.zeros(g.n)
    m_true[rng.choice(g.n, 10, replace=False)] = 1.0
    d_obs = G @ m_true + 0.01 * rng.standard_normal(g.m)
    wd = np.full(g.m, 1.0 / 0.01)
    m_prev = np.clip(rng.random(g.n) * 0.5, 0, 1)
    m_prev2 = np.clip(rng.random(g.n) * 0.5, 0, 1)
    p = irls.IrlsParams(solver="gkb", t=g.m, tp=g.m, lam=0.0, beta_depth=0.8, alpha_fixed=0.7,
                        m_min=-10.0, m_max=10.0)
    m_new, alpha, chi2, _ = irls.irls_step(g, p, 3, d_obs, wd, m_prev, m_prev2, G_dense=G)
    Wz = irls.depth_weights(g, 0.8)
    WL = irls.focusing_weights(m_prev, m_prev2, 0.0, 1e-9, 3)
    Wm = Wz * WL
    Wd = np.diag(wd)
    lhs = G.T @ Wd.T @ Wd @ G + alpha ** 2 * np.diag(Wm * Wm)
    rhs = G.T @ Wd.T @ Wd @ (d_obs - G @ m_prev)
    ref = m_prev + np.linalg.solve(lhs, rhs)
    assert np.linalg.norm(m_new - ref) <= 1e-7 * np.linalg.norm(ref)
    res = wd * (G @ m_new - d_obs)
    assert abs(chi2 - res @ res / (g.m + math.sqrt(2 * g.m))) <= 1e-12 * chi2


def test_depth_weights_values_and_layout():
    # Sec. 2.2: one weight per layer, (mean depth of the layer)^(-beta), repeated over the layer's
    # cells in the model's (layer, row, column) order.  Uneven layers 0-10-40-100 m have mean
    # depths 5, 25 and 70 m; with beta = 1 the weights are 0.2, 0.04 and 1/70, with beta = 2
    # 0.04, 0.0016 and 1/4900.
    g = geometry.Geometry(sx=3, sy=2, nz=3, dx=10.0, dy=10.0, z_edges=(0.0, 10.0, 40.0, 100.0))
    for beta, want in ((1.0, (0.2, 0.04, 1.0 / 70.0)), (2.0, (0.04, 0.0016, 1.0 / 4900.0))):
        w = irls.depth_weights(g, beta).reshape(3, 2 * 3)
        for r in range(3):
            assert np.allclose(w[r], want[r], rtol=1e-15, atol=0.0)
    assert np.array_equal(irls.depth_weights(g, 0.0), np.ones(g.n))
    # deeper layers get smaller weights for beta > 0, so W^{-1} lets deep cells take larger values
    w = irls.depth_weights(g, 0.8).reshape(3, -1)[:, 0]
    assert w[0] > w[1] > w[2]


def test_focusing_weights_reproduce_the_stabilizers():
    # eq. (WLdefn) is chosen so that sum_i (W_L)_ii^2 x_i^2 equals the stabilizer at x: the
    # minimum-support sum x^2 / (x^2 + eps^2) for lambda = 0, the smoothed l1 norm
    # x^2 / sqrt(x^2 + eps^2) for lambda = 1 (|x| as eps -> 0), and ||x||^2 (W_L = I) for lambda = 2.
    rng = np.random.default_rng(3)
    m1 = rng.standard_normal(200)
    m0 = rng.standard_normal(200)
    x = m1 - m0
    eps2 = 1e-3
    w0 = irls.focusing_weights(m1, m0, 0.0, eps2, 2)
    assert np.allclose(w0 * w0 * x * x, x * x / (x * x + eps2), rtol=1e-14, atol=0.0)
    w1 = irls.focusing_weights(m1, m0, 1.0, eps2, 2)
    assert np.allclose(w1 * w1 * x * x, x * x / np.sqrt(x * x + eps2), rtol=1e-14, atol=0.0)
    w1s = irls.focusing_weights(m1, m0, 1.0, 1e-14, 5)
    assert abs(np.sum(w1s * w1s * x * x) - np.sum(np.abs(x))) <= 1e-6 * np.sum(np.abs(x))
    assert np.allclose(irls.focusing_weights(m1, m0, 2.0, eps2, 3), 1.0, rtol=1e-15, atol=0.0)
    # the first step has no previous increment: W_L^(1) = I for any lambda
    assert np.array_equal(irls.focusing_weights(m1, m0, 0.0, eps2, 1), np.ones(200))
    # the weight depends on the increment only: no change at a cell gives eps^((lambda - 2) / 2)
    w = irls.focusing_weights(np.ones(3), np.ones(3), 0.0, 1e-4, 4)
    assert np.allclose(w, 1e-4 ** -0.5, rtol=1e-15)


@pytest.mark.parametrize("kernel", ["gravity", "magnetic"])
def test_gkb_solution_satisfies_galerkin_conditions(kernel):
    # Algorithm 1's y is the Tikhonov solution over its Krylov space (t_p well below m): the
    # normal-equation residual is orthogonal to y and to (G~^T G~)^j G~^T r~.  A solution for
    # alpha 1 % off, or y scaled by 1.001, breaks the conditions by orders of magnitude.
    g = geometry.uniform_geometry(20, 16, 4, 25.0, 25.0, 25.0, kernel=kernel, incl_deg=45.0,
                                  decl_deg=45.0)
    G = op.dense_G(g)
    rng = np.random.default_rng(8)
    wd = 1.0 / (0.05 + rng.random(g.m))
    winv = 0.5 + rng.random(g.n)
    Gt = wd[:, None] * G * winv[None, :]
    r = rng.standard_normal(g.m)
    f, fT = ops(Gt)
    t, tp = 60, 63
    _, _, S = solvers.gkb(f, fT, r, g.n, t, tp, "alpha1")
    alpha = float(S[t // 2])
    y, a, _ = solvers.gkb(f, fT, r, g.n, t, tp, "fixed", alpha)
    assert a == alpha
    assert galerkin_defects(f, fT, r, y, alpha).max() <= 1e-12
    y_off, _, _ = solvers.gkb(f, fT, r, g.n, t, tp, "fixed", 1.01 * alpha)
    assert galerkin_defects(f, fT, r, y_off, alpha).max() >= 1e-4
    assert galerkin_defects(f, fT, r, 1.001 * y, alpha).max() >= 1e-4


@pytest.mark.parametrize("kernel", ["gravity", "magnetic"])
def test_rsvd_solution_satisfies_galerkin_conditions(kernel):
    # Algorithm 2 with t = t_p: y is the Tikhonov solution over range(Q), which holds
    # G~^T G~ G~^T Omega^T c for every c (one power iteration).  alpha 1 % off, or truncation to
    # t < t_p, breaks the conditions by orders of magnitude.
    g = geometry.uniform_geometry(20, 16, 4, 25.0, 25.0, 25.0, kernel=kernel, incl_deg=45.0,
                                  decl_deg=45.0)
    G = op.dense_G(g)
    rng = np.random.default_rng(8)
    wd = 1.0 / (0.05 + rng.random(g.m))
    winv = 0.5 + rng.random(g.n)
    Gt = wd[:, None] * G * winv[None, :]
    r = rng.standard_normal(g.m)
    f, fT = ops(Gt)
    tp = 63
    omega = rng.standard_normal((tp, g.m))
    _, _, S = solvers.rsvd(f, fT, r, g.n, tp, tp, omega, "alpha1")
    alpha = float(S[tp // 2])
    y, _, _ = solvers.rsvd(f, fT, r, g.n, tp, tp, omega, "fixed", alpha)
    assert rsvd_galerkin_defects(f, fT, r, y, alpha, omega).max() <= 1e-12
    y_off, _, _ = solvers.rsvd(f, fT, r, g.n, tp, tp, omega, "fixed", 1.01 * alpha)
    assert rsvd_galerkin_defects(f, fT, r, y_off, alpha, omega).max() >= 1e-4
    y_cut, _, _ = solvers.rsvd(f, fT, r, g.n, tp - 10, tp, omega, "fixed", alpha)
    assert rsvd_galerkin_defects(f, fT, r, y_cut, alpha, omega).max() >= 1e-4
    # two power iterations: the space moves to (G~^T G~)^2 G~^T Omega^T
    y2, _, _ = solvers.rsvd(f, fT, r, g.n, tp, tp, omega, "fixed", alpha, power_iters=2)
    assert rsvd_galerkin_defects(f, fT, r, y2, alpha, omega, power_iters=2).max() <= 1e-12


def test_scaled_chi2_of_pure_noise():
    # eq. (scaledchi2) on the true model: G m_true - d_obs = -eta with eta drawn per eq. (noisydata)
    # and W_d = diag(1 / sigma), so the numerator is chi-squared with m degrees of freedom (mean m,
    # variance 2 m) and the mean of the scaled value over many draws is m / (m + sqrt(2 m)).
    # Dividing by m instead, by m + sqrt(m), or dropping the square moves the mean by 5 to 50
    # standard errors.
    from paper_2004_13904_amd import workloads as W
    g = geometry.uniform_geometry(16, 16, 2, 30.0, 30.0, 30.0)
    G = op.dense_G(g)
    m_true = np.zeros(g.n)
    m_true[: g.n // 3] = 1.0
    d_exact = G @ m_true
    S = 400
    vals = []
    for seed in range(S):
        eta, sd = W.noise(d_exact, 0.01, 0.001, 1000 + seed)
        vals.append(irls.chi2_scaled(G @ m_true, d_exact + eta, 1.0 / sd))
    m = g.m
    expect = m / (m + math.sqrt(2.0 * m))
    se = math.sqrt(2.0 * m) / (m + math.sqrt(2.0 * m)) / math.sqrt(S)
    assert abs(np.mean(vals) - expect) < 3.5 * se, (np.mean(vals), expect, se)
    # the sample variance of the numerator is 2 m as well (within its own sampling error)
    num = np.array(vals) * (m + math.sqrt(2.0 * m))
    assert abs(num.var(ddof=1) / (2.0 * m) - 1.0) < 0.25
    # a noise-free model gives zero
    assert irls.chi2_scaled(d_exact, d_exact, np.ones(m)) == 0.0


@pytest.mark.parametrize("solver", ["gkb", "rsvd"])
def test_irls_trajectory_is_iterated_tikhonov(solver):
    # A whole multi-step trajectory of the oracle's IRLS (Secs. 2.2-2.3) in the regime where it has
    # a closed form: lambda = 2 makes every focusing weight of eq. (WLdefn) 1, so W = W_z is the
    # same at every step; with alpha fixed, no bounds active and the full projected space
    # (t = t_p = m) each step adds the exact Tikhonov update of the current residual, and y = W m
    # follows iterated Tikhonov from y^(0) = 0.  A slip in how the steps chain (the residual of
    # the previous model, the W^{-1} of the update, the accumulation) breaks this at step 2.
    g = geometry.uniform_geometry(8, 8, 2, 25.0, 25.0, 25.0)
    G = op.dense_G(g)
    rng = np.random.default_rng(4)
    d_obs = G @ rng.random(g.n) + 0.01 * rng.standard_normal(g.m)
    wd = 1.0 / (0.05 + rng.random(g.m))
    w = irls.depth_weights(g, 0.8)
    A = wd[:, None] * G / w[None, :]
    alpha = 0.3 * np.linalg.svd(A, compute_uv=False)[5]
    K = 6
    ref = iterated_tikhonov(A, wd * d_obs, alpha, K)
    p = irls.IrlsParams(solver=solver, t=g.m, tp=g.m, lam=2.0, beta_depth=0.8, m_min=-1e300, m_max=1e300,
                        alpha_fixed=alpha)
    m_prev, m_prev2 = np.zeros(g.n), None
    steps = []
    for k in range(1, K + 1):
        omega = np.random.default_rng(50 + k).standard_normal((g.m, g.m))
        m_new, a, chi2, _ = irls.irls_step(g, p, k, d_obs, wd, m_prev, m_prev2, omega, G_dense=G)
        assert a == alpha
        y = w * m_new
        assert np.linalg.norm(y - ref[k - 1]) <= 1e-10 * np.linalg.norm(ref[k - 1])   # measured 4e-15
        r = wd * d_obs - A @ ref[k - 1]
        assert abs(chi2 - (r @ r) / (g.m + math.sqrt(2.0 * g.m))) <= 1e-10 * chi2
        steps.append(y)
        m_prev2, m_prev = m_prev, m_new
    # the steps move: the closed form separates them by far more than the tolerance
    assert np.linalg.norm(steps[-1] - steps[0]) >= 1e-2 * np.linalg.norm(steps[-1])


@pytest.mark.parametrize("kernel,sdiv", [("gravity", 8), ("magnetic", 4), ("gravity", 1)])
def test_one_sided_reorthogonalization_matches_algorithm_1(kernel, sdiv):
    # The device's gkb_onesided modes rest on a property of the Golub-Kahan process (Simon and Zha,
    # SIAM J. Sci. Comput. 21, 2000): when the data-side vectors h are kept orthogonal, the
    # model-side vectors a produced by the recurrence alone stay orthogonal to the level of the
    # products' rounding.  Here with the dense FP64 operator: a one-sided run of the recurrence
    # (written out below, MGS against H twice, no reorthogonalization of A) against the oracle's
    # Algorithm 1, up to t_p = m.
    g, G, wd, winv, Gt, r = small_problem(kernel, seed=2)
    tp = g.m // sdiv
    y0, a0, S0, F0 = solvers.gkb(*ops(Gt), r, g.n, tp, tp, "fixed", 0.05 * np.linalg.norm(Gt, 2),
                                  return_factors=True)
    A = np.zeros((g.n, tp))
    H = np.zeros((g.m, tp + 1))
    B = np.zeros((tp + 1, tp))
    beta = np.linalg.norm(r)
    H[:, 0] = r / beta
    a = np.zeros(g.n)
    for i in range(tp):
        b = Gt.T @ H[:, i] - beta * a
        gamma = np.linalg.norm(b)
        a = b / gamma
        A[:, i], B[i, i] = a, gamma
        c = Gt @ a - gamma * H[:, i]
        for _ in range(2):
            for j in range(i + 1):
                c = c - (H[:, j] @ c) * H[:, j]
        beta = np.linalg.norm(c)
        H[:, i + 1], B[i + 1, i] = c / beta, beta
    assert np.abs(A.T @ A - np.eye(tp)).max() <= 1e-12
    U, S, Vt = np.linalg.svd(B, full_matrices=False)
    assert np.allclose(S, S0, rtol=1e-10, atol=1e-12 * S0[0])
    alpha = 0.05 * np.linalg.norm(Gt, 2)
    y = np.linalg.norm(r) * (A @ (Vt.T @ (solvers.gamma_filter(alpha, S) * U[0, :])))
    assert np.linalg.norm(y - y0) <= 1e-10 * np.linalg.norm(y0)
