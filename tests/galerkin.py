"""Galerkin conditions of a projected Tikhonov solution (test helper, numpy only).

Algorithm 1's solution y = A_tp w minimizes ||G~ y - r~||^2 + alpha^2 ||y||^2 over the span of
the basis A_tp, the Krylov space of G~^T G~ started at G~^T r~.  So the normal-equation residual
g = G~^T (G~ y - r~) + alpha^2 y is orthogonal to every vector of that space: to y itself and to
(G~^T G~)^j G~^T r~ for j < t_p.  These conditions hold at any size and need only products with
G~ and G~^T, which the oracle's direct sums supply where its own Algorithm 1 would take minutes.
"""
import numpy as np


def galerkin_defects(apply_Gt, apply_GtT, r_tilde, y, alpha, powers=3):
    """|v^T g| / (||v|| * scale) for v = y and v = (G~^T G~)^j G~^T r~, j < powers, where scale
    sums the norms of the three terms of g (so that rounding in them gives small values)."""
    y = np.asarray(y, dtype=np.float64)
    gy = apply_Gt(y)
    gtgy = apply_GtT(gy)
    gtr = apply_GtT(r_tilde)
    g = gtgy - gtr + alpha * alpha * y
    scale = np.linalg.norm(gtgy) + np.linalg.norm(gtr) + alpha * alpha * np.linalg.norm(y)
    out = [abs(y @ g) / (np.linalg.norm(y) * scale)]
    v = gtr
    for _ in range(powers):
        out.append(abs(v @ g) / (np.linalg.norm(v) * scale))
        v = apply_GtT(apply_Gt(v))
    return np.array(out)


def rsvd_galerkin_defects(apply_Gt, apply_GtT, r_tilde, y, alpha, omega, power_iters=1, combos=2, seed=0):
    """Algorithm 2 with t = t_p: y is the Tikhonov solution over range(Q), the span of
    (G~^T G~)^q G~^T Omega^T.  Defects as in galerkin_defects for v = y and for v =
    (G~^T G~)^q G~^T Omega^T c with `combos` standard normal c (omega: t_p x m)."""
    y = np.asarray(y, dtype=np.float64)
    gtgy = apply_GtT(apply_Gt(y))
    gtr = apply_GtT(r_tilde)
    g = gtgy - gtr + alpha * alpha * y
    scale = np.linalg.norm(gtgy) + np.linalg.norm(gtr) + alpha * alpha * np.linalg.norm(y)
    out = [abs(y @ g) / (np.linalg.norm(y) * scale)]
    rng = np.random.default_rng(seed)
    for _ in range(combos):
        v = apply_GtT(omega.T @ rng.standard_normal(omega.shape[0]))
        for _ in range(power_iters):
            v = apply_GtT(apply_Gt(v))
        out.append(abs(v @ g) / (np.linalg.norm(v) * scale))
    return np.array(out)


def iterated_tikhonov(A, b, alpha, K):
    """The iterates y^(1..K) of y^(k) = y^(k-1) + (A^T A + alpha^2 I)^{-1} A^T (b - A y^(k-1)),
    y^(0) = 0, in closed form: along the right singular vector v_i (singular value s_i, data
    coefficient c_i = u_i^T b) the error c_i / s_i - y_i shrinks by alpha^2 / (s_i^2 + alpha^2)
    per step, so y^(k)_i = (c_i / s_i) (1 - (alpha^2 / (s_i^2 + alpha^2))^k)."""
    U, s, Vt = np.linalg.svd(np.asarray(A, dtype=np.float64), full_matrices=False)
    c = U.T @ np.asarray(b, dtype=np.float64)
    q = alpha * alpha / (s * s + alpha * alpha)
    return [Vt.T @ ((c / s) * (1.0 - q ** k)) for k in range(1, K + 1)]
