"""Projected solvers of the normal equations (oracle; test infrastructure only).

Written from Sec. 2.4 of the paper (Algorithms 1 and 2) in its order and notation, in FP64 NumPy:

* ``gkb``     Algorithm 1: Golub-Kahan bidiagonalization G~ A = H B with modified
              Gram-Schmidt reorthogonalization of both bases, SVD of the
              (t_p + 1) x t_p bidiagonal B, truncated UPRE over t terms, and
              y = ||r~|| A V Gamma(alpha, Sigma) U(1, :)^T.
* ``rsvd``    Algorithm 2: randomized SVD with one power iteration (three economic
              QRs), eigen-decomposition of the symmetrized B^T B, UPRE over t terms,
              y = Q V~ Gamma U~^T (B^T r~).
* ``upre``    the unbiased predictive risk estimator on a projected spectrum.
* ``alpha_one`` eq. (eq:alpha1).
* ``tikhonov_z`` the closed form eq. (normalequations) in standard form (dense).

Readings where the paper is silent (each listed in the design notes):
* UPRE (cited, not printed): for singular values s_i and coefficients c_i of the
  right-hand side in the left singular basis, i = 1..t,
      U(alpha) = sum (alpha^2 / (s_i^2 + alpha^2))^2 c_i^2 + 2 sum s_i^2 / (s_i^2 + alpha^2) - t,
  the standard-form UPRE of a whitened problem (noise variance 1 after W_d).
  GKB: c_i = ||r~|| U(1, i).  RSVD: c = U~^T (B^T r~).
* Minimizer: 400-point logarithmic grid on [1e-3 * max(s_t, 1e-14 s_1), s_1], the
  grid point with the smallest U (the larger alpha on exact ties), then golden-section
  search in log(alpha) over the two neighbouring grid cells until the bracket is below
  1e-10 in log(alpha).
* alpha^(1) of eq. (eq:alpha1) uses all t_p projected singular values of the first
  solve; the mean is over the strictly positive ones.
* GKB breakdown (beta or gamma exactly zero, Krylov space exhausted): the new basis
  vector is set to zero, which leaves y unchanged.  The paper does not discuss it.
"""
from __future__ import annotations

import math

import numpy as np

UPRE_GRID = 400
UPRE_LO = 1e-3
GOLDEN_TOL = 1e-10


def gamma_filter(alpha, s):
    """Gamma(alpha, Sigma) = diag(s_i / (s_i^2 + alpha^2)) (Sec. 2.4, Algorithms 1 and 2)."""
    s = np.asarray(s, dtype=np.float64)
    return s / (s * s + alpha * alpha)


def upre(alpha, s, c):
    """Truncated UPRE functional U(alpha) for spectrum s and coefficients c (see module doc)."""
    s = np.asarray(s, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    a2 = alpha * alpha
    f = a2 / (s * s + a2)
    return float(np.sum(f * f * c * c) + 2.0 * np.sum(s * s / (s * s + a2)) - len(s))


def upre_alpha(s, c):
    """alpha minimizing U on the grid + golden-section refinement (module doc)."""
    s = np.asarray(s, dtype=np.float64)
    s1 = float(s[0])
    lo = UPRE_LO * max(float(s[-1]), 1e-14 * s1)
    grid = np.exp(np.linspace(math.log(lo), math.log(s1), UPRE_GRID))
    vals = np.array([upre(a, s, c) for a in grid])
    best = vals.min()
    k = int(np.nonzero(vals == best)[0][-1])          # larger alpha on ties
    a = math.log(grid[max(k - 1, 0)])
    b = math.log(grid[min(k + 1, UPRE_GRID - 1)])
    g = (math.sqrt(5.0) - 1.0) / 2.0
    x1 = b - g * (b - a)
    x2 = a + g * (b - a)
    f1 = upre(math.exp(x1), s, c)
    f2 = upre(math.exp(x2), s, c)
    while b - a > GOLDEN_TOL:
        if f1 <= f2:
            b, x2, f2 = x2, x1, f1
            x1 = b - g * (b - a)
            f1 = upre(math.exp(x1), s, c)
        else:
            a, x1, f1 = x1, x2, f2
            x2 = a + g * (b - a)
            f2 = upre(math.exp(x2), s, c)
    alpha = math.exp(0.5 * (a + b))
    # never return a point worse than the best grid point
    if upre(alpha, s, c) > best:
        alpha = float(grid[k])
    return alpha


def alpha_one(n, m, s):
    """eq. (eq:alpha1): alpha^(1) = (n/m)^3.5 * s_1 / mean(s_i > 0)."""
    s = np.asarray(s, dtype=np.float64)
    pos = s[s > 0]
    return (n / m) ** 3.5 * float(s[0]) / float(pos.mean())


def _choose_alpha(mode, s_t, c_t, n, m, s_all, alpha_fixed):
    if mode == "fixed":
        return float(alpha_fixed)
    if mode == "alpha1":
        return alpha_one(n, m, s_all)
    if mode == "upre":
        return upre_alpha(s_t, c_t)
    raise ValueError(mode)


def gkb(apply_Gt, apply_GtT, r_tilde, n, t, tp, alpha_mode="upre", alpha_fixed=None,
        return_factors=False):
    """Algorithm 1.  apply_Gt(x) = G~ x (n -> m), apply_GtT(y) = G~^T y (m -> n).

    Returns (y, alpha, sigma[, factors]) with y the standard-form solution (the model
    increment is W^{-1} y) and sigma the t_p singular values of B.
    """
    r_tilde = np.asarray(r_tilde, dtype=np.float64)
    m = r_tilde.shape[0]
    a = np.zeros(n)
    B = np.zeros((tp + 1, tp))
    H = np.zeros((m, tp + 1))
    A = np.zeros((n, tp))
    beta = float(np.linalg.norm(r_tilde))
    h = r_tilde / beta
    H[:, 0] = h
    for i in range(tp):
        b = apply_GtT(h) - beta * a
        for j in range(i):                                   # MGS against A
            b = b - (A[:, j] @ b) * A[:, j]
        gamma = float(np.linalg.norm(b))
        a = b / gamma if gamma > 0 else np.zeros(n)
        B[i, i] = gamma
        A[:, i] = a
        c = apply_Gt(a) - gamma * h
        for j in range(i + 1):                               # MGS against H
            c = c - (H[:, j] @ c) * H[:, j]
        beta = float(np.linalg.norm(c))
        h = c / beta if beta > 0 else np.zeros(m)
        B[i + 1, i] = beta
        H[:, i + 1] = h
    U, S, Vt = np.linalg.svd(B, full_matrices=False)         # svds(B, t_p): U (tp+1, tp)
    rnorm = float(np.linalg.norm(r_tilde))
    c_all = rnorm * U[0, :]
    alpha = _choose_alpha(alpha_mode, S[:t], c_all[:t], n, m, S, alpha_fixed)
    y = rnorm * (A @ (Vt.T @ (gamma_filter(alpha, S) * U[0, :])))
    if return_factors:
        return y, alpha, S, dict(A=A, H=H, B=B, U=U, S=S, Vt=Vt)
    return y, alpha, S


def rsvd(apply_Gt, apply_GtT, r_tilde, n, t, tp, omega, alpha_mode="upre", alpha_fixed=None,
         return_factors=False, power_iters=1):
    """Algorithm 2 (power_iters power iterations; the paper's algorithm has one).  omega is the
    t_p x m Gaussian matrix.

    The block products are column loops over the single-vector operators, as the
    paper describes them.  Returns (y, alpha, sigma[, factors]) with sigma all t_p
    values S (sorted descending) and y in standard form.
    """
    r_tilde = np.asarray(r_tilde, dtype=np.float64)
    m = r_tilde.shape[0]
    omega = np.asarray(omega, dtype=np.float64)

    def Gt_block(X):
        return np.stack([apply_Gt(X[:, k]) for k in range(X.shape[1])], axis=1)

    def GtT_block(Y):
        return np.stack([apply_GtT(Y[:, k]) for k in range(Y.shape[1])], axis=1)

    Y = GtT_block(omega.T).T                  # Y = Omega G~        (tp x n)
    Q, _ = np.linalg.qr(Y.T)                  # Q in R^{n x tp}
    for _ in range(power_iters):
        Y = Gt_block(Q)                       # Y = G~ Q            (m x tp)
        Q, _ = np.linalg.qr(Y)                # Q in R^{m x tp}
        Y = GtT_block(Q).T                    # Y = Q^T G~          (tp x n)
        Q, _ = np.linalg.qr(Y.T)              # Q in R^{n x tp}
    Bm = Gt_block(Q)                          # B = G~ Q            (m x tp)
    Yt = Bm.T @ Bm
    lam, V = np.linalg.eigh((Yt + Yt.T) / 2.0)
    S = np.sqrt(np.abs(lam))
    order = np.argsort(-S, kind="stable")
    S = S[order]
    Vt_ = V[:, order[:t]]
    St = S[:t]
    Ut = Vt_ / St[None, :]
    btr = Bm.T @ r_tilde
    c = Ut.T @ btr
    alpha = _choose_alpha(alpha_mode, St, c, n, m, S, alpha_fixed)
    y = Q @ (Vt_ @ (gamma_filter(alpha, St) * c))
    if return_factors:
        return y, alpha, S, dict(Q=Q, B=Bm, V=Vt_, U=Ut)
    return y, alpha, S


def tikhonov_z(Gt_dense, r_tilde, alpha):
    """Standard-form solution z = (G~^T G~ + alpha^2 I)^{-1} G~^T r~ (eq. normalequations),
    computed through the equivalent m x m system G~^T (G~ G~^T + alpha^2 I)^{-1} r~."""
    Gt_dense = np.asarray(Gt_dense, dtype=np.float64)
    m = Gt_dense.shape[0]
    K = Gt_dense @ Gt_dense.T + alpha * alpha * np.eye(m)
    return Gt_dense.T @ np.linalg.solve(K, r_tilde)
