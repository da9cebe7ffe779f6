"""Focusing IRLS step and the experiment metrics (oracle; test infrastructure only).

Sec. 2.2-2.3 of the paper:
* objective eq. (globalfunction) / (dfandstab) with D = I, m_apr = 0, W_h = I,
* depth weighting W_z^(r) = (mean depth of layer r)^(-beta),
* focusing weights eq. (WLdefn) evaluated, per the IRLS description, on the
  difference of the two previous iterates:
      (W_L^(k))_ii = ((m^(k-1)_i - m^(k-2)_i)^2 + eps^2)^((lambda - 2) / 4),  W_L^(1) = I,
* standard form eq. (normalequations): G~ = W_d G W^{-1}, r~ = W_d (d_obs - G m^(k-1)),
  W = W_z W_L, the solver returns the standard-form vector z and the update is
  m^(k) = clip(m^(k-1) + W^{-1} z, m_min, m_max),
* alpha^(1) by eq. (eq:alpha1), UPRE for k > 1,
* the chi^2 test eq. (scaledchi2) on the clipped iterate.
Whole multi-step trajectories are pinned only where they have a closed form: with lambda = 2
(every focusing weight 1), alpha fixed, the bounds inactive and the full projected space, the
iterates follow iterated Tikhonov (tests/test_oracle_solvers.py).  With the focusing weights,
the UPRE alpha and active bounds: parity unpinned (single steps are pinned against the dense
closed form; a trajectory feeds rounding in alpha and the clipping into the next step).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import operator as op
from . import solvers
from .geometry import Geometry


@dataclass
class IrlsParams:
    solver: str = "gkb"          # "gkb" or "rsvd"
    t: int = 0
    tp: int = 0
    lam: float = 1.0             # lambda of eq. (WLdefn); 0 = minimum support
    eps2: float = 1e-9
    beta_depth: float = 0.8      # 0.8 gravity, 1.4 magnetic
    m_min: float = 0.0
    m_max: float = 1.0
    alpha_fixed: float = -1.0    # > 0 forces alpha at every step


def depth_weights(geom: Geometry, beta):
    """Diagonal of W_z over the model vector (constant within a layer)."""
    zmid = geom.layer_mid_depths()
    w = zmid ** (-beta)
    return np.repeat(w, geom.nx * geom.ny)


def focusing_weights(m_prev, m_prev2, lam, eps2, k):
    """Diagonal of W_L^(k)."""
    if k == 1:
        return np.ones_like(np.asarray(m_prev, dtype=np.float64))
    dm = np.asarray(m_prev, dtype=np.float64) - np.asarray(m_prev2, dtype=np.float64)
    return (dm * dm + eps2) ** ((lam - 2.0) / 4.0)


def chi2_scaled(Gm, d_obs, wd):
    """eq. (scaledchi2): ||W_d (G m - d_obs)||^2 / (m + sqrt(2 m)), m = number of data.

    Gm is the predicted data G m of the model being tested.  For pure noise of eq. (noisydata)
    whitened by W_d the numerator is chi-squared with m degrees of freedom (mean m, variance
    2 m), which is what the test pins (tests/test_oracle_solvers.py)."""
    Gm = np.asarray(Gm, dtype=np.float64)
    res = np.asarray(wd, dtype=np.float64) * (Gm - np.asarray(d_obs, dtype=np.float64))
    m = res.size
    return float(res @ res) / (m + math.sqrt(2.0 * m))


def irls_step(geom: Geometry, p: IrlsParams, k, d_obs, wd, m_prev, m_prev2, omega=None,
              table=None, G_dense=None):
    """One IRLS step k >= 1.  Returns (m_new, alpha, chi2_scaled, sigma)."""
    table = op.kernel_table(geom) if table is None and G_dense is None else table
    if G_dense is not None:
        G = lambda x: G_dense @ x
        GT = lambda y: G_dense.T @ y
    else:
        G = lambda x: op.apply_G(geom, x, table)
        GT = lambda y: op.apply_GT(geom, y, table)
    W = depth_weights(geom, p.beta_depth) * focusing_weights(m_prev, m_prev2, p.lam, p.eps2, k)
    r_tilde = wd * (d_obs - G(m_prev))
    Gt = lambda x: wd * G(x / W)
    GtT = lambda y: GT(wd * y) / W
    if p.alpha_fixed > 0:
        mode, af = "fixed", p.alpha_fixed
    else:
        mode, af = ("alpha1" if k == 1 else "upre"), None
    if p.solver == "gkb":
        z, alpha, sigma = solvers.gkb(Gt, GtT, r_tilde, geom.n, p.t, p.tp, mode, af)
    else:
        z, alpha, sigma = solvers.rsvd(Gt, GtT, r_tilde, geom.n, p.t, p.tp, omega, mode, af)
    m_new = np.clip(np.asarray(m_prev, dtype=np.float64) + z / W, p.m_min, p.m_max)
    return m_new, alpha, chi2_scaled(G(m_new), d_obs, wd), sigma


def snr_db(d_exact, d_obs):
    """eq. (SNR)."""
    return 20.0 * math.log10(np.linalg.norm(d_exact) / np.linalg.norm(d_obs - d_exact))


def relative_error(m_exact, m_k):
    """eq. (RE)."""
    return float(np.linalg.norm(m_exact - m_k) / np.linalg.norm(m_exact))
