"""Torch-facing wrappers of the projected solvers and the IRLS step (argument marshalling
only; the computation runs in libfastfocus).

* ``gkb_project``  -- Algorithm 1 of the paper (Golub-Kahan bidiagonalization).
* ``rsvd_project`` -- Algorithm 2 (randomized SVD with one power iteration).
* ``irls_step``    -- one focusing IRLS step; ``irls`` iterates it to the chi^2 test of
  eq. (scaledchi2) or K_max steps (Sec. 3.1).
All vectors are float64 CUDA tensors; the operator inside runs in the Operator's dtype.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import torch

from . import _lib as L
from .operator import _ptr, _stream

ALPHA_MODES = {"upre": 0, "alpha1": 1, "fixed": 2}


def _f64(op, t, numel, name):
    return op._vec(t, numel, name, dtype=torch.float64)


BASIS = {"f64": 1, "f32": 0}   # FF_F64, FF_F32


def workspace_bytes(op, which, tp, solver=0, basis="f64"):
    b = C.c_size_t()
    code = {"gkb": 0, "rsvd": 1, "irls": 2}[which]
    L.call("ff_workspace_size", op.h, code, int(solver), BASIS[basis], int(tp), C.byref(b))
    return b.value


def _workspace(op, which, tp, solver=0, ws=None, basis="f64"):
    need = workspace_bytes(op, which, tp, solver, basis)
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=op.device)
    return ws


def gkb_project(op, r_tilde, wd, winv, t, tp, alpha_mode="upre", alpha=None, ws=None, stream=None,
                basis="f64"):
    """Returns (y, alpha, sigma): y standard-form (model update winv * y), sigma (tp,).
    basis: "f64" (default) or "f32" storage of the GKB bases.  The handle's gkb_onesided tuning
    picks the reorthogonalization: both bases (0, Algorithm 1), the data-side basis only (1), or
    that with the model-side basis rebuilt instead of stored (2); see ff_tuning."""
    _f64(op, r_tilde, op.m, "gkb_project")
    _f64(op, wd, op.m, "gkb_project")
    _f64(op, winv, op.n, "gkb_project")
    ws = _workspace(op, "gkb", tp, 0, ws, basis)
    y = torch.empty(op.n, dtype=torch.float64, device=op.device)
    sigma = torch.empty(tp, dtype=torch.float64, device=op.device)
    a = C.c_double(float(alpha) if alpha is not None else 0.0)
    L.call("gkb_project", op.h, _ptr(r_tilde), _ptr(wd), _ptr(winv), int(t), int(tp),
           ALPHA_MODES[alpha_mode], BASIS[basis], _ptr(y), C.byref(a), _ptr(sigma), _ptr(ws), ws.numel(),
           _stream(stream))
    return y, a.value, sigma


def rsvd_project(op, r_tilde, wd, winv, t, tp, omega=None, alpha_mode="upre", alpha=None, ws=None,
                 stream=None, seed=0, power_iters=1, basis="f64"):
    """omega: (tp, m) float64 Gaussian matrix, or None to draw it on the device from `seed`
    (Philox4x32-10, see rsvd_project in include/fastfocus.h).  basis: "f64" (default) or "f32"
    storage of the n x t_p matrices.  Returns (y, alpha, sigma)."""
    _f64(op, r_tilde, op.m, "rsvd_project")
    _f64(op, wd, op.m, "rsvd_project")
    _f64(op, winv, op.n, "rsvd_project")
    if omega is not None:
        _f64(op, omega, tp * op.m, "rsvd_project")
    ws = _workspace(op, "rsvd", tp, 1, ws, basis)
    y = torch.empty(op.n, dtype=torch.float64, device=op.device)
    sigma = torch.empty(tp, dtype=torch.float64, device=op.device)
    a = C.c_double(float(alpha) if alpha is not None else 0.0)
    L.call("rsvd_project", op.h, _ptr(r_tilde), _ptr(wd), _ptr(winv), int(t), int(tp), _ptr(omega),
           int(seed), int(power_iters), ALPHA_MODES[alpha_mode], BASIS[basis], _ptr(y), C.byref(a), _ptr(sigma), _ptr(ws),
           ws.numel(), _stream(stream))
    return y, a.value, sigma


@dataclass
class IrlsParams:
    solver: str = "gkb"
    t: int = 1
    tp: int = 1
    lam: float = 1.0
    eps2: float = 1e-9
    beta_depth: float = 0.8
    m_min: float = 0.0
    m_max: float = 1.0
    alpha_fixed: float = -1.0
    power_iters: int = 1
    seed: int = 0
    basis: str = "f64"


def irls_step(op, p: IrlsParams, k, d_obs, wd, m_prev, m_prev2=None, omega=None, ws=None,
              stream=None):
    """One IRLS step k (1-based).  Returns (m_new, alpha, chi2_scaled)."""
    _f64(op, d_obs, op.m, "irls_step")
    _f64(op, wd, op.m, "irls_step")
    _f64(op, m_prev, op.n, "irls_step")
    if m_prev2 is not None:
        _f64(op, m_prev2, op.n, "irls_step")
    solver = 0 if p.solver == "gkb" else 1
    if omega is not None:
        _f64(op, omega, p.tp * op.m, "irls_step")
    ws = _workspace(op, "irls", p.tp, solver, ws, p.basis)
    prm = L.FFIrlsParams(solver, int(p.t), int(p.tp), int(k), float(p.lam), float(p.eps2),
                         float(p.beta_depth), float(p.m_min), float(p.m_max), float(p.alpha_fixed),
                         int(p.power_iters), int(p.seed), BASIS[p.basis])
    m_new = torch.empty(op.n, dtype=torch.float64, device=op.device)
    a, chi2 = C.c_double(), C.c_double()
    L.call("irls_step", op.h, C.byref(prm), _ptr(d_obs), _ptr(wd), _ptr(m_prev), _ptr(m_prev2),
           _ptr(omega), _ptr(m_new), C.byref(a), C.byref(chi2), _ptr(ws), ws.numel(),
           _stream(stream))
    return m_new, a.value, chi2.value


def irls(op, p: IrlsParams, d_obs, wd, k_max=25, omega_fn=None, callback=None, stop_at_chi2=True):
    """The IRLS iteration of Secs. 2.3 and 3.1: m^(0) = 0, steps k = 1.. until the scaled
    chi^2 of eq. (scaledchi2) is <= 1 (when stop_at_chi2) or k = k_max.  omega_fn(k) supplies
    the RSVD matrix; without it the device generator draws it from (p.seed, k).
    Returns (m, history) with history a list of (k, alpha, chi2)."""
    m_prev = torch.zeros(op.n, dtype=torch.float64, device=op.device)
    m_prev2 = torch.zeros_like(m_prev)
    ws = _workspace(op, "irls", p.tp, 0 if p.solver == "gkb" else 1, None, p.basis)
    hist = []
    for k in range(1, k_max + 1):
        omega = omega_fn(k) if (p.solver == "rsvd" and omega_fn is not None) else None
        m_new, a, chi2 = irls_step(op, p, k, d_obs, wd, m_prev, m_prev2 if k > 1 else None, omega, ws)
        hist.append((k, a, chi2))
        if callback is not None:
            callback(k, m_new, a, chi2)
        m_prev2, m_prev = m_prev, m_new
        if stop_at_chi2 and chi2 <= 1.0:
            break
    return m_prev, hist
