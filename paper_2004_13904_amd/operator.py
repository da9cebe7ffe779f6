"""Torch-facing wrapper of the layered BTTB operator (argument marshalling only).

``Operator(survey, dtype)`` builds the kernel spectra on the current HIP device; ``G``,
``GT`` and ``G_block`` enqueue the hand-written HIP passes on torch's current stream.
``GOp`` / ``GTOp`` are ``torch.autograd.Function``s whose backward is the adjoint HIP
operator (G is linear, so no activations are kept: the context holds only the handle).
"""
from __future__ import annotations

import ctypes as C
import os

import torch

from . import _lib as L


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


class Operator:
    """G and G^T of one survey geometry on one device (see include/fastfocus.h)."""

    def __init__(self, survey, dtype=torch.float32, nfft=(0, 0)):
        if not torch.cuda.is_available():
            raise L.FastFocusError("Operator", -6, "no HIP device available")
        if dtype not in (torch.float32, torch.float64):
            raise L.FastFocusError("Operator", -3, "dtype must be float32 or float64")
        geom, keep = L.make_geometry(survey, nfft)
        h = C.c_void_p()
        dt = L.FF_F32 if dtype == torch.float32 else L.FF_F64
        L.call("build_spectra", C.byref(geom), dt, _stream(), C.byref(h))
        self._attach(h, dict(survey))

    def _attach(self, h, survey):
        self.h = h
        self.survey = survey
        self.device = torch.device("cuda", torch.cuda.current_device())
        m, n, nfx, nfy, dti = C.c_int64(), C.c_int64(), C.c_int32(), C.c_int32(), C.c_int32()
        L.call("ff_spectra_info", h, C.byref(m), C.byref(n), C.byref(nfx), C.byref(nfy), C.byref(dti))
        self.m, self.n, self.nfft = m.value, n.value, (nfx.value, nfy.value)
        self.dtype = torch.float32 if dti.value == L.FF_F32 else torch.float64
        s = self.survey
        self.nx = s["sx"] + s.get("pad_xl", 0) + s.get("pad_xr", 0)
        self.ny = s["sy"] + s.get("pad_yl", 0) + s.get("pad_yr", 0)
        self.nz = s["nz"]
        self._batch_max = self.tuning["batch"]

    def save(self, path):
        """Checkpoint the spectra (and geometry) to a host file; see ff_spectra_save."""
        L.call("ff_spectra_save", self.h, os.fsencode(path))

    @classmethod
    def load(cls, path):
        """An Operator rebuilt from a spectra checkpoint (no prism or FFT evaluation)."""
        if not torch.cuda.is_available():
            raise L.FastFocusError("Operator.load", -6, "no HIP device available")
        h = C.c_void_p()
        L.call("ff_spectra_load", os.fsencode(path), _stream(), C.byref(h))
        g = L.FFGeometry()
        L.call("ff_spectra_geometry", h, C.byref(g), None)
        z = (C.c_double * (g.nz + 1))()
        L.call("ff_spectra_geometry", h, C.byref(g), z)
        survey = dict(sx=g.sx, sy=g.sy, nz=g.nz, dx=g.dx, dy=g.dy, z_edges=tuple(z),
                      kernel="gravity" if g.kernel == L.FF_GRAVITY_GZ else "magnetic",
                      incl_deg=g.incl_deg, decl_deg=g.decl_deg, field_nT=g.field_nT,
                      pad_xl=g.pad_xl, pad_xr=g.pad_xr, pad_yl=g.pad_yl, pad_yr=g.pad_yr)
        op = cls.__new__(cls)
        op._attach(h, survey)
        return op

    TUNING_KEYS = ("lg_G", "lg_GT", "row_tile", "batch", "col_batched", "rsvd_qr", "pair_fused", "gkb_graph",
                   "fft_plan_x", "fft_plan_y", "gkb_onesided")

    @property
    def batch_max(self):
        """Vectors per launch the handle's pass workspace holds (the batch build_spectra set)."""
        return self._batch_max

    @property
    def tuning(self):
        """The handle's launch tuning (see ff_tuning in include/fastfocus.h)."""
        t = L.FFTuning()
        L.call("ff_get_tuning", self.h, C.byref(t))
        return {k: getattr(t, k) for k in self.TUNING_KEYS}

    @property
    def qr_counts(self):
        """RSVD orthonormalizations on this handle so far: {"cholesky2": .., "cholesky3": ..,
        "householder": ..} (see rsvd_project in include/fastfocus.h)."""
        a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
        L.call("ff_solver_stats", self.h, C.byref(a), C.byref(b), C.byref(c))
        return {"cholesky2": a.value, "cholesky3": b.value, "householder": c.value}

    def set_tuning(self, **changes):
        """Change some tuning values (keys of ``tuning``); the others are kept."""
        cur = self.tuning
        for k, v in changes.items():
            if k not in cur:
                raise L.FastFocusError("ff_set_tuning", -1, f"unknown tuning key {k}")
            if v is not None:
                cur[k] = int(v)
        t = L.FFTuning(*[cur[k] for k in self.TUNING_KEYS])
        L.call("ff_set_tuning", self.h, C.byref(t))

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            L.load().ff_free_spectra(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- validation ------------------------------------------------------------------
    def _vec(self, t, numel, name, dtype=None):
        dtype = dtype or self.dtype
        if t.device != self.device:
            raise L.FastFocusError(name, -6, f"tensor on {t.device}, operator on {self.device}")
        if t.dtype != dtype:
            raise L.FastFocusError(name, -3, f"expected {dtype}, got {t.dtype}")
        if not t.is_contiguous():
            raise L.FastFocusError(name, -2, "tensor must be contiguous")
        if t.numel() != numel:
            raise L.FastFocusError(name, -2, f"expected {numel} values, got {t.numel()}")
        return t

    def _new(self, *shape):
        return torch.empty(*shape, dtype=self.dtype, device=self.device)

    # -- operator ----------------------------------------------------------------------
    def G(self, x, out=None, w_pre=None, w_post=None, stream=None):
        """d = w_post * G (w_pre * x); x has n values, returns m values."""
        self._vec(x, self.n, "apply_G")
        out = self._new(self.m) if out is None else self._vec(out, self.m, "apply_G")
        if w_pre is not None:
            self._vec(w_pre, self.n, "apply_G")
        if w_post is not None:
            self._vec(w_post, self.m, "apply_G")
        L.call("apply_G", self.h, _ptr(x), _ptr(out), _ptr(w_pre), _ptr(w_post), _stream(stream))
        return out

    def GT(self, d, out=None, w_pre=None, w_post=None, stream=None):
        """x = w_post * G^T (w_pre * d); d has m values, returns n values."""
        self._vec(d, self.m, "apply_GT")
        out = self._new(self.n) if out is None else self._vec(out, self.n, "apply_GT")
        if w_pre is not None:
            self._vec(w_pre, self.m, "apply_GT")
        if w_post is not None:
            self._vec(w_post, self.n, "apply_GT")
        L.call("apply_GT", self.h, _ptr(d), _ptr(out), _ptr(w_pre), _ptr(w_post), _stream(stream))
        return out

    def G_block(self, X, transpose=False, out=None, w_pre=None, w_post=None, stream=None):
        """Rows of X (k x n, or k x m when transposed) are the vectors; returns k x m (k x n)."""
        rin, rout = (self.m, self.n) if transpose else (self.n, self.m)
        if X.dim() != 2 or X.shape[1] != rin:
            raise L.FastFocusError("apply_G_block", -2, f"expected (k, {rin}), got {tuple(X.shape)}")
        k = X.shape[0]
        self._vec(X, k * rin, "apply_G_block")
        out = self._new(k, rout) if out is None else self._vec(out, k * rout, "apply_G_block")
        if w_pre is not None:
            self._vec(w_pre, rin, "apply_G_block")
        if w_post is not None:
            self._vec(w_post, rout, "apply_G_block")
        if k == 0:      # an empty batch: nothing to launch (its data pointers may be NULL)
            return out
        L.call("apply_G_block", self.h, int(bool(transpose)), k, _ptr(X), rin, _ptr(out), rout,
               _ptr(w_pre), _ptr(w_post), _stream(stream))
        return out

    def kernel_table(self, stream=None):
        """FP64 kernel table t_r(u, v), shape (nz, sy + ny - 1, sx + nx - 1)."""
        s = self.survey
        t = torch.empty(self.nz, s["sy"] + self.ny - 1, s["sx"] + self.nx - 1, dtype=torch.float64,
                        device=self.device)
        L.call("ff_kernel_table", self.h, _ptr(t), _stream(stream))
        return t


class GOp(torch.autograd.Function):
    """y = G x (x: (n,) or (k, n)); backward applies the hand-written G^T."""

    @staticmethod
    def forward(ctx, op, x):
        ctx.op = op
        x = x.contiguous()
        return op.G_block(x) if x.dim() == 2 else op.G(x)

    @staticmethod
    def backward(ctx, g):
        g = g.contiguous()
        gx = ctx.op.G_block(g, transpose=True) if g.dim() == 2 else ctx.op.GT(g)
        return None, gx


class FocusingLoss(torch.autograd.Function):
    """L = sum over models of ||wd (G m - d_obs)||^2 + alpha * sum m^2 / (m^2 + eps2), with the
    operator products and everything around them in the library (ff_focusing_loss / _grad):
    m is (n,) or (k, n); d_obs and wd have the shape of G m.  Returns a float64 scalar; the
    gradient flows to m only."""

    @staticmethod
    def forward(ctx, op, m, d_obs, wd, alpha=1.0, eps2=1e-9):
        m = m.contiguous()
        if m.dim() not in (1, 2) or m.shape[-1] != op.n:
            raise L.FastFocusError("FocusingLoss", -2, f"m must be (n,) or (k, n) with n = {op.n}")
        k = 1 if m.dim() == 1 else m.shape[0]
        op._vec(m, k * op.n, "FocusingLoss m")
        shape = (op.m,) if m.dim() == 1 else (k, op.m)
        d_obs = d_obs.contiguous()
        wd = wd.contiguous()
        for name, t in (("d_obs", d_obs), ("wd", wd)):
            if tuple(t.shape) != shape or t.dtype != m.dtype or t.device != m.device:
                raise L.FastFocusError("FocusingLoss", -2, f"{name} must be {shape} {m.dtype} on {m.device}")
        rw = torch.empty(shape, dtype=m.dtype, device=m.device)
        work = torch.empty(513, dtype=torch.float64, device=m.device)
        L.call("ff_focusing_loss", op.h, k, _ptr(m), _ptr(d_obs), _ptr(wd), float(alpha), float(eps2), _ptr(rw),
               _ptr(work), _stream())
        ctx.op, ctx.k, ctx.alpha, ctx.eps2 = op, k, float(alpha), float(eps2)
        ctx.save_for_backward(m, rw)
        return work[0]

    @staticmethod
    def backward(ctx, g):
        m, rw = ctx.saved_tensors
        g = g.to(torch.float64).contiguous()
        grad = torch.empty_like(m)
        L.call("ff_focusing_grad", ctx.op.h, ctx.k, _ptr(m), _ptr(rw), ctx.alpha, ctx.eps2, _ptr(g), _ptr(grad),
               _stream())
        return None, grad, None, None, None, None


class GTOp(torch.autograd.Function):
    """x = G^T d; backward applies G."""

    @staticmethod
    def forward(ctx, op, d):
        ctx.op = op
        d = d.contiguous()
        return op.G_block(d, transpose=True) if d.dim() == 2 else op.GT(d)

    @staticmethod
    def backward(ctx, g):
        g = g.contiguous()
        gd = ctx.op.G_block(g) if g.dim() == 2 else ctx.op.G(g)
        return None, gd


class SurveyBatch:
    """Several surveys of uneven size applied together.

    bind() builds a grouped plan (``ff_multi_create``): every survey's G x_i and G^T d_i then run
    in three grouped launches (all row transforms, all column passes, all inverse row
    transforms), captured once into a HIP graph (torch CUDA graph) and replayed.  Surveys the
    grouped kernels do not cover (double precision, embeddings above 512 x 512) make the batch
    fall back to one graph holding every survey's own launches.  ``xs`` / ``ds`` are the
    per-survey inputs; replay() refreshes ``gx`` (G x_i) and ``gtd`` (G^T d_i) in place from their
    current contents.
    """

    def __init__(self, surveys, dtype=torch.float32):
        self.ops = [Operator(s, dtype) for s in surveys]
        self.graph = None
        self.plan = None

    def bind(self, xs, ds):
        self.xs, self.ds = list(xs), list(ds)
        for op, x, d in zip(self.ops, self.xs, self.ds):
            op._vec(x, op.n, "SurveyBatch")
            op._vec(d, op.m, "SurveyBatch")
        self.gx = [op._new(op.m) for op in self.ops]
        self.gtd = [op._new(op.n) for op in self.ops]
        self._free_plan()
        n = len(self.ops)
        arr = C.c_void_p * n
        try:
            plan = C.c_void_p()
            L.call("ff_multi_create", n, arr(*[op.h.value for op in self.ops]),
                   arr(*[t.data_ptr() for t in self.xs]), arr(*[t.data_ptr() for t in self.gx]),
                   arr(*[t.data_ptr() for t in self.ds]), arr(*[t.data_ptr() for t in self.gtd]),
                   C.byref(plan))
            self.plan = plan
        except L.FastFocusError as e:
            if e.code not in (-3, -7):      # FF_EDTYPE, FF_ENOTIMPL: not covered, use per-survey launches
                raise
            self.plan = None
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            self.apply()
        torch.cuda.current_stream().wait_stream(side)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.apply()
        return self

    @property
    def grouped_launches(self):
        return self.plan is not None

    def apply(self):
        """All surveys' products on the current stream: grouped launches if planned, else eager."""
        if self.plan is not None:
            L.call("ff_multi_apply", self.plan, _stream())
        else:
            self.eager()

    def eager(self):
        """Every survey's own G and G^T launches, one survey after another."""
        for op, x, d, a, b in zip(self.ops, self.xs, self.ds, self.gx, self.gtd):
            op.G(x, out=a)
            op.GT(d, out=b)

    def replay(self):
        self.graph.replay()

    def _free_plan(self):
        if self.plan is not None and self.plan.value:
            L.load().ff_multi_free(self.plan)
        self.plan = None

    def close(self):
        self._free_plan()
        for op in self.ops:
            op.close()

    def __del__(self):
        try:
            self._free_plan()
        except Exception:
            pass
