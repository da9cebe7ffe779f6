"""The differentiable operator: torch.autograd.Functions whose backward is the hand-written
adjoint kernel, checked by gradcheck, by finite differences of the misfit + minimum-support
loss, and against the dense-G gradient of the oracle on a 16 x 16 x 4 crop."""
import numpy as np
import pytest
import torch

from gpu_common import ogeom, rel, same, to_dev, to_host
from oracle import operator as op
from paper_2004_13904_amd import workloads as W
from paper_2004_13904_amd import _lib as L
from paper_2004_13904_amd.operator import FocusingLoss, GOp, GTOp, Operator

pytestmark = pytest.mark.gpu
F64, F32 = torch.float64, torch.float32
EPS2 = 1e-9


def loss_fn(A, m, d_obs, wd, alpha):
    """||W_d (G m - d_obs)||^2 + alpha * sum m^2 / (m^2 + eps^2), summed over the batch."""
    r = wd * (GOp.apply(A, m) - d_obs)
    return (r * r).sum() + alpha * (m * m / (m * m + EPS2)).sum()


def test_gradcheck_G_and_GT():
    s = W.survey(6, 5, 3, 25, 25, 25, kernel="magnetic", incl=45, decl=45)
    A = Operator(s, F64)
    x = torch.rand(A.n, dtype=F64, device="cuda", requires_grad=True)
    d = torch.randn(A.m, dtype=F64, device="cuda", requires_grad=True)
    assert torch.autograd.gradcheck(lambda v: GOp.apply(A, v), (x,), eps=1e-6, atol=1e-8)
    assert torch.autograd.gradcheck(lambda v: GTOp.apply(A, v), (d,), eps=1e-6, atol=1e-8)
    X = torch.rand(3, A.n, dtype=F64, device="cuda", requires_grad=True)
    assert torch.autograd.gradcheck(lambda v: GOp.apply(A, v), (X,), eps=1e-6, atol=1e-8)


def crop_problem(dtype):
    s = W.survey(16, 16, 4, 20, 20, 20)        # a 16 x 16 x 4 crop of the 128 x 128 x 16 survey
    g = ogeom(s)
    G = op.dense_G(g)
    rng = np.random.default_rng(6)
    m_true = rng.random((4, g.n)) * (rng.random((4, g.n)) > 0.8)       # sparse models, batch 4
    d_obs = m_true @ G.T
    d_obs = d_obs + 0.01 * np.abs(d_obs).max() * rng.standard_normal(d_obs.shape)
    wd = 1.0 / (0.01 * np.abs(d_obs).max(axis=1, keepdims=True) + 0.01 * np.abs(d_obs))
    m0 = np.clip(m_true + 0.2 * rng.standard_normal(m_true.shape), 0, None)   # evaluation point
    m0[rng.random(m0.shape) < 0.3] = 0.0
    return s, g, G, m0, d_obs, wd


@pytest.mark.parametrize("dtype", [F64, F32])
def test_loss_gradient_matches_dense_reference(dtype):
    s, g, G, m0, d_obs, wd = crop_problem(dtype)
    alpha = 1.0
    A = Operator(s, dtype)
    m = to_dev(m0, dtype).requires_grad_(True)
    L = loss_fn(A, m, to_dev(d_obs, dtype), to_dev(wd, dtype), alpha)
    L.backward()
    # dense FP64 reference gradient: 2 G^T W_d^2 (G m - d) + alpha * 2 m eps^2 / (m^2 + eps^2)^2
    r = wd * (m0 @ G.T - d_obs)
    ref = 2.0 * (wd * r) @ G + alpha * 2.0 * m0 * EPS2 / (m0 * m0 + EPS2) ** 2
    assert rel(to_host(m.grad), ref) <= (1e-10 if dtype == F64 else 1e-5)
    ref_L = float((r * r).sum() + alpha * (m0 * m0 / (m0 * m0 + EPS2)).sum())
    assert abs(float(L.detach()) - ref_L) <= (1e-10 if dtype == F64 else 1e-5) * abs(ref_L)


def test_loss_gradient_finite_differences_full_size():
    # 128 x 128 x 16 survey, batch of 4 block models; central differences at coordinates where the
    # minimum-support term is smooth on the scale of h (m = 0 exactly, or m >= 100 eps)
    s = W.SURVEYS["gravity_diff"]
    A = Operator(s, F64)
    models = W.gravity_diff_models(s, 4, seed=5)
    rng = np.random.default_rng(8)
    m0 = models.copy()
    d_true = np.stack([to_host(A.G(to_dev(mm, F64))) for mm in models])
    d_obs = d_true + 0.01 * np.abs(d_true).max() * rng.standard_normal(d_true.shape)
    wd = np.full_like(d_obs, 1.0 / (0.01 * np.abs(d_true).max()))
    m0 = m0 * 0.9       # away from the data
    alpha = 1.0
    m = to_dev(m0, F64).requires_grad_(True)
    L = loss_fn(A, m, to_dev(d_obs, F64), to_dev(wd, F64), alpha)
    L.backward()
    grad = to_host(m.grad)
    flat = m0.reshape(-1)
    idx_zero = rng.choice(np.nonzero(flat == 0)[0], 3, replace=False)
    idx_big = rng.choice(np.nonzero(flat >= 100 * np.sqrt(EPS2))[0], 3, replace=False)
    h = 1e-6
    wd_t = to_dev(wd, F64)
    dob_t = to_dev(d_obs, F64)

    def residual(mm):
        with torch.no_grad():
            return to_host(wd_t * (GOp.apply(A, to_dev(mm, F64)) - dob_t))

    def ms(v):
        return v * v / (v * v + EPS2)

    for i in list(idx_zero) + list(idx_big):
        e = np.zeros_like(flat)
        e[i] = h
        rp = residual((flat + e).reshape(m0.shape))
        rm = residual((flat - e).reshape(m0.shape))
        # difference of squares formed from the residual difference (no cancellation in the sum)
        fd = float(((rp - rm) * (rp + rm)).sum()) / (2 * h)
        fd += alpha * (ms(flat[i] + h) - ms(flat[i] - h)) / (2 * h)
        g_i = grad.reshape(-1)[i]
        assert abs(fd - g_i) <= 1e-6 * max(1.0, abs(g_i)), (i, fd, g_i)


def test_batched_forward_backward_equals_per_vector():
    s = W.SURVEYS["gravity_diff"]
    A = Operator(s, F32)
    models = torch.tensor(W.gravity_diff_models(s, 4, seed=5), dtype=F32, device="cuda")
    X = models.clone().requires_grad_(True)
    Y = GOp.apply(A, X)
    w = torch.randn_like(Y)
    (Y * w).sum().backward()
    for c in range(4):
        same(Y[c], A.G(models[c].contiguous()))
        same(X.grad[c], A.GT(w[c].contiguous()))


@pytest.mark.parametrize("dtype", [F64, F32])
def test_fused_focusing_loss_matches_dense_reference(dtype):
    # the library's fused objective (misfit + minimum support with the operator inside) against the
    # dense FP64 loss and gradient on the crop
    s, g, G, m0, d_obs, wd = crop_problem(dtype)
    alpha = 1.0
    A = Operator(s, dtype)
    m = to_dev(m0, dtype).requires_grad_(True)
    Lf = FocusingLoss.apply(A, m, to_dev(d_obs, dtype), to_dev(wd, dtype), alpha, EPS2)
    Lf.backward()
    r = wd * (m0 @ G.T - d_obs)
    ref = 2.0 * (wd * r) @ G + alpha * 2.0 * m0 * EPS2 / (m0 * m0 + EPS2) ** 2
    ref_L = float((r * r).sum() + alpha * (m0 * m0 / (m0 * m0 + EPS2)).sum())
    tol = 1e-10 if dtype == F64 else 1e-5
    assert Lf.dtype == F64 and abs(float(Lf.detach()) - ref_L) <= tol * abs(ref_L)
    assert rel(to_host(m.grad), ref) <= tol


def test_fused_focusing_loss_equals_unfused_and_gradchecks():
    s = W.survey(7, 6, 3, 25, 25, 25, kernel="magnetic", incl=45, decl=45)
    A = Operator(s, F64)
    rng = np.random.default_rng(3)
    m0 = rng.random((2, A.n)) * (rng.random((2, A.n)) > 0.5)
    d_obs = to_dev(rng.standard_normal((2, A.m)), F64)
    wd = to_dev(0.5 + rng.random((2, A.m)), F64)
    alpha, eps2 = 0.7, 1e-3          # a smooth stabilizer at the scale of the finite differences
    m1 = to_dev(m0, F64).requires_grad_(True)
    m2 = to_dev(m0, F64).requires_grad_(True)
    L1 = FocusingLoss.apply(A, m1, d_obs, wd, alpha, eps2)
    r = wd * (GOp.apply(A, m2) - d_obs)
    L2 = (r * r).sum() + alpha * (m2 * m2 / (m2 * m2 + eps2)).sum()
    (3.0 * L1).backward()           # an upstream factor reaches the gradient
    (3.0 * L2).backward()
    assert abs(float(L1.detach()) - float(L2.detach())) <= 1e-12 * abs(float(L2.detach()))
    assert rel(to_host(m1.grad), to_host(m2.grad)) <= 1e-12
    x = to_dev(m0[0], F64).requires_grad_(True)
    assert torch.autograd.gradcheck(lambda v: FocusingLoss.apply(A, v, d_obs[0], wd[0], alpha, eps2), (x,),
                                    eps=1e-6, atol=1e-7)


def test_fused_focusing_loss_rejects_bad_arguments():
    s = W.survey(7, 6, 3, 25, 25, 25)
    A = Operator(s, F32)
    m = torch.rand(2, A.n, device="cuda")
    d = torch.randn(2, A.m, device="cuda")
    w = torch.ones(2, A.m, device="cuda")
    with pytest.raises(L.FastFocusError):
        FocusingLoss.apply(A, m, d[:, :-1].contiguous(), w, 1.0, 1e-9)      # wrong data shape
    with pytest.raises(L.FastFocusError):
        FocusingLoss.apply(A, m.double(), d.double(), w.double(), 1.0, 1e-9)   # wrong dtype
    with pytest.raises(L.FastFocusError):
        FocusingLoss.apply(A, m, d, w, 1.0, 0.0)                            # eps2 must be > 0
