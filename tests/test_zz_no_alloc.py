"""glmb_mlp_grad_noalloc, the allocation-free form of glmb_mlp_grad: the same gradient and loss
bit for bit, over two calls in a row (the second smaller, so rows of the shared scratch array
left by the first call must not leak into it), from two contexts on one device, and the
capacity limit refused before any device work."""
import numpy as np
import pytest

from oracle import proposal as pp
from paper_2512_06230_amd import scenarios as sc

pytestmark = pytest.mark.gpu

BASE = dict(dt=1.0, q=1.0, sigma_z=1.0, p_survive=0.99, det_rate=1.47, clutter_density=2e-3, gate_d2=18.42,
            birth_r_max=0.5, birth_rate=0.5, birth_sigma_v=2.0, birth_ru_max=0.5, birth_cluster_d=3.0,
            h_max=64, tau=0.0)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _data(seed, n):
    rng = np.random.default_rng(seed)
    X = np.column_stack([rng.chisquare(2, n), rng.normal(0, 1.5, n), rng.normal(0, 1.5, n), rng.uniform(0, 1, n),
                         rng.integers(0, 30, n), rng.integers(1, 6, n)]).astype(np.float32)
    y = (rng.uniform(0, 1, n) ** 3).astype(np.float32)
    w = rng.uniform(0.05, 1.0, n).astype(np.float32)
    return X, y, w


def _net(seed, X):
    params = sc.mlp_init(seed)
    norm = pp.feature_norm(X).astype(np.float32)
    return params.astype(np.float32), norm


def test_noalloc_gradient_equals_the_allocating_call(torch_cuda):
    torch = torch_cuda
    from paper_2512_06230_amd.glmb import MLP_NOALLOC_MAX, MLP_NPARAM, Tracker
    g = Tracker(BASE)
    g2 = Tracker(BASE)  # a second context on the same device shares the scratch array
    grad = torch.empty(MLP_NPARAM, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    for call, (seed, n, ctx) in enumerate([(1, 20000, g), (2, 3001, g), (3, 65, g2), (4, MLP_NOALLOC_MAX, g2),
                                           (5, 1, g)]):
        X, y, w = _data(seed, n)
        params, norm = _net(seed, X if n > 1 else np.vstack([X, X + 1]))
        P, Xd, yd, wd = (torch.as_tensor(a, device="cuda") for a in (params, X, y, w))
        grad.fill_(float("nan"))
        loss.fill_(float("nan"))
        ctx.mlp_grad_noalloc(P, norm, Xd, yd, wd, grad, loss)
        got_g, got_l = grad.cpu().numpy().copy(), loss.cpu().numpy().copy()
        ref_g, ref_l = ctx.mlp_grad(P, norm, Xd, yd, wd)
        np.testing.assert_array_equal(got_g, ref_g.cpu().numpy(), err_msg="call %d (n=%d) gradient" % (call, n))
        np.testing.assert_array_equal(got_l, ref_l.cpu().numpy(), err_msg="call %d (n=%d) loss" % (call, n))
        # and the oracle's loss (the gradient is checked element by element in the proposal tests)
        l_ref, _ = pp.loss_and_grad(params.astype(np.float64), norm.astype(np.float64), X.astype(np.float64),
                                    y.astype(np.float64), w.astype(np.float64))
        assert abs(float(got_l[0]) - l_ref) <= 1e-4 * abs(l_ref), (call, n, float(got_l[0]), l_ref)
        print("call %d: n=%d, loss %.6f, |grad| %.4e" % (call, n, float(got_l[0]), np.linalg.norm(got_g)), flush=True)
    g.close()
    g2.close()


def test_noalloc_refuses_more_samples_than_its_array(torch_cuda):
    torch = torch_cuda
    from paper_2512_06230_amd.glmb import GLMB_E_CAPACITY, MLP_NOALLOC_MAX, MLP_NPARAM, GlmbError, Tracker
    g = Tracker(BASE)
    n = MLP_NOALLOC_MAX + 1
    X, y, w = _data(7, n)
    params, norm = _net(7, X)
    P, Xd, yd, wd = (torch.as_tensor(a, device="cuda") for a in (params, X, y, w))
    grad = torch.zeros(MLP_NPARAM, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    with pytest.raises(GlmbError) as e:
        g.mlp_grad_noalloc(P, norm, Xd, yd, wd, grad, loss)
    assert e.value.status == GLMB_E_CAPACITY
    assert float(grad.abs().sum()) == 0.0 and float(loss[0]) == 0.0  # nothing was written
    g.close()
