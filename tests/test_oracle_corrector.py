"""Pins of the oracle's learned-corrector pieces (Sec. III.A, Sec. III.B /
Eq. 6): the analytic gradients of the MSE loss with respect to the filter K
and the pixel weights W, taken through B^T and the transposed row filter, are
checked against central finite differences of the oracle's own forward FDK
(the reconstruction is linear in K and in W, so the loss is quadratic in each
and the central difference is exact up to rounding); Adam is checked against
torch.optim.Adam on the CPU."""
import math

import numpy as np
import pytest
import torch

import synth

SPEC = synth.config("cone3d_crop32").with_(vol_shape=(9, 11, 13), vol_spacing=(1.0, 1.0, 1.0),
                                           det_shape=(7, 10), det_spacing=(1.6, 1.5), n_proj=9,
                                           angular_range=200 * math.pi / 180, sid=60.0, sdd=100.0)
M = 32


def _problem(ora, batch, seed=0):
    rng = np.random.default_rng(seed)
    p = rng.standard_normal((batch, SPEC.n_proj) + tuple(SPEC.det_shape))
    ref = rng.standard_normal((batch,) + tuple(SPEC.vol_shape))
    K = ora.ramp_response(M, ora.tau(SPEC)) + 0.1 * rng.standard_normal(M)
    W = 1.0 + 0.2 * rng.standard_normal(SPEC.det_shape)
    mask = (rng.random(SPEC.vol_shape) > 0.3).astype(np.float64)
    return p, ref, K, W, mask, rng


def _loss(ora, p, ref, K, W, mask):
    xs = np.stack([ora.corrector_forward(SPEC, p[b], K, W=W) for b in range(p.shape[0])])
    return ora.mse(xs, ref, np.broadcast_to(mask, xs.shape))


def _grads(ora, p, ref, K, W, mask):
    _, gx = _loss(ora, p, ref, K, W, mask)
    gq = np.stack([ora.backproject_adjoint(SPEC, gx[b]) for b in range(p.shape[0])])
    return ora.corrector_grad(SPEC, p, gq, K, W=W)


@pytest.mark.parametrize("batch", [1, 2])
def test_filter_and_weight_gradients_match_finite_differences(ora, batch):
    p, ref, K, W, mask, rng = _problem(ora, batch)
    dK, dW = _grads(ora, p, ref, K, W, mask)
    for _ in range(3):
        dk = rng.standard_normal(M)
        eps = 0.5
        fd = (_loss(ora, p, ref, K + eps * dk, W, mask)[0] - _loss(ora, p, ref, K - eps * dk, W, mask)[0]) / (2 * eps)
        an = float(dK @ dk)
        assert abs(fd - an) <= 1e-9 * abs(an)
        dw = rng.standard_normal(W.shape)
        fd = (_loss(ora, p, ref, K, W + eps * dw, mask)[0] - _loss(ora, p, ref, K, W - eps * dw, mask)[0]) / (2 * eps)
        an = float((dW * dw).sum())
        assert abs(fd - an) <= 1e-9 * abs(an)


def test_filter_gradient_single_frequency(ora):
    """Moving K along the even unit vector e_f + e_(M-f) changes the loss by
    exactly what the gradient predicts at that frequency pair (including the
    self-paired DC and Nyquist bins)."""
    p, ref, K, W, mask, _ = _problem(ora, 1, seed=4)
    dK, _ = _grads(ora, p, ref, K, W, mask)
    for f in (0, 1, 5, M // 2):
        d = np.zeros(M)
        d[f] += 1.0
        d[(M - f) % M] += 1.0
        fd = (_loss(ora, p, ref, K + d, W, mask)[0] - _loss(ora, p, ref, K - d, W, mask)[0]) / 2.0
        assert abs(fd - float(dK @ d)) <= 1e-9 * max(abs(fd), 1e-12)


def test_filter_gradient_is_even(ora):
    p, ref, K, W, mask, _ = _problem(ora, 1, seed=5)
    dK, _ = _grads(ora, p, ref, K, W, mask)
    assert np.allclose(dK, dK[(M - np.arange(M)) % M], rtol=0, atol=1e-14 * np.abs(dK).max())


def test_mse_gradient_and_value(ora):
    rng = np.random.default_rng(2)
    x, ref = rng.standard_normal(50), rng.standard_normal(50)
    mask = rng.random(50)
    L, g = ora.mse(x, ref, mask)
    assert L == pytest.approx(sum((mask[i] * (x[i] - ref[i])) ** 2 for i in range(50)) / 50, rel=1e-14)
    d = rng.standard_normal(50)
    fd = (ora.mse(x + d, ref, mask)[0] - ora.mse(x - d, ref, mask)[0]) / 2.0
    assert fd == pytest.approx(float(g @ d), rel=1e-12)


def test_adam_matches_torch_optimizer():
    from oracle import adam
    rng = np.random.default_rng(3)
    p0 = rng.standard_normal(40)
    grads = [rng.standard_normal(40) for _ in range(6)]
    lr, b1, b2, eps = 3e-2, 0.9, 0.99, 1e-6
    t_param = torch.nn.Parameter(torch.tensor(p0, dtype=torch.float64))
    opt = torch.optim.Adam([t_param], lr=lr, betas=(b1, b2), eps=eps)
    p, m, v = p0.copy(), np.zeros(40), np.zeros(40)
    for t, g in enumerate(grads, start=1):
        t_param.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        p, m, v = adam(p, g, m, v, t, lr=lr, beta1=b1, beta2=b2, eps=eps)
        assert np.allclose(p, t_param.detach().numpy(), rtol=0, atol=1e-13)


@pytest.mark.parametrize("kind", ["par2d", "fan2d"])
def test_filter_gradient_2d_matches_finite_differences(ora, kind):
    """The 2D FBP network with K as the only trainable layer (Eq. 6)."""
    base = synth.config("par2d_64") if kind == "par2d" else synth.config("fan2d_512")
    spec = base.with_(vol_shape=(14, 12), vol_spacing=(1.0, 1.1), det_shape=(19,), det_spacing=(1.3,), n_proj=11,
                      sid=40.0, sdd=70.0)
    rng = np.random.default_rng(8)
    p = rng.standard_normal((2, spec.n_proj, 19))
    ref = rng.standard_normal((2,) + spec.vol_shape)
    M = 64
    K = ora.ramp_response(M, ora.tau(spec)) + 0.1 * rng.standard_normal(M)

    def loss(Kv):
        xs = np.stack([ora.fbp(spec, p[b], K=Kv) for b in range(2)])
        return ora.mse(xs, ref)

    _, gx = loss(K)
    gq = np.stack([ora.backproject_adjoint(spec, gx[b]) for b in range(2)])
    dK, _ = ora.corrector_grad(spec, p, gq, K)
    for _ in range(3):
        d = rng.standard_normal(M)
        fd = (loss(K + 0.5 * d)[0] - loss(K - 0.5 * d)[0]) / 1.0
        assert abs(fd - float(dK @ d)) <= 1e-9 * abs(fd)
