"""Pins of the oracle's learned-guess network (oracle/learn.c) against
independent definitions: BF16 rounding of hand-picked values, the closed form
of GELU, finite differences, and torch autograd / torch.optim.Adam on the CPU
in float64 (a separate implementation of the same mathematics)."""
import numpy as np
import pytest
import torch

import oracle


def test_bf16_round_to_nearest_even():
    # 1 + 2^-8 lies halfway between 1 and 1 + 2^-7: ties go to the even mantissa (1.0)
    assert oracle.bf16(1.0 + 2.0 ** -8) == 1.0
    # 1 + 3*2^-8 lies halfway between 1 + 2^-7 (odd) and 1 + 2^-6 (even)
    assert oracle.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6
    # just above the halfway point rounds up
    assert oracle.bf16(1.0 + 2.0 ** -8 + 2.0 ** -20) == 1.0 + 2.0 ** -7
    # exactly representable values are unchanged, including sign and powers of two
    for v in (0.0, -0.0, 1.0, -2.5, 0.15625, 2.0 ** -126, 3.0 * 2.0 ** 100):
        assert oracle.bf16(v) == v
    # relative error of rounding to 8 significant bits is at most the unit roundoff 2^-8
    rng = np.random.default_rng(0)
    x = rng.standard_normal(1000) * 10.0 ** rng.uniform(-5, 5, 1000)
    r = np.array([oracle.bf16(v) for v in x])
    assert np.all(np.abs(r - x) <= 2.0 ** -8 * np.abs(x) * (1 + 1e-7))
    # and agrees with torch's own bfloat16 conversion (round to nearest even)
    t = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(r, t)


def test_gelu_closed_form_and_derivative():
    assert oracle.gelu(0.0) == 0.0
    # Phi(1) = 0.841344746068542948... (standard normal cdf)
    assert abs(oracle.gelu(1.0) - 0.8413447460685429) < 1e-15
    assert abs(oracle.gelu(-1.0) + 1.0 - 0.8413447460685429) < 1e-15  # gelu(-z) = gelu(z) - z
    assert abs(oracle.gelu(40.0) - 40.0) < 1e-12 and abs(oracle.gelu(-40.0)) < 1e-12
    assert oracle.gelu_grad(0.0) == 0.5
    for z in np.linspace(-6, 6, 49):
        h = 1e-5
        fd = (oracle.gelu(z + h) - oracle.gelu(z - h)) / (2 * h)
        assert abs(fd - oracle.gelu_grad(z)) < 1e-9


def _net(m, h, B, seed):
    rng = np.random.default_rng(seed)
    n = oracle.mlp_nparams(m, h)
    params = (rng.standard_normal(n) * 0.3).astype(np.float32)
    X = rng.standard_normal((B, m)).astype(np.float32)
    T = rng.standard_normal((B, m)).astype(np.float32)
    return params, X, T


def _torch_ref(m, h, params, X, T):
    p = torch.tensor(params.astype(np.float64), requires_grad=True)
    o = 0
    def take(k):
        nonlocal o
        v = p[o:o + k]
        o += k
        return v
    W1 = take(h * m).view(h, m); b1 = take(h); W2 = take(h * h).view(h, h); b2 = take(h)
    W3 = take(m * h).view(m, h); b3 = take(m)
    x = torch.tensor(X.astype(np.float64))
    t = torch.tensor(T.astype(np.float64))
    act = torch.nn.functional.gelu  # exact (erf) form
    y = act(act(x @ W1.T + b1) @ W2.T + b2) @ W3.T + b3
    loss = ((y - t) ** 2).mean()
    loss.backward()
    return loss.item(), y.detach().numpy(), p.grad.numpy()


@pytest.mark.parametrize("m,h,B", [(4, 6, 3), (20, 40, 37), (64, 256, 16)])
def test_mlp_without_rounding_matches_torch_autograd(m, h, B):
    params, X, T = _net(m, h, B, seed=m + h)
    loss, Y, g = oracle.mlp(m, h, params, X, T, emulate=False)
    tl, ty, tg = _torch_ref(m, h, params, X, T)
    assert abs(loss - tl) <= 1e-13 * abs(tl)
    assert np.max(np.abs(Y - ty)) <= 1e-12 * np.max(np.abs(ty))
    assert np.linalg.norm(g - tg) <= 1e-12 * np.linalg.norm(tg)


def test_mlp_gradient_against_finite_differences():
    m, h, B = 5, 7, 4
    params, X, T = _net(m, h, B, seed=3)
    _, _, g = oracle.mlp(m, h, params, X, T, emulate=False)
    rng = np.random.default_rng(1)
    for i in rng.choice(len(params), 25, replace=False):
        up, dn = params.copy(), params.copy()
        up[i] = np.float32(params[i] + np.float32(1e-2))
        dn[i] = np.float32(params[i] - np.float32(1e-2))
        lu = oracle.mlp(m, h, up, X, T, emulate=False)[0]
        ld = oracle.mlp(m, h, dn, X, T, emulate=False)[0]
        fd = (lu - ld) / (float(up[i]) - float(dn[i]))
        assert abs(fd - g[i]) <= 1e-4 * max(1.0, abs(g[i])), (i, fd, g[i])


def _rb(x):
    """FP64 -> FP32 -> BF16 (round to nearest even) -> FP64, by torch's own conversions."""
    return x.to(torch.float32).to(torch.bfloat16).to(torch.float64)


class _RoundGrad(torch.autograd.Function):
    """Identity forward; the incoming gradient is rounded to BF16 on the way back."""

    @staticmethod
    def forward(ctx, x):
        return x.view_as(x)

    @staticmethod
    def backward(ctx, g):
        return _rb(g)


class _RoundValue(torch.autograd.Function):
    """Value rounded to BF16 forward; gradient passes straight through."""

    @staticmethod
    def forward(ctx, x):
        return _rb(x)

    @staticmethod
    def backward(ctx, g):
        return g


def _torch_emulated(m, h, params, X, T):
    p = torch.tensor(params.astype(np.float64), requires_grad=True)
    sizes = [h * m, h, h * h, h, m * h, m]
    W1, b1, W2, b2, W3, b3 = torch.split(p, sizes)
    W1, W2, W3 = W1.view(h, m), W2.view(h, h), W3.view(m, h)
    rv, rg = _RoundValue.apply, _RoundGrad.apply
    act = torch.nn.functional.gelu
    x = _rb(torch.tensor(X.astype(np.float64)))
    z1 = rg(x @ rv(W1).T) + b1
    h1 = rv(act(z1))
    z2 = rg(h1 @ rv(W2).T) + b2
    h2 = rv(act(z2))
    y = rg(h2 @ rv(W3).T) + b3
    loss = ((y - torch.tensor(T.astype(np.float64))) ** 2).mean()
    loss.backward()
    return loss.item(), y.detach().numpy(), p.grad.numpy()


@pytest.mark.parametrize("m,h,B", [(20, 40, 37), (64, 256, 32)])
def test_mlp_emulated_rounding_matches_torch(m, h, B):
    """With emulation on, the oracle rounds operands and deltas to BF16 at the
    matrix products only; torch, told to round at the same places, agrees."""
    params, X, T = _net(m, h, B, seed=9)
    params *= 0.5
    l1, y1, g1 = oracle.mlp(m, h, params, X, T, emulate=True)
    tl, ty, tg = _torch_emulated(m, h, params, X, T)
    assert abs(l1 - tl) <= 1e-12 * abs(tl)
    assert np.max(np.abs(y1 - ty)) <= 1e-12 * np.max(np.abs(ty))
    assert np.linalg.norm(g1 - tg) <= 1e-12 * np.linalg.norm(tg)
    # and the rounding is a perturbation of order 2^-8, not a different function
    l0, y0, g0 = oracle.mlp(m, h, params, X, T, emulate=False)
    assert 0 < np.linalg.norm(y1 - y0) <= 2e-2 * np.linalg.norm(y0)
    assert 0 < np.linalg.norm(g1 - g0) <= 5e-2 * np.linalg.norm(g0)


def test_adam_matches_torch_optim():
    rng = np.random.default_rng(5)
    n = 50
    w = rng.standard_normal(n)
    m1, m2 = np.zeros(n), np.zeros(n)
    tw = torch.tensor(w.copy(), requires_grad=True)
    opt = torch.optim.Adam([tw], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    for t in range(1, 8):
        g = rng.standard_normal(n)
        oracle.adam(w, g, m1, m2, t, lr=1e-2)
        opt.zero_grad()
        tw.grad = torch.tensor(g)
        opt.step()
    assert np.max(np.abs(w - tw.detach().numpy())) < 1e-14
