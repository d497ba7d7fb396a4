"""Pins of the selector network's float64 reference: central finite
differences of the exact loss, closed forms at zero weights, bf16 rounding
against torch's conversion, and Adam against torch.optim.Adam."""
import numpy as np
import pytest
import torch

from oracle import mlp_ref as M


def problem(seed, B=12):
    rng = np.random.default_rng(seed)
    X = rng.random((B, M.NF))
    y = rng.integers(0, M.NC, B)
    c = rng.random((B, M.NC)) * 0.3
    c[np.arange(B), y] = 0.0
    theta = M.init_params(seed).astype(np.float64)
    theta += rng.normal(0, 0.05, theta.size)   # nonzero biases too
    return theta, X, y, c


@pytest.mark.parametrize("lam", [0.0, 2.5])
def test_grad_finite_differences(lam):
    theta, X, y, c = problem(1)
    L, g = M.grad(theta, X, y, c, lam, bf=False)
    assert L == pytest.approx(M.loss(theta, X, y, c, lam, bf=False), rel=1e-12)
    rng = np.random.default_rng(2)
    idx = np.concatenate([rng.choice(M.NPARAM, 300, replace=False),
                          np.arange(M.NPARAM - 16, M.NPARAM)])   # all of b3
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (M.loss(tp, X, y, c, lam, bf=False) - M.loss(tm, X, y, c, lam, bf=False)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 + 1e-5 * abs(fd), (i, fd, g[i])


def test_zero_weights_closed_form():
    _, X, y, c = problem(3)
    theta = np.zeros(M.NPARAM)
    L, g = M.grad(theta, X, y, c, 0.0)
    assert L == pytest.approx(np.log(16.0), rel=1e-14)
    p = M.unflatten(g)
    for name in ("W1", "b1", "W2", "b2", "W3"):
        assert not np.any(p[name]), name
    want = np.full(M.NC, 1.0 / 16) - np.bincount(y, minlength=M.NC) / y.size
    assert np.allclose(p["b3"], want, atol=1e-15)
    assert np.all(M.predict(theta, X) == 0)   # all logits tie: the first class


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(4)
    x = np.concatenate([rng.normal(0, 1, 20000), rng.normal(0, 1e-3, 5000), rng.normal(0, 1e4, 5000)])
    x32 = x.astype(np.float32)
    # ties: values exactly halfway between two bf16 numbers
    base = torch.from_numpy(rng.normal(0, 1, 2000).astype(np.float32)).to(torch.bfloat16).float().numpy()
    bits = base.view(np.uint32) | np.uint32(0x8000)
    x32 = np.concatenate([x32, bits.view(np.float32), np.float32([0.0, -0.0, 1.0, -3.0])])
    want = torch.from_numpy(x32).to(torch.bfloat16).float().numpy().astype(np.float64)
    assert np.array_equal(M.bf16(x32.astype(np.float64)), want)


def test_bf16_grad_close_to_exact():
    theta, X, y, c = problem(5, B=64)
    _, g_bf = M.grad(theta, X, y, c, 1.0, bf=True)
    _, g_ex = M.grad(theta, X, y, c, 1.0, bf=False)
    assert np.linalg.norm(g_bf - g_ex) <= 0.02 * np.linalg.norm(g_ex)


def test_adam_matches_torch():
    rng = np.random.default_rng(6)
    theta = rng.normal(0, 1, 500)
    opt = M.Adam(theta, lr=3e-3)
    t = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
    topt = torch.optim.Adam([t], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    for step in range(5):
        g = rng.normal(0, 1, 500) * (step + 1)
        opt.step(g)
        t.grad = torch.tensor(g, dtype=torch.float64)
        topt.step()
    assert np.allclose(opt.theta, t.detach().numpy(), rtol=1e-12, atol=1e-14)
