"""GPU parity of the selector network's kernels (through the C ABI) against
the float64 reference that rounds to bf16 at the same points: logits,
classes, the loss and its gradient, and Adam steps.

Tolerances.  The device accumulates in fp32 (at most 64 terms per dot
product: relative error ~64 * 2^-24 ~ 4e-6), and an activation whose fp32
value lies that close to a bf16 rounding boundary may round the other way
than in float64 (one bf16 ulp, 2^-8 relative, on about one activation in
a thousand).  Logits and gradient entries therefore agree to about 1e-3 of
their scale; the bounds below are that, with a factor of safety."""
import sys

import numpy as np
import pytest

import oracle as O
from oracle import mlp_ref as M
from paper_1502_01916_amd import gc

from test_blocks_oracle import blocks

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    return torch


@pytest.fixture(scope="module")
def ctx(torch_cuda):
    c = gc.Context(0)
    yield c
    c.close()


def theta_for(seed):
    rng = np.random.default_rng(seed)
    t = M.init_params(seed).astype(np.float64)
    t += rng.normal(0, 0.05, t.size)
    return t.astype(np.float32)


def features(seed, n):
    """Feature rows of real blocks (exact in bf16) and of uniform noise."""
    rng = np.random.default_rng(seed)
    nb = n // 2
    real = np.array([O.block_features(b) for b in blocks(seed, nb)]) if nb else np.zeros((0, 40))
    noise = rng.random((n - nb, 40))
    return np.concatenate([real, noise]).astype(np.float32)


def labels_costs(seed, n):
    rng = np.random.default_rng(seed + 1)
    y = rng.integers(0, 16, n).astype(np.uint8)
    c = (rng.random((n, 16)) * 0.5).astype(np.float32)
    c[np.arange(n), y] = 0.0
    return y, c


@pytest.mark.parametrize("n", [1, 63, 64, 65, 1000])
def test_forward(torch_cuda, ctx, n):
    torch = torch_cuda
    say("mlp forward n=%d" % n)
    theta = theta_for(n)
    X = features(n, n)
    net = gc.Mlp(ctx, 64)
    net.set_params(theta)
    assert np.array_equal(net.get_params(), theta)
    d_x = torch.from_numpy(X).cuda()
    d_z = torch.full((n + 1, 16), 7.0, dtype=torch.float32, device="cuda")
    d_c = torch.full((n + 1,), 255, dtype=torch.uint8, device="cuda")
    net.forward(d_x, n, d_z, d_c)
    torch.cuda.synchronize()
    z = d_z.cpu().numpy().astype(np.float64)
    c = d_c.cpu().numpy()
    assert np.all(z[n] == 7.0) and c[n] == 255, "write past the last row"
    ref = M.forward(theta, X.astype(np.float64))["Z3"]
    scale = max(1.0, float(np.abs(ref).max()))
    err = np.abs(z[:n] - ref)
    assert err.max() <= 5e-3 * scale, err.max()
    assert np.median(err) <= 1e-4 * scale
    # classes: equal where the reference's top two differ clearly; near a tie
    # the device may take any class within the tolerance of the maximum
    top = ref.max(axis=1)
    tol = 5e-3 * scale
    for r in range(n):
        near = np.flatnonzero(ref[r] >= top[r] - tol)
        if near.size == 1:
            assert c[r] == near[0]
        else:
            assert c[r] in near
    net.close()


@pytest.mark.parametrize("batch,lam,indexed", [(1, 0.0, False), (64, 0.0, False), (200, 2.0, True),
                                               (4096, 0.0, True), (4096, 3.0, False)])
def test_grad(torch_cuda, ctx, batch, lam, indexed):
    torch = torch_cuda
    say("mlp grad batch=%d lam=%g indexed=%s" % (batch, lam, indexed))
    rows = batch * 2 if indexed else batch
    X = features(batch, rows)
    y, c = labels_costs(batch, rows)
    theta = theta_for(batch + 7)
    idx = np.random.default_rng(batch).permutation(rows)[:batch].astype(np.uint32) if indexed else None
    net = gc.Mlp(ctx, 4096)
    net.set_params(theta)
    d_x, d_y, d_c = torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda(), torch.from_numpy(c).cuda()
    d_i = torch.from_numpy(idx.view(np.int32)).cuda() if indexed else None
    d_g = torch.zeros(M.NPARAM, dtype=torch.float32, device="cuda")
    d_l = torch.zeros(1, dtype=torch.float32, device="cuda")
    net.grad(d_x, d_y, batch, d_cost=d_c, d_index=d_i, lam=lam, d_grad=d_g, d_loss=d_l)
    torch.cuda.synchronize()
    g = d_g.cpu().numpy().astype(np.float64)
    loss = float(d_l.cpu().numpy()[0])
    sel = idx if indexed else np.arange(batch)
    L, g_ref = M.grad(theta.astype(np.float64), X[sel].astype(np.float64), y[sel].astype(np.int64),
                      c[sel].astype(np.float64), lam)
    assert loss == pytest.approx(L, rel=1e-4)
    gmax = np.abs(g_ref).max()
    bad = np.abs(g - g_ref) > 2e-3 * gmax + 1e-2 * np.abs(g_ref)
    assert not bad.any(), (np.flatnonzero(bad)[:10], g[bad][:5], g_ref[bad][:5])
    assert np.linalg.norm(g - g_ref) <= 2e-3 * np.linalg.norm(g_ref)
    net.close()


def test_adam_steps(torch_cuda, ctx):
    """Each device Adam step equals the reference update applied to the
    device's own gradient at the same parameters."""
    torch = torch_cuda
    say("mlp adam steps")
    n = 1000
    X = features(11, n)
    y, c = labels_costs(11, n)
    theta = theta_for(11)
    net = gc.Mlp(ctx, 1024)
    net.set_params(theta)
    d_x, d_y, d_c = torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda(), torch.from_numpy(c).cuda()
    opt = M.Adam(theta, lr=2e-3)
    d_g = torch.zeros(M.NPARAM, dtype=torch.float32, device="cuda")
    opts = gc.adam_opts(lr=2e-3, lam=1.5, batch=1024)
    for step in range(4):
        before = net.get_params()
        net.grad(d_x, d_y, n, d_cost=d_c, lam=1.5, d_grad=d_g)
        g = d_g.cpu().numpy().astype(np.float64)
        opt.theta = before.astype(np.float64)
        want = opt.step(g)
        net.train(d_x, d_y, n, opts, d_cost=d_c)
        got = net.get_params().astype(np.float64)
        assert np.all(np.abs(got - want) <= 1e-3 * 2e-3 + 2e-6 * np.abs(want)), step
    net.close()


def test_training_lowers_loss(torch_cuda, ctx):
    """A few passes over real blocks with their exhaustive labels."""
    torch = torch_cuda
    say("mlp training sanity")
    nb = 4096
    x = blocks(21, nb)
    d_in = gc.to_device(x.reshape(-1))
    d_f = torch.zeros((nb, 40), dtype=torch.float32, device="cuda")
    d_s = torch.zeros((nb, 16), dtype=torch.int32, device="cuda")
    d_b = torch.zeros(nb, dtype=torch.uint8, device="cuda")
    d_c = torch.zeros((nb, 16), dtype=torch.float32, device="cuda")
    ctx.block_features(d_in, nb, d_f)
    ctx.block_sizes(d_in, nb, d_s, d_b, d_c)
    net = gc.Mlp(ctx, 512)
    net.set_params(M.init_params(3))
    steps = nb // 512
    d_l = torch.zeros(steps * 20, dtype=torch.float32, device="cuda")
    opts = gc.adam_opts(lr=3e-3, lam=1.0, batch=512)
    for ep in range(20):
        perm = torch.from_numpy(np.random.default_rng(ep).permutation(nb).astype(np.int32)).cuda()
        net.train(d_f, d_b, nb, opts, d_cost=d_c, d_index=perm, d_loss=d_l[ep * steps:])
    torch.cuda.synchronize()
    l = d_l.cpu().numpy()
    assert np.all(np.isfinite(l))
    assert l[-steps:].mean() < 0.6 * l[:steps].mean(), (l[:steps].mean(), l[-steps:].mean())


def test_checkpoint_resume(torch_cuda, ctx, tmp_path):
    """Training resumed from a checkpoint continues exactly as uninterrupted
    training (the kernels are deterministic)."""
    torch = torch_cuda
    from paper_1502_01916_amd import selector
    say("mlp checkpoint resume")
    nb = 2048
    x = blocks(23, nb)
    d_in = gc.to_device(x.reshape(-1))
    T = selector.Targets(ctx, d_in, nb)
    perms = [torch.from_numpy(np.random.default_rng(e).permutation(nb).astype(np.int32)).cuda() for e in range(4)]
    opts = gc.adam_opts(lr=3e-3, lam=4.0, batch=256)
    a = gc.Mlp(ctx, 256)
    a.set_params(M.init_params(5))
    for e in range(2):
        a.train(T.feat, T.best, nb, opts, d_cost=T.cost, d_index=perms[e])
    path = str(tmp_path / "ckpt.npz")
    selector.save(a, path)
    b = selector.load(ctx, path, 256)
    assert b.get_state()[1] == a.get_state()[1] == 2 * (nb // 256)
    for e in range(2, 4):
        a.train(T.feat, T.best, nb, opts, d_cost=T.cost, d_index=perms[e])
        b.train(T.feat, T.best, nb, opts, d_cost=T.cost, d_index=perms[e])
    sa, sb = a.get_state(), b.get_state()
    assert sa[1] == sb[1]
    assert np.array_equal(sa[0], sb[0])
    a.close()
    b.close()
