"""Learned per-block codec selector: training and encoding drivers over the
C ABI (gc_block_features, gc_block_sizes, gc_mlp_*, gc_encode_blocks).

Every computation runs in the library's kernels; this module only draws the
seeded shuffles (passed to the kernels as index arrays), schedules the
learning rate and moves tensors.  The selector is not part of the paper:
it picks, for every block of 128 integers, one of the 16 codec classes of
the block container, in place of coding the block in all 16 classes."""
from __future__ import annotations

import time

import numpy as np

from . import gc


class Targets:
    """Device tensors of a training corpus: features [nb, 40] (float32),
    exhaustive classes [nb] (uint8) and relative size excesses [nb, 16]."""

    def __init__(self, ctx: gc.Context, d_in, nblocks: int):
        import torch
        self.n = int(nblocks)
        self.feat = torch.empty((self.n, gc.BLOCK_FEATURES), dtype=torch.float32, device="cuda")
        self.best = torch.empty(self.n, dtype=torch.uint8, device="cuda")
        self.cost = torch.empty((self.n, gc.BLOCK_CLASSES), dtype=torch.float32, device="cuda")
        ctx.block_features(d_in, self.n, self.feat)
        ctx.block_sizes(d_in, self.n, None, self.best, self.cost)


def init_params(seed: int) -> np.ndarray:
    """He-normal weights and zero biases of the 40-64-64-16 network, as the
    flat float32 vector of gc_mlp_set_params."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_in, fan_out in ((40, 64), (64, 64), (64, 16)):
        parts.append(rng.normal(0.0, np.sqrt(2.0 / fan_in), (fan_in, fan_out)).reshape(-1))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)


def train(ctx: gc.Context, t: Targets, epochs=30, batch=4096, lr=3e-3, lr_final=3e-4, lam=8.0, seed=0,
          model: gc.Mlp | None = None):
    """Adam over `epochs` seeded shuffles of the corpus with a geometric
    learning-rate decay from lr to lr_final.  Returns (model, per-epoch mean
    loss, seconds)."""
    import torch
    if model is None:
        model = gc.Mlp(ctx, batch)
        model.set_params(init_params(seed))
    rng = np.random.default_rng(seed)
    steps = (t.n + batch - 1) // batch
    d_loss = torch.zeros(epochs * steps, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for ep in range(epochs):
        rate = lr * (lr_final / lr) ** (ep / max(1, epochs - 1))
        perm = torch.from_numpy(rng.permutation(t.n).astype(np.int32)).cuda()
        opts = gc.adam_opts(lr=rate, lam=lam, batch=batch)
        model.train(t.feat, t.best, t.n, opts, d_cost=t.cost, d_index=perm, d_loss=d_loss[ep * steps:])
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    per_epoch = d_loss.view(epochs, steps).mean(dim=1).cpu().numpy()
    return model, per_epoch, secs


def save(model: gc.Mlp, path: str):
    """Checkpoint of the network and its Adam state (numpy .npz, no pickles)."""
    state, step = model.get_state()
    np.savez(path, state=state, step=np.uint64(step), params=np.uint64(gc.Mlp.param_count()),
             layout=np.array([40, 64, 64, 16], np.int32))


def load(ctx: gc.Context, path: str, max_batch=4096) -> gc.Mlp:
    """A network restored from save(); training continues where it stopped."""
    with np.load(path, allow_pickle=False) as z:
        if int(z["params"]) != gc.Mlp.param_count() or list(z["layout"]) != [40, 64, 64, 16]:
            raise ValueError("checkpoint of another network layout")
        model = gc.Mlp(ctx, max_batch)
        model.set_state(z["state"], int(z["step"]))
    return model


def encode(ctx: gc.Context, d_in, n: int, mode: int, model: gc.Mlp | None = None, fixed_class=0,
           with_classes=False):
    """The container of the first n integers of d_in (padded to whole
    blocks); returns (device words, words used[, classes])."""
    import torch
    nb = (n + gc.BLOCK_INTS - 1) // gc.BLOCK_INTS
    d_out = torch.empty(gc.blockmix_bound_words(n), dtype=torch.int32, device="cuda")
    d_cls = torch.empty(max(nb, 1), dtype=torch.uint8, device="cuda") if with_classes else None
    used = ctx.encode_blocks(d_in, n, mode, d_out, model=model, fixed_class=fixed_class, d_class_out=d_cls)
    return (d_out, used, d_cls) if with_classes else (d_out, used)
