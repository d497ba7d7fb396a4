"""Pins of the oracle's per-block container (the learned selector's codec
classes): round trips through the whole-list decoder, closed-form data sizes
of constant-width blocks, the size bookkeeping, the exhaustive argmin with its
tie rule, and the features recomputed here by brute force."""
import numpy as np
import pytest

import oracle as O
from paper_1502_01916_amd import synth


def blocks(seed, nb):
    """128-integer blocks with a mixed width profile: a base width per block,
    per-tuple jitter and a few wide outliers (the shape of d-gap blocks)."""
    rng = np.random.default_rng(seed)
    out = np.zeros((nb, 128), np.uint32)
    for b in range(nb):
        base = int(rng.integers(0, 29))
        w = np.clip(base + rng.integers(-3, 3, 128), 0, 32)
        v = np.where(w == 0, 0, (1 << np.maximum(w - 1, 0)).astype(np.uint64) +
                     rng.integers(0, 1 << 62, 128, dtype=np.uint64) % np.maximum((1 << np.maximum(w - 1, 0)).astype(np.uint64), 1))
        out[b] = v.astype(np.uint32)
        if rng.random() < 0.5:
            k = int(rng.integers(1, 12))
            idx = rng.choice(128, k, replace=False)
            out[b, idx] = rng.integers(1 << 20, 1 << 32, k, dtype=np.uint64).astype(np.uint32)
    return out


def bit_width(v):
    v = np.asarray(v, dtype=np.uint64)
    w = np.zeros(v.shape, np.int64)
    for t in range(32):
        w += (v >> np.uint64(t)) > 0
    return w


@pytest.mark.parametrize("kappa", range(O.NCLASS))
def test_block_round_trip(kappa):
    for x in blocks(100 + kappa, 24):
        bw, payload = O.block_encode(x, kappa)
        assert bw & 31 == kappa
        Cw, Dw, Ew = (bw >> 5) & 511, (bw >> 14) & 511, (bw >> 23) & 511
        assert Cw + Dw + Ew == payload.size
        assert O.block_size(x, kappa) == 1 + payload.size
        assert np.array_equal(O.block_decode(bw, payload), x)


@pytest.mark.parametrize("kappa", range(O.NCLASS))
def test_block_constant_width_data_size(kappa):
    """A block whose 128 integers all have width w needs 4w data words at
    least (128 w bits); the classes that code any width exactly (AFOR frames,
    PFD with no exceptions) need exactly that.  Width 0 needs no data."""
    codec = O.block_class_params(kappa).codec
    for w in range(0, 33):
        x = np.full(128, 0 if w == 0 else (1 << (w - 1)) | 1, np.uint32)
        if w == 1:
            x[:] = 1
        bw, payload = O.block_encode(x, kappa)
        Dw, Ew = (bw >> 14) & 511, (bw >> 23) & 511
        assert Dw >= 4 * w, (kappa, w, Dw)
        if codec in (O.AFOR, O.PFD):
            assert Dw == 4 * w and Ew == 0, (kappa, w, Dw, Ew)


def test_block_class_table():
    """Classes 0..15 are G-SIM, binary CG 1/2/4/8, CU CG 1/2/4/8, IU CG 4/8,
    AFOR and PFD with zeta 1/64, 1/10, 2/10, 3/10."""
    want = [(O.SIMPLE, None, None)] + \
        [(O.SCHEME, cg, O.LD_BINARY) for cg in (1, 2, 4, 8)] + \
        [(O.SCHEME, cg, O.LD_CU) for cg in (1, 2, 4, 8)] + \
        [(O.SCHEME, cg, O.LD_IU) for cg in (4, 8)] + [(O.AFOR, None, None)] + [(O.PFD, None, None)] * 4
    for kappa, (codec, cg, ld) in enumerate(want):
        p = O.block_class_params(kappa)
        assert p.codec == codec
        if cg is not None:
            assert (p.cg, p.ld) == (cg, ld)
    z = [(O.block_class_params(k).zeta_num, O.block_class_params(k).zeta_den) for k in range(12, 16)]
    assert z == [(1, 64), (1, 10), (2, 10), (3, 10)]
    with pytest.raises(ValueError):
        O.block_class_params(16)


def test_block_best_is_first_argmin():
    for x in blocks(7, 40):
        best, sizes = O.block_best(x)
        each = np.array([O.block_size(x, k) for k in range(O.NCLASS)])
        assert np.array_equal(sizes, each)
        assert best == int(np.flatnonzero(each == each.min())[0])
    # a block of zeros: every class ties at its least size, the rule keeps the first
    z = np.zeros(128, np.uint32)
    best, sizes = O.block_best(z)
    assert best == int(np.argmin(sizes))


def test_block_features_brute_force():
    for x in list(blocks(9, 30)) + [np.zeros(128, np.uint32), np.full(128, 0xFFFFFFFF, np.uint32)]:
        f = O.block_features(x)
        w = bit_width(x)
        W = int(w.max())
        tw = w.reshape(32, 4).max(axis=1)     # tuple widths
        assert f[0] == W / 32
        for b in range(33):
            assert f[1 + b] == np.count_nonzero(tw == b) / 32
        for t in range(1, 7):
            assert f[33 + t] == np.count_nonzero(w > W - t) / 128
        assert f[1:34].sum() == pytest.approx(1.0)


@pytest.mark.parametrize("n", [0, 1, 127, 128, 129, 1000, 128 * 37])
def test_blockmix_round_trip(n):
    rng = np.random.default_rng(n)
    x = blocks(n, max(1, (n + 127) // 128)).reshape(-1)[:n].copy()
    s, used = O.blockmix_encode(x)
    assert s[1] == n and s[2] == (n + 127) // 128
    assert np.array_equal(O.blockmix_decode(s), x)
    # the exhaustive container's size is the sum of the blocks' least sizes
    nb = (n + 127) // 128
    pad = np.zeros(nb * 128, np.uint32)
    pad[:n] = x
    sizes = [O.block_best(pad[b * 128:(b + 1) * 128])[1].min() for b in range(nb)]
    assert s.size == 4 + sum(sizes)
    # any fixed assignment decodes too
    if nb:
        k = rng.integers(0, O.NCLASS, nb).astype(np.uint8)
        s2, used2 = O.blockmix_encode(x, k)
        assert np.array_equal(used2, k)
        assert np.array_equal(O.blockmix_decode(s2), x)
        assert s2.size >= s.size


def test_blockmix_corpus_gain():
    """On the d-gap/TF corpus the exhaustive per-block choice is no larger
    than any single class for the whole corpus."""
    _, vals = synth.block_corpus(3, 128 * 300)
    s, used = O.blockmix_encode(vals)
    for k in range(O.NCLASS):
        sk, _ = O.blockmix_encode(vals, np.full(300, k, np.uint8))
        assert s.size <= sk.size
    assert len(np.unique(used)) > 1
