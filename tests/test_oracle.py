"""Pins for the CPU oracle: paper tables and worked examples, closed forms,
special cases that reduce to textbook routines, brute force on tiny inputs,
and round-trip identity.  CPU only."""
import itertools
import json
import os

import numpy as np
import pytest

import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def stream_bits(words, start_word, nbits):
    """Test-side LSB-first bit reader (independent of the oracle's)."""
    out = []
    for i in range(nbits):
        w = int(words[start_word + i // 32])
        out.append((w >> (i % 32)) & 1)
    return out


def areas(s):
    C, D = int(s[2]), int(s[3])
    return s[4:4 + C], s[4 + C:4 + C + D], s[4 + C + D:]


def from_tuples(tmax, k=4):
    """A list whose tuple t is (tmax[t], 0, ..., 0)."""
    x = np.zeros(len(tmax) * k, np.uint32)
    x[::k] = np.asarray(tmax, np.uint32)
    return x


# --------------------------------------------------------------------------
# Effective bit width and the quad max array.

def test_bw_matches_int_bit_length():
    rng = np.random.default_rng(11)
    edges = [0, 1, 2, 3, 4, 7, 8, 255, 256, (1 << 31) - 1, 1 << 31, (1 << 32) - 1]
    edges += [(1 << b) - 1 for b in range(33)] + [1 << b for b in range(32)]
    vals = edges + [int(v) for v in rng.integers(0, 1 << 32, 2000, dtype=np.uint64)]
    for v in vals:
        assert O.bw(v) == int(v).bit_length()


def test_pseudo_quad_max_has_quad_max_width():
    # Section 4.4: the OR of the four integers has the effective width of their max
    rng = np.random.default_rng(12)
    for _ in range(3000):
        q = rng.integers(0, 1 << 32, 4, dtype=np.uint64) >> rng.integers(0, 33, 4).astype(np.uint64)
        q = [int(v) & 0xFFFFFFFF for v in q]
        orv = q[0] | q[1] | q[2] | q[3]
        assert O.bw(orv) == O.bw(max(q))


def test_tuple_max_is_max_over_vertical_tuples():
    rng = np.random.default_rng(13)
    for k in (4, 8, 64):
        x = rng.integers(0, 1 << 32, 64 * k, dtype=np.uint64).astype(np.uint32)
        assert np.array_equal(O.tuple_max(x, k), x.reshape(-1, k).max(axis=1))


# --------------------------------------------------------------------------
# Group-Simple: Table III, Algorithm 1, the Fig. 3 example.

def test_table3_literal():
    g = gold("table3_group_simple.json")
    num, bwt = O.gsim_table()
    assert num == g["NUM"] and bwt == g["BW"]
    for n, b in zip(num, bwt):
        assert n * b <= 32                 # NUM integers of BW bits fill one component
        assert n == 32 // b                # and no more fit


def greedy_reference(widths):
    """Independent restatement of Algorithm 1's choice: the selector covering
    the most tuples (all of them fitting), ties to the narrowest width."""
    num, bwt = O.gsim_table()
    out, j, L = [], 0, len(widths)
    while j < L:
        best = None
        for i in range(10):
            cov = min(num[i], L - j)
            if all(w <= bwt[i] for w in widths[j:j + cov]):
                if cov == num[i] or cov == L - j:
                    if best is None or cov > best[0]:
                        best = (cov, i)
        out.append(best[1])
        j += best[0]
    return out


def test_algorithm1_matches_restatement():
    rng = np.random.default_rng(14)
    for trial in range(400):
        L = int(rng.integers(1, 120))
        w = rng.integers(0, 33, L) if trial % 2 else rng.integers(0, 9, L)
        q = np.array([(1 << int(b)) - 1 if b else 0 for b in w], np.uint64).astype(np.uint32)
        assert list(O.gsim_select(q)) == greedy_reference([int(b) for b in w])


def test_algorithm1_special_cases():
    assert list(O.gsim_select(np.zeros(64, np.uint32))) == [0, 0]        # all zero
    assert list(O.gsim_select(np.zeros(70, np.uint32))) == [0, 0, 0]     # partial tail
    assert list(O.gsim_select(np.array([0xFFFFFFFF], np.uint32))) == [9]
    assert list(O.gsim_select(np.array([1, 1, 1], np.uint32))) == [0]    # last selector partial
    assert list(O.gsim_select(np.zeros(0, np.uint32))) == []


def test_fig3_example_reading():
    # twenty integers (5 quadruples) whose widest needs 6 bits: selector 5, one vector
    g = gold("ld_examples.json")["group_simple_example"]
    x = np.array([63, 5, 17, 40, 1, 2, 3, 4, 9, 60, 33, 12, 0, 7, 8, 11, 63, 1, 2, 3], np.uint32)
    assert x.size == g["n"] and max(O.bw(v) for v in x) == g["max_bits"]
    s = O.encode(x, O.params(O.SIMPLE))
    ctrl, data, _ = areas(s)
    assert data.size == 4                              # one 128-bit vector
    assert int(ctrl[0]) & 0xF == g["selectors"][0]
    assert np.array_equal(O.decode(s), x)
    # the printed value 64 needs 7 bits: then selector 6 (4 quads of 8 bits) comes first
    x2 = x.copy()
    x2[0] = 64
    assert list(O.gsim_select(O.tuple_max(x2)))[0] == 6


def test_gsim_vector_layout():
    # tuple j of a selector occupies bits [j*BW, (j+1)*BW) of every component
    x = np.arange(1, 41, dtype=np.uint32)  # 10 quadruples, widths <= 6
    x[0] = 63
    s = O.encode(x, O.params(O.SIMPLE))
    ctrl, data, _ = areas(s)
    sel = int(ctrl[0]) & 0xF
    num, bwt = O.gsim_table()
    assert sel == 5 and num[sel] == 5
    for c in range(4):
        for j in range(5):
            assert (int(data[c]) >> (j * 6)) & 63 == x[4 * j + c]
            assert (int(data[4 + c]) >> (j * 6)) & 63 == x[20 + 4 * j + c]


def all_selector_sequences(widths, limit=20000):
    """Every valid Group-Simple selector sequence over the tuple widths
    (brute force; all selectors but the last are full)."""
    num, bwt = O.gsim_table()
    L = len(widths)
    out = []

    def rec(j, seq):
        if len(out) >= limit:
            return
        if j == L:
            out.append(list(seq))
            return
        for i in range(10):
            cov = min(num[i], L - j)
            if not all(w <= bwt[i] for w in widths[j:j + cov]):
                continue
            if cov < num[i] and j + cov != L:
                continue
            seq.append(i)
            rec(j + cov, seq)
            seq.pop()
    rec(0, [])
    return out


def test_gsim_bruteforce_min_and_every_sequence_decodes():
    rng = np.random.default_rng(15)
    gaps = []
    for trial in range(25):
        L = int(rng.integers(1, 9))
        w = [int(v) for v in rng.integers(0, 12, L)]
        tm = [(1 << b) - 1 if b else 0 for b in w]
        x = from_tuples(tm)
        x[1::4] = np.array(tm, np.uint32) >> 1
        seqs = all_selector_sequences(w)
        greedy = list(O.gsim_select(O.tuple_max(x)))
        assert greedy in seqs
        best = min(len(s) for s in seqs)
        assert len(greedy) >= best
        gaps.append(len(greedy) - best)
        p = O.params(O.SIMPLE)
        for seq in seqs[:: max(1, len(seqs) // 40)]:
            s = O.gsim_encode_with(x, seq, p)
            assert np.array_equal(O.decode(s), x)
    assert max(gaps) <= 2   # greedy is near the minimum on these inputs


def test_gsim_rejects_selector_that_does_not_fit():
    x = from_tuples([255, 1])
    with pytest.raises(ValueError):
        O.gsim_encode_with(x, [0], O.params(O.SIMPLE))


# --------------------------------------------------------------------------
# Group-Scheme: Table IV, eq. (1)-(2), the worked examples.

def test_table4_and_eq1_eq2():
    g = gold("table4_group_scheme.json")
    for cg, ldbits, (lo, hi) in zip(g["CG"], g["binary_ld_bits"], g["unary_range"]):
        assert ldbits == 5 - int(np.log2(cg))
        # unary range: widths 0..32 map to units lo..hi, and BW = CG * units
        units = sorted({O.gsc_units((1 << w) - 1 if w else 0, cg) for w in range(33)})
        assert units[0] == lo and units[-1] == hi and units == list(range(lo, hi + 1))
        for w in range(1, 33):
            u = O.gsc_units((1 << w) - 1, cg)
            assert cg * u >= w and cg * (u - 1) < w     # eq. (2) covers the width tightly
            assert hi - 1 < 2 ** ldbits <= 2 * hi        # binary field holds u - 1


def test_ld_of_458():
    e = gold("ld_examples.json")["length_descriptor_458"]
    assert O.gsc_units(e["value"], e["cg"]) == e["units"]
    x = from_tuples([e["value"]])
    s = O.encode(x, O.params(O.SCHEME, cg=2, ld=O.LD_CU))
    ctrl, data, _ = areas(s)
    bits = "".join(str(b) for b in stream_bits(ctrl, 0, 5))
    assert bits == e["unary_code_stream_order"]
    assert all(stream_bits(ctrl, 0, 32)[5:])           # rest of the area is 1s
    assert int(data[0]) == 458 and data.size == 4       # 10 bits in component 0
    # binary descriptor at 2-bit CG stores units - 1 in 4 bits
    s = O.encode(x, O.params(O.SCHEME, cg=2, ld=O.LD_BINARY))
    ctrl, _, _ = areas(s)
    assert int(ctrl[0]) & 0xF == e["units"] - 1


def _byte_str(word, byte_index):
    return "".join(str((int(word) >> (8 * byte_index + i)) & 1) for i in range(8))


def test_packed_unary_byte_example_cu_and_iu():
    e = gold("ld_examples.json")["packed_unary_byte"]
    # tuples with 8-bit CG units 2, 3, 1 then a 3-unit tuple whose code does not fit
    tm = [300, 70000, 5, 70000]
    assert [O.gsc_units(v, 8) for v in tm] == [2, 3, 1, 3]
    x = from_tuples(tm)
    # complete unary: the carried "11" completes in the next byte with its "0"
    s = O.encode(x, O.params(O.SCHEME, cg=8, ld=O.LD_CU))
    ctrl, _, _ = areas(s)
    assert _byte_str(ctrl[0], 0) == e["byte_stream_order"]
    assert _byte_str(ctrl[0], 1)[0] == "0"
    assert np.array_equal(O.decode(s), x)
    # incomplete unary: the same first byte, its trailing "11" is padding and
    # the 3-unit code restarts at the next byte
    s = O.encode(x, O.params(O.SCHEME, cg=8, ld=O.LD_IU))
    ctrl, _, _ = areas(s)
    assert _byte_str(ctrl[0], 0) == e["byte_stream_order"]
    assert _byte_str(ctrl[0], 1)[:3] == "110"
    assert np.array_equal(O.decode(s), x)


def test_unary_parse_of_example_byte():
    # test-side parse of the printed byte: complete codes and the carried run
    e = gold("ld_examples.json")["packed_unary_byte"]
    lds, run = [], 0
    for ch in e["byte_stream_order"]:
        if ch == "1":
            run += 1
        else:
            lds.append(run + 1)
            run = 0
    assert lds == e["complete_descriptors"] and run == e["carried_ones"]


def test_gsc_1cu_is_k_gamma():
    # 1-CU is k-Gamma (Section 5.1, k = 4): unary code of the tuple width b,
    # then b bits per integer (an all-zero tuple still takes one unit)
    rng = np.random.default_rng(16)
    x = (rng.integers(0, 1 << 20, 400, dtype=np.uint64) >> rng.integers(0, 21, 400).astype(np.uint64)).astype(np.uint32)
    s = O.encode(x, O.params(O.SCHEME, cg=1, ld=O.LD_CU))
    ctrl, data, _ = areas(s)
    W = [max(1, int(v).bit_length()) for v in O.tuple_max(x)]
    bits = stream_bits(ctrl, 0, sum(W))
    pos = 0
    for w in W:
        assert bits[pos:pos + w] == [1] * (w - 1) + [0]
        pos += w
    assert data.size == 4 * ((sum(W) + 31) // 32)


def test_binary_ld_packing_units():
    e = gold("ld_examples.json")["binary_ld_packing"]
    for cg in (1, 2, 4, 8):
        ints = e["ints_per_pattern"][str(cg)]
        pbits = e["pattern_bits"][str(cg)]
        ntup = 3 * ints // 4
        x = from_tuples([1] * ntup)
        s = O.encode(x, O.params(O.SCHEME, cg=cg, ld=O.LD_BINARY))
        # three patterns' worth of tuples use exactly three pattern units
        used = 3 * pbits
        assert int(s[2]) == ((used + 31) // 32 + 3) // 4 * 4
        fields = ints // 4
        assert fields * (5 - int(np.log2(cg))) <= e["lut_index_bits"][str(cg)]


def test_gsc_size_closed_form_and_bounds():
    rng = np.random.default_rng(17)
    x = rng.geometric(0.05, 4000).astype(np.uint32)
    tm = O.tuple_max(x)
    for cg in (1, 2, 4, 8):
        for ld in (O.LD_BINARY, O.LD_CU, O.LD_IU):
            if ld == O.LD_IU and cg < 4:
                continue
            s = O.encode(x, O.params(O.SCHEME, cg=cg, ld=ld))
            units = np.array([O.gsc_units(int(v), cg) for v in tm])
            assert int(s[3]) == 4 * ((int((cg * units).sum()) + 31) // 32)
            bpi = 32.0 * (int(s[2]) + int(s[3])) / x.size
            floor = cg + (1.0 / 4 if ld != O.LD_BINARY else (5 - np.log2(cg)) / 4)
            assert bpi >= floor - 1e-9


# --------------------------------------------------------------------------
# Group-AFOR: optimal partition by dynamic programming.

def afor_cost(tm, frames, k=4):
    bits, j = 0, 0
    for F in frames:
        b = max(int(v).bit_length() for v in tm[j:j + F])
        bits += 8 + k * F * b
        j += F
    return bits


def partitions(m):
    if m == 0:
        yield []
        return
    for F in (8, 16, 32):
        if F <= m:
            for rest in partitions(m - F):
                yield [F] + rest


def test_afor_dp_is_bruteforce_minimum():
    rng = np.random.default_rng(18)
    for trial in range(40):
        m = 8 * int(rng.integers(1, 13))
        w = rng.integers(0, 20, m) if trial % 2 else np.repeat(rng.integers(0, 20, m // 8), 8)
        tm = np.array([(1 << int(b)) - 1 if b else 0 for b in w], np.uint32)
        dp = O.afor_partition(tm)
        best = min(afor_cost(tm, p) for p in partitions(m))
        assert afor_cost(tm, dp) == best
        # canonical tie-break: at each step no larger first frame reaches the optimum
        j = 0
        for F in dp:
            for G in (32, 16):
                if G > F and j + G <= m:
                    rest = min(afor_cost(tm[j + G:], p) for p in partitions(m - j - G))
                    head = afor_cost(tm[j:j + G], [G])
                    assert head + rest > afor_cost(tm[j:], O.afor_partition(tm[j:]))
            j += F


def test_afor_every_partition_decodes():
    rng = np.random.default_rng(19)
    x = rng.geometric(0.1, 4 * 48).astype(np.uint32)
    p = O.params(O.AFOR)
    for part in partitions(48):
        s = O.afor_encode_with(x, part, p)
        assert np.array_equal(O.decode(s), x)
        assert int(s[3]) == 4 * ((sum(F * max(int(v).bit_length() for v in O.tuple_max(x)[j:j + F])
                                      for j, F in zip(np.cumsum([0] + part[:-1]), part)) + 31) // 32)


def test_afor_control_byte():
    x = from_tuples([3] * 32 + [1000] * 8)
    s = O.encode(x, O.params(O.AFOR))
    ctrl, _, _ = areas(s)
    b0, b1 = int(ctrl[0]) & 0xFF, (int(ctrl[0]) >> 8) & 0xFF
    assert (b0 & 63, b0 >> 6) == (2, 2)       # 32-tuple frame of width 2
    assert (b1 & 63, b1 >> 6) == (10, 0)      # 8-tuple frame of width 10


# --------------------------------------------------------------------------
# Group-VSEncoding: VSEncoding's frame lengths that fit a group frame (8, 12,
# 16 and 32 tuples), Group-AFOR's control byte with class 3 = 12 tuples.

def vse_partitions(m):
    if m == 0:
        yield []
        return
    for F in (8, 12, 16, 32):
        if F <= m:
            for rest in vse_partitions(m - F):
                yield [F] + rest


def test_vse_dp_is_bruteforce_minimum():
    rng = np.random.default_rng(28)
    for trial in range(40):
        m = 8 * int(rng.integers(1, 9))
        w = rng.integers(0, 20, m) if trial % 2 else np.repeat(rng.integers(0, 20, m // 4), 4)
        tm = np.array([(1 << int(b)) - 1 if b else 0 for b in w], np.uint32)
        dp = O.vse_partition(tm)
        assert sum(dp) == m and all(F in (8, 12, 16, 32) for F in dp)
        best = min(afor_cost(tm, p) for p in vse_partitions(m))
        assert afor_cost(tm, dp) == best
        # no worse than Group-AFOR, whose frame set it contains
        assert best <= afor_cost(tm, O.afor_partition(tm))
        # ties go to the larger first frame
        j = 0
        for F in dp:
            for G in (32, 16, 12):
                if G > F and j + G <= m:
                    rest = [afor_cost(tm[j + G:], p) for p in vse_partitions(m - j - G)]
                    if rest:
                        head = afor_cost(tm[j:j + G], [G])
                        assert head + min(rest) > afor_cost(tm[j:], O.vse_partition(tm[j:]))
            j += F


def test_vse_every_partition_decodes():
    rng = np.random.default_rng(29)
    x = rng.geometric(0.1, 4 * 48).astype(np.uint32)
    p = O.params(O.VSE)
    n = 0
    for part in vse_partitions(48):
        s = O.afor_encode_with(x, part, p)
        assert np.array_equal(O.decode(s), x)
        n += 1
    assert n == 41                                      # compositions of 48 into 8, 12, 16, 32
    with pytest.raises(ValueError):                    # no 12-tuple frame in Group-AFOR
        O.afor_encode_with(x, [12, 12, 8, 16], O.params(O.AFOR))


def test_vse_control_byte():
    # 12 tuples of width 2 then 12 of width 10: two 12-tuple frames cost
    # 16 + 4*12*2 + 4*12*10 = 592 bits; the best frames of 8/16/32 (8 then
    # 16) cost 16 + 4*8*2 + 4*16*10 = 720
    x = from_tuples([3] * 12 + [1000] * 12)
    s = O.encode(x, O.params(O.VSE))
    ctrl, _, _ = areas(s)
    b0, b1 = int(ctrl[0]) & 0xFF, (int(ctrl[0]) >> 8) & 0xFF
    assert (b0 & 63, b0 >> 6) == (2, 3)
    assert (b1 & 63, b1 >> 6) == (10, 3)
    assert int(s[3]) == 4 * ((12 * 2 + 12 * 10 + 31) // 32)
    assert (int(s[0]) >> 8) & 15 == 4
    a = O.encode(x, O.params(O.AFOR))
    assert O.afor_partition(O.tuple_max(x)) == [8, 16]
    assert int(a[3]) == 4 * ((8 * 2 + 16 * 10 + 31) // 32)
    assert np.array_equal(O.decode(s), x) and np.array_equal(O.decode(a), x)
    # the same byte in a Group-AFOR stream is corrupt
    bad = a.copy()
    bad[4] = int(bad[4]) | 0xC0
    assert O.decode_status(bad) == O.ECORRUPT


@pytest.mark.parametrize("k", [4, 8, 16, 32, 64])
def test_vse_roundtrip_sizes(k):
    rng = np.random.default_rng(30 + k)
    for n in (1, 7, k * 12, k * 12 + 1, 3000):
        d = np.cumsum(rng.geometric(0.05, n)).astype(np.uint32)
        s = O.encode(d, O.params(O.VSE, k=k, delta=True))
        assert np.array_equal(O.decode(s), d)
        sa = O.encode(d, O.params(O.AFOR, k=k, delta=True))
        assert s.size <= sa.size + 4                    # control padding aside


# --------------------------------------------------------------------------
# Group-PFD.

def parse_pfd_descriptors(s):
    ctrl, data, exc = areas(s)
    out = []
    for wd in ctrl:
        wd = int(wd)
        out.append(dict(b=wd & 63, wcode=(wd >> 6) & 3, first=(wd >> 8) & 0xFFF, nexc=wd >> 20))
    return out


@pytest.mark.parametrize("zeta", [(1, 10), (2, 10), (3, 10)])
def test_pfd_width_minimal_and_exception_bound(zeta):
    rng = np.random.default_rng(20)
    x = rng.geometric(0.2, 128 * 40).astype(np.uint32)
    spikes = rng.integers(0, x.size, 150)
    x[spikes] = rng.integers(1 << 12, 1 << 30, spikes.size).astype(np.uint32)
    s = O.encode(x, O.params(O.PFD, zeta=zeta))
    desc = parse_pfd_descriptors(s)
    for blk in range(40):
        tm = O.tuple_max(x[128 * blk:128 * (blk + 1)])
        W = np.array([int(v).bit_length() for v in tm])
        b = desc[blk]["b"]
        ratio = lambda bb: (W > bb).sum() / 32.0
        assert ratio(b) < zeta[0] / zeta[1]
        assert b == 0 or ratio(b - 1) >= zeta[0] / zeta[1]
        assert (W > b).sum() <= int(np.ceil(32 * zeta[0] / zeta[1])) - 1
        xb = x[128 * blk:128 * (blk + 1)]
        ex = [int(v).bit_length() for v in xb if int(v).bit_length() > b]
        if ex:
            need = max(ex)
            w = 4 << desc[blk]["wcode"]
            assert w >= need and (w == 8 or w // 2 < need)


def test_pfd_zeta_below_1_32_is_bp128():
    # no exception allowed: one b per 128 integers, the widest of the block
    rng = np.random.default_rng(21)
    x = rng.geometric(0.05, 128 * 16).astype(np.uint32)
    x[77] = 1 << 25
    s = O.encode(x, O.params(O.PFD, zeta=(1, 32)))
    desc = parse_pfd_descriptors(s)
    _, data, _ = areas(s)
    for blk, d in enumerate(desc[:16]):
        assert d["nexc"] == 0
        assert d["b"] == max(int(v).bit_length() for v in x[128 * blk:128 * (blk + 1)])
    assert data.size == 4 * sum(d["b"] for d in desc[:16])    # 128*b bits per block
    assert np.array_equal(O.decode(s), x)


def test_pfd_linked_and_bitmap_agree_and_chain_is_consistent():
    rng = np.random.default_rng(22)
    for k in (4, 8):
        x = rng.geometric(0.3, 32 * k * 12).astype(np.uint32)
        idx = rng.integers(0, x.size, 40)
        x[idx] = rng.integers(1 << 10, 1 << 31, idx.size).astype(np.uint32)
        sl = O.encode(x, O.params(O.PFD, k=k, pfd_pos=O.PFD_LINKED))
        sb = O.encode(x, O.params(O.PFD, k=k, pfd_pos=O.PFD_BITMAP))
        assert np.array_equal(O.decode(sl), x) and np.array_equal(O.decode(sb), x)
        dl, db = parse_pfd_descriptors(sl), parse_pfd_descriptors(sb)
        for a, b in zip(dl, db):
            assert a["b"] == b["b"] and a["nexc"] >= b["nexc"]   # linked adds compulsory ones


def test_pfd_compulsory_exceptions_when_b_is_small():
    # two exceptions 100 apart with b = 1: the chain needs compulsory stops
    x = np.ones(128, np.uint32)
    x[3] = 1 << 20
    x[103] = 1 << 20
    s = O.encode(x, O.params(O.PFD))
    d = parse_pfd_descriptors(s)[0]
    assert d["b"] == 1 and d["first"] == 3
    assert d["nexc"] == 2 + 99 // 2          # a stop every 2 positions
    assert np.array_equal(O.decode(s), x)


# --------------------------------------------------------------------------
# d-gaps and the prefix sum.

def test_prefix_sum_is_wrapping_cumsum_and_inverts_dgap():
    rng = np.random.default_rng(23)
    g = rng.integers(0, 1 << 32, 5000, dtype=np.uint64).astype(np.uint32)
    ref = (np.cumsum(g.astype(np.uint64)) & 0xFFFFFFFF).astype(np.uint32)
    assert np.array_equal(O.prefix_sum(g), ref)
    assert np.array_equal(O.dgap(O.prefix_sum(g)), g)
    d = np.sort(rng.choice(1 << 30, 3000, replace=False)).astype(np.uint32)
    assert np.array_equal(O.dgap(d), np.diff(d, prepend=np.uint32(0)))


# --------------------------------------------------------------------------
# Round trip over every codec, variant and layout width.

CODECS = [
    (O.SIMPLE, {}), (O.SCHEME, dict(cg=1, ld=O.LD_CU)), (O.SCHEME, dict(cg=2, ld=O.LD_CU)),
    (O.SCHEME, dict(cg=4, ld=O.LD_CU)), (O.SCHEME, dict(cg=8, ld=O.LD_CU)),
    (O.SCHEME, dict(cg=4, ld=O.LD_IU)), (O.SCHEME, dict(cg=8, ld=O.LD_IU)),
    (O.SCHEME, dict(cg=1, ld=O.LD_BINARY)), (O.SCHEME, dict(cg=2, ld=O.LD_BINARY)),
    (O.SCHEME, dict(cg=4, ld=O.LD_BINARY)), (O.SCHEME, dict(cg=8, ld=O.LD_BINARY)),
    (O.AFOR, {}), (O.PFD, {}), (O.PFD, dict(pfd_pos=O.PFD_BITMAP)),
]


@pytest.mark.parametrize("k", [4, 16, 64])
@pytest.mark.parametrize("ci", range(len(CODECS)))
def test_roundtrip(ci, k):
    codec, kw = CODECS[ci]
    rng = np.random.default_rng(100 + ci)
    for n in (0, 1, 3, 4, 5, 127, 128, 129, 1031):
        d = np.sort(rng.choice(1 << 26, n, replace=False)).astype(np.uint32)
        s = O.encode(d, O.params(codec, k=k, delta=True, **kw))
        assert np.array_equal(O.decode(s), d)
    for x in (np.zeros(700, np.uint32), np.full(700, 0xFFFFFFFF, np.uint32),
              (rng.integers(0, 1 << 32, 3000, dtype=np.uint64)
               >> rng.integers(0, 33, 3000).astype(np.uint64)).astype(np.uint32)):
        s = O.encode(x, O.params(codec, k=k, **kw))
        assert np.array_equal(O.decode(s), x)


def test_header_fields():
    s = O.encode(np.arange(10, dtype=np.uint32), O.params(O.SCHEME, k=16, cg=8, ld=O.LD_IU,
                                                          delta=True))
    p = O.parse_header(int(s[0]))
    assert (p.codec, p.k, p.cg, p.ld, p.delta) == (O.SCHEME, 16, 8, O.LD_IU, 1)
    assert int(s[1]) == 10 and int(s[2]) % 4 == 0 and int(s[3]) % 16 == 0
    assert O.parse_header(int(s[0]) | (1 << 25)) is None
    # codec 4 (Group-VSEncoding) is the last codec; 5 .. 15 are not streams
    v = O.encode(np.arange(10, dtype=np.uint32), O.params(O.VSE, k=8))
    assert O.parse_header(int(v[0])).codec == O.VSE
    for c in range(5, 16):
        assert O.parse_header((int(v[0]) & ~(15 << 8)) | (c << 8)) is None


# --------------------------------------------------------------------------
# Corrupted streams are rejected.

def test_corrupt_streams_are_rejected():
    rng = np.random.default_rng(24)
    x = rng.geometric(0.1, 2000).astype(np.uint32)
    s = O.encode(x, O.params(O.SIMPLE))
    bad = s.copy()
    bad[4] = (int(bad[4]) & ~0xF) | 12                # selector 12 does not exist
    assert O.decode_status(bad) == O.ECORRUPT
    assert O.decode_status(s[:-4]) == O.ECORRUPT      # truncated data
    s = O.encode(x, O.params(O.AFOR))
    bad = s.copy()
    bad[4] = int(bad[4]) | 0xC0                       # frame class 3
    assert O.decode_status(bad) == O.ECORRUPT
    s = O.encode(x, O.params(O.PFD))
    bad = s.copy()
    bad[4] = (int(bad[4]) & ~63) | 40                 # b = 40
    assert O.decode_status(bad) == O.ECORRUPT
    s = O.encode(x, O.params(O.SCHEME, cg=1, ld=O.LD_CU))
    bad = s.copy()
    bad[4] = 0xFFFFFFFF                               # a 33-unit code
    assert O.decode_status(bad) == O.ECORRUPT


def test_straddling_value_keeps_low_part_in_earlier_word():
    # Section 5.3.2 (unary step 2): the carried partial value is the low part,
    # completed by the next vector's bits shifted left by the carried count
    v = (1 << 20) - 3
    x = np.array([v, v - 1, v - 2, v - 3, v, v ^ 5, v ^ 9, v ^ 17], np.uint32)
    s = O.encode(x, O.params(O.SCHEME, cg=1, ld=O.LD_CU))
    _, data, _ = areas(s)
    for c in range(4):
        y = int(x[4 + c])
        assert int(data[c]) & 0xFFFFF == int(x[c])
        assert int(data[c]) >> 20 == y & 0xFFF
        assert int(data[4 + c]) & 0xFF == y >> 12
