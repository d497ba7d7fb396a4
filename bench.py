#!/usr/bin/env python3
"""Throughput of batched Group-codec decoding + d-gap prefix sum on one MI355X.

Headline workload (cfg3): 100,000 synthetic posting lists with lognormal
lengths (median 1,024, about 2^28 docIDs, universe 2^25, 70% sparse / 30%
clustered d-gaps), each coded with one of Group-Simple, Group-Scheme 1-CU,
Group-Scheme 8-IU, Group-AFOR and Group-PFD (32-tuple blocks, zeta = 1/10) in
the paper's 4-way layout.  One step decodes every list and prefix-sums it to
docIDs: the locate kernels, then per codec class the tile-sum pass, the carry
scan and the decode pass, all captured in one hipGraph (autotuned tile
sizes); `value` times the graph replays.  A second plan with the same tiles
launches the kernels directly with HIP events between the phases; it gives the
per-phase times and the dominant kernel's average duration.

Legs (each verified bit-exact against the generated lists): the same lists
decoded with one launch sequence per list, directly and replayed from a
hipGraph; the cfg2 batch (10,000 Zipf-length docID lists and their TF lists in
five codecs); the four cfg5 batches (1,000,000 lists, median 256, heavy-tailed
gaps; Group-PFD and Group-AFOR in the 4-way and 64-way layouts); every
Group-Scheme variant and BP128 beside the other codecs on cfg2; encode speed
on cfg2, GPU list encoders against the host encoder (streams checked equal);
AND queries with BM25 top-10 over the cfg2 index (decode + query per batch);
the single-list latency of cfg1.  `--workload NAME` measures one workload
alone (for profiler runs).

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gints/s decoded+prefix-summed, % HBM peak; batched vs per-list on 1 MI355X"
HBM_PEAK_GBS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")
# the sources the decode kernels are compiled from
DECODE_SRCS = [os.path.join(ROOT, "paper_1502_01916_amd", "csrc", f)
               for f in ("decode.hip", "gc_wave.h", "gc_device.h", "gc_format.h")]
CLASS_NAMES = ["group-simple", "group-scheme-unary", "group-scheme-binary", "group-afor", "group-pfd"]


def decode_sources_sha256():
    h = hashlib.sha256()
    for path in DECODE_SRCS:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def traffic_file(workload):
    return os.path.join(PROFILES, "traffic_decode_%s.txt" % workload)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def five_codecs(gc):
    """The five codecs of the cfg2 and cfg3 batches."""
    return [("group-simple", gc.SIMPLE, {}),
            ("group-scheme-1cu", gc.SCHEME, dict(cg=1, ld=gc.LD_CU)),
            ("group-scheme-8iu", gc.SCHEME, dict(cg=8, ld=gc.LD_IU)),
            ("group-afor", gc.AFOR, {}),
            ("group-pfd", gc.PFD, dict(zeta=(1, 10)))]


def all_variants(gc):
    """Every codec variant of Sections 4-6 in the 4-way layout: Group-Simple,
    the ten Group-Scheme variants (Section 5.2), Group-AFOR, Group-PFD at
    zeta = 1/10, BP128 (Group-PFD below zeta = 1/32, Section 6.3) and
    Group-VSEncoding (Group-AFOR's stream with 12-tuple frames as well)."""
    v = [("group-simple", gc.SIMPLE, {})]
    for cg in (1, 2, 4, 8):
        v.append(("gsc-%d-b" % cg, gc.SCHEME, dict(cg=cg, ld=gc.LD_BINARY)))
    for cg in (1, 2, 4, 8):
        v.append(("gsc-%d-cu" % cg, gc.SCHEME, dict(cg=cg, ld=gc.LD_CU)))
    for cg in (4, 8):
        v.append(("gsc-%d-iu" % cg, gc.SCHEME, dict(cg=cg, ld=gc.LD_IU)))
    v += [("group-afor", gc.AFOR, {}), ("group-pfd", gc.PFD, dict(zeta=(1, 10))),
          ("bp128", gc.PFD, dict(zeta=(1, 32))), ("group-vse", gc.VSE, {})]
    return v


CFG5_BATCHES = {
    "cfg5-pfd-k4": ("PFD", dict(k=4)),
    "cfg5-afor-k4": ("AFOR", dict(k=4)),
    "cfg5-pfd-k64": ("PFD", dict(k=64, pfd_pos=1)),
    "cfg5-afor-k64": ("AFOR", dict(k=64)),
}
WORKLOADS = ["cfg3", "cfg2"] + list(CFG5_BATCHES)


def kernel_name(cls, tile, carry_pass):
    """The decode kernel of a codec class as the profiler names it: tile size,
    class, and mode 2 (look-back carries) unless every carry comes from the
    tile-sum pass (mode 0)."""
    return "gc_wave_kernel<%d, %d, %d>" % (tile, cls, 0 if carry_pass == 2 else 2)


def pack_kernel_name(pack_ints):
    """The pack kernel a plan with this packed-list threshold launches."""
    return "gc_pack_kernel<2048, 512>" if pack_ints <= 2048 else "gc_pack_kernel<4096, 1024>"


def codec_class(gc, codec, kw):
    if codec == gc.SIMPLE:
        return 0
    if codec == gc.SCHEME:
        return 2 if kw.get("ld", gc.LD_CU) == gc.LD_BINARY else 1
    return 3 if codec in (gc.AFOR, gc.VSE) else 4


class Workload:
    """Streams of a batch (concatenated), the lists they decode to, and the
    codec class of every list."""

    def __init__(self, name, desc, streams, offs, lengths, cls, want):
        self.name, self.desc = name, desc
        self.streams, self.offs, self.lengths = streams, offs, lengths
        self.cls, self.want = cls, want
        self.ints = int(lengths.sum())

    def class_bytes(self, c, packed=None):
        """Algorithmic bytes of one decode pass of class c: its streams read
        once, its integers written once (lists the pack kernel decodes
        excluded)."""
        m = self.cls == c
        if packed is not None:
            m = m & ~packed
        return self.bytes_of(m)

    def bytes_of(self, m):
        words = int(np.sum((self.offs[1:] - self.offs[:-1])[m]))
        return 4 * words + 4 * int(self.lengths[m].sum())

    def path_bytes(self):
        return 4 * int(self.streams.size) + 4 * self.ints


def concat_parts(parts):
    streams = np.concatenate([p[0] for p in parts])
    offs, base = [np.zeros(1, np.int64)], 0
    for s, o in parts:
        o = o.astype(np.int64)
        offs.append(o[1:] + base)
        base += int(o[-1])
    return streams, np.concatenate(offs)


def build_cfg3(gc, synth):
    t = time.time()
    lengths, docs, cidx = synth.cfg3()
    codecs = five_codecs(gc)
    cod = np.array([codecs[c][1] for c in cidx], np.int32)
    plist = [gc.params(delta=True, **codecs[c][2]) for c in cidx]
    s, offs = gc.encode_lists(docs, lengths, cod, plist)
    cls = np.array([codec_class(gc, codecs[c][1], codecs[c][2]) for c in cidx], np.int32)
    log("cfg3: %d lists, %d docIDs, %.2f bits/int (%.1fs)" % (lengths.size, docs.size, 32.0 * s.size / docs.size,
                                                             time.time() - t))
    desc = ("100,000 posting lists, lognormal lengths (median 1,024, max 2^22), 2.68e8 docIDs, universe 2^25, "
            "70% sparse / 30% clustered d-gaps; each list in one of Group-Simple, Group-Scheme 1-CU, "
            "Group-Scheme 8-IU, Group-AFOR, Group-PFD (zeta 1/10), 4-way layout; all lists decoded and "
            "prefix-summed per step; seed 3")
    return Workload("cfg3", desc, s, offs.astype(np.int64), lengths, cls, docs)


def build_cfg2(gc, synth, variants=None):
    t = time.time()
    lengths, docs, tfs = synth.cfg2()
    parts, cls, want = [], [], []
    for name, codec, kw in (variants or five_codecs(gc)):
        for flat, delta in ((docs, True), (tfs, False)):
            s, offs = gc.encode_lists(flat, lengths, codec, gc.params(delta=delta, **kw))
            parts.append((s, offs))
            cls.append(np.full(lengths.size, codec_class(gc, codec, kw), np.int32))
            want.append(flat)
    s, offs = concat_parts(parts)
    L = np.tile(lengths, len(parts))
    log("cfg2: %d streams, %d integers, %.2f bits/int (%.1fs)" % (L.size, int(L.sum()), 32.0 * s.size / L.sum(),
                                                                 time.time() - t))
    desc = ("10,000 posting lists (Zipf lengths in [128, 2^22], 2^26 docIDs, universe 2^25, 70% sparse / 30% "
            "clustered d-gaps) plus their TF lists (geometric p=0.4), each coded with Group-Simple, Group-Scheme "
            "1-CU, Group-Scheme 8-IU, Group-AFOR and Group-PFD (zeta 1/10), 4-way layout; all 100,000 streams "
            "decoded per step, docID lists prefix-summed; seed 2")
    return Workload("cfg2", desc, s, offs, L, np.concatenate(cls), np.concatenate(want)), (lengths, docs, tfs)


_CFG5 = None


def build_cfg5(gc, synth, name, spec=None):
    """The cfg5 lists in the format of CFG5_BATCHES[name], or of `spec`
    (codec name, params) under that name."""
    global _CFG5
    t = time.time()
    if _CFG5 is None:
        _CFG5 = synth.cfg5()
    lengths, docs = _CFG5
    codec_name, kw = spec if spec else CFG5_BATCHES[name]
    codec = getattr(gc, codec_name)
    s, offs = gc.encode_lists(docs, lengths, codec, gc.params(delta=True, **kw))
    log("%s: %d lists, %d docIDs, %.2f bits/int (%.1fs)" % (name, lengths.size, docs.size,
                                                           32.0 * s.size / docs.size, time.time() - t))
    desc = ("1,000,000 posting lists, lognormal lengths (median 256, max 2^22), 5.37e8 docIDs, Pareto(1.2) "
            "d-gaps with 20%% dense runs of gap 1; Group-%s, %d-way layout%s; all lists decoded and "
            "prefix-summed per step; seed 6"
            % ("PFD (zeta 1/10)" if codec_name == "PFD" else "AFOR", kw["k"],
               ", bitmap exceptions" if kw.get("pfd_pos") else ""))
    cls = np.full(lengths.size, codec_class(gc, codec, kw), np.int32)
    return Workload(name, desc, s, offs.astype(np.int64), lengths, cls, docs)


def read_traffic(workload, units, kernel, alg_bytes):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary of `workload`: one block per plan profiled (blocks begin with a
    `kernel:` line), the one taken on the current decode kernel source, this
    workload, this kernel and a plan that gives the kernel the same
    algorithmic bytes per launch."""
    path = traffic_file(workload)
    if not os.path.exists(path):
        return None
    blocks, kv = [], None
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                if k.strip() == "kernel":
                    kv = {}
                    blocks.append(kv)
                if kv is not None:
                    kv[k.strip()] = v.strip()
    for kv in blocks:
        if (kv.get("decode_sources_sha256") == decode_sources_sha256() and kv.get("workload_units") == str(units)
                and kv.get("kernel") == kernel and kv.get("algorithmic_bytes_per_launch") == str(int(alg_bytes))):
            try:
                return float(kv["hbm_bytes_per_launch"])
            except (KeyError, ValueError):
                return None
    return None


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_threads():
    """Worker processes for the CPU baseline: the cores this process may use,
    at most 16 (the host share of one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


_CPU_WL = None


def _cpu_worker(args):
    """Decodes lists order[k], order[k + stride], ... with the C oracle for
    about `seconds`; returns (lists, integers, seconds)."""
    import oracle as O
    order, k, stride, seconds = args
    wl = _CPU_WL
    done_i = done_l = 0
    t0 = time.perf_counter()
    for idx in range(k, len(order), stride):
        li = order[idx]
        done_i += O.decode(wl.streams[int(wl.offs[li]):int(wl.offs[li + 1])]).size
        done_l += 1
        if time.perf_counter() - t0 > seconds:
            break
    return done_l, done_i, time.perf_counter() - t0


def cpu_baseline(wl, seconds):
    """The plain C oracle decoding (and prefix-summing) a random sample of the
    workload's streams: first in this process, then in one forked worker
    process per host core (lists dealt round-robin), each for about
    `seconds` seconds."""
    global _CPU_WL
    import multiprocessing as mp
    _CPU_WL = wl
    order = np.random.default_rng(123).permutation(wl.lengths.size)
    one = _cpu_worker((order, 0, 1, seconds))
    nt = cpu_threads()
    with mp.get_context("fork").Pool(nt) as pool:
        res = pool.map(_cpu_worker, [(order, k, nt, seconds) for k in range(nt)])
    wall = max(r[2] for r in res)    # the slowest worker's decode time (pool start-up excluded)
    lists = sum(r[0] for r in res)
    ints = sum(r[1] for r in res)
    return dict(value=round(ints / wall / 1e9, 4), unit="Gints/s", cores=nt, kind="oracle",
                per_core_value=round(one[1] / one[2] / 1e9, 4),
                hardware_concurrency=os.cpu_count(), cpu_model=cpu_model(),
                sample="lists of the %s workload drawn at random, each decoded and prefix-summed by the plain C "
                       "oracle: %d lists (%d integers) on %d worker processes, the slowest busy %.2f s; in one "
                       "process: %d lists (%d integers) in %.2f s"
                       % (wl.name, lists, ints, nt, wall, one[0], one[1], one[2]))


def cfg1_latency(gc, synth, ctx, torch, reps=30):
    """One list of 2^20 docIDs (mean gap 16) in Group-Simple, decoded and
    prefix-summed by gc_decode: the single-list latency, timed with HIP events
    around each call."""
    docs = synth.cfg1()
    s = gc.encode(docs, gc.SIMPLE, gc.params(delta=True))
    d_s = gc.to_device(s)
    d_o = torch.empty(docs.size, dtype=torch.int32, device="cuda")
    for _ in range(3):
        ctx.decode(d_s, s.size, s[:4], d_o)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for e0, e1 in ev:
        e0.record()
        ctx.decode(d_s, s.size, s[:4], d_o)
        e1.record()
    torch.cuda.synchronize()
    us = sorted(1e3 * e0.elapsed_time(e1) for e0, e1 in ev)
    rc, det = ctx.sync_status()
    ok = rc == gc.OK and np.array_equal(gc.to_host(d_o), docs)
    med = us[len(us) // 2]
    return dict(ints=int(docs.size), bits_per_int=round(32.0 * s.size / docs.size, 3), median_us=round(med, 2),
                min_us=round(us[0], 2), gints_s=round(docs.size / med / 1e3, 2), verified_bit_exact=bool(ok))


def timed(run, steps, warmup, torch):
    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        run()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


class Measured:
    pass


def pack_option(gc, v):
    """--pack-ints: 'auto' (0, autotuned), 'off' or a threshold."""
    return 0 if v == "auto" else gc.PACK_OFF if v == "off" else int(v)


def measure(gc, torch, ctx, wl, args, keep_device=False):
    """Times one workload: an autotuned plan replayed from a hipGraph (the
    value), then a plan with the same tiles and HIP events between the phases
    (per-phase times, the dominant decode kernel's duration); verifies the
    output bit-exact."""
    descs, headers, out_offs = gc.batch_layout(wl.streams, wl.offs, wl.lengths, align=4)
    d_s = gc.to_device(wl.streams)
    d_o = torch.empty(int(out_offs[-1]), dtype=torch.int32, device="cuda")
    t = time.time()
    plan = gc.Plan(ctx, descs, headers, d_s, d_o, tile_ints=args.tile, locate_stream=args.locate_stream,
                   pfd_tile_ints=args.pfd_tile or (4096 if args.tile else 0),
                   autotune=args.tile == 0, use_graph=True, carry_pass=args.carry_pass,
                   graph_serial=args.graph_serial,
                   pack_ints=pack_option(gc, args.pack_ints))
    cfg = plan.config()
    log("%s plan: %s (%.1fs)" % (wl.name, cfg, time.time() - t))
    tplan = gc.Plan(ctx, descs, headers, d_s, d_o, class_tiles=cfg["class_tiles"],
                    locate_stream=args.locate_stream, timing_slots=args.steps + args.warmup,
                    carry_pass=args.carry_pass, pack_ints=cfg["pack_ints"] or gc.PACK_OFF,
                    pack_groups=cfg["pack_groups"])
    packed = plan.packed_lists(wl.lengths.size)
    elapsed = timed(lambda: plan.decode_batch(d_s, d_o), args.steps, args.warmup, torch)
    t_events = timed(lambda: tplan.decode_batch(d_s, d_o), args.steps, args.warmup, torch)
    tm = tplan.timings(args.steps)
    rc, detail = ctx.sync_status()
    if rc != gc.OK:
        raise SystemExit("%s: device reported %d (detail %d)" % (wl.name, rc, detail))
    got = gc.unpad(gc.to_host(d_o), out_offs, wl.lengths)
    verified = bool(np.array_equal(got, wl.want))
    del got
    if not verified:
        raise SystemExit("%s: decoded output differs from the generated lists" % wl.name)
    m = Measured()
    m.cfg, m.verified, m.descs = cfg, verified, descs
    m.ms_per_step = 1e3 * elapsed / args.steps
    m.value = wl.ints / (elapsed / args.steps) / 1e9
    m.path_gbs = wl.path_bytes() / (elapsed / args.steps) / 1e9
    dec = tm["decode"].mean(axis=0)
    pack_ms = float(tm["pack"].mean())
    m.dec = dec
    # the dominant kernel: the longest decode pass, or the pack kernel
    m.cls = int(np.argmax(dec))
    if cfg["packs"] and pack_ms > dec[m.cls]:
        m.cls = -1
        m.cls_bytes = wl.bytes_of(packed)
        m.dec_avg = pack_ms
        m.kname = pack_kernel_name(cfg["pack_ints"])
    else:
        m.cls_bytes = wl.class_bytes(m.cls, packed)
        m.dec_avg = float(dec[m.cls])
        m.kname = kernel_name(m.cls, cfg["class_tiles"][m.cls], args.carry_pass)
    m.achieved = m.cls_bytes / (m.dec_avg * 1e-3) / 1e9
    present = [c for c in range(5) if np.any((wl.cls == c) & ~packed)]
    m.phases = {
        "note": "from a second plan with the same tiles and HIP events between the phases",
        "gpu_total": round(float(tm["total"].mean()), 4),
        "events_ms_per_step": round(1e3 * t_events / args.steps, 4),
        "locate": ({CLASS_NAMES[c]: round(float(tm["locate"][:, c].mean()), 4) for c in present}
                   if args.locate_stream else {"all classes": round(float(tm["locate"].sum(axis=1).mean()), 4)}),
        "sum_and_carry": {CLASS_NAMES[c]: round(float(tm["sum"][:, c].mean()), 4) for c in present},
        "decode": {CLASS_NAMES[c]: round(float(dec[c]), 4) for c in present},
        "decode_hbm_frac": {CLASS_NAMES[c]: round(wl.class_bytes(c, packed) / (float(dec[c]) * 1e-3) / 1e9
                                                  / HBM_PEAK_GBS, 4) for c in present},
    }
    if cfg["packs"]:
        m.phases["pack"] = round(pack_ms, 4)
        m.phases["pack_lists"] = int(packed.sum())
        m.phases["pack_ints"] = int(wl.lengths[packed].sum())
        m.phases["pack_hbm_frac"] = round(wl.bytes_of(packed) / (pack_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    log("%s: step %.3f ms, %.1f Gints/s, path %.0f GB/s (%.1f%% of HBM); dominant %s %.3f ms, %.0f GB/s; "
        "phases %s" % (wl.name, m.ms_per_step, m.value, m.path_gbs, 100 * m.path_gbs / HBM_PEAK_GBS,
                       m.kname, m.dec_avg, m.achieved, m.phases))
    tplan.close()
    if keep_device:
        m.plan, m.d_s, m.d_o, m.out_offs = plan, d_s, d_o, out_offs
    else:
        plan.close()
        del d_s, d_o
    return m


def leg_record(wl, m):
    return dict(workload=wl.desc, value=round(m.value, 3), unit="Gints/s", ms_per_step=round(m.ms_per_step, 4),
                ints_per_step=wl.ints, lists=int(wl.lengths.size), bits_per_int=round(32.0 * wl.streams.size / wl.ints, 3),
                path_hbm_frac=round(m.path_gbs / HBM_PEAK_GBS, 4), class_tile_ints=m.cfg["class_tiles"],
                pack_ints=m.cfg["pack_ints"], packs=m.cfg["packs"],
                pack_groups_per_cu=(None if m.cfg["pack_groups"] == 0x80000000 else m.cfg["pack_groups"]),
                dominant_kernel=m.kname, dominant_kernel_ms=round(m.dec_avg, 4),
                dominant_kernel_hbm_frac=round(m.achieved / HBM_PEAK_GBS, 4), phases_ms=m.phases,
                verified_bit_exact=m.verified)


def per_list_legs(gc, torch, ctx, wl, m, args):
    """One launch sequence per list (the same kernels): every list of the
    workload queued directly on one stream; and, on the first 10,000 lists,
    those launches replayed from one hipGraph beside the batched plan of the
    same lists."""
    res = {}
    plan, d_s, d_o = m.plan, m.d_s, m.d_o
    plan.decode_each(d_s, d_o)
    torch.cuda.synchronize()
    reps = 2
    t = timed(lambda: plan.decode_each(d_s, d_o), reps, 0, torch) / reps
    rc, det = ctx.sync_status()
    ok = rc == gc.OK and np.array_equal(gc.unpad(gc.to_host(d_o), m.out_offs, wl.lengths), wl.want)
    res["per_list"] = dict(value=round(wl.ints / t / 1e9, 3), unit="Gints/s", ms_per_run=round(1e3 * t, 2),
                           batched_speedup=round(m.value / (wl.ints / t / 1e9), 2), verified_bit_exact=bool(ok),
                           note="one launch sequence per list, all %d lists queued on one stream" % wl.lengths.size)
    # a subset captured in a graph
    nsub = min(10_000, wl.lengths.size)
    s_end = int(wl.offs[nsub])
    sub_l = wl.lengths[:nsub]
    descs, headers, out_offs = gc.batch_layout(wl.streams[:s_end], wl.offs[:nsub + 1], sub_l, align=4)
    ds2 = gc.to_device(wl.streams[:s_end])
    do2 = torch.full((int(out_offs[-1]),), -1, dtype=torch.int32, device="cuda")
    want = wl.want[:int(sub_l.sum())]
    p2 = gc.Plan(ctx, descs, headers, ds2, do2, class_tiles=m.cfg["class_tiles"], use_graph=True,
                 carry_pass=args.carry_pass)
    t_b = timed(lambda: p2.decode_batch(ds2, do2), 10, 2, torch) / 10
    t_d = timed(lambda: p2.decode_each(ds2, do2), 2, 1, torch) / 2
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        p2.decode_each(ds2, do2)
    do2.fill_(-1)
    t_g = timed(g.replay, 5, 1, torch) / 5
    rc, det = ctx.sync_status()
    ok = rc == gc.OK and np.array_equal(gc.unpad(gc.to_host(do2), out_offs, sub_l), want)
    n2 = int(sub_l.sum())
    res["per_list_graph"] = dict(
        lists=nsub, ints=n2, verified_bit_exact=bool(ok),
        batched_gints_s=round(n2 / t_b / 1e9, 3), per_list_direct_gints_s=round(n2 / t_d / 1e9, 3),
        per_list_graph_gints_s=round(n2 / t_g / 1e9, 3), batched_speedup_vs_graph=round(t_g / t_b, 2),
        note="the first %d lists of the workload: the batched plan, one launch sequence per list queued "
             "directly, and those per-list launches replayed from one hipGraph" % nsub)
    log("per-list: %s" % res)
    del g
    p2.close()
    del ds2, do2
    return res


def encode_leg(gc, torch, cfg2_data, reps=3):
    """Encode speed (Section 7.3.2, Table VII's encode columns) on the cfg2
    lists, docIDs and TFs, in the five codecs (4-way layout): the GPU list
    encoders (gc_encode_lists_gpu, input already on the device, streams
    written to device memory, sizes read back) against the host encoder on
    every host core (gc_encode_lists); the streams are checked equal."""
    lengths, docs, tfs = cfg2_data
    d_docs, d_tfs = gc.to_device(docs), gc.to_device(tfs)
    out = {}
    for name, codec, kw in five_codecs(gc):
        ints = 0
        t_gpu = t_host = 0.0
        same = True
        for flat, d_flat, delta in ((docs, d_docs, True), (tfs, d_tfs, False)):
            p = gc.params(delta=delta, **kw)
            got, goffs = gc.encode_lists_gpu(d_flat, lengths, codec, p)   # warm-up, sizes the output
            d_out = torch.empty(int(goffs[-1]), dtype=torch.int32, device="cuda")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                got, goffs = gc.encode_lists_gpu(d_flat, lengths, codec, p, d_out=d_out)
            torch.cuda.synchronize()
            t_gpu += (time.perf_counter() - t0) / reps
            t0 = time.perf_counter()
            want, woffs = gc.encode_lists(flat, lengths, codec, p)
            t_host += time.perf_counter() - t0
            same = same and np.array_equal(goffs, woffs) and np.array_equal(gc.to_host(got), want)
            ints += flat.size
            del got, d_out
        out[name] = dict(gpu_gints_s=round(ints / t_gpu / 1e9, 3), host_gints_s=round(ints / t_host / 1e9, 3),
                         gpu_ms=round(1e3 * t_gpu, 3), host_ms=round(1e3 * t_host, 2),
                         host_threads=os.cpu_count(), identical=bool(same))
        log("encode %-18s %s" % (name, out[name]))
    return out


def query_leg(gc, torch, ctx, synth, cfg2_data, nq=1000, reps=5):
    """Query processing (Section 7.4, Table X): 1,000 AND queries of 2 to 4
    terms (drawn by list length) over the cfg2 index, docIDs and TFs in one
    codec; per batch, one graph replay decodes the lists of the batch's
    distinct terms, then the AND / BM25 top-10 kernels run.  Reports
    queries/s and the share of the batch spent decoding (the paper finds
    decoding 15-35% of query time on its CPU); checks a sample of queries
    against the float64 reference."""
    from oracle import query_ref as Q
    lengths, docs, tfs = cfg2_data
    queries = synth.queries(lengths, seed=7, nq=nq)
    terms = np.unique(queries[queries >= 0])
    remap = np.full(lengths.size, -1, np.int64)
    remap[terms] = np.arange(terms.size)
    qloc = np.where(queries >= 0, remap[np.maximum(queries, 0)], -1)
    sub_len = lengths[terms]
    lo = np.concatenate([[0], np.cumsum(lengths)])
    sub_docs = np.concatenate([docs[lo[t]:lo[t + 1]] for t in terms])
    sub_tfs = np.concatenate([tfs[lo[t]:lo[t + 1]] for t in terms])
    doclen = synth.doc_lengths(ndocs=synth.U25)
    d_doclen = torch.from_numpy(doclen.view(np.int16)).cuda()
    avgdl = float(doclen.mean())
    out = {}
    for name, codec, kw in five_codecs(gc):
        s_d, o_d = gc.encode_lists(sub_docs, sub_len, codec, gc.params(delta=True, **kw))
        s_t, o_t = gc.encode_lists(sub_tfs, sub_len, codec, gc.params(**kw))
        streams = np.concatenate([s_d, s_t])
        offs = np.concatenate([o_d[:-1], o_t + o_d[-1]]).astype(np.int64)
        descs, headers, out_offs = gc.batch_layout(streams, offs, np.concatenate([sub_len, sub_len]), align=4)
        n = terms.size
        half = int(out_offs[n])
        d_s = gc.to_device(streams)
        arena = torch.empty(int(out_offs[-1]), dtype=torch.int32, device="cuda")
        plan = gc.Plan(ctx, descs, headers, d_s, arena, use_graph=True)
        term_off = torch.from_numpy(out_offs[:n].astype(np.int64)).cuda()
        qp = gc.QueryPlan(sub_len, qloc, synth.U25, avgdl, topk=10)
        d_doc = torch.empty(nq * 10, dtype=torch.int32, device="cuda")
        d_sc = torch.empty(nq * 10, dtype=torch.float32, device="cuda")
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        dec = qry = 0.0
        for r in range(reps + 1):
            ev[0].record()
            plan.decode_batch(d_s, arena)
            ev[1].record()
            qp.run(arena, arena[half:], term_off, d_doclen, d_doc, d_sc)
            ev[2].record()
            torch.cuda.synchronize()
            if r:
                dec += ev[0].elapsed_time(ev[1]) / reps
                qry += ev[1].elapsed_time(ev[2]) / reps
        rc, det = ctx.sync_status()
        got_d = gc.to_host(d_doc).reshape(nq, 10)
        got_s = d_sc.cpu().numpy().reshape(nq, 10)
        sample = np.random.default_rng(1).choice(nq, 50, replace=False)
        ok = rc == gc.OK
        sub_doc_lists = [sub_docs[int(o):int(o) + int(L)] for o, L in zip(np.concatenate([[0], np.cumsum(sub_len)]), sub_len)]
        sub_tf_lists = [sub_tfs[int(o):int(o) + int(L)] for o, L in zip(np.concatenate([[0], np.cumsum(sub_len)]), sub_len)]
        for q in sample:
            want = Q.and_topk(sub_doc_lists, sub_tf_lists, qloc[q], doclen, synth.U25, avgdl, k=10)
            nw = len(want)
            ok = ok and bool(np.all(got_d[q, nw:] == 0xFFFFFFFF)) and bool(
                np.allclose(got_s[q, :nw], [s for s, _ in want], rtol=2e-5, atol=0))
        total = dec + qry
        out[name] = dict(queries_per_s=round(nq / (total * 1e-3), 1), ms_per_batch=round(total, 4),
                         decode_ms=round(dec, 4), query_ms=round(qry, 4),
                         decode_share=round(dec / total, 4), terms=int(n), postings=int(2 * sub_len.sum()),
                         verified_sample=bool(ok))
        log("query %-18s %s" % (name, out[name]))
        qp.close()
        plan.close()
        del d_s, arena
    return out


def variants_leg(gc, torch, ctx, synth, args, cfg2_data):
    """Section 7.2's trade-off on the cfg2 lists: every variant's bits/int,
    Gints/s and decode-pass % of HBM (docIDs and TFs of one variant per
    batch)."""
    lengths, docs, tfs = cfg2_data
    out = {}
    for name, codec, kw in all_variants(gc):
        parts = []
        for flat, delta in ((docs, True), (tfs, False)):
            parts.append(gc.encode_lists(flat, lengths, codec, gc.params(delta=delta, **kw)))
        s, offs = concat_parts(parts)
        L = np.tile(lengths, 2)
        c = codec_class(gc, codec, kw)
        wl = Workload(name, name, s, offs, L, np.full(L.size, c, np.int32), np.concatenate([docs, tfs]))
        m = measure(gc, torch, ctx, wl, args)
        out[name] = dict(gints_s=round(m.value, 2), bits_per_int_docids=round(32.0 * parts[0][0].size / docs.size, 3),
                         bits_per_int_tf=round(32.0 * parts[1][0].size / tfs.size, 3),
                         path_hbm_frac=round(m.path_gbs / HBM_PEAK_GBS, 4),
                         decode_ms=round(m.dec_avg, 4), decode_hbm_frac=round(m.achieved / HBM_PEAK_GBS, 4))
        log("%-14s %s" % (name, out[name]))
        del wl, s
    return out


def widths_leg(gc, torch, ctx, synth, args):
    """The cfg5 lists in Group-AFOR and Group-PFD at the layout widths between
    the paper's 4-way layout and the 64-way one (Section 3.1's k-way layout):
    bits/int, Gints/s and % of HBM for k = 8, 16 and 32 (4 and 64 are the
    cfg5 batches of the full run)."""
    out = {}
    for codec_name in ("AFOR", "PFD"):
        for k in (8, 16, 32):
            name = "cfg5-%s-k%d" % (codec_name.lower(), k)
            w5 = build_cfg5(gc, synth, name, (codec_name, dict(k=k)))
            rec = leg_record(w5, measure(gc, torch, ctx, w5, args))
            out[name] = {key: rec[key] for key in ("bits_per_int", "value", "path_hbm_frac", "dominant_kernel",
                                                   "dominant_kernel_hbm_frac", "pack_ints", "verified_bit_exact")}
            log("%-16s %s" % (name, out[name]))
            del w5
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="cfg3", choices=WORKLOADS,
                    help="the workload timed for `value`; any other than cfg3 is measured alone (no legs)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--graph-serial", action="store_true",
                    help="graph: one chain of kernels instead of branches for the pack kernel and each class")
    ap.add_argument("--no-extra", action="store_true", help="skip every leg")
    ap.add_argument("--tile", type=int, default=0, help="force the wave-tile size (0 = autotune)")
    ap.add_argument("--pack-ints", default="auto",
                    help="packed-list threshold: auto (autotuned), off, or 1 .. 4096 integers")
    ap.add_argument("--pfd-tile", type=int, default=0, help="force the Group-PFD tile size (with --tile)")
    ap.add_argument("--locate-stream", action="store_true",
                    help="run the locate kernels on a second stream, ahead of the other kernels")
    ap.add_argument("--leg", choices=("encode", "query", "variants", "widths"),
                    help="run only this leg (cfg2: the list encoders, AND queries, or every codec variant; "
                         "widths: the cfg5 lists at k = 8, 16, 32) and print its record")
    ap.add_argument("--carry-pass", type=int, default=0, choices=(0, 1, 2, 3),
                    help="carries of delta lists: 1 look-back in the decode pass, 2 tile-sum pass and carry "
                         "scan, 3 look-back for lists of up to 64 tiles and the tile-sum pass for longer ones, "
                         "0 the library default")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the decode path is built and measured on a single "
              "MI355X (lists shard across GPUs with no exchange); --gpus %d is not supported"
              % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1502_01916_amd import gc, synth
    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    gc.lib()
    if args.leg:
        data = synth.cfg2() if args.leg != "widths" else None
        if args.leg == "encode":
            rec = encode_leg(gc, torch, data)
        elif args.leg == "variants":
            rec = variants_leg(gc, torch, gc.Context(0), synth, args, data)
        elif args.leg == "widths":
            rec = widths_leg(gc, torch, gc.Context(0), synth, args)
        else:
            rec = query_leg(gc, torch, gc.Context(0), synth, data)
        print(json.dumps({"leg": args.leg + ("_cfg5" if args.leg == "widths" else "_cfg2"), "record": rec}),
              flush=True)
        return
    legs = args.workload == "cfg3" and not args.no_extra

    cfg2_data = None
    if args.workload == "cfg3":
        wl = build_cfg3(gc, synth)
    elif args.workload == "cfg2":
        wl, cfg2_data = build_cfg2(gc, synth)
    else:
        wl = build_cfg5(gc, synth, args.workload)
    ctx = gc.Context(0)
    m = measure(gc, torch, ctx, wl, args, keep_device=True)
    traffic = read_traffic(wl.name, len(m.descs), m.kname, m.cls_bytes)

    extra = {}
    if legs:
        extra.update(per_list_legs(gc, torch, ctx, wl, m, args))
    m.plan.close()
    del m.d_s, m.d_o
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(wl, args.cpu_seconds)
        log("cpu oracle: %s" % cpu)
    if legs:
        w2, cfg2_data = build_cfg2(gc, synth)
        extra["cfg2"] = leg_record(w2, measure(gc, torch, ctx, w2, args))
        del w2
        for name in CFG5_BATCHES:
            w5 = build_cfg5(gc, synth, name)
            extra[name] = leg_record(w5, measure(gc, torch, ctx, w5, args))
            del w5
        extra["variants_cfg2"] = variants_leg(gc, torch, ctx, synth, args, cfg2_data)
        extra["encode_cfg2"] = encode_leg(gc, torch, cfg2_data)
        extra["query_cfg2"] = query_leg(gc, torch, ctx, synth, cfg2_data)
        extra["cfg1_latency"] = cfg1_latency(gc, synth, ctx, torch)
        log("cfg1 single list: %s" % extra["cfg1_latency"])

    line = {
        "metric": METRIC,
        "value": round(m.value, 3),
        "unit": "Gints/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(m.ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": wl.desc,
            "name": wl.name,
            "lists": len(m.descs),
            "ints_per_step": wl.ints,
            "stream_bytes": 4 * int(wl.streams.size),
            "bits_per_int": round(32.0 * wl.streams.size / wl.ints, 3),
            "tile_ints": m.cfg["tile_ints"],
            "pfd_tile_ints": m.cfg["pfd_tile_ints"],
            "class_tile_ints": m.cfg["class_tiles"],
            "tiles": m.cfg["tiles"],
            "sum_tiles": m.cfg["sum_tiles"],
            "pack_ints": m.cfg["pack_ints"],
            "packs": m.cfg["packs"],
            "packed_lists": m.cfg["packed_lists"],
            "pack_groups_per_cu": (None if m.cfg["pack_groups"] == gc.PACK_GROUPS_ALL else m.cfg["pack_groups"]),
            "verified_bit_exact": m.verified,
        },
        "path_hbm_frac": round(m.path_gbs / HBM_PEAK_GBS, 4),
        "roofline": {
            "bound": "hbm",
            "kernel": m.kname,
            "achieved": round(m.achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(m.achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "algorithmic_bytes_per_launch": m.cls_bytes,
            "avg_kernel_ms": round(m.dec_avg, 4),
        },
        "phases_ms": m.phases,
        "cpu_baseline": cpu,
    }
    line.update(extra)
    # plain copy of a known size, so counter runs of this command can be
    # scaled against it
    src = torch.empty(1 << 26, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
