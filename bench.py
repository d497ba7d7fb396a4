#!/usr/bin/env python3
"""Throughput of batched Group-codec decoding + d-gap prefix sum on one MI355X.

Workload: 10,000 synthetic posting lists (Zipf lengths clipped to
[128, 2^22], 2^26 docIDs, universe 2^25, 70% sparse / 30% clustered d-gaps)
and their TF lists, each coded with Group-Simple, Group-Scheme 1-CU,
Group-Scheme 8-IU, Group-AFOR and Group-PFD (32-tuple blocks, zeta = 1/10) in
the paper's 4-way layout: 100,000 streams, about 6.7e8 integers.  One step
decodes every stream (docID lists prefix-summed): the locate kernels, then per
codec class the tile-sum pass, the carry scan and the decode pass, all captured
in one hipGraph; `value` times the graph replays.  A second plan with the same
tiles launches the kernels directly with HIP events between the phases; it
gives the per-phase times and the dominant kernel's average duration.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gints/s decoded+prefix-summed, % HBM peak; batched vs per-list on 1 MI355X"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_decode_cfg2.txt")
# the sources the decode kernels are compiled from
DECODE_SRCS = [os.path.join(ROOT, "paper_1502_01916_amd", "csrc", f)
               for f in ("decode.hip", "gc_wave.h", "gc_device.h", "gc_format.h")]


def decode_sources_sha256():
    h = hashlib.sha256()
    for path in DECODE_SRCS:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def variants(gc):
    return [("group-simple", gc.SIMPLE, {}),
            ("group-scheme-1cu", gc.SCHEME, dict(cg=1, ld=gc.LD_CU)),
            ("group-scheme-8iu", gc.SCHEME, dict(cg=8, ld=gc.LD_IU)),
            ("group-afor", gc.AFOR, {}),
            ("group-pfd", gc.PFD, dict(zeta=(1, 10)))]


CLASS_NAMES = ["group-simple", "group-scheme-unary", "group-scheme-binary", "group-afor", "group-pfd"]


def kernel_name(cls, tile, carry_pass):
    """The decode kernel of a codec class as the profiler names it: tile size,
    class, and mode 2 (look-back carries) unless every carry comes from the
    tile-sum pass (mode 0)."""
    return "gc_wave_kernel<%d, %d, %d>" % (tile, cls, 0 if carry_pass == 2 else 2)


def codec_class(gc, codec, kw):
    if codec == gc.SIMPLE:
        return 0
    if codec == gc.SCHEME:
        return 2 if kw.get("ld", gc.LD_CU) == gc.LD_BINARY else 1
    return 3 if codec == gc.AFOR else 4


def class_bytes(gc, parts, cls):
    """Algorithmic bytes of one decode pass of a class: its streams read once
    and its integers written once."""
    b = 0
    for p in parts:
        if p["cls"] == cls:
            b += 4 * int(p["streams"].size) + 4 * int(p["flat"].size)
    return b


def build_workload(gc, synth):
    t = time.time()
    lengths, docs, tfs = synth.cfg2()
    log("cfg2 generated: %d lists, %d docIDs (%.1fs)" % (lengths.size, docs.size, time.time() - t))
    parts = []
    for name, codec, kw in variants(gc):
        for kind, flat, delta in (("docids", docs, True), ("tf", tfs, False)):
            t = time.time()
            s, offs = gc.encode_lists(flat, lengths, codec, gc.params(delta=delta, **kw))
            parts.append(dict(name=name, kind=kind, codec=codec, streams=s, offs=offs,
                              lengths=lengths, flat=flat, cls=codec_class(gc, codec, kw)))
            log("encoded %-18s %-6s %.2f bits/int (%.1fs)" % (name, kind, 32.0 * s.size / flat.size,
                                                              time.time() - t))
    return parts


def concat(parts):
    streams = np.concatenate([p["streams"] for p in parts])
    offs, base = [np.zeros(1, np.int64)], 0
    for p in parts:
        o = p["offs"].astype(np.int64)
        offs.append(o[1:] + base)
        base += int(o[-1])
    lengths = np.concatenate([p["lengths"] for p in parts])
    return streams, np.concatenate(offs), lengths


def read_traffic(units, kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, if it was taken on the current decode kernel source and this
    workload."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    with open(TRAFFIC_FILE) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    sha = decode_sources_sha256()
    if (kv.get("decode_sources_sha256") != sha or kv.get("workload_units") != str(units)
            or kv.get("kernel") != kernel):
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_threads():
    """Worker processes for the CPU baseline: the cores this process may use,
    at most 16 (the host share of one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


_CPU_PARTS = None


def _cpu_worker(args):
    """Decodes lists order[k], order[k + stride], ... with the C oracle for
    about `seconds`; returns (lists, integers, seconds)."""
    import oracle as O
    order, k, stride, seconds = args
    done_i = done_l = 0
    t0 = time.perf_counter()
    for idx in range(k, len(order), stride):
        pi, li = order[idx]
        p = _CPU_PARTS[pi]
        done_i += O.decode(p["streams"][int(p["offs"][li]):int(p["offs"][li + 1])]).size
        done_l += 1
        if time.perf_counter() - t0 > seconds:
            break
    return done_l, done_i, time.perf_counter() - t0


def cpu_baseline(parts, seconds):
    """The plain C oracle decoding (and prefix-summing) a random sample of the
    same streams: first in this process, then in one forked worker process per
    host core (lists dealt round-robin), each for about `seconds` seconds."""
    global _CPU_PARTS
    import multiprocessing as mp
    _CPU_PARTS = parts
    rng = np.random.default_rng(123)
    order = [(pi, li) for pi in range(len(parts)) for li in range(parts[pi]["lengths"].size)]
    rng.shuffle(order)
    one = _cpu_worker((order, 0, 1, seconds))
    nt = cpu_threads()
    with mp.get_context("fork").Pool(nt) as pool:
        res = pool.map(_cpu_worker, [(order, k, nt, seconds) for k in range(nt)])
    # the slowest worker's decode time (pool start-up excluded)
    wall = max(r[2] for r in res)
    lists = sum(r[0] for r in res)
    ints = sum(r[1] for r in res)
    return dict(value=round(ints / wall / 1e9, 4), unit="Gints/s", cores=nt, kind="oracle",
                per_core_value=round(one[1] / one[2] / 1e9, 4),
                sample="lists drawn at random from the same 100,000 streams, each decoded and "
                       "prefix-summed by the plain C oracle: %d lists (%d integers) on %d worker processes, the "
                       "slowest busy %.2f s; in one process: %d lists (%d integers) in %.2f s"
                       % (lists, ints, nt, wall, one[0], one[1], one[2]))


def cfg1_latency(gc, synth, ctx, torch, reps=30):
    """One list of 2^20 docIDs (mean gap 16) in Group-Simple, decoded and
    prefix-summed by gc_decode (locate, tile sums, carry scan, decode):
    the single-list latency, timed with HIP events around each call."""
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


def timed(plan, d_s, d_o, steps, warmup, torch):
    for _ in range(warmup):
        plan.decode_batch(d_s, d_o)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.decode_batch(d_s, d_o)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true", help="skip per-list and per-codec runs")
    ap.add_argument("--tile", type=int, default=0, help="force the wave-tile size (0 = autotune)")
    ap.add_argument("--pfd-tile", type=int, default=0, help="force the Group-PFD tile size (with --tile)")
    ap.add_argument("--locate-stream", action="store_true",
                    help="run the locate kernels on a second stream, ahead of the other kernels")
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

    parts = build_workload(gc, synth)
    streams, offs, lengths = concat(parts)
    descs, headers, out_offs = gc.batch_layout(streams, offs, lengths, align=4)
    total = int(lengths.sum())
    out_len = int(out_offs[-1])
    stream_bytes = 4 * int(streams.size)
    ctx = gc.Context(0)
    d_s = gc.to_device(streams)
    d_o = torch.empty(out_len, dtype=torch.int32, device="cuda")
    t = time.time()
    # the timed plan: autotuned tiles, the whole run captured in one hipGraph
    plan = gc.Plan(ctx, descs, headers, d_s, d_o, tile_ints=args.tile, locate_stream=args.locate_stream,
                   pfd_tile_ints=args.pfd_tile or (4096 if args.tile else 0),
                   autotune=args.tile == 0, use_graph=True, carry_pass=args.carry_pass)
    cfg = plan.config()
    log("plan: %s (%.1fs)" % (cfg, time.time() - t))
    # the same tiles with HIP events between the phases (direct launches), for
    # the per-phase times and the dominant kernel's duration
    tplan = gc.Plan(ctx, descs, headers, d_s, d_o, class_tiles=cfg["class_tiles"],
                    locate_stream=args.locate_stream, timing_slots=args.steps + args.warmup,
                    carry_pass=args.carry_pass)

    elapsed = timed(plan, d_s, d_o, args.steps, args.warmup, torch)
    t_events = timed(tplan, d_s, d_o, args.steps, args.warmup, torch)
    tm = tplan.timings(args.steps)
    rc, detail = ctx.sync_status()
    if rc != gc.OK:
        raise SystemExit("device reported %d (detail %d)" % (rc, detail))
    got = gc.unpad(gc.to_host(d_o), out_offs, lengths)
    want = np.concatenate([p["flat"] for p in parts])
    verified = bool(np.array_equal(got, want))
    del got, want
    ms_per_step = 1e3 * elapsed / args.steps
    value = total / (elapsed / args.steps) / 1e9
    # the dominant kernel: the decode pass of the class that takes longest
    dec = tm["decode"].mean(axis=0)
    cls = int(np.argmax(dec))
    cls_bytes = class_bytes(gc, parts, cls)
    dec_avg = float(dec[cls])
    achieved = cls_bytes / (dec_avg * 1e-3) / 1e9
    log("step %.3f ms  %.1f Gints/s  (with events between phases %.3f ms, GPU %.3f ms; per class locate %s, "
        "sum+carry %s, decode %s)  verified=%s"
        % (ms_per_step, value, 1e3 * t_events / args.steps, tm["total"].mean(), np.round(tm["locate"].mean(axis=0), 3),
           np.round(tm["sum"].mean(axis=0), 3), np.round(dec, 3), verified))
    log("dominant kernel: %s decode pass %.3f ms, %.0f GB/s" % (CLASS_NAMES[cls], dec_avg, achieved))
    if not verified:
        raise SystemExit("decoded output differs from the generated lists")
    kname = kernel_name(cls, cfg["class_tiles"][cls], args.carry_pass)
    traffic = read_traffic(len(descs), kname)

    extra = {}
    if not args.no_extra:
        # one launch sequence per list, same kernels (the per-list baseline)
        plan.decode_each(d_s, d_o)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = 2
        for _ in range(reps):
            plan.decode_each(d_s, d_o)
        torch.cuda.synchronize()
        per_list = total / ((time.perf_counter() - t0) / reps) / 1e9
        extra["per_list"] = dict(value=round(per_list, 3), unit="Gints/s",
                                 batched_speedup=round(value / per_list, 2))
        log("per-list launches: %.2f Gints/s, batched speedup %.1fx" % (per_list, value / per_list))
        per = {}
        for i in range(0, len(parts), 2):
            sub = parts[i:i + 2]
            s2, o2, l2 = concat(sub)
            de2, h2, oo2 = gc.batch_layout(s2, o2, l2, align=4)
            ds2 = gc.to_device(s2)
            do2 = torch.empty(int(oo2[-1]), dtype=torch.int32, device="cuda")
            p2 = gc.Plan(ctx, de2, h2, ds2, do2, class_tiles=cfg["class_tiles"], timing_slots=args.steps,
                         carry_pass=args.carry_pass)
            el = timed(p2, ds2, do2, args.steps, 2, torch)
            t2 = p2.timings(args.steps)
            c2 = sub[0]["cls"]
            n2 = int(l2.sum())
            gbs = class_bytes(gc, sub, c2) / (float(t2["decode"][:, c2].mean()) * 1e-3) / 1e9
            per[sub[0]["name"]] = dict(gints_s=round(n2 / (el / args.steps) / 1e9, 2),
                                       bits_per_int_docids=round(32.0 * sub[0]["streams"].size / n2 * 2, 3),
                                       bits_per_int_tf=round(32.0 * sub[1]["streams"].size / n2 * 2, 3),
                                       locate_ms=round(float(t2["locate"][:, c2].mean()), 4),
                                       sum_ms=round(float(t2["sum"][:, c2].mean()), 4),
                                       decode_ms=round(float(t2["decode"][:, c2].mean()), 4),
                                       decode_kernel_gbs=round(gbs, 1),
                                       hbm_frac=round(gbs / HBM_PEAK_GBS, 4))
            log("%-18s %s" % (sub[0]["name"], per[sub[0]["name"]]))
            p2.close()
            del ds2, do2
        extra["per_codec"] = per
        extra["cfg1_latency"] = cfg1_latency(gc, synth, ctx, torch)
        log("cfg1 single list: %s" % extra["cfg1_latency"])

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(parts, args.cpu_seconds)
        log("cpu oracle: %.4f Gints/s on %d threads, %.4f on one (%s)"
            % (cpu["value"], cpu["cores"], cpu["per_core_value"], cpu["sample"]))

    line = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Gints/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": "10,000 posting lists (Zipf lengths in [128, 2^22], 2^26 docIDs, universe "
                        "2^25, 70% sparse / 30% clustered d-gaps) plus their TF lists (geometric "
                        "p=0.4), each coded with Group-Simple, Group-Scheme 1-CU, Group-Scheme "
                        "8-IU, Group-AFOR and Group-PFD (zeta 1/10), 4-way layout; all 100,000 "
                        "streams decoded per step (locate, tile sums, carry scans, decode passes), "
                        "docID lists prefix-summed; seed 2",
            "lists": len(descs),
            "ints_per_step": total,
            "stream_bytes": stream_bytes,
            "bits_per_int": round(32.0 * streams.size / total, 3),
            "tile_ints": cfg["tile_ints"],
            "pfd_tile_ints": cfg["pfd_tile_ints"],
            "class_tile_ints": cfg["class_tiles"],
            "tiles": cfg["tiles"],
            "sum_tiles": cfg["sum_tiles"],
            "verified_bit_exact": verified,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": kname,
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "algorithmic_bytes_per_launch": cls_bytes,
            "avg_kernel_ms": round(dec_avg, 4),
        },
        "phases_ms": {
            "note": "from a second plan with the same tiles and HIP events between the phases",
            "gpu_total": round(float(tm["total"].mean()), 4),
            "locate": ({CLASS_NAMES[c]: round(float(tm["locate"][:, c].mean()), 4)
                        for c in range(5) if dec[c] > 0} if args.locate_stream
                       else {"all classes": round(float(tm["locate"].sum(axis=1).mean()), 4)}),
            "sum_and_carry": {CLASS_NAMES[c]: round(float(tm["sum"][:, c].mean()), 4)
                              for c in range(5) if dec[c] > 0},
            "decode": {CLASS_NAMES[c]: round(float(dec[c]), 4) for c in range(5) if dec[c] > 0},
        },
        "cpu_baseline": cpu,
    }
    line.update(extra)
    # plain copy of a known size, so counter runs of this command can be
    # scaled against it
    src = torch.empty(1 << 26, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    plan.close()
    tplan.close()
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
