"""Thin ctypes binding of libgc (include/gc.h): argument marshalling only.

Every decode step runs in libgc's HIP kernels; this module only converts
numpy arrays and torch device tensors into pointers and sizes.  Importing it
does not load the library; the first call does, and raises if libgc.so has
not been built (``python -m paper_1502_01916_amd.build``) -- there is no CPU
fallback.

Device buffers are torch tensors (int32 storage holding uint32 bit patterns);
streams are ``torch.cuda.current_stream().cuda_stream`` unless given.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

SIMPLE, SCHEME, AFOR, PFD, VSE = 0, 1, 2, 3, 4   # VSE: Group-VSEncoding (decoded by the AFOR class)
LD_BINARY, LD_CU, LD_IU = 0, 1, 2
PFD_LINKED, PFD_BITMAP = 0, 1
DELTA = 1
# decode kernel classes (gc_plan_timings columns)
CLS_SIMPLE, CLS_SCHEME_UNARY, CLS_SCHEME_BINARY, CLS_AFOR, CLS_PFD = range(5)
CLASSES = 5
TIMING_FIELDS = 2 + 3 * CLASSES
PACK_OFF = 0x80000000   # gc_plan_opts.pack_ints: no packed lists
PACK_GROUPS_ALL = 0x80000000   # gc_plan_opts.pack_groups: one wave per pack
OK, EINVAL, ENOSPC, ECORRUPT, EDEVICE, EUNSUPPORTED, ENOMEM = 0, -1, -2, -3, -4, -5, -6
_NAMES = {0: "GC_OK", -1: "GC_EINVAL", -2: "GC_ENOSPC", -3: "GC_ECORRUPT", -4: "GC_EDEVICE",
          -5: "GC_EUNSUPPORTED", -6: "GC_ENOMEM"}

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libgc.so")
_lib = None
_lock = threading.Lock()


class GcError(RuntimeError):
    def __init__(self, fn, code, detail=None):
        self.code = code
        self.detail = detail
        msg = "%s returned %s" % (fn, _NAMES.get(code, code))
        if detail:
            msg += " (detail %d)" % detail
        super().__init__(msg)


class Params(ctypes.Structure):
    _fields_ = [("k", ctypes.c_uint32), ("cg", ctypes.c_uint8), ("ld", ctypes.c_uint8),
                ("pfd_pos", ctypes.c_uint8), ("reserved", ctypes.c_uint8),
                ("zeta_num", ctypes.c_uint16), ("zeta_den", ctypes.c_uint16),
                ("flags", ctypes.c_uint32)]


class ListDesc(ctypes.Structure):
    _fields_ = [("stream_off_words", ctypes.c_uint64), ("stream_words", ctypes.c_uint64),
                ("out_off", ctypes.c_uint64), ("n", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class CtxOpts(ctypes.Structure):
    _fields_ = [("max_list_ints", ctypes.c_uint64), ("reserved", ctypes.c_uint32 * 2)]


class PlanOpts(ctypes.Structure):
    _fields_ = [("tile_ints", ctypes.c_uint32), ("pfd_tile_ints", ctypes.c_uint32),
                ("use_graph", ctypes.c_uint32), ("autotune", ctypes.c_uint32),
                ("timing_slots", ctypes.c_uint32), ("schedule", ctypes.c_uint32),
                ("class_tile_ints", ctypes.c_uint32 * 5), ("carry_pass", ctypes.c_uint32),
                ("pack_ints", ctypes.c_uint32), ("graph_serial", ctypes.c_uint32),
                ("pack_groups", ctypes.c_uint32)]


# how the tiles of a delta list get their carries (gc_plan_opts.carry_pass)
CARRY_DEFAULT, CARRY_LOOKBACK, CARRY_SUM_PASS, CARRY_HYBRID = 0, 1, 2, 3


class BM25Params(ctypes.Structure):
    _fields_ = [("k1", ctypes.c_float), ("b", ctypes.c_float), ("avgdl", ctypes.c_float),
                ("topk", ctypes.c_uint32), ("ndocs", ctypes.c_uint32), ("reserved", ctypes.c_uint32 * 2)]


class AdamOpts(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float), ("lam", ctypes.c_float), ("batch", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32 * 2)]


def adam_opts(lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, lam=0.0, batch=4096):
    return AdamOpts(lr, beta1, beta2, eps, lam, batch)


def params(k=4, cg=1, ld=LD_CU, pfd_pos=PFD_LINKED, zeta=(1, 10), delta=False):
    return Params(int(k), int(cg), int(ld), int(pfd_pos), 0, int(zeta[0]), int(zeta[1]),
                  DELTA if delta else 0)


def lib():
    """Loads libgc.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libgc.so is not built: run python -m paper_1502_01916_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        vp, sz, u32p = ctypes.c_void_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_uint32)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        i = ctypes.c_int
        f32p = ctypes.POINTER(ctypes.c_float)
        L.gc_version.restype = ctypes.c_char_p
        L.gc_encoded_bound_words.argtypes = [sz, i, ctypes.POINTER(Params)]
        L.gc_encoded_bound_words.restype = sz
        L.gc_encode.argtypes = [u32p, sz, i, ctypes.POINTER(Params), u32p, sz, ctypes.POINTER(sz)]
        L.gc_encoded_bound_words_lists.argtypes = [u64p, sz, ctypes.POINTER(ctypes.c_int),
                                                   ctypes.POINTER(Params), i]
        L.gc_encoded_bound_words_lists.restype = sz
        L.gc_encode_lists.argtypes = [u32p, u64p, sz, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(Params),
                                      i, u32p, sz, u64p, i]
        L.gc_ctx_create.argtypes = [i, ctypes.POINTER(vp)]
        L.gc_ctx_create_opts.argtypes = [i, ctypes.POINTER(CtxOpts), ctypes.POINTER(vp)]
        L.gc_ctx_destroy.argtypes = [vp]
        L.gc_decode.argtypes = [vp, vp, sz, u32p, vp, vp]
        L.gc_decode_noalloc.argtypes = [vp, vp, sz, u32p, vp, vp]
        L.gc_query_plan_create.argtypes = [vp, sz, vp, ctypes.c_uint32, ctypes.c_uint32,
                                           ctypes.POINTER(BM25Params), ctypes.POINTER(vp)]
        L.gc_query_plan_destroy.argtypes = [vp]
        L.gc_query_run.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
        L.gc_encode_lists_gpu.argtypes = [vp, ctypes.POINTER(ctypes.c_uint64), sz, i, ctypes.POINTER(Params), vp,
                                          sz, ctypes.POINTER(ctypes.c_uint64), vp]
        L.gc_plan_create.argtypes = [vp, ctypes.POINTER(ListDesc), sz, u32p, ctypes.POINTER(PlanOpts),
                                     vp, vp, ctypes.POINTER(vp)]
        L.gc_plan_destroy.argtypes = [vp]
        L.gc_decode_batch.argtypes = [vp, vp, vp, vp]
        L.gc_decode_each.argtypes = [vp, vp, vp, vp]
        L.gc_plan_config.argtypes = [vp, u32p, u32p, u64p, u64p]
        L.gc_plan_class_tiles.argtypes = [vp, u32p]
        L.gc_plan_pack_config.argtypes = [vp, u32p, u64p, u64p, u32p]
        L.gc_plan_packed_lists.argtypes = [vp, vp, sz]
        L.gc_plan_timings.argtypes = [vp, ctypes.c_uint32, f32p, u32p]
        L.gc_plan_timings.restype = ctypes.c_int
        L.gc_sync_status.argtypes = [vp, vp, u32p]
        L.gc_block_features.argtypes = [vp, vp, sz, vp, vp]
        L.gc_block_sizes.argtypes = [vp, vp, sz, vp, vp, vp, vp]
        L.gc_blockmix_bound_words.argtypes = [sz]
        L.gc_blockmix_bound_words.restype = sz
        L.gc_blockmix_encode.argtypes = [vp, vp, sz, vp, vp, sz, ctypes.POINTER(sz), vp]
        L.gc_mlp_param_count.restype = sz
        L.gc_mlp_create.argtypes = [vp, ctypes.c_uint32, ctypes.POINTER(vp)]
        L.gc_mlp_destroy.argtypes = [vp]
        L.gc_mlp_set_params.argtypes = [vp, f32p, sz, vp]
        L.gc_mlp_get_params.argtypes = [vp, f32p, sz, vp]
        L.gc_mlp_forward.argtypes = [vp, vp, sz, vp, vp, vp]
        L.gc_mlp_get_state.argtypes = [vp, f32p, sz, ctypes.POINTER(ctypes.c_uint64), vp]
        L.gc_mlp_set_state.argtypes = [vp, f32p, sz, ctypes.c_uint64, vp]
        L.gc_mlp_grad.argtypes = [vp, vp, vp, vp, vp, ctypes.c_uint32, ctypes.c_float, vp, vp, vp]
        L.gc_mlp_train.argtypes = [vp, vp, vp, vp, vp, sz, ctypes.POINTER(AdamOpts), vp, vp]
        L.gc_encode_blocks.argtypes = [vp, vp, sz, i, vp, ctypes.c_uint32, vp, sz, ctypes.POINTER(sz), vp, vp]
        for f in ("gc_encode", "gc_encode_lists", "gc_ctx_create", "gc_ctx_create_opts", "gc_ctx_destroy",
                  "gc_decode", "gc_decode_noalloc", "gc_encode_lists_gpu", "gc_query_plan_create",
                  "gc_query_plan_destroy", "gc_query_run",
                  "gc_plan_create", "gc_plan_destroy", "gc_decode_batch", "gc_decode_each",
                  "gc_plan_config", "gc_plan_class_tiles", "gc_plan_pack_config", "gc_plan_packed_lists",
                  "gc_sync_status", "gc_block_features",
                  "gc_block_sizes", "gc_blockmix_encode", "gc_mlp_create", "gc_mlp_destroy", "gc_mlp_set_params",
                  "gc_mlp_get_params", "gc_mlp_forward", "gc_mlp_grad", "gc_mlp_train", "gc_encode_blocks",
                  "gc_mlp_get_state", "gc_mlp_set_state"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
        return L


def _check(fn, rc, detail=None):
    if rc != OK:
        raise GcError(fn, rc, detail)


def _u32(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


def version():
    return lib().gc_version().decode()


# ---------------------------------------------------------------------------
# Host encoding.

def encoded_bound_words(n, codec, p: Params):
    return lib().gc_encoded_bound_words(n, codec, ctypes.byref(p))


def encode(x, codec, p: Params):
    """gc_encode: one uint32 list -> one stream (numpy uint32 words)."""
    x = np.ascontiguousarray(x, dtype=np.uint32)
    cap = encoded_bound_words(x.size, codec, p)
    out = np.zeros(max(cap, 4), np.uint32)
    w = ctypes.c_size_t()
    _check("gc_encode", lib().gc_encode(_u32(x), x.size, codec, ctypes.byref(p), _u32(out), out.size,
                                        ctypes.byref(w)))
    return out[:w.value].copy()


def encode_lists(flat, lengths, codecs, plist, nthreads=0):
    """gc_encode_lists: many lists (concatenated in `flat`) on all host cores.
    `codecs` is one codec per list; `plist` one Params or one per list.
    Returns (streams_flat, stream_offsets[nlists+1])."""
    flat = np.ascontiguousarray(flat, dtype=np.uint32)
    lengths = np.asarray(lengths, dtype=np.int64)
    nl = lengths.size
    in_offs = np.zeros(nl + 1, np.uint64)
    np.cumsum(lengths, out=in_offs[1:])
    cod = np.ascontiguousarray(np.broadcast_to(np.asarray(codecs, dtype=np.int32), (nl,)))
    one = isinstance(plist, Params)
    parr = (Params * (1 if one else nl))()
    if one:
        parr[0] = plist
    else:
        for i, p in enumerate(plist):
            parr[i] = p
    cap = lib().gc_encoded_bound_words_lists(in_offs.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), nl,
                                             cod.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), parr, int(one))
    out = np.zeros(cap, np.uint32)
    offs = np.zeros(nl + 1, np.uint64)
    rc = lib().gc_encode_lists(_u32(flat), in_offs.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), nl,
                               cod.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), parr, int(one),
                               _u32(out), out.size, offs.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                               int(nthreads))
    _check("gc_encode_lists", rc)
    return out[:int(offs[-1])], offs


def encode_lists_gpu(d_flat, lengths, codec, p, d_out=None, stream=None):
    """gc_encode_lists_gpu: the lists concatenated in the device tensor
    d_flat (int32), one codec / Params for all, encoded on the GPU.  Returns
    (d_streams, stream_offsets[nlists+1]); d_streams is d_out (or a new
    tensor sized by gc_encoded_bound_words_lists) cut to the streams."""
    import torch
    lengths = np.asarray(lengths, dtype=np.int64)
    nl = lengths.size
    in_offs = np.zeros(nl + 1, np.uint64)
    np.cumsum(lengths, out=in_offs[1:])
    if d_out is None:
        cod = np.full(nl, int(codec), np.int32)
        parr = (Params * 1)()
        parr[0] = p
        cap = lib().gc_encoded_bound_words_lists(in_offs.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), nl,
                                                 cod.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), parr, 1)
        d_out = torch.empty(max(int(cap), 1), dtype=torch.int32, device=d_flat.device)
    offs = np.zeros(nl + 1, np.uint64)
    rc = lib().gc_encode_lists_gpu(_ptr(d_flat), in_offs.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), nl,
                                   int(codec), ctypes.byref(p), _ptr(d_out), int(d_out.numel()),
                                   offs.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), _stream_handle(stream))
    _check("gc_encode_lists_gpu", rc)
    return d_out[:int(offs[-1])], offs


# ---------------------------------------------------------------------------
# Device decoding.

def _stream_handle(stream):
    if stream is not None:
        return ctypes.c_void_p(stream)
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """gc_ctx_create_opts / gc_decode / gc_sync_status / gc_ctx_destroy.
    max_list_ints: the longest list decode() and the block encoders accept
    (0 = the library's default, 2^24)."""

    def __init__(self, device=0, max_list_ints=0):
        self._h = ctypes.c_void_p()
        opts = CtxOpts(int(max_list_ints))
        _check("gc_ctx_create_opts", lib().gc_ctx_create_opts(int(device), ctypes.byref(opts),
                                                                ctypes.byref(self._h)))

    def decode(self, d_stream, stream_words, header, d_out, stream=None):
        """gc_decode: `header` is the host copy of the stream's first 4 words."""
        hdr = np.ascontiguousarray(header, dtype=np.uint32)[:4]
        _check("gc_decode", lib().gc_decode(self._h, _ptr(d_stream), int(stream_words), _u32(hdr),
                                            _ptr(d_out), _stream_handle(stream)))

    def decode_noalloc(self, d_stream, stream_words, header, d_out, stream=None):
        """gc_decode_noalloc: gc_decode with the library's fixed device
        scratch (lists of up to 2^22 integers); allocates nothing."""
        hdr = np.ascontiguousarray(header, dtype=np.uint32)[:4]
        _check("gc_decode_noalloc", lib().gc_decode_noalloc(self._h, _ptr(d_stream), int(stream_words), _u32(hdr),
                                                            _ptr(d_out), _stream_handle(stream)))

    def sync_status(self, stream=None):
        """Returns (status, detail) of the first device error since the last call."""
        d = ctypes.c_uint32()
        rc = lib().gc_sync_status(self._h, _stream_handle(stream), ctypes.byref(d))
        return rc, d.value

    def check(self, stream=None):
        rc, d = self.sync_status(stream)
        _check("gc_sync_status", rc, d)

    # ---- per-block container (learned codec selector) ----
    def block_features(self, d_in, nblocks, d_feat, stream=None):
        """gc_block_features: d_in int32 [nblocks*128], d_feat float32 [nblocks, 40]."""
        _check("gc_block_features", lib().gc_block_features(self._h, _ptr(d_in), int(nblocks), _ptr(d_feat),
                                                              _stream_handle(stream)))

    def block_sizes(self, d_in, nblocks, d_sizes=None, d_best=None, d_cost=None, stream=None):
        """gc_block_sizes: d_sizes int32 [nblocks, 16], d_best uint8 [nblocks], d_cost float32
        [nblocks, 16]; any may be None."""
        _check("gc_block_sizes", lib().gc_block_sizes(
            self._h, _ptr(d_in), int(nblocks), None if d_sizes is None else _ptr(d_sizes),
            None if d_best is None else _ptr(d_best), None if d_cost is None else _ptr(d_cost),
            _stream_handle(stream)))

    def blockmix_encode(self, d_in, n, d_class, d_out, stream=None):
        """gc_blockmix_encode: returns the container's length in words."""
        used = ctypes.c_size_t()
        _check("gc_blockmix_encode", lib().gc_blockmix_encode(
            self._h, _ptr(d_in), int(n), _ptr(d_class), _ptr(d_out), int(d_out.numel()), ctypes.byref(used),
            _stream_handle(stream)))
        return used.value

    def encode_blocks(self, d_in, n, mode, d_out, model=None, fixed_class=0, d_class_out=None, stream=None):
        """gc_encode_blocks: returns the container's length in words."""
        used = ctypes.c_size_t()
        _check("gc_encode_blocks", lib().gc_encode_blocks(
            self._h, _ptr(d_in), int(n), int(mode), None if model is None else model._h, int(fixed_class),
            _ptr(d_out), int(d_out.numel()), ctypes.byref(used),
            None if d_class_out is None else _ptr(d_class_out), _stream_handle(stream)))
        return used.value

    def close(self):
        if self._h:
            lib().gc_ctx_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """gc_plan_create / gc_decode_batch / gc_decode_each / gc_plan_destroy."""

    def __init__(self, ctx: Context, descs, headers, d_streams=None, d_out=None, tile_ints=0,
                 pfd_tile_ints=0, use_graph=False, autotune=False, timing_slots=0, locate_stream=False,
                 carry_pass=CARRY_DEFAULT, class_tiles=None, pack_ints=0, graph_serial=False, pack_groups=0):
        self.ctx = ctx
        nl = len(descs)
        arr = (ListDesc * max(nl, 1))()
        for i, d in enumerate(descs):
            arr[i] = d
        hdr = np.ascontiguousarray(headers, dtype=np.uint32).reshape(-1)
        ct = (ctypes.c_uint32 * 5)(*[int(t) for t in (class_tiles if class_tiles is not None else [0] * 5)])
        opts = PlanOpts(int(tile_ints), int(pfd_tile_ints), int(bool(use_graph)), int(bool(autotune)),
                        int(timing_slots), int(bool(locate_stream)), ct, int(carry_pass), int(pack_ints),
                        int(bool(graph_serial)), int(pack_groups))
        self._h = ctypes.c_void_p()
        rc = lib().gc_plan_create(ctx._h, arr, nl, _u32(hdr), ctypes.byref(opts),
                                  _ptr(d_streams) if d_streams is not None else None,
                                  _ptr(d_out) if d_out is not None else None, ctypes.byref(self._h))
        _check("gc_plan_create", rc)

    def decode_batch(self, d_streams, d_out, stream=None):
        _check("gc_decode_batch", lib().gc_decode_batch(self._h, _ptr(d_streams), _ptr(d_out),
                                                        _stream_handle(stream)))

    def decode_each(self, d_streams, d_out, stream=None):
        _check("gc_decode_each", lib().gc_decode_each(self._h, _ptr(d_streams), _ptr(d_out),
                                                      _stream_handle(stream)))

    def timings(self, max_runs):
        """Per-run kernel times (ms) of the last runs, oldest first: a dict of
        arrays -- total (runs,), and locate, sum, decode (runs, CLASSES) with
        classes in the order SIMPLE, SCHEME unary, SCHEME binary, AFOR, PFD."""
        a = (ctypes.c_float * (max(max_runs, 1) * TIMING_FIELDS))()
        n = ctypes.c_uint32()
        _check("gc_plan_timings", lib().gc_plan_timings(self._h, int(max_runs), a, ctypes.byref(n)))
        m = np.array(a[:n.value * TIMING_FIELDS], dtype=np.float64).reshape(n.value, TIMING_FIELDS)
        return dict(total=m[:, 0], locate=m[:, 1:1 + CLASSES], sum=m[:, 1 + CLASSES:1 + 2 * CLASSES],
                    decode=m[:, 1 + 2 * CLASSES:1 + 3 * CLASSES], pack=m[:, 1 + 3 * CLASSES])

    def config(self):
        """Chosen tile sizes, decode tiles per run and the tiles of those the
        sum pass decodes too."""
        t, pt = ctypes.c_uint32(), ctypes.c_uint32()
        n, ns = ctypes.c_uint64(), ctypes.c_uint64()
        _check("gc_plan_config", lib().gc_plan_config(self._h, ctypes.byref(t), ctypes.byref(pt),
                                                      ctypes.byref(n), ctypes.byref(ns)))
        ct = (ctypes.c_uint32 * CLASSES)()
        _check("gc_plan_class_tiles", lib().gc_plan_class_tiles(self._h, ct))
        pi, npk, npl, pg = ctypes.c_uint32(), ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint32()
        _check("gc_plan_pack_config", lib().gc_plan_pack_config(self._h, ctypes.byref(pi), ctypes.byref(npk),
                                                                ctypes.byref(npl), ctypes.byref(pg)))
        return dict(tile_ints=t.value, pfd_tile_ints=pt.value, tiles=n.value, sum_tiles=ns.value,
                    class_tiles=[int(x) for x in ct], pack_ints=pi.value, packs=npk.value,
                    packed_lists=npl.value, pack_groups=pg.value)

    def packed_lists(self, nlists):
        """gc_plan_packed_lists: a bool array, True for the lists the pack
        kernel decodes."""
        out = np.zeros(int(nlists), dtype=np.uint8)
        _check("gc_plan_packed_lists", lib().gc_plan_packed_lists(self._h, out.ctypes.data_as(ctypes.c_void_p),
                                                                  int(nlists)))
        return out.astype(bool)

    def close(self):
        if self._h:
            lib().gc_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_layout(streams_flat, stream_offs, lengths, align=1):
    """List descriptors and headers for streams concatenated in `streams_flat`
    (offsets from encode_lists).  List i decodes to out_offs[i] .. +lengths[i]
    of one output buffer; with align > 1 every list starts on a multiple of
    `align` integers.  Returns (descs, headers, out_offs) with out_offs[-1] the
    buffer length."""
    lengths = np.asarray(lengths, dtype=np.int64)
    padded = (lengths + align - 1) // align * align
    out_offs = np.zeros(lengths.size + 1, np.int64)
    np.cumsum(padded, out=out_offs[1:])
    so = np.asarray(stream_offs, dtype=np.int64)
    descs = [ListDesc(int(so[i]), int(so[i + 1] - so[i]), int(out_offs[i]), int(lengths[i]), 0)
             for i in range(lengths.size)]
    idx = so[:-1, None] + np.arange(4)[None, :]
    headers = streams_flat[idx.reshape(-1)].reshape(-1, 4) if lengths.size else np.zeros((0, 4), np.uint32)
    return descs, np.ascontiguousarray(headers, dtype=np.uint32), out_offs


def unpad(out, out_offs, lengths):
    """Concatenates the decoded lists of a batch output laid out by batch_layout."""
    lengths = np.asarray(lengths, dtype=np.int64)
    if np.array_equal(np.diff(out_offs), lengths):
        return out[:int(lengths.sum())]
    return np.concatenate([out[int(o):int(o) + int(L)] for o, L in zip(out_offs[:-1], lengths)])


SELECT_EXHAUSTIVE, SELECT_LEARNED, SELECT_FIXED = 0, 1, 2


def _opt(t):
    return None if t is None else _ptr(t)


class Mlp:
    """The selector network: gc_mlp_create / set/get_params / forward / grad /
    train / destroy.  Device tensors in, device tensors out."""

    def __init__(self, ctx: Context, max_batch=4096):
        self.ctx = ctx
        self._h = ctypes.c_void_p()
        _check("gc_mlp_create", lib().gc_mlp_create(ctx._h, int(max_batch), ctypes.byref(self._h)))

    @staticmethod
    def param_count():
        return int(lib().gc_mlp_param_count())

    def set_params(self, theta, stream=None):
        t = np.ascontiguousarray(theta, dtype=np.float32)
        _check("gc_mlp_set_params", lib().gc_mlp_set_params(
            self._h, t.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), t.size, _stream_handle(stream)))

    def get_params(self, stream=None):
        t = np.zeros(self.param_count(), np.float32)
        _check("gc_mlp_get_params", lib().gc_mlp_get_params(
            self._h, t.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), t.size, _stream_handle(stream)))
        return t

    def get_state(self, stream=None):
        """(state floats [3 * params]: parameters, Adam m, Adam v; step)."""
        st = np.zeros(3 * self.param_count(), np.float32)
        step = ctypes.c_uint64()
        _check("gc_mlp_get_state", lib().gc_mlp_get_state(
            self._h, st.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), st.size, ctypes.byref(step),
            _stream_handle(stream)))
        return st, int(step.value)

    def set_state(self, state, step, stream=None):
        st = np.ascontiguousarray(state, dtype=np.float32)
        _check("gc_mlp_set_state", lib().gc_mlp_set_state(
            self._h, st.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), st.size, int(step), _stream_handle(stream)))

    def forward(self, d_feat, n, d_logits=None, d_class=None, stream=None):
        _check("gc_mlp_forward", lib().gc_mlp_forward(self._h, _ptr(d_feat), int(n), _opt(d_logits),
                                                      _opt(d_class), _stream_handle(stream)))

    def grad(self, d_feat, d_label, batch, d_cost=None, d_index=None, lam=0.0, d_grad=None, d_loss=None,
             stream=None):
        _check("gc_mlp_grad", lib().gc_mlp_grad(self._h, _ptr(d_feat), _ptr(d_label), _opt(d_cost), _opt(d_index),
                                                int(batch), float(lam), _opt(d_grad), _opt(d_loss),
                                                _stream_handle(stream)))

    def train(self, d_feat, d_label, nindex, opts: AdamOpts, d_cost=None, d_index=None, d_loss=None, stream=None):
        _check("gc_mlp_train", lib().gc_mlp_train(self._h, _ptr(d_feat), _ptr(d_label), _opt(d_cost),
                                                  _opt(d_index), int(nindex), ctypes.byref(opts), _opt(d_loss),
                                                  _stream_handle(stream)))

    def close(self):
        if self._h:
            lib().gc_mlp_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


BLOCK_INTS = 128
BLOCK_CLASSES = 16
BLOCK_FEATURES = 40


def blockmix_bound_words(n):
    return int(lib().gc_blockmix_bound_words(int(n)))


def to_device(a_u32, device="cuda"):
    """numpy uint32 -> torch int32 device tensor with the same bits."""
    import torch
    return torch.from_numpy(np.ascontiguousarray(a_u32, dtype=np.uint32).view(np.int32)).to(device)


def to_host(t):
    return t.cpu().numpy().view(np.uint32)


class QueryPlan:
    """gc_query_plan_create / gc_query_run / gc_query_plan_destroy: AND
    queries with BM25 top-k over decoded lists.  term_len: length of every
    term's list (host); queries: (nq, terms_per_query) term indices, -1 =
    none."""

    def __init__(self, term_len, queries, ndocs, avgdl, topk=10, k1=1.2, b=0.75):
        tl = np.ascontiguousarray(term_len, dtype=np.uint32)
        qt = np.ascontiguousarray(queries, dtype=np.int32)
        self.nq, self.tpq, self.topk = int(qt.shape[0]), int(qt.shape[1]), int(topk)
        bp = BM25Params(float(k1), float(b), float(avgdl), int(topk), int(ndocs))
        self._h = ctypes.c_void_p()
        _check("gc_query_plan_create", lib().gc_query_plan_create(
            tl.ctypes.data_as(ctypes.c_void_p), tl.size, qt.ctypes.data_as(ctypes.c_void_p), self.tpq, self.nq,
            ctypes.byref(bp), ctypes.byref(self._h)))

    def run(self, d_docs, d_tfs, d_term_off, d_doclen, d_top_doc, d_top_score, stream=None):
        """d_docs / d_tfs: decoded arenas (int32), d_term_off: int64 offsets,
        d_doclen: int16 document lengths; outputs (nq * topk) int32 / float32."""
        _check("gc_query_run", lib().gc_query_run(self._h, _ptr(d_docs), _ptr(d_tfs), _ptr(d_term_off),
                                                  _ptr(d_doclen), _ptr(d_top_doc), _ptr(d_top_score),
                                                  _stream_handle(stream)))

    def close(self):
        if self._h:
            lib().gc_query_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
