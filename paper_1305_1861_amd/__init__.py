"""Exact frequent-k-mer counting on AMD Instinct MI355X (gfx950).

Thin Python binding of ``libturtle.so`` (C ABI declared in
``include/turtle.h``).  The functions carry the C names and only marshal
arguments: every step of the counting path runs in the library's HIP kernels.
PyTorch is used for device memory and streams only.

The method is the exact-count path of Turtle (Roy, Bhattacharya & Schliep,
arXiv 1305.1861, §2.1): 2-bit extraction of canonical k-mers, a
pattern-blocked Bloom screen of k-mers seen once, and sort-and-compact
counting of the survivors.

If the library has not been built the functions raise ``RuntimeError``; there
is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libturtle.so")

TK_OK, TK_EINVAL, TK_ENOMEM, TK_EDEVICE, TK_EOVERFLOW = 0, -1, -2, -3, -4
TK_FLAG_TIMING = 1
TK_FLAG_GLOBAL_FILTER = 2
STAGES = ("pack", "screen", "collect", "sort", "compact", "partition", "bucket", "fallback", "gather")

_u64 = ctypes.c_uint64
_u32 = ctypes.c_uint32
_vp = ctypes.c_void_p


class tk_options(ctypes.Structure):
    _fields_ = [("bloom_beta", _u32), ("bloom_table_bits", _u32), ("bloom_bits", _u32),
                ("flags", _u32), ("bloom_blocks", _u64), ("bloom_seed", _u64),
                ("part_bits", ctypes.c_int32), ("shard_count", _u32), ("shard_index", _u32),
                ("bucket_tile", _u32)]


class tk_result(ctypes.Structure):
    _fields_ = [("n", _u64), ("k", _u32), ("key_words", _u32),
                ("keys", ctypes.POINTER(_u64)), ("counts", ctypes.POINTER(_u32)),
                ("n_windows", _u64), ("n_collected", _u64), ("n_distinct", _u64),
                ("n_singletons", _u64), ("n_below_c", _u64), ("bloom_blocks", _u64),
                ("sort_passes", _u32), ("part_bits", ctypes.c_int32), ("n_fallback", _u64),
                ("stage_ms", ctypes.c_double * len(STAGES))]


class TurtleError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: {detail} (status {status})")
        self.status = status


_lib = None


def load_library():
    """Load libturtle.so; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_1305_1861_amd.build` (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    sigs = {
        "tk_default_options": (ctypes.c_int, [P(tk_options)]),
        "tk_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "tk_last_error": (ctypes.c_char_p, []),
        "tk_count": (ctypes.c_int, [_vp, _vp, _u64, ctypes.c_int, _u32, P(tk_options),
                                    P(P(tk_result))]),
        "tk_result_free": (None, [P(tk_result)]),
        "tk_workspace_size": (ctypes.c_int, [_u64, _u64, ctypes.c_int, _u32, P(tk_options),
                                             P(ctypes.c_size_t)]),
        "tk_count_device": (ctypes.c_int, [_vp, _vp, _u64, _u64, ctypes.c_int, _u32,
                                           P(tk_options), _vp, ctypes.c_size_t, _vp,
                                           P(tk_result)]),
        "tk_count_device_static": (ctypes.c_int, [_vp, _vp, _u64, _u64, ctypes.c_int, _u32,
                                                  P(tk_options), _vp, _vp, _u64, _vp, P(tk_result)]),
        "tk_batch_workspace_size": (ctypes.c_int, [_u64, _vp, _vp, _vp, _vp, P(tk_options),
                                                   P(ctypes.c_size_t)]),
        "tk_count_batch_device": (ctypes.c_int, [_vp, _vp, _u64, _vp, _vp, _vp, _vp,
                                                 P(tk_options), _vp, ctypes.c_size_t, _vp, _vp]),
        "tk_count_phased": (ctypes.c_int, [_vp, _vp, _u64, ctypes.c_int, _u32, _u64, _u64, P(tk_options),
                                           P(P(tk_result)), P(ctypes.c_size_t)]),
        "tk_pattern_table": (ctypes.c_int, [P(tk_options), _vp, _u64]),
        "tk_bloom_blocks": (ctypes.c_int, [_u64, _u64, ctypes.c_int, P(tk_options), P(_u64)]),
        "tk_part_bits": (ctypes.c_int, [_u64, _u64, ctypes.c_int, P(tk_options), P(ctypes.c_int)]),
        "tk_pack_device": (ctypes.c_int, [_vp, _vp, _u64, _u64, ctypes.c_int, _vp, _vp, _vp,
                                          _vp, _vp]),
        "tk_sort_scratch_size": (ctypes.c_int, [_u64, ctypes.c_int, P(ctypes.c_size_t)]),
        "tk_sort_keys_device": (ctypes.c_int, [_vp, _vp, _u64, ctypes.c_int, ctypes.c_int, _vp,
                                               ctypes.c_size_t, _vp, P(_vp)]),
        "tk_compact_scratch_size": (ctypes.c_int, [_u64, P(ctypes.c_size_t)]),
        "tk_compact_device": (ctypes.c_int, [_vp, _u64, ctypes.c_int, _u32, _vp, _vp, _vp,
                                             ctypes.c_size_t, _vp, P(_u64)]),
    }
    for name, (res, args) in sigs.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    """Names of the C entry points the binding expects the library to export."""
    return ["tk_default_options", "tk_strerror", "tk_last_error", "tk_count", "tk_result_free",
            "tk_workspace_size", "tk_count_device", "tk_count_device_static", "tk_batch_workspace_size", "tk_count_batch_device",
            "tk_count_phased", "tk_pattern_table", "tk_bloom_blocks", "tk_part_bits",
            "tk_pack_device", "tk_sort_scratch_size", "tk_sort_keys_device",
            "tk_compact_scratch_size", "tk_compact_device"]


def _check(status: int, where: str):
    if status != TK_OK:
        lib = load_library()
        detail = (lib.tk_last_error() or b"").decode() or lib.tk_strerror(status).decode()
        raise TurtleError(status, where, detail)


def _opts(opts) -> tk_options | None:
    if opts is None:
        return None
    if isinstance(opts, tk_options):
        return opts
    o = tk_default_options()
    for key, val in dict(opts).items():
        setattr(o, key, val)
    return o


def _optp(o):
    return ctypes.byref(o) if o is not None else None


def tk_default_options() -> tk_options:
    o = tk_options()
    _check(load_library().tk_default_options(ctypes.byref(o)), "tk_default_options")
    return o


def tk_strerror(status: int) -> str:
    return load_library().tk_strerror(status).decode()


def tk_last_error() -> str:
    return (load_library().tk_last_error() or b"").decode()


def tk_workspace_size(n_bases: int, n_reads: int, k: int, c: int, opts=None) -> int:
    o = _opts(opts)
    out = ctypes.c_size_t(0)
    _check(load_library().tk_workspace_size(n_bases, n_reads, k, c, _optp(o), ctypes.byref(out)),
           "tk_workspace_size")
    return int(out.value)


def tk_bloom_blocks(n_bases: int, n_reads: int, k: int, opts=None) -> int:
    o = _opts(opts)
    out = _u64(0)
    _check(load_library().tk_bloom_blocks(n_bases, n_reads, k, _optp(o), ctypes.byref(out)),
           "tk_bloom_blocks")
    return int(out.value)


def tk_part_bits(n_bases: int, n_reads: int, k: int, opts=None) -> int:
    o = _opts(opts)
    out = ctypes.c_int(0)
    _check(load_library().tk_part_bits(n_bases, n_reads, k, _optp(o), ctypes.byref(out)), "tk_part_bits")
    return int(out.value)


def tk_pattern_table(opts=None) -> np.ndarray:
    o = _opts(opts)
    bits = o.bloom_table_bits if o is not None and o.bloom_table_bits else 10
    out = np.zeros(1 << bits, np.uint64)
    _check(load_library().tk_pattern_table(_optp(o), out.ctypes.data, out.size), "tk_pattern_table")
    return out


@dataclass
class Counts:
    """Result of a counting call.  ``keys`` is ``uint64[n, key_words]``
    ({hi, lo} rows when ``key_words`` is 2); ``counts`` is ``uint32[n]``.
    For device results both are torch tensors (int64 / int32 bit patterns)
    that view the workspace; for host results both are numpy arrays."""
    keys: object
    counts: object
    k: int
    key_words: int
    n_windows: int
    n_collected: int
    n_distinct: int
    n_singletons: int
    n_below_c: int
    bloom_blocks: int
    sort_passes: int
    part_bits: int
    n_fallback: int
    stage_ms: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.counts.shape[0])


def _stats(r: tk_result) -> dict:
    return dict(k=int(r.k), key_words=int(r.key_words), n_windows=int(r.n_windows),
                n_collected=int(r.n_collected), n_distinct=int(r.n_distinct),
                n_singletons=int(r.n_singletons), n_below_c=int(r.n_below_c),
                bloom_blocks=int(r.bloom_blocks), sort_passes=int(r.sort_passes),
                part_bits=int(r.part_bits), n_fallback=int(r.n_fallback),
                stage_ms={s: float(r.stage_ms[i]) for i, s in enumerate(STAGES)})


def tk_count(bases: np.ndarray, offsets: np.ndarray, k: int, c: int, opts=None) -> Counts:
    """Count a library held in host memory (numpy ``uint8`` bases, ``uint64`` offsets)."""
    lib = load_library()
    b = np.ascontiguousarray(bases, dtype=np.uint8)
    off = np.ascontiguousarray(offsets, dtype=np.uint64)
    o = _opts(opts)
    res = ctypes.POINTER(tk_result)()
    _check(lib.tk_count(b.ctypes.data if b.size else None, off.ctypes.data, off.size - 1, k, c,
                        _optp(o), ctypes.byref(res)), "tk_count")
    try:
        r = res.contents
        n, kw = int(r.n), int(r.key_words)
        keys = np.ctypeslib.as_array(r.keys, shape=(max(n, 1) * kw,))[:n * kw].copy().reshape(n, kw)
        counts = np.ctypeslib.as_array(r.counts, shape=(max(n, 1),))[:n].copy()
        return Counts(keys, counts, **_stats(r))
    finally:
        lib.tk_result_free(res)


def tk_count_phased(bases: np.ndarray, offsets: np.ndarray, k: int, c: int, chunk_bases: int,
                    sac_capacity: int = 0, opts=None) -> Counts:
    """Phased sort-and-compact over a library in host memory, streamed in
    chunks of at most ``chunk_bases`` bases; ``sac_capacity`` bounds the
    resident (key, count) array (0: no bound).  The result's
    ``device_bytes`` is the device memory the call used."""
    lib = load_library()
    b = np.ascontiguousarray(bases, dtype=np.uint8)
    off = np.ascontiguousarray(offsets, dtype=np.uint64)
    o = _opts(opts)
    res = ctypes.POINTER(tk_result)()
    used = ctypes.c_size_t(0)
    _check(lib.tk_count_phased(b.ctypes.data if b.size else None, off.ctypes.data, off.size - 1, k, c,
                               chunk_bases, sac_capacity, _optp(o), ctypes.byref(res), ctypes.byref(used)),
           "tk_count_phased")
    try:
        r = res.contents
        n, kw = int(r.n), int(r.key_words)
        keys = np.ctypeslib.as_array(r.keys, shape=(max(n, 1) * kw,))[:n * kw].copy().reshape(n, kw)
        counts = np.ctypeslib.as_array(r.counts, shape=(max(n, 1),))[:n].copy()
        out = Counts(keys, counts, **_stats(r))
        out.device_bytes = int(used.value)
        return out
    finally:
        lib.tk_result_free(res)


def _torch():
    import torch
    return torch


def _stream_handle(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _check_device_reads(bases, offsets, n_bases_min: int = 0, n_offsets_min: int = 1):
    """Reject arguments the library would otherwise trust: the C side reads
    ``n_bases`` bytes of ``bases`` and ``n_reads + 1`` 8-byte ``offsets``."""
    torch = _torch()
    if not isinstance(bases, torch.Tensor) or not isinstance(offsets, torch.Tensor):
        raise ValueError("bases and offsets must be torch tensors")
    if bases.dtype != torch.uint8:
        raise ValueError(f"bases must be uint8, not {bases.dtype}")
    if offsets.dtype not in (torch.int64, getattr(torch, "uint64", torch.int64)):
        raise ValueError(f"offsets must be int64 or uint64 (8-byte) values, not {offsets.dtype}")
    if not bases.is_contiguous() or not offsets.is_contiguous():
        raise ValueError("bases and offsets must be contiguous")
    if offsets.numel() < n_offsets_min:
        raise ValueError(f"offsets holds {offsets.numel()} values, at least {n_offsets_min} needed")
    if bases.numel() < n_bases_min:
        raise ValueError(f"bases holds {bases.numel()} bytes, at least {n_bases_min} needed")
    if bases.device.type != "cuda" or offsets.device != bases.device:
        raise ValueError("bases and offsets must be CUDA tensors on one device")


def _check_workspace(workspace, need: int, device):
    torch = _torch()
    if not isinstance(workspace, torch.Tensor) or workspace.dtype != torch.uint8 or not workspace.is_contiguous():
        raise ValueError("workspace must be a contiguous uint8 tensor")
    if workspace.numel() < need:
        raise ValueError(f"workspace of {workspace.numel()} bytes is below the {need} needed")
    if workspace.device != device:
        raise ValueError("workspace must be on the device of the reads")


def tk_count_device(bases, offsets, k: int, c: int, opts=None, workspace=None, stream=None) -> Counts:
    """Count a library held in device memory.

    ``bases``: CUDA ``uint8`` tensor; ``offsets``: CUDA ``int64``/``uint64``
    tensor of n_reads + 1 values.  ``workspace``: optional CUDA ``uint8``
    tensor of at least ``tk_workspace_size`` bytes (allocated here if None).
    Returned keys/counts are views into the workspace.
    """
    torch = _torch()
    lib = load_library()
    _check_device_reads(bases, offsets)
    n_bases = int(bases.numel())
    n_reads = int(offsets.numel()) - 1
    o = _opts(opts)
    need = tk_workspace_size(n_bases, n_reads, k, c, o)
    if workspace is None:
        workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=bases.device)
    _check_workspace(workspace, need, bases.device)
    r = tk_result()
    _check(lib.tk_count_device(ctypes.c_void_p(bases.data_ptr()) if n_bases else None,
                               ctypes.c_void_p(offsets.data_ptr()), n_bases, n_reads, k, c,
                               _optp(o), ctypes.c_void_p(workspace.data_ptr()),
                               workspace.numel(), _stream_handle(stream), ctypes.byref(r)),
           "tk_count_device")
    n, kw = int(r.n), int(r.key_words)
    base = workspace.data_ptr()
    ko = ctypes.cast(r.keys, ctypes.c_void_p).value - base if n else 0
    co = ctypes.cast(r.counts, ctypes.c_void_p).value - base if n else 0
    keys = workspace[ko:ko + n * kw * 8].view(torch.int64).view(n, kw)
    counts = workspace[co:co + n * 4].view(torch.int32)
    out = Counts(keys, counts, **_stats(r))
    out.workspace = workspace
    return out


STATIC_WORKSPACE_BYTES = 256 << 20


def tk_count_device_static(bases, offsets, k: int, c: int, out_keys, out_counts, opts=None,
                           stream=None) -> Counts:
    """Count a library held in device memory with the library's static
    workspace (no device allocation anywhere in the call).  ``out_keys``:
    CUDA int64 tensor of at least n_records * key_words entries;
    ``out_counts``: CUDA int32 tensor of at least n_records entries (n_bases
    entries always suffice).  Returned keys/counts view these tensors."""
    torch = _torch()
    lib = load_library()
    _check_device_reads(bases, offsets)
    n_bases = int(bases.numel())
    n_reads = int(offsets.numel()) - 1
    kw = 1 if k <= 31 else 2
    for t, dt in ((out_keys, torch.int64), (out_counts, torch.int32)):
        if not isinstance(t, torch.Tensor) or t.dtype != dt or not t.is_contiguous() or t.device != bases.device:
            raise ValueError(f"output buffers must be contiguous {dt} tensors on the device of the reads")
    cap = min(int(out_keys.numel()) // kw, int(out_counts.numel()))
    o = _opts(opts)
    r = tk_result()
    _check(lib.tk_count_device_static(ctypes.c_void_p(bases.data_ptr()) if n_bases else None,
                                      ctypes.c_void_p(offsets.data_ptr()), n_bases, n_reads, k, c, _optp(o),
                                      ctypes.c_void_p(out_keys.data_ptr()), ctypes.c_void_p(out_counts.data_ptr()),
                                      cap, _stream_handle(stream), ctypes.byref(r)),
           "tk_count_device_static")
    n = int(r.n)
    return Counts(out_keys[:n * kw].view(n, kw), out_counts[:n], **_stats(r))


def _batch_arrays(lib_bases, lib_reads, k, c):
    lb = np.ascontiguousarray(np.asarray(lib_bases, dtype=np.uint64))
    lr = np.ascontiguousarray(np.asarray(lib_reads, dtype=np.uint64))
    n_libs = lb.size - 1
    if n_libs < 1 or lr.size != lb.size:
        raise ValueError("lib_bases and lib_reads need n_libs + 1 entries each")
    cc = np.full(n_libs, c, np.uint32) if np.isscalar(c) else np.ascontiguousarray(np.asarray(c, dtype=np.uint32))
    kk = np.full(n_libs, k, np.int32) if np.isscalar(k) else np.ascontiguousarray(np.asarray(k, dtype=np.int32))
    if cc.size != n_libs or kk.size != n_libs:
        raise ValueError("k and c need one value (or one per library)")
    return n_libs, lb, lr, kk, cc


def _batch_options(opts, lb, kk):
    """Explicit options, else the autotuner's cached choice for the batch's
    largest library (batch-wide options only; every library keeps the size
    rule's D) when the cache file ``$TK_TUNE_CACHE`` is set, else None."""
    if opts is not None or not os.environ.get("TK_TUNE_CACHE"):
        return _opts(opts)
    from .tune import cached_options
    sizes = np.diff(lb.astype(np.int64))
    j = int(np.argmax(sizes))
    return cached_options(int(kk[j]), int(sizes[j]), with_part_bits=False)


def tk_batch_workspace_size(lib_bases, lib_reads, k, c, opts=None) -> int:
    """Workspace bytes of tk_count_batch_device for these library boundaries
    (``k`` and ``c``: one value or one per library)."""
    n_libs, lb, lr, kk, cc = _batch_arrays(lib_bases, lib_reads, k, c)
    o = _batch_options(opts, lb, kk)
    out = ctypes.c_size_t(0)
    _check(load_library().tk_batch_workspace_size(n_libs, lb.ctypes.data, lr.ctypes.data, kk.ctypes.data,
                                                  cc.ctypes.data, _optp(o), ctypes.byref(out)),
           "tk_batch_workspace_size")
    return int(out.value)


def tk_count_batch_device(bases, offsets, lib_bases, lib_reads, k, c, opts=None, workspace=None,
                          stream=None) -> list:
    """Count a batch of libraries held in device memory (one bases/offsets
    pair; library j owns reads lib_reads[j]..lib_reads[j+1] and bases
    lib_bases[j]..lib_bases[j+1]).  ``k`` and ``c``: one value or one per
    library.  ``opts=None``: the autotuner's cached choice when
    ``$TK_TUNE_CACHE`` names a cache file (see ``tune``), else the defaults.
    Returns one Counts per library, viewing the workspace."""
    torch = _torch()
    lib = load_library()
    n_libs, lb, lr, kk, cc = _batch_arrays(lib_bases, lib_reads, k, c)
    _check_device_reads(bases, offsets, int(lb[-1]), int(lr[-1]) + 1)
    o = _batch_options(opts, lb, kk)
    need = tk_batch_workspace_size(lb, lr, kk, cc, o)
    if workspace is None:
        workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=bases.device)
    _check_workspace(workspace, need, bases.device)
    res = (tk_result * n_libs)()
    n_bases = int(bases.numel())
    _check(lib.tk_count_batch_device(ctypes.c_void_p(bases.data_ptr()) if n_bases else None,
                                     ctypes.c_void_p(offsets.data_ptr()), n_libs, lb.ctypes.data, lr.ctypes.data,
                                     kk.ctypes.data, cc.ctypes.data, _optp(o), ctypes.c_void_p(workspace.data_ptr()),
                                     workspace.numel(), _stream_handle(stream), res),
           "tk_count_batch_device")
    base = workspace.data_ptr()
    outs = []
    for r in res:
        n, kw = int(r.n), int(r.key_words)
        ko = ctypes.cast(r.keys, ctypes.c_void_p).value - base if n else 0
        co = ctypes.cast(r.counts, ctypes.c_void_p).value - base if n else 0
        keys = workspace[ko:ko + n * kw * 8].view(torch.int64).view(n, kw)
        counts = workspace[co:co + n * 4].view(torch.int32)
        out = Counts(keys, counts, **_stats(r))
        out.workspace = workspace
        outs.append(out)
    return outs


def tk_pack_device(bases, offsets, k: int, stream=None):
    """2-bit packing stage: returns (packed int64[n_words], valid int32[n_words], n_windows)."""
    torch = _torch()
    lib = load_library()
    n_bases = int(bases.numel())
    n_reads = int(offsets.numel()) - 1
    n_words = (n_bases + 31) // 32
    dev = bases.device
    packed = torch.empty(max(n_words, 1), dtype=torch.int64, device=dev)
    valid = torch.empty(max(n_words, 1), dtype=torch.int32, device=dev)
    scratch = torch.empty(max(n_words, 1), dtype=torch.int32, device=dev)
    nw = torch.zeros(1, dtype=torch.int64, device=dev)
    _check(lib.tk_pack_device(ctypes.c_void_p(bases.data_ptr()) if n_bases else None,
                              ctypes.c_void_p(offsets.data_ptr()), n_bases, n_reads, k,
                              ctypes.c_void_p(packed.data_ptr()), ctypes.c_void_p(valid.data_ptr()),
                              ctypes.c_void_p(scratch.data_ptr()), ctypes.c_void_p(nw.data_ptr()),
                              _stream_handle(stream)), "tk_pack_device")
    return packed[:n_words], valid[:n_words], nw


def tk_sort_keys_device(keys, key_words: int, key_bits: int, stream=None):
    """Radix-sort stage on a CUDA int64 tensor of n * key_words words; returns the sorted tensor."""
    torch = _torch()
    lib = load_library()
    n = int(keys.numel()) // key_words
    keys = keys.contiguous()
    alt = torch.empty_like(keys)
    need = ctypes.c_size_t(0)
    _check(lib.tk_sort_scratch_size(n, key_words, ctypes.byref(need)), "tk_sort_scratch_size")
    scratch = torch.empty(max(int(need.value), 256), dtype=torch.uint8, device=keys.device)
    out = ctypes.c_void_p(0)
    _check(lib.tk_sort_keys_device(ctypes.c_void_p(keys.data_ptr()), ctypes.c_void_p(alt.data_ptr()),
                                   n, key_words, key_bits, ctypes.c_void_p(scratch.data_ptr()),
                                   scratch.numel(), _stream_handle(stream), ctypes.byref(out)),
           "tk_sort_keys_device")
    return keys if out.value == keys.data_ptr() else alt


def tk_compact_device(keys, key_words: int, c: int, stream=None):
    """Run-length stage on sorted keys: (out_keys, out_counts, stats dict)."""
    torch = _torch()
    lib = load_library()
    n = int(keys.numel()) // key_words
    keys = keys.contiguous()
    out_keys = torch.empty(max(n, 1) * key_words, dtype=torch.int64, device=keys.device)
    out_counts = torch.empty(max(n, 1), dtype=torch.int32, device=keys.device)
    need = ctypes.c_size_t(0)
    _check(lib.tk_compact_scratch_size(n, ctypes.byref(need)), "tk_compact_scratch_size")
    scratch = torch.empty(max(int(need.value), 256), dtype=torch.uint8, device=keys.device)
    stats = (_u64 * 4)()
    _check(lib.tk_compact_device(ctypes.c_void_p(keys.data_ptr()) if n else None, n, key_words, c,
                                 ctypes.c_void_p(out_keys.data_ptr()),
                                 ctypes.c_void_p(out_counts.data_ptr()),
                                 ctypes.c_void_p(scratch.data_ptr()), scratch.numel(),
                                 _stream_handle(stream), stats), "tk_compact_device")
    m = int(stats[0])
    return (out_keys[:m * key_words].view(m, key_words), out_counts[:m],
            dict(n_out=m, n_distinct=int(stats[1]), n_singletons=int(stats[2]),
                 n_below_c=int(stats[3])))
