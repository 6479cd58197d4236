"""Exact multi-pattern log matching on MI355X (failureless-trie walk, arXiv 1704.02278).

A thin ctypes binding over ``libglop.so`` (the C-ABI in ``include/glop.h``).
It only marshals arguments: tensors become device pointers, lists of bytes
become pointer arrays; every step of the matching runs in the library's HIP
kernels.  There is no fallback: if the library is missing, importing this
package raises ImportError.

Functions with the C names (``glop_build``, ``glop_match`` ...) mirror the
C-ABI one to one; ``Dict`` is a convenience wrapper for torch tensors.
"""

from __future__ import annotations

import ctypes
from pathlib import Path

# torch first: it loads its HIP runtime (soname libamdhip64.so.7), which
# libglop.so then binds to, so streams and events are shared with torch.
import torch  # noqa: F401

_PKG = Path(__file__).resolve().parent
LIB_PATH = _PKG / "libglop.so"

if not LIB_PATH.exists():
    raise ImportError(f"{LIB_PATH} is not built; run `python paper_1704_02278_amd/build.py`")

GLOP_OK = 0
GLOP_EINVAL = -1
GLOP_ENOMEM = -2
GLOP_EHIP = -3
GLOP_ETOOLONG = -4
GLOP_ENODEV = -5
GLOP_EINTERNAL = -6
GLOP_SERVE_BATCHED = 0
GLOP_SERVE_PLAIN = 1
GLOP_PREFIX_FULL = 0xFFFFFFFF
GLOP_FILTER_AUTO = 0
GLOP_FILTER_NONE = 1
GLOP_FILTER_QGRAM = 2
GLOP_LAYOUT_AUTO = 0
GLOP_LAYOUT_DENSE = 1
GLOP_LAYOUT_HYBRID = 2
GLOP_PLACE_AUTO = 0
GLOP_PLACE_GLOBAL = 1
GLOP_PLACE_LDS = 2
GLOP_MAX_PATTERN_LEN = 65535
MATCH_RECORD_BYTES = 16


class glop_match_t(ctypes.Structure):
    _fields_ = [("offset", ctypes.c_uint64), ("pattern_id", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class glop_build_opts(ctypes.Structure):
    _fields_ = [("filter", ctypes.c_int32), ("stride", ctypes.c_uint32), ("qgram", ctypes.c_uint32),
                ("bitmap_log2", ctypes.c_uint32), ("probe_bits", ctypes.c_uint32), ("tile_kib", ctypes.c_uint32),
                ("prefix_len", ctypes.c_uint32), ("candidates", ctypes.c_uint32), ("layout", ctypes.c_uint32),
                ("placement", ctypes.c_uint32)]


class glop_chunk_t(ctypes.Structure):
    _fields_ = [("text", ctypes.c_void_p), ("len", ctypes.c_uint64)]


class glop_batch_match_t(ctypes.Structure):
    _fields_ = [("offset", ctypes.c_uint64), ("pattern_id", ctypes.c_uint32), ("chunk", ctypes.c_uint32)]


class glop_events_t(ctypes.Structure):
    _fields_ = [("scan_begin", ctypes.c_void_p), ("scan_end", ctypes.c_void_p), ("emit_end", ctypes.c_void_p)]


class glop_tune_result_t(ctypes.Structure):
    _fields_ = [("opts", glop_build_opts), ("ms", ctypes.c_float), ("auto_ms", ctypes.c_float),
                ("evaluated", ctypes.c_uint32), ("from_cache", ctypes.c_uint32)]


class glop_server_opts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("max_inflight", ctypes.c_uint32), ("max_batch_requests", ctypes.c_uint32),
                ("max_batch_bytes", ctypes.c_uint64), ("hbm_budget_bytes", ctypes.c_uint64),
                ("count_payload", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class glop_completion_t(ctypes.Structure):
    _fields_ = [("request_id", ctypes.c_uint64), ("tag", ctypes.c_uint64), ("dict", ctypes.c_uint32),
                ("truncated", ctypes.c_uint32), ("matches", ctypes.c_uint64), ("records", ctypes.c_uint64),
                ("d_records", ctypes.c_void_p), ("arrival_ns", ctypes.c_int64), ("launch_ns", ctypes.c_int64),
                ("done_ns", ctypes.c_int64), ("batch_requests", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class glop_info_t(ctypes.Structure):
    _fields_ = [
        ("num_patterns", ctypes.c_uint32), ("min_len", ctypes.c_uint32), ("max_len", ctypes.c_uint32),
        ("num_classes", ctypes.c_uint32), ("num_states", ctypes.c_uint64), ("table_bytes", ctypes.c_uint64),
        ("outlist_ids", ctypes.c_uint64), ("filter", ctypes.c_int32), ("stride", ctypes.c_uint32),
        ("qgram", ctypes.c_uint32), ("bitmap_log2", ctypes.c_uint32), ("probe_bits", ctypes.c_uint32),
        ("tile_kib", ctypes.c_uint32), ("filter_keys", ctypes.c_uint64),
        ("prefix_len", ctypes.c_uint32), ("candidates", ctypes.c_uint32),
        ("device_bytes", ctypes.c_uint64), ("device", ctypes.c_int32),
        ("prefix_keys", ctypes.c_uint32), ("prefix_slots", ctypes.c_uint32), ("prefix_depth", ctypes.c_uint32),
        ("filter2_log2", ctypes.c_uint32), ("layout", ctypes.c_uint32), ("placement", ctypes.c_uint32),
        ("dense_states", ctypes.c_uint64),
    ]


_u8pp = ctypes.POINTER(ctypes.c_void_p)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_vp = ctypes.c_void_p
_u64 = ctypes.c_uint64

_lib = ctypes.CDLL(str(LIB_PATH))
_SIGNATURES = {
    "glop_build": (_vp, [_u8pp, _u32p, ctypes.c_uint32]),
    "glop_build_ex": (_vp, [_u8pp, _u32p, ctypes.c_uint32, ctypes.POINTER(glop_build_opts)]),
    "glop_compile": (_vp, [_u8pp, _u32p, ctypes.c_uint32, ctypes.POINTER(glop_build_opts)]),
    "glop_free": (None, [_vp]),
    "glop_match": (ctypes.c_int, [_vp, _vp, _u64, _vp, _u64, _vp, _vp]),
    "glop_workspace_bytes": (_u64, [_vp, _u64]),
    "glop_match_ws": (ctypes.c_int, [_vp, _vp, _u64, _vp, _u64, _vp, _vp, _vp, _u64, _vp,
                                     ctypes.POINTER(glop_events_t)]),
    "glop_match_host": (ctypes.c_int, [_vp, _vp, _u64, _vp, _u64, _vp, _vp, _u64, _vp]),
    "glop_match_static": (ctypes.c_int, [_vp, _vp, _u64, _vp, _u64, _vp, _vp, _vp]),
    "glop_static_max_len": (_u64, [_vp]),
    "glop_batch_workspace_bytes": (_u64, [_vp, ctypes.c_uint32, _u64]),
    "glop_match_batch": (ctypes.c_int, [_vp, _vp, ctypes.c_uint32, _u64, _vp, _u64, _vp, _vp, _vp, _vp, _vp, _u64,
                                        _vp]),
    "glop_match_batch_sliced": (ctypes.c_int, [_vp, _vp, ctypes.c_uint32, _u64, _vp, _u64, _vp, _vp, _vp, _vp, _vp,
                                               _vp, _vp, _u64, _vp]),
    "glop_cpu_walk": (ctypes.c_int, [_vp, _vp, _u64, _vp, _u64, _vp, _vp, ctypes.c_int]),
    "glop_get_info": (ctypes.c_int, [_vp, ctypes.POINTER(glop_info_t)]),
    "glop_num_patterns": (ctypes.c_uint32, [_vp]),
    "glop_max_len": (ctypes.c_uint32, [_vp]),
    "glop_stream_read": (ctypes.c_int, [_vp, _u64, _vp, _vp]),
    "glop_autotune": (ctypes.c_int, [_u8pp, _u32p, ctypes.c_uint32, _vp, _u64, _vp,
                                     ctypes.POINTER(glop_tune_result_t)]),
    "glop_server_create": (_vp, [ctypes.POINTER(glop_server_opts)]),
    "glop_server_add_dict": (ctypes.c_int, [_vp, _vp, ctypes.POINTER(ctypes.c_uint32)]),
    "glop_server_submit": (ctypes.c_int, [_vp, ctypes.c_uint32, _vp, _u64, _u64, ctypes.c_int64,
                                          ctypes.POINTER(_u64)]),
    "glop_server_poll": (ctypes.c_int, [_vp, ctypes.POINTER(glop_completion_t), ctypes.c_uint32, ctypes.c_uint32,
                                        ctypes.POINTER(ctypes.c_uint32)]),
    "glop_server_release": (ctypes.c_int, [_vp, _u64]),
    "glop_server_destroy": (None, [_vp]),
    "glop_now_ns": (ctypes.c_int64, []),
    "glop_server_run_trace": (ctypes.c_int, [_vp, ctypes.c_uint32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                             _vp, _vp, ctypes.POINTER(ctypes.c_int64)]),
    "glop_last_error": (ctypes.c_int, []),
    "glop_last_error_message": (ctypes.c_char_p, []),
    "glop_strerror": (ctypes.c_char_p, [ctypes.c_int]),
}
for _name, (_res, _args) in _SIGNATURES.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args
    globals()[_name] = _f

EXPORTED = tuple(_SIGNATURES)


class GlopError(RuntimeError):
    def __init__(self, code: int, what: str):
        msg = (glop_last_error_message() or b"").decode(errors="replace")
        super().__init__(f"{what}: {glop_strerror(code).decode()} ({code}): {msg}")
        self.code = code


def _check(rc: int, what: str):
    if rc != GLOP_OK:
        raise GlopError(rc, what)


def _pattern_arrays(patterns):
    pats = [bytes(p) for p in patterns]
    keep = [ctypes.create_string_buffer(p, len(p)) for p in pats]
    ptrs = (ctypes.c_void_p * max(1, len(pats)))(*[ctypes.addressof(b) for b in keep])
    lens = (ctypes.c_uint32 * max(1, len(pats)))(*[len(p) for p in pats])
    return keep, ptrs, lens, len(pats)


def _opts(filter=GLOP_FILTER_AUTO, stride=0, qgram=0, bitmap_log2=0, probe_bits=0, tile_kib=0, prefix_len=0,
          candidates=False, layout=GLOP_LAYOUT_AUTO, placement=GLOP_PLACE_AUTO):
    return glop_build_opts(int(filter), int(stride), int(qgram), int(bitmap_log2), int(probe_bits), int(tile_kib),
                           int(prefix_len), 1 if candidates else 0, int(layout), int(placement))


class Dict:
    """A compiled dictionary on the current device (or host-only with ``device=False``)."""

    def __init__(self, patterns, *, device: bool = True, filter=GLOP_FILTER_AUTO, stride=0, qgram=0,
                 bitmap_log2=0, probe_bits=0, tile_kib=0, prefix_len=0, candidates=False, layout=GLOP_LAYOUT_AUTO,
                 placement=GLOP_PLACE_AUTO):
        keep, ptrs, lens, n = _pattern_arrays(patterns)
        opts = _opts(filter, stride, qgram, bitmap_log2, probe_bits, tile_kib, prefix_len, candidates, layout,
                     placement)
        fn = glop_build_ex if device else glop_compile
        h = fn(ctypes.cast(ptrs, _u8pp), lens, n, ctypes.byref(opts))
        if not h:
            raise GlopError(glop_last_error(), "glop_build_ex" if device else "glop_compile")
        self._h = ctypes.c_void_p(h)
        self.num_patterns = int(glop_num_patterns(self._h))
        self.max_len = int(glop_max_len(self._h))
        self.pattern_lengths = [len(p) for p in patterns]
        del keep

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        out = glop_info_t()
        _check(glop_get_info(self._h, ctypes.byref(out)), "glop_get_info")
        return {name: getattr(out, name) for name, _ in glop_info_t._fields_}

    def workspace_bytes(self, length: int) -> int:
        return int(glop_workspace_bytes(self._h, int(length)))

    def match_into(self, text, out, counts, *, max_matches=None, total=None, workspace=None, stream=None,
                   events=None, length=None):
        """Enqueue a match into caller-owned tensors (no allocation, no sync).

        text: uint8 CUDA tensor; out: int64 CUDA tensor [cap, 2] (16-byte
        records); counts: int64 CUDA tensor [n]; total: int64 CUDA tensor [1]
        or None; workspace: uint8 CUDA tensor of >= workspace_bytes(len)
        bytes (None = let the library allocate on the stream).
        """
        import torch

        n = int(text.numel()) if length is None else int(length)
        cap = int(out.shape[0]) if max_matches is None else int(max_matches)
        s = (stream if stream is not None else torch.cuda.current_stream()).cuda_stream
        if workspace is None:
            _check(glop_match(self._h, text.data_ptr(), n, out.data_ptr(), cap, counts.data_ptr(), s),
                   "glop_match")
            return
        ev = None
        if events is not None:
            ev = ctypes.byref(glop_events_t(*events))
        _check(glop_match_ws(self._h, text.data_ptr(), n, out.data_ptr(), cap, counts.data_ptr(),
                             total.data_ptr() if total is not None else None, workspace.data_ptr(),
                             int(workspace.numel()), s, ev), "glop_match_ws")

    def match(self, text, max_matches=None, stream=None):
        """Match a uint8 CUDA tensor; returns (offsets i64[M], ids i64[M], counts i64[n], total).

        With ``max_matches=None`` the output is sized to fit every match (a
        second pass runs if the first guess was short; this synchronises).
        ``offsets`` and ``ids`` are views of the 16-byte records (the id column
        holds pattern_id with the zero ``reserved`` word above it).
        """
        import torch

        dev = text.device
        n = int(text.numel())
        counts = torch.empty(max(1, self.num_patterns), dtype=torch.int64, device=dev)
        total = torch.zeros(1, dtype=torch.int64, device=dev)
        ws = torch.empty(self.workspace_bytes(n) + 256, dtype=torch.uint8, device=dev)
        ws = ws[(-ws.data_ptr()) % 256:]
        cap = max(1024, n // 1024) if max_matches is None else int(max_matches)
        out = torch.empty((max(cap, 1), 2), dtype=torch.int64, device=dev)
        self.match_into(text, out, counts, max_matches=cap, total=total, workspace=ws, stream=stream)
        got = int(total.item())
        if max_matches is None and got > cap:
            cap = got
            out = torch.empty((cap, 2), dtype=torch.int64, device=dev)
            self.match_into(text, out, counts, max_matches=cap, total=total, workspace=ws, stream=stream)
            got = int(total.item())
        k = min(cap, got)
        return out[:k, 0], out[:k, 1], counts[: self.num_patterns], got

    def match_host(self, text, max_matches=None, chunk_bytes=0, stream=None):
        """Match a host (numpy uint8) text streamed through pinned buffers
        (glop_match_host); returns (offsets, ids, counts, total) on the device,
        like ``match``.  ``max_matches=None`` sizes the output (a second pass
        streams the text again if the first guess was short)."""
        import numpy as np
        import torch

        t = np.ascontiguousarray(text, dtype=np.uint8)
        n = int(t.size)
        dev = torch.device("cuda", torch.cuda.current_device())
        counts = torch.empty(max(1, self.num_patterns), dtype=torch.int64, device=dev)
        total = torch.zeros(1, dtype=torch.int64, device=dev)
        cap = max(1024, n // 1024) if max_matches is None else int(max_matches)
        out = torch.empty((max(cap, 1), 2), dtype=torch.int64, device=dev)
        s = (stream if stream is not None else torch.cuda.current_stream()).cuda_stream
        _check(glop_match_host(self._h, t.ctypes.data if n else None, n, out.data_ptr(), cap, counts.data_ptr(),
                               total.data_ptr(), int(chunk_bytes), s), "glop_match_host")
        got = int(total.item())
        if max_matches is None and got > cap:
            cap = got
            out = torch.empty((cap, 2), dtype=torch.int64, device=dev)
            _check(glop_match_host(self._h, t.ctypes.data if n else None, n, out.data_ptr(), cap,
                                   counts.data_ptr(), total.data_ptr(), int(chunk_bytes), s), "glop_match_host")
            got = int(total.item())
        k = min(cap, got)
        return out[:k, 0], out[:k, 1], counts[: self.num_patterns], got

    def batch_workspace_bytes(self, nchunks: int, max_total_bytes: int) -> int:
        return int(glop_batch_workspace_bytes(self._h, int(nchunks), int(max_total_bytes)))

    def match_batch_into(self, chunk_table, nchunks, max_total_bytes, out, chunk_first, chunk_count, counts, total,
                         workspace, *, max_matches=None, stream=None):
        """Enqueue a batch into caller-owned CUDA tensors (no allocation, no sync).

        chunk_table: int64 CUDA tensor [nchunks, 2] of (device pointer, length);
        out: int64 CUDA tensor [cap, 2] (16-byte records: offset, pattern id |
        chunk << 32); chunk_first, chunk_count: int64 [nchunks]; counts: int64
        [n]; total: int64 [1]; workspace: uint8 CUDA tensor, 256-byte aligned.
        """
        import torch

        cap = int(out.shape[0]) if max_matches is None else int(max_matches)
        s = (stream if stream is not None else torch.cuda.current_stream()).cuda_stream
        _check(glop_match_batch(self._h, chunk_table.data_ptr(), int(nchunks), int(max_total_bytes),
                                out.data_ptr(), cap, chunk_first.data_ptr(), chunk_count.data_ptr(),
                                counts.data_ptr(), total.data_ptr(), workspace.data_ptr(), int(workspace.numel()),
                                s), "glop_match_batch")

    def match_batch_sliced_into(self, chunk_table, nchunks, max_total_bytes, out, slice_first, slice_cap,
                                chunk_first, chunk_count, counts, total, workspace, *, stream=None):
        """``match_batch_into`` with a fixed output slice per chunk: chunk c's
        first min(count, slice_cap[c]) records go to out[slice_first[c]:]
        (slice_first, slice_cap: int64 CUDA tensors [nchunks])."""
        import torch

        s = (stream if stream is not None else torch.cuda.current_stream()).cuda_stream
        _check(glop_match_batch_sliced(self._h, chunk_table.data_ptr(), int(nchunks), int(max_total_bytes),
                                       out.data_ptr(), int(out.shape[0]), slice_first.data_ptr(),
                                       slice_cap.data_ptr(), chunk_first.data_ptr(), chunk_count.data_ptr(),
                                       counts.data_ptr(), total.data_ptr(), workspace.data_ptr(),
                                       int(workspace.numel()), s), "glop_match_batch_sliced")

    def match_batch(self, chunks, max_matches=None, stream=None):
        """Match a list of uint8 CUDA tensors as one batch.

        Returns (offsets, ids, chunk_ids, chunk_first, chunk_count, counts,
        total); the first three are views of the records (chunk order, then
        offset, then id).  With ``max_matches=None`` the output is sized to
        fit (this synchronises).
        """
        import torch

        dev = chunks[0].device
        n = len(chunks)
        table = torch.tensor([[c.data_ptr() if c.numel() else 0, c.numel()] for c in chunks], dtype=torch.int64)
        table = table.to(dev)
        total_bytes = sum(int(c.numel()) for c in chunks)
        first = torch.empty(n, dtype=torch.int64, device=dev)
        count = torch.empty(n, dtype=torch.int64, device=dev)
        counts = torch.empty(max(1, self.num_patterns), dtype=torch.int64, device=dev)
        total = torch.zeros(1, dtype=torch.int64, device=dev)
        wsb = self.batch_workspace_bytes(n, total_bytes)
        ws = torch.empty(wsb + 256, dtype=torch.uint8, device=dev)
        ws = ws[(-ws.data_ptr()) % 256:]
        cap = max(1024, total_bytes // 1024) if max_matches is None else int(max_matches)
        out = torch.empty((max(cap, 1), 2), dtype=torch.int64, device=dev)
        self.match_batch_into(table, n, total_bytes, out, first, count, counts, total, ws, max_matches=cap,
                              stream=stream)
        got = int(total.item())
        if max_matches is None and got > cap:
            cap = got
            out = torch.empty((cap, 2), dtype=torch.int64, device=dev)
            self.match_batch_into(table, n, total_bytes, out, first, count, counts, total, ws, max_matches=cap,
                                  stream=stream)
            got = int(total.item())
        k = min(cap, got)
        rec = out[:k]
        return (rec[:, 0], rec[:, 1] & 0xFFFFFFFF, rec[:, 1] >> 32, first, count, counts[: self.num_patterns],
                got)

    def cpu_walk(self, text, threads: int = 1, max_matches=None):
        """Failureless-trie walk on the host (baseline); returns numpy arrays like ``match``."""
        import numpy as np

        t = np.frombuffer(bytes(text), dtype=np.uint8) if not isinstance(text, np.ndarray) else text
        t = np.ascontiguousarray(t)
        counts = np.zeros(max(1, self.num_patterns), dtype=np.uint64)
        total = ctypes.c_uint64(0)
        if max_matches is None:
            _check(glop_cpu_walk(self._h, t.ctypes.data, t.size, None, 0, counts.ctypes.data,
                                 ctypes.byref(total), threads), "glop_cpu_walk")
            max_matches = total.value
        rec = np.zeros((max(1, max_matches), 2), dtype=np.uint64)
        _check(glop_cpu_walk(self._h, t.ctypes.data, t.size, rec.ctypes.data, max_matches, counts.ctypes.data,
                             ctypes.byref(total), threads), "glop_cpu_walk")
        k = min(max_matches, total.value)
        return rec[:k, 0], rec[:k, 1] & np.uint64(0xFFFFFFFF), counts[: self.num_patterns], int(total.value)

    def close(self):
        if getattr(self, "_h", None):
            glop_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build(patterns, **opts) -> Dict:
    return Dict(patterns, **opts)


def stream_read(data, sink, stream=None):
    """Enqueue one read of a 16-byte aligned uint8 CUDA tensor (the HBM read
    ceiling the matcher is compared with); ``sink`` is an int64 CUDA tensor [1]."""
    import torch

    s = (stream if stream is not None else torch.cuda.current_stream()).cuda_stream
    _check(glop_stream_read(data.data_ptr(), int(data.numel()), sink.data_ptr(), s), "glop_stream_read")


def autotune(patterns, sample, stream=None) -> dict:
    """Time build options for ``patterns`` on ``sample`` (a uint8 CUDA tensor of
    representative text) and return the fastest: {"opts": {...}, "ms",
    "auto_ms", "evaluated", "from_cache"}.  ``Dict(patterns, **r["opts"])``
    builds with them."""
    import torch

    keep, ptrs, lens, n = _pattern_arrays(patterns)
    s = (stream if stream is not None else torch.cuda.current_stream()).cuda_stream
    r = glop_tune_result_t()
    _check(glop_autotune(ctypes.cast(ptrs, _u8pp), lens, n, sample.data_ptr(), int(sample.numel()), s,
                         ctypes.byref(r)), "glop_autotune")
    del keep
    o = r.opts
    return {"opts": {"filter": o.filter, "stride": o.stride, "qgram": o.qgram, "bitmap_log2": o.bitmap_log2,
                     "probe_bits": o.probe_bits, "tile_kib": o.tile_kib, "prefix_len": o.prefix_len,
                     "layout": o.layout, "placement": o.placement},
            "ms": float(r.ms), "auto_ms": float(r.auto_ms), "evaluated": int(r.evaluated),
            "from_cache": bool(r.from_cache)}


class Server:
    """Resident dictionaries matched as requests arrive (continuous batching).

    ``Server(dicts, mode=GLOP_SERVE_BATCHED, hbm_budget_bytes=..., ...)`` with
    ``dicts`` a list of ``Dict``; ``submit`` / ``poll`` / ``release`` map to the
    C calls, and ``run_trace`` replays an open-loop trace natively.
    """

    def __init__(self, dicts, *, mode=GLOP_SERVE_BATCHED, max_inflight=0, max_batch_requests=0, max_batch_bytes=0,
                 hbm_budget_bytes=0, count_payload=True):
        o = glop_server_opts(mode, max_inflight, max_batch_requests, max_batch_bytes, hbm_budget_bytes,
                             1 if count_payload else 0, 0)
        h = glop_server_create(ctypes.byref(o))
        if not h:
            raise GlopError(glop_last_error(), "glop_server_create")
        self._s = ctypes.c_void_p(h)
        self.dicts = list(dicts)
        for d in self.dicts:
            k = ctypes.c_uint32()
            _check(glop_server_add_dict(self._s, d.handle, ctypes.byref(k)), "glop_server_add_dict")

    def submit(self, dict_index, text, tag=0, length=None, arrival_ns=-1) -> int:
        rid = ctypes.c_uint64()
        n = int(text.numel()) if length is None else int(length)
        _check(glop_server_submit(self._s, dict_index, text.data_ptr() if n else None, n, tag, arrival_ns,
                                  ctypes.byref(rid)), "glop_server_submit")
        return rid.value

    def poll(self, max_n=256, wait_us=1000):
        buf = (glop_completion_t * max_n)()
        got = ctypes.c_uint32()
        _check(glop_server_poll(self._s, buf, max_n, wait_us, ctypes.byref(got)), "glop_server_poll")
        return [buf[k] for k in range(got.value)]

    def release(self, request_id):
        _check(glop_server_release(self._s, request_id), "glop_server_release")

    def run_trace(self, dicts, texts, lengths, at_ns, copy_out=None, copy_base=None, copy_cap=None):
        """Replay n requests (device pointers ``texts``); returns (latency_ns, matches,
        truncated, batch_requests, wall_ns) as numpy arrays / int."""
        import numpy as np

        n = len(lengths)
        dk = np.ascontiguousarray(dicts, dtype=np.uint32)
        tx = np.ascontiguousarray(texts, dtype=np.uint64)
        ln = np.ascontiguousarray(lengths, dtype=np.uint64)
        at = np.ascontiguousarray(at_ns, dtype=np.int64)
        lat = np.zeros(n, dtype=np.int64)
        mt = np.zeros(n, dtype=np.uint64)
        tr = np.zeros(n, dtype=np.uint32)
        br = np.zeros(n, dtype=np.uint32)
        wall = ctypes.c_int64()
        cb = cc = None
        if copy_out is not None:
            cb = np.ascontiguousarray(copy_base, dtype=np.uint64)
            cc = np.ascontiguousarray(copy_cap, dtype=np.uint64)
        _check(glop_server_run_trace(self._s, n, dk.ctypes.data, tx.ctypes.data, ln.ctypes.data, at.ctypes.data,
                                     copy_out.data_ptr() if copy_out is not None else None,
                                     cb.ctypes.data if cb is not None else None,
                                     cc.ctypes.data if cc is not None else None,
                                     lat.ctypes.data, mt.ctypes.data, tr.ctypes.data, br.ctypes.data,
                                     ctypes.byref(wall)), "glop_server_run_trace")
        return lat, mt, tr, br, int(wall.value)

    def close(self):
        if getattr(self, "_s", None):
            glop_server_destroy(self._s)
            self._s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

