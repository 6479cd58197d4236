"""CPU oracle for exact multi-pattern matching -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU matcher
(``paper_1704_02278_amd``) and neither imports the other.

``match(text, patterns)`` returns the plain definition of the result that the
failureless-trie walk (Section 5) reaches: every (offset, pattern id) with
``text[offset : offset + len(p)] == p``, ascending by offset then id, plus the
per-pattern counts.  The arithmetic lives in ``glop_oracle.c`` (plain C).
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "glop_oracle.c"
_LIB = _HERE / "libglop_oracle.so"


def compile_oracle(src: Path, dst: Path) -> Path:
    tmp = dst.with_name(dst.name + ".tmp")
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread", str(src), "-o", str(tmp)],
                   check=True)
    os.replace(tmp, dst)
    return dst


def build_library(force: bool = False) -> Path:
    if force or not _LIB.exists() or _LIB.stat().st_mtime < _SRC.stat().st_mtime:
        compile_oracle(_SRC, _LIB)
    return _LIB


def _bind(path: Path):
    lib = ctypes.CDLL(str(path))
    u64p = ctypes.POINTER(ctypes.c_uint64)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    lib.oracle_match.restype = ctypes.c_uint64
    lib.oracle_match.argtypes = [
        ctypes.c_void_p, ctypes.c_uint64,            # text, N
        ctypes.c_void_p, u64p, u32p, ctypes.c_uint32,  # patterns
        ctypes.c_int, ctypes.c_int,                  # bucketed, threads
        ctypes.c_uint64, u64p, u32p,                 # cap, out_off, out_id
        u64p,                                        # counts
    ]
    return lib


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not _LIB.exists():
            build_library()
        _lib = _bind(_LIB)
    return _lib


def _as_u8(buf) -> np.ndarray:
    if isinstance(buf, np.ndarray):
        assert buf.dtype == np.uint8
        return np.ascontiguousarray(buf)
    return np.frombuffer(bytes(buf), dtype=np.uint8)


def flatten_patterns(patterns):
    lens = np.array([len(p) for p in patterns], dtype=np.uint32)
    offs = np.zeros(len(patterns), dtype=np.uint64)
    if len(patterns) > 1:
        offs[1:] = np.cumsum(lens[:-1], dtype=np.uint64)
    blob = np.frombuffer(b"".join(bytes(p) for p in patterns) or b"\0", dtype=np.uint8)
    return blob, offs, lens


def match(text, patterns, *, bucketed: bool | int = True, threads: int | None = None,
          cap: int | None = None, lib=None):
    """(offsets u64[M'], ids u32[M'], counts u64[n], total M).

    ``bucketed``: False/0 = every pattern at every offset; True/1 = only the
    patterns whose first byte is the text byte; 2 = only the 1-byte patterns
    and those whose first two bytes are the next two text bytes.  All three
    give the same result.  ``cap`` limits how many pairs are returned (None =
    all, found by a count pass first); the counts and ``total`` are always
    complete.
    """
    lib = lib or _load()
    t = _as_u8(text)
    blob, offs, lens = flatten_patterns(patterns)
    if threads is None:
        threads = min(16, os.cpu_count() or 1)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    counts = np.zeros(len(patterns), dtype=np.uint64)
    args = (t.ctypes.data, t.size, blob.ctypes.data, offs.ctypes.data_as(u64p),
            lens.ctypes.data_as(u32p), len(patterns), int(bucketed), threads)
    if cap is None:
        total = lib.oracle_match(*args, 0, None, None, counts.ctypes.data_as(u64p))
        if total == 2 ** 64 - 1:
            raise ValueError("invalid oracle input (empty pattern?)")
        cap = total
    out_off = np.zeros(max(cap, 1), dtype=np.uint64)
    out_id = np.zeros(max(cap, 1), dtype=np.uint32)
    total = lib.oracle_match(*args, cap, out_off.ctypes.data_as(u64p), out_id.ctypes.data_as(u32p),
                             counts.ctypes.data_as(u64p))
    if total == 2 ** 64 - 1:
        raise ValueError("invalid oracle input (empty pattern?)")
    k = min(cap, total)
    return out_off[:k], out_id[:k], counts, int(total)
