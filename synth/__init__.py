"""Seeded synthetic workloads for the log matcher (patterns, log text, plants).

This module only draws bytes; it holds none of the matching arithmetic.  The
CPU oracle's tests and the GPU path's tests and benchmark take their inputs
from here, so both sides always see identical data.

The paper's own inputs (Section 6: 100 MB Mersenne-Twister logs, random
patterns checked for uniqueness with SHA-256) are not available; these seeded
generators stand in for them with the shapes of the workloads studied here:

* ``tiny``   -- 16 patterns of 4-16 B over 1 MiB of log lines, 1 plant / 4 KiB
* ``medium`` -- 1,000 patterns of 8-64 B (30 % share a 4-12 B prefix with an
  earlier pattern, 5 % are exact prefixes of a longer one) over 1 GiB,
  1 plant / 64 KiB
* ``large``  -- 20,000 patterns, Zipf(1.2) lengths on 4-128 B, 40 % shared
  prefixes, over 4 GiB, 1 plant / 16 KiB
* ``batched`` (``make_chunks``) -- the medium dictionary over 4,096 independent
  texts whose sizes are lognormal (median 256 KiB, sigma 2.16) clipped to
  [1 KiB, 64 MiB], about 8 GiB in all, 1 plant / 64 KiB in each
* served (``make_served``, ``served_trace``) -- 8 resident dictionaries of
  100 ... 20,000 patterns (the medium recipe up to 1,000 patterns, the large
  one above), a 256 MiB planted text pool per dictionary, and request traces
  with Poisson arrivals, a uniform dictionary tag and lognormal sizes (median
  256 KiB, sigma 2.16) clipped to [4 KiB, 16 MiB], each request a slice of its
  dictionary's pool

Every random draw comes from MT19937-64 substreams (``synth.c``) selected by
(seed, stream, block), so the output does not depend on thread counts.
"""

from __future__ import annotations

import ctypes
import dataclasses
import hashlib
import os
import subprocess
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "synth.c"
_LIB = _HERE / "libsynth.so"

BASE_SEED = 170402278

# Substream ids (one per purpose) -- offsets added to a workload's index.
STREAM_PATTERNS = 1 << 20
STREAM_TEXT = 2 << 20
STREAM_PLANTS = 3 << 20
# Chunked workloads: sizes, then (text, plants) per chunk.
STREAM_CHUNK_SIZES = 4 << 20
STREAM_CHUNKS = 5 << 20
# Served workload: dictionaries, pools and traces.
STREAM_SERVED = 6 << 20


def build_library(force: bool = False) -> Path:
    """Compile ``libsynth.so`` with gcc (plain C, pthreads)."""
    if force or not _LIB.exists() or _LIB.stat().st_mtime < _SRC.stat().st_mtime:
        tmp = _LIB.with_suffix(".so.tmp")
        subprocess.run(
            ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread", str(_SRC), "-o", str(tmp)],
            check=True,
        )
        os.replace(tmp, _LIB)
    return _LIB


class _TextCfg(ctypes.Structure):
    _fields_ = [
        ("line_min", ctypes.c_uint32),
        ("line_max", ctypes.c_uint32),
        ("word_min", ctypes.c_uint32),
        ("word_max", ctypes.c_uint32),
        ("byte_lo", ctypes.c_uint32),
        ("byte_hi", ctypes.c_uint32),
        ("block_bytes", ctypes.c_uint64),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not _LIB.exists():
            build_library()
        lib = ctypes.CDLL(str(_LIB))
        u64p = ctypes.POINTER(ctypes.c_uint64)
        lib.synth_substream_seed.restype = ctypes.c_uint64
        lib.synth_substream_seed.argtypes = [ctypes.c_uint64] * 3
        lib.synth_mt64_raw.restype = None
        lib.synth_mt64_raw.argtypes = [ctypes.c_uint64, ctypes.c_uint64, u64p]
        lib.synth_stream.restype = None
        lib.synth_stream.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, u64p]
        lib.synth_text.restype = ctypes.c_int
        lib.synth_text.argtypes = [
            ctypes.c_uint64,
            ctypes.c_uint64,
            ctypes.c_void_p,
            ctypes.c_uint64,
            ctypes.POINTER(_TextCfg),
            ctypes.c_int,
        ]
        _lib = lib
    return _lib


def mt64_raw(mt_seed: int, count: int) -> np.ndarray:
    """First ``count`` outputs of MT19937-64 seeded with ``mt_seed``."""
    out = np.empty(count, dtype=np.uint64)
    _load().synth_mt64_raw(mt_seed, count, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    return out


def stream(seed: int, stream_id: int, count: int) -> np.ndarray:
    out = np.empty(count, dtype=np.uint64)
    _load().synth_stream(seed, stream_id, count, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    return out


class Draws:
    """Sequential consumer of one substream (32-bit draws, high half first)."""

    def __init__(self, seed: int, stream_id: int, chunk: int = 1 << 16):
        self.seed, self.stream_id = seed, stream_id
        self._raw = np.empty(0, dtype=np.uint64)
        self._u32: list[int] = []
        self._pos = 0
        self._chunk = chunk

    def _grow(self):
        n = max(self._chunk, 2 * self._raw.size)
        self._raw = stream(self.seed, self.stream_id, n)
        hi = (self._raw >> np.uint64(32)).astype(np.uint32)
        lo = (self._raw & np.uint64(0xFFFFFFFF)).astype(np.uint32)
        self._u32 = np.stack([hi, lo], axis=1).reshape(-1).tolist()

    def u32(self) -> int:
        if self._pos >= len(self._u32):
            self._grow()
        v = self._u32[self._pos]
        self._pos += 1
        return v

    def randint(self, lo: int, hi: int) -> int:
        """Uniform integer in [lo, hi] (inclusive)."""
        return lo + ((self.u32() * (hi - lo + 1)) >> 32)

    def unit(self) -> float:
        """Uniform float in [0, 1) with 53 bits."""
        return ((self.u32() << 21) ^ (self.u32() >> 11)) / float(1 << 53)

    def bytes_in(self, n: int, lo: int, hi: int) -> bytes:
        return bytes(self.randint(lo, hi) for _ in range(n))


@dataclasses.dataclass(frozen=True)
class PatternSpec:
    n: int
    len_min: int
    len_max: int
    zipf_s: float = 0.0          # 0 => uniform lengths; else P(len_min-1+r) ~ r^-s
    shared_frac: float = 0.0     # share a k-byte prefix with an earlier pattern
    shared_kmin: int = 4
    shared_kmax: int = 12
    exact_prefix_frac: float = 0.0  # exact prefix of an earlier, longer pattern
    byte_lo: int = 0x20
    byte_hi: int = 0x7E


@dataclasses.dataclass(frozen=True)
class TextSpec:
    n_bytes: int
    line_min: int = 60
    line_max: int = 200
    word_min: int = 1
    word_max: int = 12
    byte_lo: int = 0x21
    byte_hi: int = 0x7E
    block_bytes: int = 1 << 20
    plant_every: int = 0  # bytes of text per planted occurrence (0 = none)


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    index: int
    patterns: PatternSpec
    text: TextSpec


WORKLOADS = {
    "tiny": Workload(
        "tiny", 1,
        PatternSpec(n=16, len_min=4, len_max=16),
        TextSpec(n_bytes=1 << 20, plant_every=4 << 10),
    ),
    "medium": Workload(
        "medium", 2,
        PatternSpec(n=1000, len_min=8, len_max=64, shared_frac=0.30, exact_prefix_frac=0.05),
        TextSpec(n_bytes=1 << 30, plant_every=64 << 10),
    ),
    "large": Workload(
        "large", 3,
        PatternSpec(n=20000, len_min=4, len_max=128, zipf_s=1.2, shared_frac=0.40),
        TextSpec(n_bytes=4 << 30, plant_every=16 << 10),
    ),
}


def _length_sampler(spec: PatternSpec, d: Draws):
    if spec.zipf_s <= 0.0:
        return lambda: d.randint(spec.len_min, spec.len_max)
    r = np.arange(1, spec.len_max - spec.len_min + 2, dtype=np.float64)
    cdf = np.cumsum(r ** (-spec.zipf_s))
    cdf /= cdf[-1]
    cdf_list = cdf.tolist()

    def draw():
        u = d.unit()
        k = int(np.searchsorted(cdf_list, u, side="right"))
        return spec.len_min + min(k, len(cdf_list) - 1)

    return draw


def gen_patterns(spec: PatternSpec, seed: int = BASE_SEED, stream_id: int = STREAM_PATTERNS) -> list[bytes]:
    """Distinct patterns following ``spec``; duplicates are redrawn."""
    d = Draws(seed, stream_id)
    draw_len = _length_sampler(spec, d)
    pats: list[bytes] = []
    seen: set[bytes] = set()
    while len(pats) < spec.n:
        length = draw_len()
        u = d.unit()
        p = None
        if pats and u < spec.exact_prefix_frac:
            src = pats[d.randint(0, len(pats) - 1)]
            if len(src) > spec.len_min:
                p = src[: d.randint(spec.len_min, len(src) - 1)]
        elif pats and u < spec.exact_prefix_frac + spec.shared_frac:
            src = pats[d.randint(0, len(pats) - 1)]
            k = d.randint(spec.shared_kmin, spec.shared_kmax)
            k = min(k, length - 1, len(src) - 1)
            if k >= spec.shared_kmin:
                p = src[:k] + d.bytes_in(length - k, spec.byte_lo, spec.byte_hi)
        if p is None:
            p = d.bytes_in(length, spec.byte_lo, spec.byte_hi)
        if p in seen:
            continue
        seen.add(p)
        pats.append(p)
    return pats


def gen_text(spec: TextSpec, seed: int = BASE_SEED, stream_id: int = STREAM_TEXT,
             threads: int | None = None, out: np.ndarray | None = None) -> np.ndarray:
    """Synthetic log text of exactly ``spec.n_bytes`` bytes (no plants)."""
    if out is None:
        out = np.empty(spec.n_bytes, dtype=np.uint8)
    assert out.dtype == np.uint8 and out.size == spec.n_bytes and out.flags.c_contiguous
    cfg = _TextCfg(spec.line_min, spec.line_max, spec.word_min, spec.word_max,
                   spec.byte_lo, spec.byte_hi, spec.block_bytes)
    if threads is None:
        threads = min(16, os.cpu_count() or 1)
    rc = _load().synth_text(seed, stream_id, out.ctypes.data, spec.n_bytes, ctypes.byref(cfg), threads)
    if rc != 0:
        raise ValueError("invalid text configuration")
    return out


_NL_MARGIN = 512


def plant(text: np.ndarray, patterns: list[bytes], every: int, seed: int = BASE_SEED,
          stream_id: int = STREAM_PLANTS, draw_chunk: int = 1 << 16) -> list[tuple[int, int]]:
    """Overwrite ``text`` with one occurrence per ``every``-byte slot.

    Each plant picks a pattern uniformly, lies wholly inside its slot (so plants
    never overlap) and inside one line (it never covers a newline).  Returns the
    sorted list of (offset, pattern id) planted.  ``draw_chunk`` only sizes the
    draw buffer (the draws themselves do not depend on it).
    """
    if every <= 0 or not patterns:
        return []
    n = text.size
    nslots = n // every
    if nslots == 0:
        return []
    d = Draws(seed, stream_id, chunk=draw_chunk)
    plants = []
    for m in range(nslots):
        lo, hi = m * every, (m + 1) * every
        for _attempt in range(64):
            j = d.randint(0, len(patterns) - 1)
            p = patterns[j]
            if len(p) > every:
                continue
            o = d.randint(lo, hi - len(p))
            # Newlines near o (lines are far shorter than the search margin).
            w_lo, w_hi = max(0, o - _NL_MARGIN), min(n, o + len(p) + _NL_MARGIN)
            nl = np.flatnonzero(text[w_lo:w_hi] == 0x0A) + w_lo
            k = int(np.searchsorted(nl, o))
            if k < nl.size:
                nxt = int(nl[k])
            elif w_hi == n:
                nxt = n
            else:
                continue
            if o + len(p) > nxt:
                # Slide back inside the line, or forward into the following line.
                if k > 0:
                    start = int(nl[k - 1]) + 1
                elif w_lo == 0:
                    start = 0
                else:
                    continue
                if nxt - len(p) >= max(start, lo):
                    o = nxt - len(p)
                else:
                    o = nxt + 1
                    if k + 1 < nl.size:
                        nxt2 = int(nl[k + 1])
                    elif w_hi == n:
                        nxt2 = n
                    else:
                        continue
                    if o + len(p) > min(nxt2, hi):
                        continue
            text[o:o + len(p)] = np.frombuffer(p, dtype=np.uint8)
            plants.append((o, j))
            break
    return plants


def sha256_bytes(buf) -> str:
    return hashlib.sha256(memoryview(buf)).hexdigest()


def sha256_patterns(patterns) -> str:
    """SHA-256 of a pattern set in id order: each pattern as its length (4-byte
    little-endian) followed by its bytes, so no two different lists collide by
    concatenation."""
    h = hashlib.sha256()
    for p in patterns:
        h.update(len(p).to_bytes(4, "little"))
        h.update(bytes(p))
    return h.hexdigest()


def make_workload(name: str, seed: int = BASE_SEED, n_bytes: int | None = None,
                  threads: int | None = None):
    """(patterns, text, plants) for a named workload; ``n_bytes`` may shrink the text."""
    w = WORKLOADS[name]
    tspec = w.text if n_bytes is None else dataclasses.replace(w.text, n_bytes=n_bytes)
    pats = gen_patterns(w.patterns, seed, STREAM_PATTERNS + w.index)
    text = gen_text(tspec, seed, STREAM_TEXT + w.index, threads=threads)
    plants = plant(text, pats, tspec.plant_every, seed, STREAM_PLANTS + w.index)
    return pats, text, plants


@dataclasses.dataclass(frozen=True)
class ChunkSpec:
    count: int
    median: int
    sigma: float
    size_min: int
    size_max: int
    plant_every: int


CHUNKED = {
    # Many independent texts matched as one batch, against the medium dictionary.
    "batched": ("medium", ChunkSpec(count=4096, median=256 << 10, sigma=2.16, size_min=1 << 10,
                                    size_max=64 << 20, plant_every=64 << 10)),
}


def chunk_sizes(spec: ChunkSpec, seed: int = BASE_SEED, stream_id: int = STREAM_CHUNK_SIZES) -> list[int]:
    """Lognormal sizes (Box-Muller normals from one substream), clipped."""
    d = Draws(seed, stream_id)
    out = []
    mu = np.log(spec.median)
    for _ in range(spec.count):
        u1 = 1.0 - d.unit()  # (0, 1]
        u2 = d.unit()
        z = float(np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2))
        size = int(round(float(np.exp(mu + spec.sigma * z))))
        out.append(min(max(size, spec.size_min), spec.size_max))
    return out


def make_chunks(name: str = "batched", seed: int = BASE_SEED, count: int | None = None,
                threads: int | None = None):
    """(patterns, text, offsets, sizes, plants): chunk k is text[offsets[k]:offsets[k]+sizes[k]],
    generated and planted on its own; ``plants[k]`` lists its (offset in chunk, id).
    ``count`` keeps only the first chunks (smaller test cases of the same draw)."""
    dict_name, spec = CHUNKED[name]
    w = WORKLOADS[dict_name]
    pats = gen_patterns(w.patterns, seed, STREAM_PATTERNS + w.index)
    sizes = chunk_sizes(spec, seed)
    if count is not None:
        sizes = sizes[:count]
    offsets = np.zeros(len(sizes), dtype=np.int64)
    if sizes:
        offsets[1:] = np.cumsum(sizes[:-1])
    text = np.empty(int(sum(sizes)), dtype=np.uint8)
    plants = []
    for k, (o, n) in enumerate(zip(offsets.tolist(), sizes)):
        view = text[o:o + n]
        tspec = dataclasses.replace(w.text, n_bytes=n, plant_every=spec.plant_every)
        gen_text(tspec, seed, STREAM_CHUNKS + 2 * k, threads=threads, out=view)
        plants.append(plant(view, pats, spec.plant_every, seed, STREAM_CHUNKS + 2 * k + 1,
                            draw_chunk=64 + 4 * (n // spec.plant_every)))
    return pats, text, offsets, sizes, plants


SERVED_SIZES = (100, 500, 1000, 2000, 5000, 10000, 15000, 20000)


def served_spec(n: int) -> PatternSpec:
    """Dictionary recipe by size: medium's up to 1,000 patterns, large's above."""
    base = WORKLOADS["medium" if n <= 1000 else "large"].patterns
    return dataclasses.replace(base, n=n)


def make_served(pool_bytes: int = 256 << 20, seed: int = BASE_SEED, sizes=SERVED_SIZES, threads: int | None = None):
    """(dictionaries, pools): one pattern list and one planted text pool per size."""
    dicts, pools = [], []
    for k, n in enumerate(sizes):
        pats = gen_patterns(served_spec(n), seed, STREAM_SERVED + 16 * k)
        spec = dataclasses.replace(WORKLOADS["medium"].text, n_bytes=pool_bytes)
        pool = gen_text(spec, seed, STREAM_SERVED + 16 * k + 1, threads=threads)
        plant(pool, pats, spec.plant_every, seed, STREAM_SERVED + 16 * k + 2)
        dicts.append(pats)
        pools.append(pool)
    return dicts, pools


def served_trace(rate: float, count: int, ndicts: int, pool_bytes: int, seed: int = BASE_SEED,
                 size_min: int = 4 << 10, size_max: int = 16 << 20, median: int = 256 << 10,
                 sigma: float = 2.16, trace_id: int = 0):
    """Open-loop request trace: (arrival ns, dictionary, size, offset in its pool), arrivals ascending."""
    d = Draws(seed, STREAM_SERVED + 1024 + trace_id)
    t = 0.0
    at, dk, sz, off = [], [], [], []
    mu = float(np.log(median))
    for _ in range(count):
        t += -np.log(1.0 - d.unit()) / rate
        u1, u2 = 1.0 - d.unit(), d.unit()
        z = float(np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2))
        n = min(max(int(round(float(np.exp(mu + sigma * z)))), size_min), min(size_max, pool_bytes))
        k = d.randint(0, ndicts - 1)
        at.append(int(t * 1e9))
        dk.append(k)
        sz.append(n)
        off.append(d.randint(0, pool_bytes - n))
    return (np.array(at, dtype=np.int64), np.array(dk, dtype=np.uint32), np.array(sz, dtype=np.uint64),
            np.array(off, dtype=np.uint64))

