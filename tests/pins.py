"""Pins of the CPU oracle against facts fixed outside it.

``pin_failures(lib)`` runs every quick pin against an oracle library handle and
returns the names of those that fail.  The regular tests require an empty list;
the mutation test requires a non-empty one for each planted mistake.

Pins:
  * hand-derived examples (``golden/hand_examples.txt``), plain and both
    bucketings (first byte, first two bytes), with 1 and 3 threads;
  * brute force by Python slicing on random tiny inputs over 1-3 letter
    alphabets (forces overlaps, duplicates and prefix chains);
  * single-pattern special case against two library routines: overlapping
    ``re`` look-ahead search and a ``bytes.find`` loop;
  * truncation: a capacity below the total returns the first pairs in order
    with complete counts.
"""

from __future__ import annotations

import random
import re

import numpy as np

import oracle
from brute import brute_matches
from golden_io import load_examples


MODES = (0, 1, 2)  # plain, first-byte buckets, two-byte buckets


def _run(lib, text: bytes, pats, bucketed: int, threads: int, cap=None):
    off, ids, counts, total = oracle.match(text, pats, bucketed=bucketed, threads=threads, cap=cap, lib=lib)
    return list(zip(off.tolist(), ids.tolist())), counts.tolist(), total


def _random_case(rng: random.Random):
    alpha = b"abc"[: rng.randint(1, 3)]
    n = rng.randint(1, 8)
    pats = []
    for _ in range(n):
        r = rng.random()
        if pats and r < 0.2:
            pats.append(rng.choice(pats))                      # duplicate
        elif pats and r < 0.4:
            src = rng.choice(pats)
            pats.append(src[: rng.randint(1, len(src))])       # prefix of another
        else:
            pats.append(bytes(rng.choice(alpha) for _ in range(rng.randint(1, 8))))
    text = bytes(rng.choice(alpha) for _ in range(rng.randint(0, 256)))
    return text, pats


def _single_pattern_refs(text: bytes, p: bytes):
    via_re = [m.start() for m in re.finditer(b"(?=" + re.escape(p) + b")", text)]
    via_find, k = [], text.find(p)
    while k != -1:
        via_find.append(k)
        k = text.find(p, k + 1)
    return via_re, via_find


def pin_failures(lib, n_random: int = 150, seed: int = 1704) -> list[str]:
    failed: list[str] = []
    for ex in load_examples():
        for bucketed in MODES:
            for threads in (1, 3):
                got, counts, total = _run(lib, ex.text, ex.patterns, bucketed, threads)
                if got != ex.matches or counts != ex.counts or total != len(ex.matches):
                    failed.append(f"hand:{ex.name}:b{int(bucketed)}:t{threads}")
    rng = random.Random(seed)
    for k in range(n_random):
        text, pats = _random_case(rng)
        want, want_counts = brute_matches(text, pats)
        for bucketed in MODES:
            got, counts, total = _run(lib, text, pats, bucketed, 1 + k % 4)
            if got != want or counts != want_counts or total != len(want):
                failed.append(f"brute:{k}:b{int(bucketed)}")
    for k in range(40):
        alpha = b"ab"[: 1 + k % 2]
        text = bytes(rng.choice(alpha) for _ in range(rng.randint(0, 300)))
        p = bytes(rng.choice(alpha) for _ in range(rng.randint(1, 5)))
        via_re, via_find = _single_pattern_refs(text, p)
        for bucketed in MODES:
            got, counts, total = _run(lib, text, [p], bucketed, 2)
            if not (via_re == via_find == [o for o, _ in got]) or counts != [len(via_re)]:
                failed.append(f"single:{k}:b{int(bucketed)}")
    text, pats = b"abababab", [b"ab", b"b", b"aba"]
    want, want_counts = brute_matches(text, pats)
    for cap in (0, 1, len(want) - 1):
        for bucketed in (1, 2):
            got, counts, total = _run(lib, text, pats, bucketed, 2, cap=cap)
            if got != want[:cap] or counts != want_counts or total != len(want):
                failed.append(f"cap:{cap}:b{bucketed}")
    return failed


def workload_invariant_failures(text: np.ndarray, pats: list[bytes], plants, off, ids, counts, total) -> list[str]:
    """Properties that any correct result on a synthetic workload must have."""
    failed = []
    off = np.asarray(off, dtype=np.uint64)
    ids = np.asarray(ids, dtype=np.uint32)
    if off.size != total or int(np.sum(counts)) != total:
        failed.append("sum(counts) == |M| == len(output)")
    key = off.astype(np.uint64) * np.uint64(1 << 32) + ids.astype(np.uint64)
    if off.size > 1 and not np.all(key[1:] > key[:-1]):
        failed.append("strictly ascending (offset, id)")
    pair_set = set(zip(off.tolist(), ids.tolist()))
    if not all((o, j) in pair_set for o, j in plants):
        failed.append("every planted occurrence reported")
    tb = text.tobytes() if isinstance(text, np.ndarray) else bytes(text)
    if not all(tb[o:o + len(pats[j])] == pats[j] for o, j in pair_set):
        failed.append("every reported pair is a true occurrence")
    # Prefix closure: where a pattern occurs, every pattern that is a prefix of it occurs too.
    by_bytes = {}
    for j, p in enumerate(pats):
        by_bytes.setdefault(p, []).append(j)
    prefixes_of = {}
    for j, p in enumerate(pats):
        prefixes_of[j] = [a for L in range(1, len(p)) for a in by_bytes.get(p[:L], [])]
    for o, j in pair_set:
        if not all((o, a) in pair_set for a in prefixes_of[j]):
            failed.append("prefix closure")
            break
    return failed
