"""Truncated-trie engine on the host (glop_compile + glop_cpu_walk, no GPU).

prefix_len = 8 builds the trie from each pattern's first 8 bytes (the
truncation of Sections 2 and 5); the verify stage must restore the exact
result, and `candidates` must report exactly the truncated matches, i.e. the
oracle run on the truncated patterns.
"""

import random

import numpy as np
import pytest

import oracle
from brute import brute_matches
from golden_io import load_examples

glop = pytest.importorskip("paper_1704_02278_amd")


def host_dict(patterns, **opts):
    return glop.Dict(patterns, device=False, **opts)


def walk(d, text):
    off, ids, counts, total = d.cpu_walk(text)
    return list(zip(off.tolist(), ids.tolist())), counts.tolist(), total


def test_hand_examples_exact_with_truncation():
    for ex in load_examples():
        for L in (1, 2, 8):
            got, counts, total = walk(host_dict(ex.patterns, prefix_len=L), ex.text)
            assert got == ex.matches and counts == ex.counts and total == len(ex.matches), (ex.name, L)


def test_shared_long_prefixes_are_told_apart():
    pats = [b"abcdefghXY", b"abcdefghZ", b"abcdefgh", b"abcdefghXYZ", b"bcdefghX", b"hXY"]
    text = b"..abcdefghXYZ..abcdefghZ..abcdefghX..abcdefgh"
    want, want_counts = brute_matches(text, pats)
    for L in (3, 8, 9, 200):
        got, counts, total = walk(host_dict(pats, prefix_len=L), text)
        assert got == want and counts == want_counts, L


def test_random_cases_exact_and_candidates():
    rng = random.Random(8)
    for _ in range(150):
        alpha = b"ab"[: rng.randint(1, 2)] + b"c"
        pats = [bytes(rng.choice(alpha) for _ in range(rng.randint(1, 14))) for _ in range(rng.randint(1, 8))]
        text = bytes(rng.choice(alpha) for _ in range(rng.randint(0, 300)))
        L = rng.randint(1, 9)
        got, counts, _ = walk(host_dict(pats, prefix_len=L), text)
        assert (got, counts) == brute_matches(text, pats), (pats, text, L)
        cand, counts, _ = walk(host_dict(pats, prefix_len=L, candidates=True), text)
        assert (cand, counts) == brute_matches(text, [p[:L] for p in pats]), (pats, text, L)


def test_candidates_equal_the_oracle_on_truncated_patterns():
    import synth

    pats, text, _ = synth.make_workload("medium", n_bytes=2 << 20)
    d = host_dict(pats, prefix_len=8, candidates=True)
    off, ids, counts, total = d.cpu_walk(text, threads=4)
    w_off, w_ids, w_counts, w_total = oracle.match(text, [p[:8] for p in pats], bucketed=True)
    assert total == w_total and np.array_equal(off, w_off.astype(np.uint64))
    assert np.array_equal(ids, w_ids.astype(np.uint64)) and np.array_equal(counts, w_counts)
    exact = host_dict(pats, prefix_len=8).cpu_walk(text, threads=4)
    e_off, e_ids, e_counts, e_total = oracle.match(text, pats, bucketed=True)
    assert exact[3] == e_total <= total and np.array_equal(exact[0], e_off.astype(np.uint64))


def test_prefix_options_are_checked_and_reported():
    with pytest.raises(glop.GlopError):
        host_dict([b"abc"], prefix_len=256)
    with pytest.raises(glop.GlopError):
        host_dict([b"abc"], candidates=True)
    info = host_dict([b"abcdefghij", b"xyz"], prefix_len=8).info()
    assert info["prefix_len"] == 8 and info["candidates"] == 0 and info["max_len"] == 10 and info["min_len"] == 3
    info = host_dict([b"abcdefghij", b"abcdefghkl"], prefix_len=8, candidates=True).info()
    assert info["candidates"] == 1 and info["num_states"] == 9  # root + 8 shared prefix states


def test_automatic_engine_rule():
    # Every pattern fits in 8 bytes: truncation would change nothing.
    assert host_dict([b"abc", b"abcdefgh"]).info()["prefix_len"] == 0
    # Longer patterns with distinct heads: 8-byte prefixes plus verification.
    assert host_dict([b"abcdefghij", b"bcdefghijk"]).info()["prefix_len"] == 8
    # 16 patterns may share one 8-byte head; 17 may not.
    share16 = [b"commonhd" + bytes([65 + k]) for k in range(16)]
    assert host_dict(share16).info()["prefix_len"] == 8
    assert host_dict(share16 + [b"commonhdZZ"]).info()["prefix_len"] == 0
    # Explicit choices win.
    assert host_dict(share16 + [b"commonhdZZ"], prefix_len=8).info()["prefix_len"] == 8
    assert host_dict([b"abcdefghij"], prefix_len=glop.GLOP_PREFIX_FULL).info()["prefix_len"] == 0
