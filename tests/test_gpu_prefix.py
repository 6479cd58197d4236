"""Truncated-trie engine on the GPU (needs an MI355X).

prefix_len = 8: the trie holds the first 8 bytes of every pattern and a GPU
verify stage compares the rest, so records must equal the oracle bit for bit;
candidates = 1 must equal the oracle run on the truncated patterns.
"""

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

glop = pytest.importorskip("paper_1704_02278_amd")
from gpu_util import assert_same, gpu_match, oracle_match, say, to_device  # noqa: E402


def _variants(pats):
    out = [dict(), dict(filter=glop.GLOP_FILTER_NONE), dict(filter=glop.GLOP_FILTER_QGRAM, stride=1)]
    if min(min(len(p), 8) for p in pats) >= 7:
        out.append(dict(filter=glop.GLOP_FILTER_QGRAM, stride=4, qgram=4))
    return out


@pytest.mark.parametrize("name,n_bytes", [("tiny", None), ("medium", 32 << 20), ("large", 8 << 20)])
def test_exact_with_verify_stage(name, n_bytes):
    pats, text, _ = synth.make_workload(name, n_bytes=n_bytes)
    want = oracle_match(text, pats)
    cand = oracle_match(text, [p[:8] for p in pats])
    for opts in _variants(pats):
        say("prefix8", name, opts)
        assert_same(gpu_match(glop.Dict(pats, prefix_len=8, **opts), to_device(text, 3)), want, f"{name} {opts}")
        assert_same(gpu_match(glop.Dict(pats, prefix_len=8, candidates=True, **opts), to_device(text, 3)), cand,
                    f"{name} candidates {opts}")


def test_verify_near_the_text_end_and_dense_candidates():
    pats = [b"abcdefghXY", b"abcdefghZ", b"abcdefgh", b"abcdefghXYZ", b"bcdefghX"]
    base = b"abcdefghXYZ-abcdefghZ-" * 3000
    for tail in (b"abcdefghX", b"abcdefghXY", b"abcdefgh", b"abcdefghZ"):
        text = np.frombuffer(base + tail, dtype=np.uint8)
        want = oracle_match(text, pats)
        for opts in ({}, {"filter": glop.GLOP_FILTER_NONE}):
            say("prefix8 tail", tail, opts)
            assert_same(gpu_match(glop.Dict(pats, prefix_len=8, **opts), to_device(text, 7)), want, f"tail {tail}")


def test_batched_with_prefix_engine():
    pats, text, _ = synth.make_workload("medium", n_bytes=8 << 20)
    pieces = [text[k * 300_000:(k + 1) * 300_000 + 17 * k] for k in range(20)]
    buf = torch.from_numpy(np.concatenate(pieces)).cuda()
    chunks, pos = [], 0
    for p in pieces:
        chunks.append(buf[pos:pos + p.size])
        pos += p.size
    d = glop.Dict(pats, prefix_len=8)
    say("prefix8 batched")
    off, ids, cid, first, count, counts, total = d.match_batch(chunks)
    off, ids, cid = off.cpu().numpy(), ids.cpu().numpy(), cid.cpu().numpy()
    pos = 0
    for k, p in enumerate(pieces):
        w_off, w_ids, _, w_total = oracle_match(p, pats)
        assert int(count[k]) == w_total and int(first[k]) == pos
        assert np.array_equal(off[pos:pos + w_total].astype(np.uint64), w_off)
        assert np.array_equal(ids[pos:pos + w_total].astype(np.uint64), w_ids)
        assert np.all(cid[pos:pos + w_total] == k)
        pos += w_total
    assert total == pos
