"""Full-size workloads through the launch configuration bench.py times (needs an MI355X).

* medium (1 GiB, 1,000 patterns): every record and count compared with the
  first-byte-bucketed oracle over the whole text.
* medium dictionary over 2 GiB + 8 KiB of text: one tile more than 256 CUs x
  1,024 tiles, so the single text is split into two rounds of work items;
  every record and count against the oracle.
* large (4 GiB, 20,000 patterns): every record and count compared with the
  two-byte-bucketed oracle over the whole text (the first-byte bucketing would
  take most of an hour of host time on this dictionary); the output's
  properties (true occurrences, strictly ascending, plants present) are checked
  as well.
* batched (4,096 independent texts, about 7.7 GiB, medium dictionary) through
  glop_match_batch: every chunk's records, its position and record count, and
  the batch's per-pattern counts, against one oracle run over the chunks laid
  end to end, keeping the occurrences that lie wholly inside one chunk (the
  union of the per-chunk results, since the oracle is the plain definition).
"""

import numpy as np
import pytest

import oracle
import synth

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

glop = pytest.importorskip("paper_1704_02278_amd")
from chunks import split_by_chunk  # noqa: E402
from gpu_util import assert_same, gpu_match, oracle_match, say, to_device  # noqa: E402


def test_medium_full_size_bit_exact():
    pats, text, plants = synth.make_workload("medium")
    say("fullsize medium", text.size)
    dev_text = to_device(text)
    got = gpu_match(glop.Dict(pats), dev_text)
    want = oracle_match(text, pats)
    assert want[3] >= len(plants)
    assert_same(got, want, "medium 1 GiB")
    # The default is 4 KiB tiles here; the 8 KiB kernels at the same size.
    say("fullsize medium, 8 KiB tiles", text.size)
    assert_same(gpu_match(glop.Dict(pats, tile_kib=8), dev_text), want, "medium 1 GiB, 8 KiB tiles")


def _properties(text, pats, plants, off, ids, counts, total):
    assert off.size == total == int(counts.sum())
    key = off * np.uint64(1 << 32) + ids
    assert np.all(key[1:] > key[:-1]), "records not strictly ascending"
    tb = memoryview(text)
    assert all(bytes(tb[o:o + len(pats[j])]) == pats[j] for o, j in zip(off.tolist(), ids.tolist()))
    got = set(zip(off.tolist(), ids.tolist()))
    assert all((o, j) in got for o, j in plants), "a planted occurrence is missing"


def test_medium_dictionary_two_rounds_bit_exact():
    n = (2 << 30) + 8192
    pats, text, plants = synth.make_workload("medium", n_bytes=n)
    say("fullsize medium dictionary, two rounds of items", text.size)
    got = gpu_match(glop.Dict(pats), to_device(text))
    want = oracle_match(text, pats, bucketed=2)
    assert want[3] >= len(plants)
    assert_same(got, want, "medium dictionary, 2 GiB + 8 KiB")


def test_large_full_size_bit_exact():
    pats, text, plants = synth.make_workload("large")
    say("fullsize large", text.size)
    got = gpu_match(glop.Dict(pats), to_device(text))
    _properties(text, pats, plants, *got)
    say("fullsize large: oracle (two-byte buckets)")
    want = oracle_match(text, pats, bucketed=2)
    assert_same(got, want, "large 4 GiB")


def test_batched_full_size_bit_exact():
    import torch

    pats, text, offs, sizes, plants = synth.make_chunks("batched")
    say("fullsize batched", len(sizes), text.size)
    buf = torch.from_numpy(text).to("cuda")
    chunks = [buf[o:o + n] for o, n in zip(offs.tolist(), sizes)]
    d = glop.Dict(pats)
    g_off, g_ids, g_cid, first, count, counts, total = d.match_batch(chunks)
    g_off, g_ids, g_cid = (x.cpu().numpy().astype(np.uint64) for x in (g_off, g_ids, g_cid))
    first, count = first.cpu().numpy(), count.cpu().numpy()
    counts = counts.cpu().numpy().astype(np.uint64)
    del buf, chunks

    say("fullsize batched: oracle over the concatenation")
    w_off, w_ids, _, _ = oracle_match(text, pats)
    k, w_rel, w_ids = split_by_chunk(w_off, w_ids, [len(p) for p in pats], offs, sizes)
    w_rel = w_rel.astype(np.uint64)
    per_chunk = np.bincount(k, minlength=len(sizes))

    assert total == w_rel.size
    assert np.array_equal(count, per_chunk)
    assert np.array_equal(first, np.concatenate([[0], np.cumsum(per_chunk)[:-1]]))
    assert np.array_equal(g_cid, k.astype(np.uint64))
    assert np.array_equal(g_off, w_rel)
    assert np.array_equal(g_ids, w_ids.astype(np.uint64))
    assert np.array_equal(counts, np.bincount(w_ids.astype(np.int64), minlength=len(pats)).astype(np.uint64))
    assert all(len(p) <= c for p, c in zip(plants, per_chunk.tolist()))

