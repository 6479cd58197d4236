"""The CPU oracle, pinned to facts outside itself (CPU only)."""

import os
import shutil
from pathlib import Path

import numpy as np
import pytest

import oracle
import synth
from pins import pin_failures, workload_invariant_failures
from golden_io import load_examples


def test_golden_examples_parse():
    exs = load_examples()
    assert len(exs) >= 10
    for ex in exs:
        assert ex.cite and len(ex.counts) == len(ex.patterns)
        assert sum(ex.counts) == len(ex.matches)


def test_oracle_meets_every_pin():
    assert pin_failures(oracle._load()) == []


def test_empty_pattern_rejected():
    with pytest.raises(ValueError):
        oracle.match(b"abc", [b"a", b""])


def test_empty_dictionary():
    off, ids, counts, total = oracle.match(b"abc", [])
    assert total == 0 and off.size == 0 and counts.size == 0


def test_thread_count_does_not_change_result():
    pats, text, _ = synth.make_workload("tiny", n_bytes=256 << 10)
    ref = oracle.match(text, pats, bucketed=True, threads=1)
    for t in (2, 5, 8):
        got = oracle.match(text, pats, bucketed=True, threads=t)
        assert np.array_equal(ref[0], got[0]) and np.array_equal(ref[1], got[1])
        assert np.array_equal(ref[2], got[2]) and ref[3] == got[3]


@pytest.mark.parametrize("name,n_bytes", [("tiny", None), ("medium", 4 << 20), ("large", 2 << 20)])
def test_oracle_invariants_on_workloads(name, n_bytes):
    pats, text, plants = synth.make_workload(name, n_bytes=n_bytes)
    off, ids, counts, total = oracle.match(text, pats, bucketed=True)
    assert total >= len(plants) > 0
    assert workload_invariant_failures(text, pats, plants, off, ids, counts, total) == []


def _same(a, b):
    return (np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
            and a[3] == b[3])


def test_plain_equals_bucketed_on_workload_slices():
    for name, nb in (("tiny", None), ("medium", 1 << 20), ("large", 96 << 10)):
        pats, text, _ = synth.make_workload(name, n_bytes=nb)
        a = oracle.match(text, pats, bucketed=0)
        assert _same(a, oracle.match(text, pats, bucketed=1))
        assert _same(a, oracle.match(text, pats, bucketed=2))


@pytest.mark.slow
def test_two_byte_buckets_equal_first_byte_buckets_on_large_slice():
    """The two-byte bucketing, which the full-size large-dictionary GPU test
    compares against, equals the first-byte bucketing (itself equal to the
    plain loop above) on 256 MiB of the 20,000-pattern workload."""
    pats, text, plants = synth.make_workload("large", n_bytes=256 << 20)
    a = oracle.match(text, pats, bucketed=1)
    b = oracle.match(text, pats, bucketed=2)
    assert a[3] >= len(plants) > 0
    assert _same(a, b)


# Plausible mistakes, planted in a copy of the oracle source; the pins must
# catch every one.  (old text, new text) pairs.
MUTANTS = {
    "fit-off-by-one": ("if (len > pb->n_text - i) return 0;", "if (len >= pb->n_text - i) return 0;"),
    "short-compare": ("(size_t)len) == 0;", "(size_t)len - 1) == 0;"),
    "drop-last-pattern": ("for (uint32_t j = 0; j < pb->n_pat; j++)\n                if (occurs_at",
                          "for (uint32_t j = 0; j + 1 < pb->n_pat; j++)\n                if (occurs_at"),
    "bucket-drops-last": ("k < pb->bucket_at[first + 1]; k++", "k + 1 < pb->bucket_at[first + 1]; k++"),
    "count-not-accumulated": ("if (r->counts) r->counts[j] += 1;", "if (r->counts) r->counts[j] = 1;"),
    "range-order-shift": ("rs[t].out_base = total;\n        total += rs[t].found;",
                          "total += rs[t].found;\n        rs[t].out_base = total;"),
    "range-split-gap": ("rs[t].hi = n_text * (uint64_t)(t + 1) / (uint64_t)threads;",
                        "rs[t].hi = n_text * (uint64_t)(t + 1) / (uint64_t)threads - (t + 1 < threads);"),
    "one-match-per-offset": ("if (occurs_at(pb, i, j)) record(r, i, j);\n            }",
                             "if (occurs_at(pb, i, j)) { record(r, i, j); break; }\n            }"),
    "reversed-compare": ("memcmp(pb->text + i, pb->pat_bytes + pb->pat_off[j], (size_t)len) == 0",
                         "memcmp(pb->text + i + 1, pb->pat_bytes + pb->pat_off[j], (size_t)len) == 0"),
    # two-byte buckets
    "pair-key-swapped": ("uint32_t key = (uint32_t)pb->text[i] * 256u + pb->text[i + 1];",
                         "uint32_t key = (uint32_t)pb->text[i + 1] * 256u + pb->text[i];"),
    "pair-drops-short-list": ("uint64_t a = 0, a_end = pb->n_short, b = 0, b_end = 0;",
                              "uint64_t a = 0, a_end = 0, b = 0, b_end = 0;"),
    "pair-no-last-offset": ("    if (i + 1 < pb->n_text) {\n        uint32_t key",
                            "    if (i + 1 >= pb->n_text) return;\n    {\n        uint32_t key"),
    "pair-short-list-first": ("if (b == b_end || (a < a_end && pb->short_ids[a] < pb->pair_ids[b]))",
                              "if (a < a_end)"),
    "pair-bucket-drops-last": ("b_end = pb->pair_at[key + 1];", "b_end = pb->pair_at[key + 1] - (b < pb->pair_at[key + 1]);"),
    "pair-short-by-length-2": ("if (pat_len[j] == 1)\n                short_ids[n_short++] = j;",
                               "if (pat_len[j] <= 2)\n                short_ids[n_short++] = j;"),
}


@pytest.mark.parametrize("mutant", sorted(MUTANTS))
def test_pins_catch_planted_mistake(mutant, tmp_path):
    src = Path(oracle.__file__).resolve().parent / "glop_oracle.c"
    text = src.read_text()
    old, new = MUTANTS[mutant]
    assert text.count(old) == 1, f"mutation site for {mutant} not found exactly once"
    mut_src = tmp_path / "mutant.c"
    mut_src.write_text(text.replace(old, new))
    lib = oracle._bind(oracle.compile_oracle(mut_src, tmp_path / "libmutant.so"))
    assert pin_failures(lib, n_random=60) != [], f"no pin detects mutant {mutant}"


def test_concatenated_oracle_split_equals_per_chunk_oracle():
    """The batched tests' reference: one oracle run over chunks laid end to end,
    split by chunk, equals the oracle run on each chunk alone."""
    from chunks import split_by_chunk

    pats, text, offs, sizes, _ = synth.make_chunks(count=24)
    off, ids, _, _ = oracle.match(text, pats, bucketed=True)
    k, rel, kid = split_by_chunk(off, ids, [len(p) for p in pats], offs, sizes)
    for c, (o, n) in enumerate(zip(offs.tolist(), sizes)):
        w_off, w_ids, _, w_total = oracle.match(text[o:o + n], pats, bucketed=True)
        sel = k == c
        assert np.array_equal(rel[sel], w_off.astype(np.int64)) and np.array_equal(kid[sel], w_ids.astype(np.int64))
    # An occurrence that crosses a chunk boundary is found in the concatenation and dropped.
    text = np.frombuffer(b"abcab" + b"cabc" + b"c", dtype=np.uint8)
    pats = [b"ca", b"bc", b"c"]
    off, ids, _, _ = oracle.match(text, pats, bucketed=False)
    k, rel, kid = split_by_chunk(off, ids, [len(p) for p in pats], [0, 5, 9], [5, 4, 1])
    got = list(zip(k.tolist(), rel.tolist(), kid.tolist()))
    assert got == [(0, 1, 1), (0, 2, 0), (0, 2, 2), (1, 0, 0), (1, 0, 2), (1, 2, 1), (1, 3, 2), (2, 0, 2)]
    assert (4, 1) in set(zip(off.tolist(), ids.tolist()))  # "bc" across the first boundary
