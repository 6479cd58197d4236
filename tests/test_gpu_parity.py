"""HIP path vs the CPU oracle, bit-exact (needs an MI355X).

Every case goes through the C-ABI (``glop_build_ex`` / ``glop_match_ws``) via
the ctypes binding.  Sizes span several 8 KiB tiles with ragged tails; edge
cases cover empty inputs, unaligned text, tile-boundary straddles, dense
matches (the staging-overflow path), truncation and binary bytes.
"""

import random

import numpy as np
import pytest
import torch

import synth
from brute import brute_matches
from golden_io import load_examples

pytestmark = pytest.mark.gpu

glop = pytest.importorskip("paper_1704_02278_amd")
from gpu_util import assert_same, build_variant, gpu_match, oracle_match, say, to_device, variants_for  # noqa: E402


def test_hand_examples_every_variant():
    for ex in load_examples():
        for opts in variants_for(ex.patterns):
            say("hand", ex.name, opts)
            d = build_variant(ex.patterns, opts)
            if d is None:
                continue
            off, ids, counts, total = gpu_match(d, to_device(ex.text))
            assert list(zip(off.tolist(), ids.tolist())) == ex.matches, (ex.name, opts)
            assert counts.tolist() == ex.counts and total == len(ex.matches), (ex.name, opts)


def test_random_small_cases_vs_brute_force():
    rng = random.Random(4242)
    for k in range(60):
        alpha = b"abc"[: rng.randint(1, 3)]
        pats = [bytes(rng.choice(alpha) for _ in range(rng.randint(1, 9))) for _ in range(rng.randint(1, 7))]
        text = bytes(rng.choice(alpha) for _ in range(rng.randint(0, 3000)))
        want, want_counts = brute_matches(text, pats)
        for opts in variants_for(pats):
            say("random", k, len(text), opts)
            d = build_variant(pats, opts)
            if d is None:
                continue
            off, ids, counts, total = gpu_match(d, to_device(text, shift=k % 16))
            assert list(zip(off.tolist(), ids.tolist())) == want, (k, opts)
            assert counts.tolist() == want_counts and total == len(want), (k, opts)


def test_dense_tile_totals_are_stable_over_repeated_calls():
    """A dense single-tile text (every other byte starts a match, so the tile's
    535 starts are walked in nine batches by all the workgroup's waves), matched
    2,000 times in two-call pairs as gpu_match makes them: every total must be
    the brute-force count.  Before the kernels waited for their LDS atomics at
    each barrier, the record count read after the last walk phase missed the
    last batch of one wave in about one call in 300."""
    rng = random.Random(4242)
    for _ in range(21):  # the 21st small case of the random test above
        alpha = b"abc"[: rng.randint(1, 3)]
        pats = [bytes(rng.choice(alpha) for _ in range(rng.randint(1, 9))) for _ in range(rng.randint(1, 7))]
        text = bytes(rng.choice(alpha) for _ in range(rng.randint(0, 3000)))
    want, _ = brute_matches(text, pats)
    assert len(want) == 1093
    t = to_device(text, shift=4)
    for opts in (dict(), dict(layout=glop.GLOP_LAYOUT_HYBRID)):
        d = build_variant(pats, opts)
        ws = torch.empty(d.workspace_bytes(len(text)) + 256, dtype=torch.uint8, device="cuda")
        ws = ws[(-ws.data_ptr()) % 256:]
        total = torch.zeros(1, dtype=torch.int64, device="cuda")
        counts = torch.empty(d.num_patterns, dtype=torch.int64, device="cuda")
        bad = []
        for it in range(1000):
            for cap in (1024, len(want)):
                out = torch.empty((cap, 2), dtype=torch.int64, device="cuda")
                d.match_into(t, out, counts, max_matches=cap, total=total, workspace=ws)
                got = int(total.item())
                if got != len(want):
                    bad.append((it, cap, got))
        assert not bad, (opts, len(bad), bad[:5])


@pytest.mark.parametrize("name,n_bytes", [("tiny", None), ("medium", 48 << 20), ("large", 8 << 20)])
def test_workload_parity(name, n_bytes):
    pats, text, plants = synth.make_workload(name, n_bytes=n_bytes)
    want = oracle_match(text, pats)
    assert want[3] >= len(plants)
    t = to_device(text)
    for opts in variants_for(pats):
        say("workload", name, text.size, opts)
        d = build_variant(pats, opts)
        if d is not None:
            assert_same(gpu_match(d, t), want, f"{name} {opts}")


def test_unaligned_text_and_ragged_lengths():
    pats, text, _ = synth.make_workload("tiny", n_bytes=200_000)
    d = glop.Dict(pats)
    for shift in range(16):
        for n in (0, 1, 3, 4, 15, 16, 17, 1023, 1024, 1025, 8191, 8192, 8193, 8192 * 3 + 7, 200_000 - shift):
            sub = text[shift:shift + n]
            say("unaligned", shift, n)
            assert_same(gpu_match(d, to_device(sub, shift=shift)), oracle_match(sub, pats), f"shift {shift} n {n}")


@pytest.mark.parametrize("tile,short", [(8192, (b"HIS", b"ISTO")), (4096, (b"ISTO",)), (4096, ())])
def test_tile_boundary_straddles(tile, short):
    # One plant per tile, at every offset from 40 bytes before to 8 after the
    # tile's end, so occurrences straddle wave-tile and round boundaries.  The
    # 4 KiB cases have a shortest pattern of 4 bytes (stride 1) or 26 (stride
    # 4): the filters whose short texts run 4 KiB tiles by default.
    rng = np.random.default_rng(7)
    pats = [b"HISTORY-of-a-long-pattern-" + bytes([65 + k]) * (k + 1) for k in range(6)] + list(short)
    deltas = list(range(-40, 9))
    text = rng.integers(0x61, 0x7B, size=tile * (len(deltas) + 2), dtype=np.uint8)
    for m, dlt in enumerate(deltas, start=1):
        p = pats[m % 6]
        o = m * tile + dlt
        text[o:o + len(p)] = np.frombuffer(p, dtype=np.uint8)
    want = oracle_match(text, pats)
    for shift in (0, 5, 13):
        for opts in variants_for(pats):
            say("straddle", tile, len(short), shift, opts)
            d = build_variant(pats, opts)
            if d is not None:
                assert_same(gpu_match(d, to_device(text, shift=shift)), want, f"{opts}")


def test_dense_matches_take_the_overflow_path():
    pats = [b"a", b"aa", b"aaa", b"b"]
    text = b"a" * 70_000 + b"b" + b"a" * 33
    want = oracle_match(text, pats)
    for opts in variants_for(pats):
        say("dense", opts)
        d = build_variant(pats, opts)
        if d is not None:
            assert_same(gpu_match(d, to_device(text)), want, f"dense {opts}")


def test_truncation_keeps_sorted_prefix_and_full_counts():
    pats, text, _ = synth.make_workload("tiny")
    want = oracle_match(text, pats)
    d = glop.Dict(pats)
    t = to_device(text)
    for cap in (0, 1, 7, want[3] - 1, want[3], want[3] + 5):
        say("truncate", cap)
        off, ids, counts, total = gpu_match(d, t, max_matches=cap)
        k = min(cap, want[3])
        assert total == want[3] and np.array_equal(counts, want[2])
        assert np.array_equal(off, want[0][:k]) and np.array_equal(ids, want[1][:k])


def test_empty_inputs():
    say("empty")
    d = glop.Dict([b"abc", b"de"])
    off, ids, counts, total = gpu_match(d, to_device(b""))
    assert total == 0 and off.size == 0 and counts.tolist() == [0, 0]
    off, ids, counts, total = gpu_match(d, to_device(b"a"))  # shorter than every pattern
    assert total == 0 and counts.tolist() == [0, 0]
    e = glop.Dict([])
    off, ids, counts, total = gpu_match(e, to_device(b"abcabc"))
    assert total == 0 and off.size == 0


def test_binary_bytes():
    rng = np.random.default_rng(11)
    text = rng.integers(0, 4, size=300_000, dtype=np.uint8) * np.uint8(85)  # 0x00 0x55 0xAA 0xFF
    pats = [bytes((rng.integers(0, 4, size=int(L)) * 85).astype(np.uint8)) for L in rng.integers(1, 12, size=40)]
    pats += [b"\x00\xff", b"\xff\xff\xff\xff\xff\xff\xff\xff", b"\x00"]
    want = oracle_match(text, pats)
    for opts in variants_for(pats):
        say("binary", opts)
        d = build_variant(pats, opts)
        if d is not None:
            assert_same(gpu_match(d, to_device(text, shift=3)), want, f"binary {opts}")


def test_repeated_runs_are_identical():
    pats, text, _ = synth.make_workload("medium", n_bytes=8 << 20)
    d = glop.Dict(pats)
    t = to_device(text)
    first = gpu_match(d, t)
    for k in range(5):
        say("repeat", k)
        assert_same(gpu_match(d, t), first, f"repeat {k}")


def test_dense_hits_at_stride4_fill_the_workgroup_list():
    # A period-7 text that every 4-byte word of the pattern hits: over 1,000
    # hit words per 8 KiB tile, so each workgroup's deferred hit list fills
    # (later tiles walk at once) and tiles exceed their staging slots (the
    # emit kernel rescans them).  24 MiB gives each workgroup > 8 tiles.
    pats = [b"abcdefg", b"cdefgab", b"zzzzzzzz"]
    text = (b"abcdefg" * ((24 << 20) // 7 + 1))[: 24 << 20]
    want = oracle_match(text, pats)
    assert want[3] > 3_000_000
    t = to_device(text, shift=1)
    for opts in (dict(), dict(filter=glop.GLOP_FILTER_QGRAM, stride=4, qgram=4, probe_bits=1)):
        say("dense-stride4", opts)
        d = glop.Dict(pats, **opts)
        assert d.info()["stride"] == 4
        assert_same(gpu_match(d, t), want, f"dense stride4 {opts}")
    # Stride 1 lists surviving offsets the same way: the list fills after two
    # tiles, later tiles walk at once, and the emit kernel rescans them all.
    for opts in (dict(filter=glop.GLOP_FILTER_QGRAM, stride=1),
                 dict(filter=glop.GLOP_FILTER_QGRAM, stride=1, probe_bits=1)):
        say("dense-stride1", opts)
        d = glop.Dict(pats, **opts)
        assert d.info()["stride"] == 1
        assert_same(gpu_match(d, t), want, f"dense stride1 {opts}")


@pytest.mark.parametrize("n_pats,lo,hi", [(900, 8, 14), (2500, 8, 14), (900, 7, 12), (1500, 7, 12),
                                           (450, 4, 6), (900, 4, 6)])
def test_prefix_table_on_both_sides_of_the_lds_limit(n_pats, lo, hi):
    # The scan kernel uses the prefix table (8-byte keys when every pattern
    # has 8 bytes, else 4-byte keys) when it fits in LDS: up to 2,048 slots at
    # stride 4, 1,024 at stride 1, at most half full; otherwise its walks start
    # at the root.  These dictionaries land on both sides of both limits, with
    # both key lengths.  A 16-letter alphabet makes most offsets start some
    # pattern's first bytes.
    rng = np.random.default_rng(n_pats * 31 + lo)
    alpha = np.frombuffer(b"etaoinshrdlucmfw", dtype=np.uint8)
    pats = [bytes(alpha[rng.integers(0, 16, size=int(L))]) for L in rng.integers(lo, hi + 1, size=n_pats)]
    text = alpha[rng.integers(0, 16, size=3 << 20)]
    text[::97] = 0x0A  # lines, which the planter keeps occurrences inside
    assert len(synth.plant(text, pats, 2048, seed=5, stream_id=9)) > 1000
    want = oracle_match(text, pats)
    info = glop.Dict(pats).info()
    depth = 8 if lo >= 8 else 4
    assert info["prefix_depth"] == depth and info["prefix_keys"] == len({p[:depth] for p in pats})
    say("prefix-table", n_pats, lo, hi, info["prefix_slots"], info["stride"], want[3])
    t = to_device(text, shift=5)
    for opts in variants_for(pats):
        say("prefix-table", n_pats, opts)
        d = build_variant(pats, opts)
        if d is not None:
            assert_same(gpu_match(d, t), want, f"prefix table {n_pats} {opts}")


def test_item_count_flips_with_the_text_alignment():
    # 2 MiB is 256 tiles of 8 KiB when aligned (256 items of one tile on 256
    # CUs) but 257 tiles 15 bytes off (129 items of two): the launch's tile
    # count follows the text's own alignment, and its workspace layout must
    # still fit the size the library asks for (allocated here to the byte).
    pats, text, _ = synth.make_workload("medium", n_bytes=(2 << 20) + 64)
    d = glop.Dict(pats)
    for n in ((2 << 20) - 15, (2 << 20) - 1, 2 << 20, (2 << 20) + 1, (2 << 20) + 17):
        sub = text[:n]
        want = oracle_match(sub, pats)
        for shift in (0, 1, 15):
            say("alignment flip", n, shift)
            t = to_device(sub, shift=shift)
            nbytes = d.workspace_bytes(n)
            ws_buf = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
            ws = ws_buf[(-ws_buf.data_ptr()) % 256:][:nbytes]
            out = torch.empty((want[3] + 64, 2), dtype=torch.int64, device="cuda")
            counts = torch.empty(len(pats), dtype=torch.int64, device="cuda")
            total = torch.empty(1, dtype=torch.int64, device="cuda")
            d.match_into(t, out, counts, total=total, workspace=ws)
            torch.cuda.synchronize()
            got = (out[:want[3], 0].cpu().numpy().astype(np.uint64), out[:want[3], 1].cpu().numpy().astype(np.uint64),
                   counts.cpu().numpy().astype(np.uint64), int(total[0]))
            assert_same(got, want, f"n {n} shift {shift}")


def test_total_written_to_pinned_host_memory():
    # glop_match_ws may take a pinned host word for the total: the emit kernel
    # writes it directly (the server's single-request path relies on this).
    pats, text, _ = synth.make_workload("medium", n_bytes=6 << 20)
    want = oracle_match(text, pats)
    d = glop.Dict(pats)
    t = to_device(text)
    out = torch.empty((want[3] + 64, 2), dtype=torch.int64, device="cuda")
    counts = torch.empty(len(pats), dtype=torch.int64, device="cuda")
    ws = torch.empty(d.workspace_bytes(t.numel()) + 256, dtype=torch.uint8, device="cuda")
    ws = ws[(-ws.data_ptr()) % 256:][:d.workspace_bytes(t.numel())]
    host_total = torch.full((1,), -1, dtype=torch.int64).pin_memory()
    for k in range(3):
        say("pinned total", k)
        host_total.fill_(-1)
        d.match_into(t, out, counts, total=host_total, workspace=ws)
        torch.cuda.synchronize()
        assert int(host_total[0]) == want[3]
    assert np.array_equal(out[:want[3], 0].cpu().numpy().astype(np.uint64), want[0])


def test_table_layouts_and_placements_on_the_large_dictionary():
    """The whole-pattern trie of the large dictionary (325,458 states): the
    automatic layout is hybrid (about 6 MB instead of 125 MB), and dense, hybrid
    and (where it fits) LDS-placed rows all give the oracle's result; dense
    rows that cannot fit in LDS are refused at build."""
    pats, text, _ = synth.make_workload("large", n_bytes=6 << 20)
    want = oracle_match(text, pats, bucketed=2)
    t = to_device(text, shift=7)
    full = glop.GLOP_PREFIX_FULL
    auto = glop.Dict(pats, prefix_len=full)
    assert auto.info()["layout"] == glop.GLOP_LAYOUT_HYBRID and auto.info()["table_bytes"] < 8e6
    for opts in (dict(prefix_len=full), dict(prefix_len=full, layout=glop.GLOP_LAYOUT_DENSE),
                 dict(layout=glop.GLOP_LAYOUT_HYBRID), dict(layout=glop.GLOP_LAYOUT_HYBRID, filter=glop.GLOP_FILTER_NONE)):
        say("layout", opts)
        assert_same(gpu_match(glop.Dict(pats, **opts), t), want, f"large {opts}")
    with pytest.raises(glop.GlopError) as e:
        glop.Dict(pats, prefix_len=full, placement=glop.GLOP_PLACE_LDS)
    assert e.value.code == glop.GLOP_EINVAL


def test_lds_placed_rows_on_the_tiny_dictionary():
    pats, text, _ = synth.make_workload("tiny")
    want = oracle_match(text, pats)
    t = to_device(text, shift=1)
    auto = glop.Dict(pats, prefix_len=glop.GLOP_PREFIX_FULL)
    assert auto.info()["placement"] == glop.GLOP_PLACE_LDS  # a few KB of rows fit beside the filter
    for opts in (dict(prefix_len=glop.GLOP_PREFIX_FULL), dict(placement=glop.GLOP_PLACE_GLOBAL),
                 dict(placement=glop.GLOP_PLACE_LDS, layout=glop.GLOP_LAYOUT_HYBRID),
                 dict(placement=glop.GLOP_PLACE_LDS, filter=glop.GLOP_FILTER_NONE)):
        say("placement", opts)
        d = glop.Dict(pats, **opts)
        assert d.info()["placement"] == opts.get("placement", glop.GLOP_PLACE_LDS)
        assert_same(gpu_match(d, t), want, f"tiny {opts}")
