"""C-ABI library: exports, the trie compiler and argument errors (CPU only).

The trie compiler is checked through ``glop_cpu_walk``, the failureless walk
over the compiled tables on the host, against the oracle; no GPU is touched.
"""

import ctypes
import random
import re
from pathlib import Path

import numpy as np
import pytest

import oracle
import synth
from brute import brute_matches
from golden_io import load_examples

ROOT = Path(__file__).resolve().parent.parent
glop = pytest.importorskip("paper_1704_02278_amd", reason="libglop.so not built")


def header_functions():
    text = (ROOT / "include" / "glop.h").read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(glop_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    names = header_functions()
    assert "glop_build" in names and "glop_match" in names and len(names) >= 12
    lib = ctypes.CDLL(str(glop.LIB_PATH))
    missing = [n for n in names if not hasattr(lib, n)]
    assert missing == []
    assert set(names) == set(glop.EXPORTED)


def host_dict(patterns, **opts):
    return glop.Dict(patterns, device=False, **opts)


def test_hand_examples_through_compiled_trie():
    for ex in load_examples():
        d = host_dict(ex.patterns)
        off, ids, counts, total = d.cpu_walk(ex.text)
        assert list(zip(off.tolist(), ids.tolist())) == ex.matches, ex.name
        assert counts.tolist() == ex.counts and total == len(ex.matches)


@pytest.mark.parametrize("layout", [glop.GLOP_LAYOUT_DENSE, glop.GLOP_LAYOUT_HYBRID])
def test_random_small_cases_against_brute_force(layout):
    # Patterns up to 9 bytes over 1-3 letters: with the hybrid layout the trie
    # goes well below its dense rows (depth <= 2), through states with one
    # and with several children.
    rng = random.Random(99)
    for _ in range(200):
        alpha = b"abc"[: rng.randint(1, 3)]
        pats = [bytes(rng.choice(alpha) for _ in range(rng.randint(1, 9))) for _ in range(rng.randint(1, 7))]
        text = bytes(rng.choice(alpha) for _ in range(rng.randint(0, 200)))
        want, want_counts = brute_matches(text, pats)
        d = host_dict(pats, layout=layout, prefix_len=glop.GLOP_PREFIX_FULL)
        off, ids, counts, total = d.cpu_walk(text, threads=rng.randint(1, 4))
        assert list(zip(off.tolist(), ids.tolist())) == want
        assert counts.tolist() == want_counts and total == len(want)


@pytest.mark.parametrize("name,n_bytes", [("tiny", None), ("medium", 2 << 20), ("large", 1 << 20)])
def test_hybrid_layout_walks_like_the_dense_table(name, n_bytes):
    """The hybrid layout, walked in its device form on the host (dense rows to
    depth 2, then nodes), against the oracle; it is a small fraction of the
    dense table and keeps every state."""
    pats, text, _ = synth.make_workload(name, n_bytes=n_bytes)
    o_off, o_ids, o_counts, o_total = oracle.match(text, pats, bucketed=2)
    for prefix in (0, glop.GLOP_PREFIX_FULL):
        dense = host_dict(pats, prefix_len=prefix, layout=glop.GLOP_LAYOUT_DENSE).info()
        d = host_dict(pats, prefix_len=prefix, layout=glop.GLOP_LAYOUT_HYBRID)
        info = d.info()
        assert info["layout"] == glop.GLOP_LAYOUT_HYBRID and info["num_states"] == dense["num_states"]
        assert 1 < info["dense_states"] < info["num_states"]
        assert info["table_bytes"] < dense["table_bytes"] / 3
        off, ids, counts, total = d.cpu_walk(text, threads=8)
        assert total == o_total
        assert np.array_equal(off, o_off.astype(np.uint64)) and np.array_equal(ids, o_ids.astype(np.uint64))
        assert np.array_equal(counts, o_counts)


def test_automatic_layout_is_hybrid_only_for_large_tables():
    large, _, _ = synth.make_workload("large", n_bytes=1 << 16)
    medium, _, _ = synth.make_workload("medium", n_bytes=1 << 16)
    big = host_dict(large, prefix_len=glop.GLOP_PREFIX_FULL).info()  # 125 MB dense
    assert big["layout"] == glop.GLOP_LAYOUT_HYBRID and big["table_bytes"] < 8e6
    assert host_dict(large).info()["layout"] == glop.GLOP_LAYOUT_DENSE  # 8-byte prefixes: 30.5 MB
    m = host_dict(medium).info()
    assert m["layout"] == glop.GLOP_LAYOUT_DENSE and m["dense_states"] == m["num_states"]


@pytest.mark.parametrize("name,n_bytes", [("tiny", None), ("medium", 2 << 20), ("large", 1 << 20)])
def test_compiled_trie_matches_oracle_on_workloads(name, n_bytes):
    pats, text, _ = synth.make_workload(name, n_bytes=n_bytes)
    o_off, o_ids, o_counts, o_total = oracle.match(text, pats)
    off, ids, counts, total = host_dict(pats).cpu_walk(text, threads=8)
    assert total == o_total
    assert np.array_equal(off, o_off.astype(np.uint64)) and np.array_equal(ids, o_ids.astype(np.uint64))
    assert np.array_equal(counts, o_counts)


def test_state_count_is_distinct_prefixes_plus_root():
    pats = synth.gen_patterns(synth.WORKLOADS["medium"].patterns, 5, 77)
    prefixes = {p[:k] for p in pats for k in range(1, len(p) + 1)}
    info = host_dict(pats, prefix_len=glop.GLOP_PREFIX_FULL).info()
    assert info["num_states"] == len(prefixes) + 1
    # The automatic engine truncates this dictionary to 8-byte prefixes.
    heads = {p[:k] for p in pats for k in range(1, min(8, len(p)) + 1)}
    auto = host_dict(pats).info()
    assert auto["prefix_len"] == 8 and auto["num_states"] == len(heads) + 1
    assert info["num_classes"] == len({b for p in pats for b in p}) + 1
    assert info["min_len"] == 8 and info["max_len"] <= 64
    # medium dictionary: 4-byte q-grams probed at every aligned word
    assert info["filter"] == glop.GLOP_FILTER_QGRAM and info["stride"] == 4 and info["qgram"] == 4


def test_prefix_table_holds_the_distinct_prefixes():
    """The walk's first D steps come from an exact table of the patterns'
    D-byte prefixes: D = 8 when every pattern is at least 8 bytes long, else 4;
    no table when some pattern is shorter than 4 bytes."""
    pats = synth.gen_patterns(synth.WORKLOADS["medium"].patterns, 5, 77)
    assert min(map(len, pats)) >= 8
    info = host_dict(pats).info()
    assert info["prefix_depth"] == 8 and info["prefix_keys"] == len({p[:8] for p in pats})
    slots = info["prefix_slots"]
    assert slots >= 2 * info["prefix_keys"] and slots & (slots - 1) == 0 and slots >= 64
    mid = host_dict(pats + [b"abcdefg"]).info()
    assert mid["prefix_depth"] == 4 and mid["prefix_keys"] == len({p[:4] for p in pats + [b"abcdefg"]})
    short = host_dict(pats + [b"abc"]).info()
    assert short["prefix_keys"] == 0 and short["prefix_slots"] == 0 and short["prefix_depth"] == 0
    # Patterns of exactly 4 bytes end on the table's own states; a longer
    # pattern through one of them adds no key.
    four = host_dict([b"GET ", b"POST", b"GET /x"]).info()
    assert four["prefix_depth"] == 4 and four["prefix_keys"] == 2 and four["prefix_slots"] == 64
    # The whole-pattern trie keys on the same prefixes (its walks go on below).
    full = host_dict(pats, prefix_len=glop.GLOP_PREFIX_FULL).info()
    assert full["prefix_depth"] == 8 and full["prefix_keys"] == info["prefix_keys"]


def test_second_filter_only_where_stride_one_walks_follow():
    """The second filter (checked before stride-1 walks) exists for stride-1
    dictionaries whose first filter does not use the second hash."""
    large = synth.gen_patterns(synth.WORKLOADS["large"].patterns, 300, 5)
    assert min(map(len, large)) < 7
    info = host_dict(large).info()
    assert info["stride"] == 1 and info["probe_bits"] == 3 and info["filter2_log2"] == 17
    assert host_dict(large, probe_bits=1).info()["filter2_log2"] == 17
    assert host_dict(large, probe_bits=2).info()["filter2_log2"] == 0
    assert host_dict(large, filter=glop.GLOP_FILTER_NONE).info()["filter2_log2"] == 0
    medium = synth.gen_patterns(synth.WORKLOADS["medium"].patterns, 300, 5)
    assert host_dict(medium).info()["stride"] == 4 and host_dict(medium).info()["filter2_log2"] == 0
    assert host_dict(medium, stride=1).info()["filter2_log2"] == 17


def test_automatic_options():
    assert host_dict([b"abcdefg"]).info()["stride"] == 4
    assert host_dict([b"abcdef"]).info()["stride"] == 1
    i = host_dict([b"ab", b"abcdef"]).info()
    assert i["qgram"] == 2 and i["stride"] == 1
    assert host_dict([]).info()["filter"] == glop.GLOP_FILTER_NONE


def test_build_errors():
    with pytest.raises(glop.GlopError) as e:
        host_dict([b"abc", b""])
    assert e.value.code == glop.GLOP_EINVAL
    with pytest.raises(glop.GlopError) as e:
        host_dict([b"x" * (glop.GLOP_MAX_PATTERN_LEN + 1)])
    assert e.value.code == glop.GLOP_ETOOLONG
    for bad in (dict(stride=4, qgram=4, filter=glop.GLOP_FILTER_QGRAM),  # needs length >= 7
                dict(qgram=5, filter=glop.GLOP_FILTER_QGRAM),
                dict(bitmap_log2=25, filter=glop.GLOP_FILTER_QGRAM),
                dict(stride=4, filter=glop.GLOP_FILTER_NONE),
                dict(filter=7), dict(layout=3), dict(placement=3)):
        with pytest.raises(glop.GlopError) as e:
            host_dict([b"abcd"], **bad)
        assert e.value.code == glop.GLOP_EINVAL


def test_match_on_host_only_handle_is_refused():
    d = host_dict([b"abc"])
    rc = glop.glop_match(d.handle, None, 0, None, 0, ctypes.c_void_p(8), None)
    assert rc == glop.GLOP_ENODEV
    rc = glop.glop_match(d.handle, None, 5, None, 0, ctypes.c_void_p(8), None)
    assert rc == glop.GLOP_EINVAL  # NULL text with len > 0 is caught first


def test_workspace_grows_with_length():
    d = host_dict([b"abc"])
    a, b = d.workspace_bytes(1 << 20), d.workspace_bytes(1 << 30)
    assert 0 < a < b and b % 256 == 0


def test_workspace_never_shrinks_as_the_text_grows():
    # A workspace sized for one length serves every shorter text (the
    # host-streamed form sizes one for its largest piece, and a launch lays
    # out at most what the query sized): across tile and round boundaries the
    # size never drops as the length grows.
    d = host_dict([b"abc"])
    lens = sorted({max(0, k * 8192 + e) for k in (0, 1, 255, 256, 257, 1024, 1025, 4096)
                   for e in range(-20, 21)})
    sizes = [d.workspace_bytes(n) for n in lens]
    assert all(a <= b for a, b in zip(sizes, sizes[1:]))
    assert all(s % 256 == 0 for s in sizes)


def test_size_getters_and_stream_probe_argument_checks():
    d = host_dict([b"abc", b"de", b"fghij"])
    assert glop.glop_num_patterns(d.handle) == 3 == d.num_patterns
    assert glop.glop_max_len(d.handle) == 5 == d.max_len
    assert glop.glop_num_patterns(None) == 0 and glop.glop_max_len(None) == 0
    # Rejected before any device work: no sink, or data that is not 16-byte aligned.
    assert glop.glop_stream_read(None, 0, None, None) == glop.GLOP_EINVAL
    assert glop.glop_stream_read(17, 64, 4096, None) == glop.GLOP_EINVAL
    assert glop.glop_stream_read(None, 16, 4096, None) == glop.GLOP_EINVAL


def test_autotune_argument_checks_need_no_device():
    pats = [b"abc", b"abd"]
    keep, ptrs, lens, n = glop._pattern_arrays(pats)
    r = glop.glop_tune_result_t()
    u8pp = glop._u8pp
    assert glop.glop_autotune(ctypes.cast(ptrs, u8pp), lens, n, 4096, 64, None, None) == glop.GLOP_EINVAL
    assert glop.glop_autotune(ctypes.cast(ptrs, u8pp), lens, n, None, 64, None, ctypes.byref(r)) == glop.GLOP_EINVAL
    assert glop.glop_autotune(ctypes.cast(ptrs, u8pp), lens, n, 4096, 0, None, ctypes.byref(r)) == glop.GLOP_EINVAL
    assert glop.glop_strerror(glop.GLOP_EINTERNAL) == b"internal consistency check failed"


def test_server_create_argument_checks():
    bad = glop.glop_server_opts(7, 0, 0, 0, 0, 1, 0)
    assert not glop.glop_server_create(ctypes.byref(bad))
    assert glop.glop_last_error() == glop.GLOP_EINVAL
    assert glop.glop_server_add_dict(None, None, None) == glop.GLOP_EINVAL
    assert glop.glop_server_release(None, 1) == glop.GLOP_EINVAL
    assert glop.glop_server_submit(None, 0, None, 0, 0, -1, None) == glop.GLOP_EINVAL
    got = ctypes.c_uint32()
    assert glop.glop_server_poll(None, None, 0, 0, ctypes.byref(got)) == glop.GLOP_EINVAL
    glop.glop_server_destroy(None)  # ignored
    t0 = glop.glop_now_ns()
    assert glop.glop_now_ns() >= t0 > 0


def test_tile_sizes():
    with pytest.raises(glop.GlopError):
        host_dict([b"abcdefgh"], tile_kib=16)
    assert host_dict([b"abcdefgh"], tile_kib=8).info()["tile_kib"] == 8
    # 4 KiB tiles for the automatic filters: stride 4 with two hash bits (a
    # shortest pattern of 7 bytes or more), stride 1 blocked (shorter ones).
    long4 = host_dict([b"abcdefgh", b"bcdefghij"], tile_kib=4).info()
    assert (long4["tile_kib"], long4["stride"], long4["probe_bits"]) == (4, 4, 2)
    short4 = host_dict([b"abcd", b"bcdefghij"], tile_kib=4).info()
    assert (short4["tile_kib"], short4["stride"], short4["probe_bits"]) == (4, 1, 3)
    # Other filters have no 4 KiB kernels.
    for opts in (dict(probe_bits=1), dict(stride=1, probe_bits=2), dict(filter=glop.GLOP_FILTER_NONE),
                 dict(qgram=2, stride=1)):
        with pytest.raises(glop.GlopError):
            host_dict([b"abcdefgh"], tile_kib=4, **opts)
    # The workspace holds per-tile results: twice the tiles, about twice the bytes.
    n = 64 << 20
    w8 = host_dict([b"abcdefgh"], tile_kib=8).workspace_bytes(n)
    w4 = host_dict([b"abcdefgh"], tile_kib=4).workspace_bytes(n)
    assert 1.8 * w8 < w4 < 2.2 * w8
    # Automatic: 4 KiB tiles for stride 4 with two hash bits, 8 KiB otherwise.
    assert host_dict([b"abcdefgh", b"bcdefghij"]).info()["tile_kib"] == 4
    assert host_dict([b"abcd", b"bcdefghij"]).info()["tile_kib"] == 8
    assert host_dict([b"abcdefgh"], probe_bits=1).info()["tile_kib"] == 8


def test_stride1_tile_follows_text_length():
    # The automatic stride-1 blocked filter runs 4 KiB tiles on texts of at
    # most 640 KiB per CU and 8 KiB above: its workspace is that of the
    # explicit tile at each length (a host-built handle counts one CU).
    pats = [b"abcd", b"bcdefghij"]
    auto, t4, t8 = host_dict(pats), host_dict(pats, tile_kib=4), host_dict(pats, tile_kib=8)
    assert (auto.info()["stride"], auto.info()["probe_bits"]) == (1, 3)
    for n in (1, 4096, 64 << 10, 640 << 10):
        assert auto.workspace_bytes(n) == t4.workspace_bytes(n), n
    for n in ((640 << 10) + 1, 1 << 30, 64 << 30):
        assert auto.workspace_bytes(n) == t8.workspace_bytes(n), n
    # The stride-4 filter keeps 4 KiB tiles at every length.
    long_auto, long4 = host_dict([b"abcdefgh", b"bcdefghij"]), host_dict([b"abcdefgh", b"bcdefghij"], tile_kib=4)
    for n in (4096, 1 << 30, 64 << 30):
        assert long_auto.workspace_bytes(n) == long4.workspace_bytes(n), n
    # The static workspace's text limit is the last length that fits.
    limit = int(glop.glop_static_max_len(auto.handle))
    assert auto.workspace_bytes(limit) <= 32 << 20 < auto.workspace_bytes(limit + 1)


def test_batch_tile_follows_batch_size():
    # Automatic dictionaries run 4 KiB batch tiles when the batch's byte bound
    # is at most 64 KiB per CU and the filter has 4 KiB kernels, else 8 KiB; a
    # given tile_kib holds at every size (a host-built handle counts one CU).
    for pats in ([b"abcdefgh", b"bcdefghij"], [b"abcd", b"bcdefghij"]):
        auto, t4, t8 = host_dict(pats), host_dict(pats, tile_kib=4), host_dict(pats, tile_kib=8)
        for n in (1, 4096, 64 << 10):
            assert auto.batch_workspace_bytes(3, n) == t4.batch_workspace_bytes(3, n), n
        for n in ((64 << 10) + 1, 640 << 10, 1 << 30):
            assert auto.batch_workspace_bytes(3, n) == t8.batch_workspace_bytes(3, n), n
        assert t4.batch_workspace_bytes(3, 1 << 30) > 1.8 * t8.batch_workspace_bytes(3, 1 << 30)
    # Filters without 4 KiB kernels keep 8 KiB.
    other, other8 = host_dict([b"abcdefgh"], probe_bits=1), host_dict([b"abcdefgh"], probe_bits=1, tile_kib=8)
    assert other.batch_workspace_bytes(3, 4096) == other8.batch_workspace_bytes(3, 4096)
