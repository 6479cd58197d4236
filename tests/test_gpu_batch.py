"""Batched matching (glop_match_batch) vs the oracle per chunk (needs an MI355X).

Every chunk of a batch must give exactly what the oracle gives for that chunk
alone: records (offsets relative to the chunk) in order, the chunk's record
count and position, and the batch's per-pattern counts.
"""

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

glop = pytest.importorskip("paper_1704_02278_amd")
from gpu_util import build_variant, oracle_match, say, variants_for  # noqa: E402


def _chunks_in_one_buffer(pieces, shift=3):
    """Upload byte strings back to back (at odd offsets) into one device buffer."""
    sizes = [len(p) for p in pieces]
    buf = torch.zeros(sum(sizes) + 64 * len(pieces) + 256, dtype=torch.uint8, device="cuda")
    views, pos = [], shift
    host = bytearray(buf.numel())
    for k, p in enumerate(pieces):
        host[pos:pos + len(p)] = p
        views.append((pos, len(p)))
        pos += len(p) + 1 + (k * 7) % 13
    buf.copy_(torch.frombuffer(bytes(host), dtype=torch.uint8))
    return buf, [buf[o:o + n] for o, n in views]


def _check_batch(d, pats, pieces, chunks, res):
    off, ids, cid, first, count, counts, total = res
    off, ids, cid = off.cpu().numpy(), ids.cpu().numpy(), cid.cpu().numpy()
    first, count = first.cpu().numpy(), count.cpu().numpy()
    want_counts = np.zeros(len(pats), dtype=np.uint64)
    pos = 0
    for c, p in enumerate(pieces):
        w_off, w_ids, w_counts, w_total = oracle_match(p, pats, threads=4)
        want_counts += w_counts
        assert first[c] == pos and count[c] == w_total, f"chunk {c}: first/count"
        seg = slice(pos, pos + w_total)
        assert np.array_equal(off[seg].astype(np.uint64), w_off), f"chunk {c}: offsets"
        assert np.array_equal(ids[seg].astype(np.uint64), w_ids), f"chunk {c}: ids"
        assert np.all(cid[seg] == c)
        pos += w_total
    assert total == pos and np.array_equal(counts.cpu().numpy().astype(np.uint64), want_counts)


def _mixed_pieces(text, rng, n):
    # Around both tile sizes (small batches run 4 KiB tiles, larger ones 8 KiB).
    sizes = [0, 1, 3, 7, 8, 4095, 4096, 4097, 8191, 8192, 8193, 16383, 16384, 16385, 1 << 16]
    sizes += [int(x) for x in np.exp(rng.uniform(0, np.log(300_000), size=n - len(sizes)))]
    pieces, pos = [], 0
    for s in sizes:
        if pos + s > text.size:
            pos = 0
        pieces.append(text[pos:pos + s].tobytes())
        pos += s + int(rng.integers(0, 5000))
    return pieces


@pytest.mark.parametrize("name", ["tiny", "medium"])
def test_batch_equals_each_chunk_alone(name):
    rng = np.random.default_rng(5)
    pats, text, _ = synth.make_workload(name, n_bytes=24 << 20)
    pieces = _mixed_pieces(text, rng, 150)
    buf, chunks = _chunks_in_one_buffer(pieces)
    variants = variants_for(pats) + [dict(prefix_len=glop.GLOP_PREFIX_FULL)]
    for opts in variants:
        say("batch", name, len(pieces), opts)
        d = build_variant(pats, opts)
        if d is not None:
            _check_batch(d, pats, pieces, chunks, d.match_batch(chunks))


def test_batch_truncation_and_positions():
    pats, text, _ = synth.make_workload("tiny", n_bytes=2 << 20)
    pieces = [text[k * 100_000:(k + 1) * 100_000].tobytes() for k in range(20)]
    buf, chunks = _chunks_in_one_buffer(pieces)
    d = glop.Dict(pats)
    full = d.match_batch(chunks)
    for cap in (0, 1, 57, full[6] - 1):
        say("batch-truncate", cap)
        off, ids, cid, first, count, counts, total = d.match_batch(chunks, max_matches=cap)
        assert total == full[6] and off.numel() == min(cap, total)
        assert torch.equal(first, full[3]) and torch.equal(count, full[4]) and torch.equal(counts, full[5])
        assert torch.equal(off, full[0][:cap]) and torch.equal(ids, full[1][:cap]) and torch.equal(cid, full[2][:cap])


def test_batch_over_capacity_reports_max_total():
    pats, text, _ = synth.make_workload("tiny", n_bytes=1 << 20)
    pieces = [text[: 300_000].tobytes(), text[300_000: 700_000].tobytes()]
    buf, chunks = _chunks_in_one_buffer(pieces)
    d = glop.Dict(pats)
    dev = buf.device
    table = torch.tensor([[c.data_ptr(), c.numel()] for c in chunks], dtype=torch.int64).to(dev)
    small = 200_000  # far below the 700,000 bytes the chunks hold
    ws = torch.empty(d.batch_workspace_bytes(2, small) + 256, dtype=torch.uint8, device=dev)
    ws = ws[(-ws.data_ptr()) % 256:]
    out = torch.empty((1024, 2), dtype=torch.int64, device=dev)
    first = torch.full((2,), 7, dtype=torch.int64, device=dev)
    count = torch.full((2,), 7, dtype=torch.int64, device=dev)
    counts = torch.full((len(pats),), 7, dtype=torch.int64, device=dev)
    total = torch.zeros(1, dtype=torch.int64, device=dev)
    say("batch-overflow")
    d.match_batch_into(table, 2, small, out, first, count, counts, total, ws)
    torch.cuda.synchronize()
    assert total.item() == -1  # UINT64_MAX read as int64
    assert first.tolist() == [0, 0] and count.tolist() == [0, 0] and int(counts.sum()) == 0


def test_batch_dense_chunks_take_the_rescan_path():
    pats = [b"abcdefg", b"cdefgab", b"bcdefga"]
    pieces = [(b"abcdefg" * 9000)[: 60_000 + 17 * k] for k in range(12)] + [b"", b"abc", b"xyz" * 1000]
    buf, chunks = _chunks_in_one_buffer(pieces, shift=5)
    for opts in (dict(), dict(prefix_len=glop.GLOP_PREFIX_FULL), dict(filter=glop.GLOP_FILTER_QGRAM, stride=1)):
        say("batch-dense", opts)
        d = glop.Dict(pats, **opts)
        _check_batch(d, pats, pieces, chunks, d.match_batch(chunks))


def test_batch_graph_replays_with_a_new_chunk_table():
    pats, text, _ = synth.make_workload("medium", n_bytes=16 << 20)
    rng = np.random.default_rng(9)
    pieces_a = _mixed_pieces(text, rng, 60)
    pieces_b = list(reversed(_mixed_pieces(text[1000:], rng, 60)))
    buf_a, chunks_a = _chunks_in_one_buffer(pieces_a)
    buf_b, chunks_b = _chunks_in_one_buffer(pieces_b, shift=11)
    n = 60
    cap_bytes = max(sum(map(len, pieces_a)), sum(map(len, pieces_b)))
    d = glop.Dict(pats)
    dev = buf_a.device
    table_a = torch.tensor([[c.data_ptr() if c.numel() else 0, c.numel()] for c in chunks_a], dtype=torch.int64).to(dev)
    table_b = torch.tensor([[c.data_ptr() if c.numel() else 0, c.numel()] for c in chunks_b], dtype=torch.int64).to(dev)
    table = table_a.clone()
    ws = torch.empty(d.batch_workspace_bytes(n, cap_bytes) + 256, dtype=torch.uint8, device=dev)
    ws = ws[(-ws.data_ptr()) % 256:]
    out = torch.empty((200_000, 2), dtype=torch.int64, device=dev)
    first = torch.empty(n, dtype=torch.int64, device=dev)
    count = torch.empty(n, dtype=torch.int64, device=dev)
    counts = torch.empty(len(pats), dtype=torch.int64, device=dev)
    total = torch.zeros(1, dtype=torch.int64, device=dev)

    def snapshot():
        torch.cuda.synchronize()
        t = int(total.item())
        return (out[:t].clone(), first.clone(), count.clone(), counts.clone(), t)

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):  # warm-up outside capture
        d.match_batch_into(table, n, cap_bytes, out, first, count, counts, total, ws)
    torch.cuda.current_stream().wait_stream(s)
    eager_a = snapshot()
    table.copy_(table_b)
    d.match_batch_into(table, n, cap_bytes, out, first, count, counts, total, ws)
    eager_b = snapshot()

    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        d.match_batch_into(table, n, cap_bytes, out, first, count, counts, total, ws)
    for k, (tbl, want) in enumerate([(table_a, eager_a), (table_b, eager_b), (table_a, eager_a), (table_b, eager_b)]):
        say("graph-replay", k)
        table.copy_(tbl)
        out.zero_()
        torch.cuda.synchronize()
        g.replay()
        got = snapshot()
        assert got[4] == want[4]
        for a, b in zip(got[:4], want[:4]):
            assert torch.equal(a, b), f"replay {k} differs from the eager result"
    _check_batch(d, pats, pieces_b, chunks_b,
                 (out[:eager_b[4], 0], out[:eager_b[4], 1] & 0xFFFFFFFF, out[:eager_b[4], 1] >> 32,
                  first, count, counts, eager_b[4]))


SENTINEL = -0x0123456789ABCDEF


def test_batch_sliced_outputs_each_chunk_into_its_own_slice():
    """glop_match_batch_sliced: chunk c's first min(count, cap_c) records land in
    its own slice and nothing else is written, whatever the other chunks hold:
    dense chunks (the emit kernel's rescan path) beside sparse ones, chunks that
    span several work items (their first record lies in an earlier item), caps
    of 0, 1, below, at and above the chunk's count."""
    rng = np.random.default_rng(11)
    pats, text, _ = synth.make_workload("medium", n_bytes=8 << 20)
    pats = pats + [b"abcdefgh", b"bcdefgha"]
    dense = (b"abcdefgh" * 80_000)
    pieces = [dense[:300_000], text[:200_000].tobytes(), dense[3:900_003], text[300_000:301_000].tobytes(), b"",
              text[400_000:1_400_000].tobytes(), dense[:20_000], text[2_000_000:2_000_007].tobytes()]
    pieces += _mixed_pieces(text, rng, 40)
    buf, chunks = _chunks_in_one_buffer(pieces)
    want = [oracle_match(p, pats, threads=4) for p in pieces]
    caps = []
    for k, (_, _, _, w_total) in enumerate(want):
        choice = k % 5
        caps.append([0, 1, max(0, w_total - 3), w_total, w_total + 5][choice])
    gap = 3
    slice_first = np.zeros(len(pieces), dtype=np.int64)
    slice_first[1:] = np.cumsum(np.array(caps, dtype=np.int64) + gap)[:-1]
    n_out = int(slice_first[-1] + caps[-1] + gap)
    dev = buf.device
    table = torch.tensor([[c.data_ptr() if c.numel() else 0, c.numel()] for c in chunks], dtype=torch.int64).to(dev)
    total_bytes = sum(len(p) for p in pieces)
    for opts in (dict(), dict(filter=glop.GLOP_FILTER_QGRAM, stride=1), dict(prefix_len=glop.GLOP_PREFIX_FULL)):
        say("batch-sliced", len(pieces), opts)
        d = glop.Dict(pats, **opts)
        ws = torch.empty(d.batch_workspace_bytes(len(pieces), total_bytes) + 256, dtype=torch.uint8, device=dev)
        ws = ws[(-ws.data_ptr()) % 256:]
        out = torch.full((n_out, 2), SENTINEL, dtype=torch.int64, device=dev)
        first = torch.empty(len(pieces), dtype=torch.int64, device=dev)
        count = torch.empty(len(pieces), dtype=torch.int64, device=dev)
        counts = torch.empty(len(pats), dtype=torch.int64, device=dev)
        total = torch.zeros(1, dtype=torch.int64, device=dev)
        sf = torch.from_numpy(slice_first).to(dev)
        sc = torch.tensor(caps, dtype=torch.int64, device=dev)
        d.match_batch_sliced_into(table, len(pieces), total_bytes, out, sf, sc, first, count, counts, total, ws)
        torch.cuda.synchronize()
        o = out.cpu().numpy()
        written = np.zeros(n_out, dtype=bool)
        pos = 0
        want_counts = np.zeros(len(pats), dtype=np.uint64)
        for c, (w_off, w_ids, w_counts, w_total) in enumerate(want):
            assert int(count[c]) == w_total and int(first[c]) == pos, f"chunk {c}: count/first"
            k = min(w_total, caps[c])
            seg = o[slice_first[c]:slice_first[c] + k]
            assert np.array_equal(seg[:, 0].astype(np.uint64), w_off[:k]), f"chunk {c}: offsets"
            assert np.array_equal((seg[:, 1] & 0xFFFFFFFF).astype(np.uint64), w_ids[:k]), f"chunk {c}: ids"
            assert np.all(seg[:, 1] >> 32 == c), f"chunk {c}: chunk field"
            written[slice_first[c]:slice_first[c] + k] = True
            pos += w_total
            want_counts += w_counts
        assert np.all(o[~written] == SENTINEL), "a record was written outside its chunk's slice"
        assert int(total.item()) == pos
        assert np.array_equal(counts.cpu().numpy().astype(np.uint64), want_counts)
