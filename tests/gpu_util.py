"""Helpers for the GPU parity tests: run the HIP path, compare with the oracle."""

from __future__ import annotations

import sys

import numpy as np
import torch

import oracle
import paper_1704_02278_amd as glop


def say(*parts):
    print("[case]", *parts, flush=True)
    sys.stdout.flush()


def variants_for(patterns):
    """Build options valid for this dictionary (every one must give the same result)."""
    out = [dict()]
    if patterns:
        minlen = min(len(p) for p in patterns)
        if max(len(p) for p in patterns) > 8:
            # The whole-pattern trie: walks go on below the prefix table's depth.
            out.append(dict(prefix_len=glop.GLOP_PREFIX_FULL))
        out.append(dict(filter=glop.GLOP_FILTER_NONE))
        out.append(dict(filter=glop.GLOP_FILTER_QGRAM, stride=1))
        out.append(dict(filter=glop.GLOP_FILTER_QGRAM, stride=1, probe_bits=1))
        out.append(dict(filter=glop.GLOP_FILTER_QGRAM, stride=1, probe_bits=3))
        if minlen >= 4:
            out.append(dict(filter=glop.GLOP_FILTER_QGRAM, stride=1, qgram=4, probe_bits=4))
        if minlen >= 4:
            # Both tile sizes of the automatic filters: short texts and small
            # batches default to 4 KiB tiles, so 8 KiB ones are asked for.
            out.append(dict(filter=glop.GLOP_FILTER_QGRAM, stride=1, qgram=4, probe_bits=3, tile_kib=4))
            out.append(dict(filter=glop.GLOP_FILTER_QGRAM, stride=1, qgram=4, probe_bits=3, tile_kib=8))
        if minlen >= 7:
            out.append(dict(filter=glop.GLOP_FILTER_QGRAM, stride=4, qgram=4, tile_kib=4))
            out.append(dict(filter=glop.GLOP_FILTER_QGRAM, stride=4, qgram=4, tile_kib=8))
            out.append(dict(filter=glop.GLOP_FILTER_QGRAM, stride=4, qgram=4))
            out.append(dict(filter=glop.GLOP_FILTER_QGRAM, stride=4, qgram=4, probe_bits=1))
            out.append(dict(filter=glop.GLOP_FILTER_QGRAM, stride=4, qgram=4, probe_bits=3))
        if minlen >= 2:
            out.append(dict(filter=glop.GLOP_FILTER_QGRAM, stride=1, qgram=1, bitmap_log2=12))
        # Table layouts and placements: dense rows to depth 2 and nodes below
        # (for both engines), the dense rows read from device memory, and (when
        # they fit beside the scan kernel's tables) from LDS.
        out.append(dict(layout=glop.GLOP_LAYOUT_HYBRID))
        if max(len(p) for p in patterns) > 8:
            out.append(dict(layout=glop.GLOP_LAYOUT_HYBRID, prefix_len=glop.GLOP_PREFIX_FULL))
        out.append(dict(placement=glop.GLOP_PLACE_GLOBAL))
        out.append(dict(placement=glop.GLOP_PLACE_LDS, filter=glop.GLOP_FILTER_QGRAM, stride=1))
        out.append(dict(placement=glop.GLOP_PLACE_LDS, layout=glop.GLOP_LAYOUT_HYBRID))
    return out


def build_variant(patterns, opts):
    """A device dictionary with `opts`, or None when the dictionary cannot take
    them (dense rows placed in LDS that do not fit there)."""
    try:
        return glop.Dict(patterns, **opts)
    except glop.GlopError as e:
        if opts.get("placement") == glop.GLOP_PLACE_LDS and e.code == glop.GLOP_EINVAL:
            return None
        raise


def to_device(text, shift: int = 0) -> torch.Tensor:
    """Upload text so that its first byte sits `shift` bytes past a 256-byte boundary."""
    arr = np.frombuffer(bytes(text), dtype=np.uint8) if not isinstance(text, np.ndarray) else text
    buf = torch.empty(arr.size + 512, dtype=torch.uint8, device="cuda")
    start = ((-buf.data_ptr()) % 256) + shift
    t = buf[start:start + arr.size]
    if arr.size:
        t.copy_(torch.from_numpy(np.ascontiguousarray(arr)))
    return t


SENTINEL = -0x0123456789ABCDEF


def gpu_match(d: glop.Dict, text_dev: torch.Tensor, max_matches=None):
    """Match through glop_match_ws into outputs pre-filled with a sentinel, so a
    record the kernels fail to write cannot pass as one left behind by an
    earlier call in the same memory; the first pass sizes the output."""
    n = int(text_dev.numel())
    dev = text_dev.device
    ws = torch.empty(d.workspace_bytes(n) + 256, dtype=torch.uint8, device=dev)
    ws = ws[(-ws.data_ptr()) % 256:]
    total = torch.zeros(1, dtype=torch.int64, device=dev)
    cap = max(1024, n // 1024) if max_matches is None else int(max_matches)
    while True:
        out = torch.full((max(cap, 1), 2), SENTINEL, dtype=torch.int64, device=dev)
        counts = torch.full((max(1, d.num_patterns),), SENTINEL, dtype=torch.int64, device=dev)
        d.match_into(text_dev, out, counts, max_matches=cap, total=total, workspace=ws)
        got = int(total.item())
        if max_matches is not None or got <= cap:
            break
        cap = got
    # A call that failed inside the kernels reports a total of all ones.
    assert got >= 0, f"the call reported a failure (total {got:#x}, capacity {cap})"
    k = min(cap, got)
    o = out[:k].cpu().numpy()
    past = out[k:].cpu().numpy()
    written = np.flatnonzero(np.any(past != SENTINEL, axis=1))
    assert written.size == 0, (f"a record was written past the total: total {got}, capacity {cap}, "
                               f"{written.size} rows written past it, first {past[written[:4]].tolist()}")
    return (o[:, 0].astype(np.uint64), o[:, 1].astype(np.uint64),  # the id with its zero reserved word
            counts[: d.num_patterns].cpu().numpy().astype(np.uint64), got)


def oracle_match(text, patterns, threads=None, bucketed=1):
    off, ids, counts, total = oracle.match(text, patterns, bucketed=bucketed, threads=threads)
    return off.astype(np.uint64), ids.astype(np.uint64), counts.astype(np.uint64), int(total)


def assert_same(got, want, what=""):
    g_off, g_ids, g_counts, g_total = got
    w_off, w_ids, w_counts, w_total = want
    assert g_total == w_total, f"{what}: total {g_total} != {w_total}"
    assert np.array_equal(g_counts, w_counts), f"{what}: counts differ"
    assert g_off.size == w_off.size, f"{what}: {g_off.size} records vs {w_off.size}"
    if not (np.array_equal(g_off, w_off) and np.array_equal(g_ids, w_ids)):
        bad = int(np.flatnonzero((g_off != w_off) | (g_ids != w_ids))[0])
        raise AssertionError(f"{what}: first difference at record {bad}: gpu ({g_off[bad]}, {g_ids[bad]}) "
                             f"oracle ({w_off[bad]}, {w_ids[bad]})")
