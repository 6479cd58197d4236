"""The boundary's two headline calls on the GPU, through ctypes and nothing else.

glop_build(patterns, lengths, n) compiles and uploads a dictionary with every
option automatic; glop_match(h, text, len, out, max_matches, counts, stream)
takes its device scratch from the stream-ordered allocator of `stream` (the
construct and search phases of Section 4, with the problem statement of
Section 1: the occurrences and their counts).  Both are compared with the
oracle on a tiny and a 48 MiB medium text, on a stream other than the default
one, at capacities 0, 1, total - 1 and total: the first max_matches records in
order are written, nothing past them, and the counts are always complete.
"""

import ctypes

import numpy as np
import pytest
import synth

pytestmark = pytest.mark.gpu

glop = pytest.importorskip("paper_1704_02278_amd")
import torch  # noqa: E402

from gpu_util import oracle_match, say, to_device  # noqa: E402

SENTINEL = -0x0123456789ABCDEF


def _build(pats):
    keep = [ctypes.create_string_buffer(p, len(p)) for p in pats]
    ptrs = (ctypes.c_void_p * len(pats))(*[ctypes.addressof(b) for b in keep])
    lens = (ctypes.c_uint32 * len(pats))(*[len(p) for p in pats])
    h = glop.glop_build(ctypes.cast(ptrs, glop._u8pp), lens, len(pats))
    del keep  # glop_build copies the patterns
    assert h, glop.glop_last_error_message()
    return ctypes.c_void_p(h)


@pytest.mark.parametrize("name,n_bytes", [("tiny", None), ("medium", 48 << 20)])
def test_glop_build_and_glop_match_against_oracle(name, n_bytes):
    pats, text, plants = synth.make_workload(name, n_bytes=n_bytes)
    w_off, w_ids, w_counts, w_total = oracle_match(text, pats)
    assert w_total >= len(plants) > 1
    h = _build(pats)
    try:
        assert glop.glop_num_patterns(h) == len(pats)
        assert glop.glop_max_len(h) == max(len(p) for p in pats)
        t = to_device(text, shift=5)
        stream = torch.cuda.Stream()
        for cap in (0, 1, w_total - 1, w_total):
            say("headline C-ABI", name, text.size, "max_matches", cap)
            out = torch.full((cap + 8, 2), SENTINEL, dtype=torch.int64, device="cuda")
            counts = torch.full((len(pats),), SENTINEL, dtype=torch.int64, device="cuda")
            torch.cuda.synchronize()
            rc = glop.glop_match(h, t.data_ptr(), t.numel(), out.data_ptr() if cap else None, cap,
                                 counts.data_ptr(), stream.cuda_stream)
            assert rc == glop.GLOP_OK, glop.glop_last_error_message()
            stream.synchronize()
            o = out.cpu().numpy()
            assert np.array_equal(counts.cpu().numpy().astype(np.uint64), w_counts)
            assert np.array_equal(o[:cap, 0].astype(np.uint64), w_off[:cap])
            assert np.array_equal((o[:cap, 1] & 0xFFFFFFFF).astype(np.uint64), w_ids[:cap])
            assert np.all(o[:cap, 1] >> 32 == 0), "reserved word not zero"
            assert np.all(o[cap:] == SENTINEL), "a record was written past max_matches"
    finally:
        glop.glop_free(h)


def test_glop_match_empty_text_and_short_text():
    """len == 0 and a text shorter than every pattern: no records, counts zeroed."""
    pats = [b"abcd", b"bcdef"]
    h = _build(pats)
    try:
        stream = torch.cuda.Stream()
        for text in (b"", b"abc"):
            say("headline C-ABI, short text", len(text))
            counts = torch.full((2,), SENTINEL, dtype=torch.int64, device="cuda")
            t = to_device(text) if text else None
            rc = glop.glop_match(h, t.data_ptr() if t is not None else None, len(text), None, 0,
                                 counts.data_ptr(), stream.cuda_stream)
            assert rc == glop.GLOP_OK, glop.glop_last_error_message()
            stream.synchronize()
            assert counts.cpu().tolist() == [0, 0]
    finally:
        glop.glop_free(h)
