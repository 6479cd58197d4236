"""Host-streamed matching (needs an MI355X): the same result as one device call.

glop_match_host cuts a host text into pieces that overlap by the longest
pattern minus one byte, uploads them through pinned buffers and matches each
into one output.  Records, counts and the total must equal glop_match on the
whole text already in device memory, for piece sizes that put many
occurrences across piece boundaries, and the oracle on the tiny workload.
"""

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

glop = pytest.importorskip("paper_1704_02278_amd")
from gpu_util import assert_same, oracle_match, say  # noqa: E402


def _host(d, text, **kw):
    off, ids, counts, total = d.match_host(text, **kw)
    torch.cuda.synchronize()
    return (off.cpu().numpy().astype(np.uint64), (ids.cpu().numpy() & 0xFFFFFFFF).astype(np.uint64),
            counts.cpu().numpy().astype(np.uint64), int(total))


def _device(d, text):
    off, ids, counts, total = d.match(torch.from_numpy(text).cuda())
    torch.cuda.synchronize()
    return (off.cpu().numpy().astype(np.uint64), (ids.cpu().numpy() & 0xFFFFFFFF).astype(np.uint64),
            counts.cpu().numpy().astype(np.uint64), int(total))


def test_tiny_against_the_oracle():
    pats, text, _ = synth.make_workload("tiny")
    d = glop.Dict(pats)
    want = oracle_match(text, pats)
    for chunk in (4096, 5000, 65536, 0):
        say("host-stream tiny", chunk)
        assert_same(_host(d, text, chunk_bytes=chunk), want, f"tiny chunk {chunk}")


@pytest.mark.parametrize("name,n_bytes", [("medium", 24 << 20), ("large", 12 << 20)])
def test_pieces_equal_one_device_call(name, n_bytes):
    pats, text, _ = synth.make_workload(name, n_bytes=n_bytes)
    d = glop.Dict(pats)
    want = _device(d, text)
    for chunk in (4096 * 3 + 1, 1 << 20, 7 << 20, 0):
        say("host-stream", name, chunk)
        assert_same(_host(d, text, chunk_bytes=chunk), want, f"{name} chunk {chunk}")


def test_boundary_occurrences_and_truncation():
    # Occurrences written across every piece boundary, and a capacity that cuts the output.
    pats = [b"boundary-spanning", b"span", b"ning", b"y-s"]
    rng = np.random.default_rng(3)
    text = rng.integers(0x61, 0x7B, size=3 << 20, dtype=np.uint8)
    chunk = 1 << 16
    for k in range(1, text.size // chunk):
        o = k * chunk - 9
        text[o:o + len(pats[0])] = np.frombuffer(pats[0], dtype=np.uint8)
    d = glop.Dict(pats)
    want = _device(d, text)
    assert want[3] >= 4 * (text.size // chunk - 1)
    say("host-stream boundaries")
    assert_same(_host(d, text, chunk_bytes=chunk), want, "boundaries")
    cut = want[3] // 3
    off, ids, counts, total = _host(d, text, chunk_bytes=chunk, max_matches=cut)
    assert total == want[3] and off.size == cut and np.array_equal(counts, want[2])
    assert np.array_equal(off, want[0][:cut]) and np.array_equal(ids, want[1][:cut])


def test_empty_and_short_texts():
    d = glop.Dict([b"abcdef", b"xyz"])
    for text in (b"", b"ab", b"xyz", b"abcdefxyz" * 1000):
        t = np.frombuffer(text, dtype=np.uint8)
        say("host-stream short", len(text))
        got = _host(d, t, chunk_bytes=4096)
        want = oracle_match(t, [b"abcdef", b"xyz"])
        assert_same(got, want, f"len {len(text)}")
