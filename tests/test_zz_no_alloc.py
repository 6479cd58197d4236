"""glop_match_static, the entry point for callers that cannot allocate (needs an MI355X).

It runs the single-text kernels with the library's static per-device
workspace; its records, counts and total must equal glop_match_ws with a
caller's workspace, bit for bit, on two calls in a row (the second on a
smaller text, so any stale workspace contents from the first would show), and
a text too long for the static workspace is refused before anything runs.
"""

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

glop = pytest.importorskip("paper_1704_02278_amd")
from gpu_util import oracle_match, say, to_device  # noqa: E402

SENTINEL = -0x0123456789ABCDEF


def _with_workspace(d, t, cap):
    out = torch.full((cap + 4, 2), SENTINEL, dtype=torch.int64, device="cuda")
    counts = torch.full((d.num_patterns,), SENTINEL, dtype=torch.int64, device="cuda")
    total = torch.zeros(1, dtype=torch.int64, device="cuda")
    ws = torch.empty(d.workspace_bytes(t.numel()) + 256, dtype=torch.uint8, device="cuda")
    ws = ws[(-ws.data_ptr()) % 256:]
    d.match_into(t, out, counts, max_matches=cap, total=total, workspace=ws)
    torch.cuda.synchronize()
    return out.cpu().numpy(), counts.cpu().numpy(), int(total.item())


def _static(d, t, cap, stream):
    out = torch.full((cap + 4, 2), SENTINEL, dtype=torch.int64, device="cuda")
    counts = torch.full((d.num_patterns,), SENTINEL, dtype=torch.int64, device="cuda")
    total = torch.zeros(1, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    rc = glop.glop_match_static(d.handle, t.data_ptr(), t.numel(), out.data_ptr(), cap, counts.data_ptr(),
                                total.data_ptr(), stream.cuda_stream)
    assert rc == glop.GLOP_OK, glop.glop_last_error_message()
    stream.synchronize()
    return out.cpu().numpy(), counts.cpu().numpy(), int(total.item())


@pytest.mark.parametrize("name,sizes", [("medium", (40 << 20, (3 << 20) + 333)), ("large", (24 << 20, 77_777))])
def test_static_workspace_equals_caller_workspace(name, sizes):
    pats, text, _ = synth.make_workload(name, n_bytes=max(sizes) + 5000)
    d = glop.Dict(pats)
    stream = torch.cuda.Stream()
    for k, n in enumerate(sizes):
        host = text[5000 - 1000 * k: 5000 - 1000 * k + n]  # the second text is another span, not a prefix
        t = to_device(host, shift=3 + k)
        w_off, w_ids, w_counts, w_total = oracle_match(host, pats, bucketed=2 if name == "large" else 1)
        for cap in (w_total, max(0, w_total // 3)):
            say("static workspace", name, n, "max_matches", cap)
            ref = _with_workspace(d, t, cap)
            got = _static(d, t, cap, stream)
            assert got[2] == ref[2] == w_total
            assert np.array_equal(got[1], ref[1])
            assert np.array_equal(got[1].astype(np.uint64), w_counts)
            assert np.array_equal(got[0], ref[0]), "records differ from glop_match_ws"
            assert np.array_equal(got[0][:cap, 0].astype(np.uint64), w_off[:cap])
            assert np.all(got[0][cap:] == SENTINEL)


def test_static_workspace_refuses_a_text_too_long():
    pats = [b"abcd", b"bcdef"]
    d = glop.Dict(pats)
    limit = int(glop.glop_static_max_len(d.handle))
    assert (1 << 30) <= limit < (1 << 32)
    say("static workspace limit", limit)
    counts = torch.zeros(2, dtype=torch.int64, device="cuda")
    # A real buffer of that length, so the call would stay in bounds even if it ran.
    buf = torch.zeros(limit + 1, dtype=torch.uint8, device="cuda")
    rc = glop.glop_match_static(d.handle, buf.data_ptr(), limit + 1, None, 0, counts.data_ptr(), None, None)
    assert rc == glop.GLOP_ETOOLONG
    torch.cuda.synchronize()
    assert "static workspace" in glop.glop_last_error_message().decode()
