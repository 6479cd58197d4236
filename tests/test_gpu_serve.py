"""Served matching (needs an MI355X): results alone equal results in the mix.

A trace of requests over several resident dictionaries is replayed through the
server (batched, plain and under a small HBM budget that forces queueing); every
request's records must equal, bit for bit, what the same text gives when
matched alone, and a sample is checked against the oracle.
"""

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

glop = pytest.importorskip("paper_1704_02278_amd")
from gpu_util import oracle_match, say  # noqa: E402

POOL = 16 << 20
SIZES = (100, 500, 2000, 5000)


@pytest.fixture(scope="module")
def served():
    dicts, pools = synth.make_served(pool_bytes=POOL, sizes=SIZES)
    dev_pools = [torch.from_numpy(p).cuda() for p in pools]
    handles = [glop.Dict(p) for p in dicts]
    at, dk, sz, off = synth.served_trace(200_000.0, 400, len(SIZES), POOL, size_max=2 << 20, trace_id=7)
    return dicts, pools, dev_pools, handles, (at, dk, sz, off)


def _alone(handles, dev_pools, dk, sz, off):
    """Each request matched on its own (plain glop_match_ws through the binding)."""
    out = []
    for k in range(len(sz)):
        t = dev_pools[dk[k]][int(off[k]):int(off[k]) + int(sz[k])]
        o, i, _, total = handles[dk[k]].match(t)
        out.append((o.cpu().numpy(), i.cpu().numpy(), total))
    return out


def _replay(handles, dev_pools, trace, **server_opts):
    at, dk, sz, off = trace
    texts = [dev_pools[dk[k]].data_ptr() + int(off[k]) for k in range(len(sz))]
    caps = np.maximum(64, sz // 256).astype(np.uint64)
    base = np.zeros(len(sz), dtype=np.uint64)
    base[1:] = np.cumsum(caps)[:-1]
    copy_out = torch.zeros((int(caps.sum()), 2), dtype=torch.int64, device="cuda")
    srv = glop.Server(handles, **server_opts)
    try:
        lat, matches, trunc, batch, wall = srv.run_trace(dk, texts, sz, at, copy_out, base, caps)
    finally:
        srv.close()
    rec = copy_out.cpu().numpy()
    got = [(rec[int(base[k]):int(base[k]) + int(matches[k]), 0], rec[int(base[k]):int(base[k]) + int(matches[k]), 1],
            int(matches[k])) for k in range(len(sz))]
    assert not trunc.any()
    assert np.all(lat > 0)
    return got, batch


def _same(got, want, what):
    for k, ((go, gi, gt), (wo, wi, wt)) in enumerate(zip(got, want)):
        assert gt == wt, f"{what}: request {k}: {gt} matches vs {wt} alone"
        assert np.array_equal(go, wo) and np.array_equal(gi & 0xFFFFFFFF, wi), f"{what}: request {k} records differ"


def test_batched_mix_equals_alone_and_oracle(served):
    dicts, pools, dev_pools, handles, trace = served
    at, dk, sz, off = trace
    say("serve batched", len(sz))
    got, batch = _replay(handles, dev_pools, trace, mode=glop.GLOP_SERVE_BATCHED)
    assert batch.max() > 1, "no two requests shared a batch"
    alone = _alone(handles, dev_pools, dk, sz, off)
    _same(got, alone, "batched")
    for k in range(0, len(sz), 40):
        host = pools[dk[k]][int(off[k]):int(off[k]) + int(sz[k])]
        w_off, w_ids, _, w_total = oracle_match(host, dicts[dk[k]], threads=8)
        assert got[k][2] == w_total
        assert np.array_equal(got[k][0].astype(np.uint64), w_off) and np.array_equal(
            (got[k][1] & 0xFFFFFFFF).astype(np.uint64), w_ids)


def test_plain_mode_and_small_budget_give_the_same_results(served):
    dicts, pools, dev_pools, handles, trace = served
    at, dk, sz, off = trace
    alone = _alone(handles, dev_pools, dk, sz, off)
    say("serve plain", len(sz))
    got, batch = _replay(handles, dev_pools, trace, mode=glop.GLOP_SERVE_PLAIN)
    assert batch.max() == 1
    _same(got, alone, "plain")
    say("serve small budget", len(sz))
    got, batch = _replay(handles, dev_pools, trace, mode=glop.GLOP_SERVE_BATCHED, hbm_budget_bytes=12 << 20)
    _same(got, alone, "small budget")


def test_submit_poll_release(served):
    dicts, pools, dev_pools, handles, trace = served
    srv = glop.Server(handles, hbm_budget_bytes=8 << 20)
    try:
        with pytest.raises(glop.GlopError):
            srv.submit(0, dev_pools[0], length=POOL)  # larger than the whole budget
        with pytest.raises(glop.GlopError):
            srv.submit(len(SIZES), dev_pools[0], length=4096)  # no such dictionary
        reqs = {}
        for k in range(12):
            n = 4096 * (k + 1) * 7
            t = dev_pools[k % len(SIZES)][k * 1000:k * 1000 + n]
            rid = srv.submit(k % len(SIZES), t, tag=100 + k)
            reqs[rid] = (k % len(SIZES), t, 100 + k)
        seen = {}
        for _ in range(2000):
            for c in srv.poll(wait_us=2000):
                seen[c.request_id] = c
            if len(seen) == len(reqs):
                break
        assert set(seen) == set(reqs)
        for rid, c in seen.items():
            dict_index, t, tag = reqs[rid]
            assert c.tag == tag and c.dict == dict_index and not c.truncated
            o, i, _, total = handles[dict_index].match(t)
            assert c.matches == c.records == total
            if total:
                view = _device_records(c.d_records, total)
                assert torch.equal(view[:, 0], o) and torch.equal(view[:, 1] & 0xFFFFFFFF, i & 0xFFFFFFFF)
            srv.release(rid)
        with pytest.raises(glop.GlopError):
            srv.release(next(iter(reqs)))  # already released
    finally:
        srv.close()


def _device_records(ptr, n):
    """Copy n 16-byte records at a device address into a new tensor."""
    out = torch.empty((n, 2), dtype=torch.int64, device="cuda")
    hip = glop.ctypes.CDLL("libamdhip64.so.7")
    hip.hipMemcpy.argtypes = [glop.ctypes.c_void_p, glop.ctypes.c_void_p, glop.ctypes.c_size_t, glop.ctypes.c_int]
    rc = hip.hipMemcpy(out.data_ptr(), ptr, n * 16, 3)  # device to device
    assert rc == 0
    return out


def test_dense_request_in_a_batch_gets_what_it_gets_alone():
    """A request with more occurrences than its output capacity (max(64,
    len / 256) records) shares a batch with sparse requests: it is cut at its
    own capacity and flagged truncated, as when matched alone, and the requests
    after it keep all their records."""
    pats = [b"abab", b"babab", b"xq7#z"]
    rng = np.random.default_rng(3)
    sparse = [bytes(rng.integers(0x20, 0x7F, size=n, dtype=np.uint8)) + b"xq7#z" for n in (5000, 70_000, 300)]
    texts = [b"ab" * 40_000] + sparse + [b"abab" * 3000, sparse[1]]
    # The first request (256 MiB, no occurrence) holds the only stream slot
    # while the others, all due at once, queue behind it and go out together.
    dev = [torch.full((256 << 20,), ord("k"), dtype=torch.uint8, device="cuda")]
    dev += [torch.frombuffer(bytearray(t), dtype=torch.uint8).cuda() for t in texts]
    h = glop.Dict(pats)
    alone = []
    for t in dev:
        cap = max(64, t.numel() // 256)
        o, i, _, total = h.match(t)
        alone.append((o[:cap].cpu().numpy(), (i[:cap] & 0xFFFFFFFF).cpu().numpy(), total, cap))
    assert alone[1][2] > alone[1][3] and alone[5][2] > alone[5][3], "the dense requests must exceed their capacity"
    caps = np.array([a[3] for a in alone], dtype=np.uint64)
    base = np.zeros(len(dev), dtype=np.uint64)
    base[1:] = np.cumsum(caps)[:-1]
    copy_out = torch.full((int(caps.sum()), 2), -1, dtype=torch.int64, device="cuda")
    srv = glop.Server([h], max_inflight=1)
    try:
        say("serve dense request in a batch")
        lat, matches, trunc, batch, _ = srv.run_trace(np.zeros(len(dev)), [t.data_ptr() for t in dev],
                                                      [t.numel() for t in dev], np.zeros(len(dev)), copy_out, base,
                                                      caps)
    finally:
        srv.close()
    assert batch[1:].max() > 1, "the queued requests did not share a batch"
    rec = copy_out.cpu().numpy()
    for k, (w_off, w_ids, w_total, cap) in enumerate(alone):
        assert matches[k] == w_total, f"request {k}: matches"
        assert bool(trunc[k]) == (w_total > cap), f"request {k}: truncated flag"
        got = rec[int(base[k]):int(base[k]) + min(w_total, cap)]
        assert np.array_equal(got[:, 0], w_off) and np.array_equal(got[:, 1] & 0xFFFFFFFF, w_ids), \
            f"request {k}: records differ from the request matched alone"
