#!/usr/bin/env python3
"""Throughput of exact multi-pattern matching on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload medium]

A step is one glop_match_ws call (scan + emit kernels: filter, trie walks,
ordered output, counts) over the whole synthetic text, which is resident in
HBM before timing starts.  Throughput follows Eq. 1 of the paper (8 N / t,
reported here also as N / t in GB/s) with N the text bytes of the call.

Prints one JSON line.  The CPU baseline is the oracle (test infrastructure,
bucketed memcmp) timed on a bounded sample of the same text on host cores.
"""

from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time
from pathlib import Path

import numpy as np

ROOT = Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s

WORKLOAD_LABEL = {
    "tiny": "plain matcher: 16 patterns (4-16 B) over 1 MiB synthetic log text",
    "medium": "plain matcher: 1,000 patterns (8-64 B, 30% shared prefixes, 5% exact prefixes) over 1 GiB synthetic log text",
    "large": "plain matcher: 20,000 patterns (Zipf(1.2) lengths 4-128 B, 40% shared prefixes) over 4 GiB synthetic log text",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


class HipEvents:
    """Raw hipEvent_t handles from the HIP runtime torch loaded (shared with libglop)."""

    def __init__(self):
        self.hip = ctypes.CDLL("libamdhip64.so.7")
        self.hip.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
        self.hip.hipEventDestroy.argtypes = [ctypes.c_void_p]

    def create(self):
        e = ctypes.c_void_p()
        rc = self.hip.hipEventCreate(ctypes.byref(e))
        if rc != 0:
            raise RuntimeError(f"hipEventCreate failed ({rc})")
        return e.value

    def elapsed_ms(self, a, b) -> float:
        ms = ctypes.c_float()
        rc = self.hip.hipEventElapsedTime(ctypes.byref(ms), a, b)
        if rc != 0:
            raise RuntimeError(f"hipEventElapsedTime failed ({rc})")
        return float(ms.value)

    def destroy(self, e):
        self.hip.hipEventDestroy(e)


def _profiling():
    """The rocprofv3 summary helper, loaded by path (it reads CSV only)."""
    import importlib.util

    spec = importlib.util.spec_from_file_location("_glop_profiling", ROOT / "paper_1704_02278_amd" / "profiling.py")
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def measured_traffic(workload: str):
    """HBM bytes per scan launch from the committed rocprofv3 counter runs, or
    None if they were taken on other kernel sources or another workload."""
    path = ROOT / "profiles" / f"glop_scan_kernel_{workload}_traffic.json"
    if not path.exists():
        return None
    rec = json.loads(path.read_text())
    if rec.get("kernel_sources_sha256") != _profiling().kernel_sources_sha256():
        return None
    return int(rec["traffic_bytes_per_launch"])


def cpu_threads() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def host_info() -> dict:
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "usable_cpus": cpu_threads(), "model": model}


def cpu_baseline(text: np.ndarray, pats, target_s: float) -> dict:
    import oracle

    threads = cpu_threads()
    probe = min(text.size, 4 << 20)
    t0 = time.perf_counter()
    oracle.match(text[:probe], pats, bucketed=True, threads=threads)
    dt = max(time.perf_counter() - t0, 1e-3)
    n = int(min(text.size, max(probe, probe * target_s / dt)))
    n = max(probe, n - n % (1 << 20)) if n >= (1 << 20) else n
    t0 = time.perf_counter()
    _, _, _, total = oracle.match(text[:n], pats, bucketed=True, threads=threads)
    dt = time.perf_counter() - t0
    return {"value": round(n / dt / 1e9, 6), "unit": "GB/s", "cores": threads, "kind": "oracle", "host": host_info(),
            "sample": f"first {n / 2**20:.0f} MiB of the same text, bucketed memcmp oracle, {threads} threads, "
                      f"{dt:.1f} s, {total} matches"}


def cpu_trie_baseline(d, text: np.ndarray, target_s: float) -> dict:
    threads = cpu_threads()
    out = {}
    for thr in (1, threads):
        probe = min(text.size, 1 << 20)
        t0 = time.perf_counter()
        d.cpu_walk(text[:probe], threads=thr, max_matches=0)
        dt = max(time.perf_counter() - t0, 1e-4)
        n = int(min(text.size, max(probe, probe * target_s / dt)))
        t0 = time.perf_counter()
        d.cpu_walk(text[:n], threads=thr, max_matches=0)
        dt = time.perf_counter() - t0
        out[f"threads_{thr}"] = {"value": round(n / dt / 1e9, 6), "unit": "GB/s", "bytes": n}
    return {"kind": "failureless-trie walk on the host (the CPU side of the paper's comparison)", **out}


def bench_host_stream(d, text: np.ndarray, reps: int = 3, chunk_bytes: int = 64 << 20) -> dict:
    """The same text matched from host memory (glop_match_host): pageable and
    pinned sources, end to end (host text in, device result out), next to the
    plain pinned H2D copy rate of the same bytes."""
    import torch

    n = int(text.size)
    pinned = torch.empty(n, dtype=torch.uint8, pin_memory=True)
    pinned.numpy()[:] = text
    dev = torch.empty(n, dtype=torch.uint8, device="cuda")
    for _ in range(2):
        dev.copy_(pinned, non_blocking=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        dev.copy_(pinned, non_blocking=True)
    torch.cuda.synchronize()
    h2d = n * reps / (time.perf_counter() - t0) / 1e9
    del dev
    out = {"chunk_bytes": chunk_bytes, "h2d_pinned_GBps": round(h2d, 2)}
    for name, src in (("pageable", text), ("pinned", pinned.numpy())):
        d.match_host(src, chunk_bytes=chunk_bytes)  # warm-up (sizes the output)
        t0 = time.perf_counter()
        for _ in range(reps):
            d.match_host(src, chunk_bytes=chunk_bytes, max_matches=1 << 20)
        dt = (time.perf_counter() - t0) / reps
        out[name] = {"ms": round(dt * 1e3, 3), "GBps": round(n / dt / 1e9, 2), "frac_of_h2d": round(n / dt / 1e9 / h2d, 3)}
    return out


def bench_batched(reps: int) -> dict:
    """Many independent texts: one batched call (graph replay) vs one plain call per text.

    Plain is timed twice: the per-chunk glop_match_ws calls issued from Python
    (eager) and the same calls captured once in a graph and replayed (no host
    launch cost).  Both write every chunk's records; the batched result must
    equal them chunk by chunk (checked outside the timed regions).
    """
    import torch

    import paper_1704_02278_amd as glop
    import synth

    t0 = time.perf_counter()
    pats, text, offs, sizes, plants = synth.make_chunks("batched")
    nchunks, nbytes = len(sizes), int(text.size)
    log(f"[bench] batched: {nchunks} chunks, {nbytes} bytes, generated in {time.perf_counter() - t0:.1f} s")
    dev = torch.device("cuda:0")
    buf = torch.from_numpy(text).to(dev)
    del text
    chunks = [buf[o:o + n] for o, n in zip(offs.tolist(), sizes)]
    d = glop.Dict(pats)
    npat = len(pats)
    stream = torch.cuda.current_stream()

    # Plain: one glop_match_ws per chunk into its own slice of one output buffer.
    caps = [16 + n // 2048 for n in sizes]
    bases = np.zeros(nchunks + 1, dtype=np.int64)
    bases[1:] = np.cumsum(caps)
    out_plain = torch.zeros((int(bases[-1]), 2), dtype=torch.int64, device=dev)
    totals = torch.zeros(nchunks, dtype=torch.int64, device=dev)
    counts_plain = torch.empty(npat, dtype=torch.int64, device=dev)
    ws_bytes = d.workspace_bytes(max(sizes))
    ws_buf = torch.empty(ws_bytes + 256, dtype=torch.uint8, device=dev)
    ws = ws_buf[(-ws_buf.data_ptr()) % 256:][:ws_bytes]
    outs = [out_plain[int(bases[k]):int(bases[k + 1])] for k in range(nchunks)]
    tots = [totals[k:k + 1] for k in range(nchunks)]

    def plain_all():
        for k in range(nchunks):
            d.match_into(chunks[k], outs[k], counts_plain, total=tots[k], workspace=ws, stream=stream)

    # Batched: one glop_match_batch over the chunk table.
    table = torch.tensor([[c.data_ptr(), c.numel()] for c in chunks], dtype=torch.int64).to(dev)
    cap_b = int(bases[-1])
    out_b = torch.zeros((cap_b, 2), dtype=torch.int64, device=dev)
    first = torch.empty(nchunks, dtype=torch.int64, device=dev)
    count = torch.empty(nchunks, dtype=torch.int64, device=dev)
    counts_b = torch.empty(npat, dtype=torch.int64, device=dev)
    total_b = torch.zeros(1, dtype=torch.int64, device=dev)
    wsb_bytes = d.batch_workspace_bytes(nchunks, nbytes)
    wsb_buf = torch.empty(wsb_bytes + 256, dtype=torch.uint8, device=dev)
    wsb = wsb_buf[(-wsb_buf.data_ptr()) % 256:][:wsb_bytes]

    def batched():
        d.match_batch_into(table, nchunks, nbytes, out_b, first, count, counts_b, total_b, wsb, stream=stream)

    def timed(fn, n, back_to_back=4):
        # Each sample is `back_to_back` calls issued one after another between
        # two events, divided by their number: the device time per call with
        # the queue kept full, so a graph launch's host-side submission is not
        # counted as device time before its first kernel (the eager form's
        # later kernels are queued while its first one runs).
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        ms = []
        for _ in range(n):
            torch.cuda.synchronize()
            a.record(stream)
            for _ in range(back_to_back):
                fn()
            b.record(stream)
            torch.cuda.synchronize()
            ms.append(a.elapsed_time(b) / back_to_back)
        return np.array(ms)

    # Warm-up, then capture both forms as graphs (the capture stream is torch's).
    plain_all()
    batched()
    torch.cuda.synchronize()
    g_plain, g_batch = torch.cuda.CUDAGraph(), torch.cuda.CUDAGraph()
    cs = torch.cuda.Stream()
    cs.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(cs):
        with torch.cuda.graph(g_plain, stream=cs):
            for k in range(nchunks):
                d.match_into(chunks[k], outs[k], counts_plain, total=tots[k], workspace=ws, stream=cs)
        with torch.cuda.graph(g_batch, stream=cs):
            d.match_batch_into(table, nchunks, nbytes, out_b, first, count, counts_b, total_b, wsb, stream=cs)
    torch.cuda.current_stream().wait_stream(cs)
    torch.cuda.synchronize()

    t_eager = timed(plain_all, max(2, reps // 5), back_to_back=1)
    t_plain_graph = timed(g_plain.replay, max(2, reps // 5), back_to_back=1)
    t_batch_graph = timed(g_batch.replay, reps)
    t_batch_eager = timed(batched, reps)

    # Same records chunk by chunk (plain slices vs batched segments), same totals.
    tb = int(total_b.item())
    assert 0 <= tb <= cap_b, tb
    tot = totals.cpu().numpy()
    fst, cnt = first.cpu().numpy(), count.cpu().numpy()
    assert np.array_equal(cnt, tot) and tb == int(tot.sum())
    assert all(len(p) <= t for p, t in zip(plants, tot.tolist()))
    ob, op = out_b[:tb].cpu().numpy(), out_plain.cpu().numpy()
    idx_plain = np.concatenate([np.arange(bases[k], bases[k] + tot[k]) for k in range(nchunks)])
    assert np.array_equal(ob[:, 0], op[idx_plain, 0])
    assert np.array_equal(ob[:, 1] & 0xFFFFFFFF, op[idx_plain, 1])
    assert np.array_equal(ob[:, 1] >> 32, np.repeat(np.arange(nchunks), tot))
    assert np.array_equal(fst, np.concatenate([[0], np.cumsum(tot)[:-1]]))

    def rate(ms):
        return round(nbytes / (float(np.median(ms)) / 1e3) / 1e9, 2)

    return {
        "workload": "4,096 independent log texts (lognormal sizes, median 256 KiB, sigma 2.16, 1 KiB-64 MiB), "
                    "1,000-pattern dictionary",
        "chunks": nchunks, "bytes": nbytes, "matches": tb, "reps": reps,
        "batched_graph": {"ms_median": round(float(np.median(t_batch_graph)), 4),
                          "ms_min": round(float(t_batch_graph.min()), 4), "GBps": rate(t_batch_graph),
                          "hbm_frac": round(rate(t_batch_graph) / HBM_PEAK_GBS, 4)},
        "batched_eager": {"ms_median": round(float(np.median(t_batch_eager)), 4), "GBps": rate(t_batch_eager)},
        "plain_graph": {"ms_median": round(float(np.median(t_plain_graph)), 4), "GBps": rate(t_plain_graph),
                        "launches": 2 * nchunks},
        "plain_eager": {"ms_median": round(float(np.median(t_eager)), 4), "GBps": rate(t_eager)},
        "speedup_vs_plain_graph": round(float(np.median(t_plain_graph) / np.median(t_batch_graph)), 2),
        "speedup_vs_plain_eager": round(float(np.median(t_eager) / np.median(t_batch_graph)), 2),
    }


def bench_served(requests: int, rates=(1000.0, 5000.0, 20000.0)) -> dict:
    """Open-loop traces over 8 resident dictionaries: continuous batching vs one
    plain call per request (FIFO, one stream).  Latency = result visible on the
    host minus scheduled arrival; payloads are already in HBM."""
    import torch

    import paper_1704_02278_amd as glop
    import synth

    pool = 256 << 20
    t0 = time.perf_counter()
    dicts, pools = synth.make_served(pool_bytes=pool)
    log(f"[bench] served: {len(dicts)} dictionaries ({', '.join(str(len(d)) for d in dicts)} patterns), "
        f"{len(pools)} x {pool >> 20} MiB pools, generated in {time.perf_counter() - t0:.1f} s")
    dev_pools = [torch.from_numpy(p).cuda() for p in pools]
    del pools
    t0 = time.perf_counter()
    handles = [glop.Dict(d) for d in dicts]
    log(f"[bench] served: dictionaries built in {time.perf_counter() - t0:.1f} s")

    def pct(a, q):
        return round(float(np.percentile(a, q)) / 1e6, 4)

    def run(mode, trace, budget=0):
        at, dk, sz, off = trace
        texts = np.array([dev_pools[dk[k]].data_ptr() + int(off[k]) for k in range(len(sz))], dtype=np.uint64)
        srv = glop.Server(handles, mode=mode, hbm_budget_bytes=budget)
        try:
            lat, matches, trunc, batch, wall = srv.run_trace(dk, texts, sz, at)
        finally:
            srv.close()
        assert not trunc.any()
        res = {"p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99), "mean_ms": round(float(lat.mean()) / 1e6, 4),
               "GBps": round(float(sz.sum()) / (wall / 1e9) / 1e9, 2), "wall_s": round(wall / 1e9, 3)}
        if mode == glop.GLOP_SERVE_BATCHED:
            res["mean_batch_requests"] = round(float(batch.mean()), 2)
        return res, matches

    out = {"workload": f"{len(dicts)} resident dictionaries ({'/'.join(str(len(d)) for d in dicts)} patterns); "
                       f"Poisson arrivals; sizes lognormal (median 256 KiB, sigma 2.16) in [4 KiB, 16 MiB]",
           "requests_per_rate": requests, "rates": {}}
    for k, rate in enumerate(rates):
        trace = synth.served_trace(rate, requests, len(dicts), pool, trace_id=k)
        log(f"[bench] served: {rate:.0f} req/s, {requests} requests, {int(trace[2].sum()) / 2**30:.1f} GiB ...")
        b, mb = run(glop.GLOP_SERVE_BATCHED, trace)
        p, mp = run(glop.GLOP_SERVE_PLAIN, trace)
        assert np.array_equal(mb, mp), "batched and plain disagree on a request's match count"
        out["rates"][f"{rate:.0f}"] = {"offered_GBps": round(float(trace[2].sum()) / (trace[0][-1] / 1e9) / 1e9, 2),
                                       "batched": b, "plain": p, "matches": int(mb.sum())}
    trace = synth.served_trace(rates[-1], requests, len(dicts), pool, trace_id=len(rates))
    log("[bench] served: 256 MiB budget ...")
    b, _ = run(glop.GLOP_SERVE_BATCHED, trace, budget=256 << 20)
    out["budget_256MiB"] = {"rate": rates[-1], "batched": b}
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="medium", choices=sorted(WORKLOAD_LABEL))
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target length of the CPU oracle sample")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU baselines (profiling runs)")
    ap.add_argument("--copy-probe", action="store_true", help="also time a plain device copy of the text")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched (many texts) comparison")
    ap.add_argument("--batched-reps", type=int, default=10)
    ap.add_argument("--no-served", action="store_true", help="skip the served (continuous batching) traces")
    ap.add_argument("--no-host-stream", action="store_true", help="skip the host-streamed input measurement")
    ap.add_argument("--no-alt", action="store_true", help="skip the alternative engine/filter configurations")
    ap.add_argument("--served-requests", type=int, default=20000)
    ap.add_argument("--prefix-len", default="auto",
                    help="trie depth of the timed dictionary: auto (the library's default), full, or a byte count")
    ap.add_argument("--layout", default="auto", choices=["auto", "dense", "hybrid"],
                    help="transition-table layout of the timed dictionary")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the matcher has no multi-GPU path",
              file=sys.stderr)
        return 2

    import torch

    import paper_1704_02278_amd as glop
    import synth

    t0 = time.perf_counter()
    pats, text, plants = synth.make_workload(args.workload)
    log(f"[bench] workload {args.workload}: {len(pats)} patterns, {text.size} bytes, {len(plants)} plants, "
        f"generated in {time.perf_counter() - t0:.1f} s")
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    dict_opts = {}
    if args.prefix_len != "auto":
        dict_opts["prefix_len"] = glop.GLOP_PREFIX_FULL if args.prefix_len == "full" else int(args.prefix_len)
    if args.layout != "auto":
        dict_opts["layout"] = {"dense": glop.GLOP_LAYOUT_DENSE, "hybrid": glop.GLOP_LAYOUT_HYBRID}[args.layout]
    d = glop.Dict(pats, **dict_opts)
    info = d.info()
    log(f"[bench] dictionary: {info}")
    t_dev = torch.from_numpy(text).to(dev)
    n = t_dev.numel()
    cap = max(1 << 16, 4 * len(plants) + (n >> 12))
    out = torch.empty((cap, 2), dtype=torch.int64, device=dev)
    counts = torch.empty(len(pats), dtype=torch.int64, device=dev)
    total = torch.zeros(1, dtype=torch.int64, device=dev)
    ws_bytes = d.workspace_bytes(n)
    ws_buf = torch.empty(ws_bytes + 256, dtype=torch.uint8, device=dev)
    ws = ws_buf[(-ws_buf.data_ptr()) % 256:][:ws_bytes]
    stream = torch.cuda.current_stream()
    hev = HipEvents()
    # The throughput loop carries no events (a timed event record between two
    # launches costs several microseconds of GPU time).  A second loop of the
    # same K calls records, around every call, the start and end of the scan
    # kernel and the end of the emit kernel: the scan kernel's duration for the
    # roofline and the per-call latency.
    call_evs = [(hev.create(), hev.create(), hev.create()) for _ in range(args.steps)]

    # Settle before the W warmup calls: matching right after the device was
    # idle runs a few percent slower for the first milliseconds (measured: the
    # same 100 timed calls 1.6 % slower after 3 warmup calls than after 50), so
    # 50 ms of untimed calls come first, whatever W is.
    t_settle = time.perf_counter()
    while time.perf_counter() - t_settle < 0.05:
        for _ in range(8):
            d.match_into(t_dev, out, counts, total=total, workspace=ws, stream=stream)
        torch.cuda.synchronize()
    for _ in range(args.warmup):
        d.match_into(t_dev, out, counts, total=total, workspace=ws, stream=stream)
    torch.cuda.synchronize()
    got_total = int(total.item())
    if got_total > cap:
        raise RuntimeError(f"output capacity {cap} below {got_total} matches")

    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for k in range(args.steps):
        d.match_into(t_dev, out, counts, total=total, workspace=ws, stream=stream)
    end.record(stream)
    torch.cuda.synchronize()
    wall_ms = start.elapsed_time(end)
    ms_per_step = wall_ms / args.steps
    # Kernel durations and per-call latency (scan start to emit end), own loop.
    for k in range(args.steps):
        d.match_into(t_dev, out, counts, total=total, workspace=ws, stream=stream, events=call_evs[k])
    torch.cuda.synchronize()
    scan_ms = np.array([hev.elapsed_ms(a_, b_) for a_, b_, _ in call_evs])
    step_ms = np.array([hev.elapsed_ms(a_, c_) for a_, _, c_ in call_evs])
    for trio in call_evs:
        for x in trio:
            hev.destroy(x)

    # Correctness of the timed result (outside the timed region).
    off = out[:got_total, 0].cpu().numpy()
    ids = out[:got_total, 1].cpu().numpy()
    cnt = counts.cpu().numpy()
    assert int(total.item()) == got_total == int(cnt.sum())
    assert got_total >= len(plants)
    key = off.astype(np.uint64) * np.uint64(1 << 32) + ids.astype(np.uint64)
    assert np.all(key[1:] > key[:-1])
    tb = memoryview(text)
    assert all(bytes(tb[o:o + len(pats[j])]) == pats[j] for o, j in zip(off.tolist(), ids.tolist()))

    # Algorithmic bytes of one call (the method's, not the implementation's):
    # the text read once, a 16-byte record per match, an 8-byte count per
    # pattern; the time is the scan kernel's (the dominant kernel).
    scan_bytes = n + 16 * got_total + 8 * len(pats)
    scan_avg = float(scan_ms.mean())
    achieved = scan_bytes / (scan_avg / 1e3) / 1e9
    value = n / (ms_per_step / 1e3) / 1e9

    # Read-stream ceiling of this device, same session: one read of the text.
    sink = torch.zeros(1, dtype=torch.int64, device=dev)
    assert t_dev.data_ptr() % 16 == 0
    for _ in range(3):
        glop.stream_read(t_dev, sink, stream)
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(20):
        glop.stream_read(t_dev, sink, stream)
    b.record(stream)
    torch.cuda.synchronize()
    read_ms = a.elapsed_time(b) / 20
    read_gbs = (n - n % 16) / (read_ms / 1e3) / 1e9

    copy = None
    if args.copy_probe:
        dst = torch.empty_like(t_dev)
        for _ in range(3):
            dst.copy_(t_dev)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(20):
            dst.copy_(t_dev)
        b.record()
        torch.cuda.synchronize()
        cms = a.elapsed_time(b) / 20
        copy = {"ms": round(cms, 4), "GBps_read_plus_write": round(2 * n / (cms / 1e3) / 1e9, 1)}
        del dst

    result = {
        "metric": "match throughput GB/s (% HBM peak), batched/served vs plain; p50/p99 latency",
        "value": round(value, 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic (seeded MT19937-64 log lines and patterns, planted occurrences)",
        "config": {"workload": WORKLOAD_LABEL[args.workload], "patterns": len(pats), "text_bytes": n,
                   "form": "plain (one glop_match_ws call per step)",
                   **({"dictionary_options": {"prefix_len": args.prefix_len, "layout": args.layout}}
                      if dict_opts else {})},
        "sha256": {"text": synth.sha256_bytes(text), "patterns": synth.sha256_patterns(pats)},
        "gbps_eq1": round(8 * value, 2),
        "hbm_frac": round(value / HBM_PEAK_GBS, 5),
        "step_ms_mean": round(float(step_ms.mean()), 5),
        "step_ms_p50": round(float(np.percentile(step_ms, 50)), 5),
        "step_ms_p99": round(float(np.percentile(step_ms, 99)), 5),
        "matches": got_total,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": None if dict_opts else measured_traffic(args.workload),
                     "kernel": "glop_scan_kernel", "kernel_ms_avg": round(scan_avg, 5),
                     "kernel_event_samples": int(scan_ms.size),
                     "algorithmic_bytes_per_launch": int(scan_bytes)},
        "read_stream_ceiling": {"GBps": round(read_gbs, 1), "ms": round(read_ms, 5),
                                "value_frac": round(value / read_gbs, 4), "scan_frac": round(achieved / read_gbs, 4),
                                "kernel": "glop_stream_read_kernel (same load shape as the scan)"},
        "dictionary": {k: info[k] for k in ("num_states", "num_classes", "stride", "qgram", "bitmap_log2",
                                            "probe_bits", "filter_keys", "table_bytes", "prefix_len")},
        "paper_context": "20 Gbps (2.5 GB/s) PFAC texture-memory kernel on a Tesla K20m, 100 MB logs, "
                         "patterns truncated to 8 bytes (Sections 7-8); other hardware and problem",
    }
    if copy:
        result["copy_probe"] = copy
    # Other exact configurations of the same match on the same text: the
    # truncated-trie engine (prefix 8 + GPU verify) and the blocked filter.
    def time_dict(dd):
        wsd, need = ws, dd.workspace_bytes(n)  # smaller tiles need more workspace
        if need > ws.numel():
            wbuf = torch.empty(need + 256, dtype=torch.uint8, device=dev)
            wsd = wbuf[(-wbuf.data_ptr()) % 256:][:need]
        # The same settling as the main loop: a leg timed right after the
        # device idled (building the dictionary, tuning) read 6 % slow.
        t_set = time.perf_counter()
        while time.perf_counter() - t_set < 0.05:
            for _ in range(8):
                dd.match_into(t_dev, out, counts, total=total, workspace=wsd, stream=stream)
            torch.cuda.synchronize()
        for _ in range(args.warmup):
            dd.match_into(t_dev, out, counts, total=total, workspace=wsd, stream=stream)
        torch.cuda.synchronize()
        assert int(total.item()) == got_total, "configurations disagree on the match count"
        a_ = torch.cuda.Event(enable_timing=True)
        b_ = torch.cuda.Event(enable_timing=True)
        a_.record(stream)
        for _ in range(args.steps):
            dd.match_into(t_dev, out, counts, total=total, workspace=wsd, stream=stream)
        b_.record(stream)
        torch.cuda.synchronize()
        return a_.elapsed_time(b_) / args.steps

    alt = () if args.no_alt else (
        ("full_trie", dict(prefix_len=glop.GLOP_PREFIX_FULL), "trie of the whole patterns"),
        ("prefix8", dict(prefix_len=8), "trie of 8-byte prefixes + GPU verify of the rest"),
        ("blocked_filter", dict(probe_bits=3), "two filter bits in one word (one LDS read per probe)"))
    for key, opts, what in alt:
        dd = glop.Dict(pats, **opts)
        ms_alt = time_dict(dd)
        result[key] = {"ms_per_step": round(ms_alt, 5), "GBps": round(n / (ms_alt / 1e3) / 1e9, 2),
                       "vs_default": round(ms_per_step / ms_alt, 3), "num_states": dd.info()["num_states"],
                       "config": what}
        del dd

    if not args.no_alt:
        # The autotuner on an independent sample of the same recipe and size
        # (another seed), then the chosen options on the benchmark text.
        import dataclasses

        w = synth.WORKLOADS[args.workload]
        spec = dataclasses.replace(w.text, n_bytes=n)
        sample_text = synth.gen_text(spec, synth.BASE_SEED + 1, synth.STREAM_TEXT + w.index)
        synth.plant(sample_text, pats, spec.plant_every, synth.BASE_SEED + 1, synth.STREAM_PLANTS + w.index)
        sample = torch.from_numpy(sample_text).to(dev)
        t0 = time.perf_counter()
        tuned = glop.autotune(pats, sample)
        tune_s = time.perf_counter() - t0
        del sample
        dt_ = glop.Dict(pats, **tuned["opts"])
        ms_tuned = time_dict(dt_)
        del dt_
        result["autotune"] = {"opts": tuned["opts"], "evaluated": tuned["evaluated"], "seconds": round(tune_s, 2),
                              "sample_ms_auto": round(tuned["auto_ms"], 5), "sample_ms_tuned": round(tuned["ms"], 5),
                              "ms_per_step": round(ms_tuned, 5), "GBps": round(n / (ms_tuned / 1e3) / 1e9, 2),
                              "sample": "a text of the same recipe, size and dictionary, another seed"}

    if not args.no_host_stream:
        log("[bench] host-streamed input ...")
        result["host_streamed"] = bench_host_stream(d, text)
    if not args.no_batched and args.workload == "medium":
        del out, ws_buf, t_dev
        torch.cuda.empty_cache()
        log("[bench] batched comparison ...")
        result["batched"] = bench_batched(args.batched_reps)
    if not args.no_served and args.workload == "medium":
        torch.cuda.empty_cache()
        result["served"] = bench_served(args.served_requests)
    if not args.no_cpu:
        log("[bench] timing the CPU oracle on a sample ...")
        result["cpu_baseline"] = cpu_baseline(text, pats, args.cpu_seconds)
        log("[bench] timing the CPU trie walk ...")
        result["cpu_trie_walk"] = cpu_trie_baseline(d, text, 4.0)
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
