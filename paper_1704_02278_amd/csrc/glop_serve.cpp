// Served matching: resident dictionaries, continuous batching under an HBM
// budget, and an open-loop trace driver.  Built on the public C-ABI
// (glop_match_batch / glop_match_ws); see glop.h for the contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "glop.h"

namespace {

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

constexpr uint64_t align256(uint64_t v) { return (v + 255) & ~255ull; }

// Waiting without sleeping: a small call's GPU time is 20 µs or less, while a
// condition-variable sleep costs tens of microseconds to wake from (and a
// short timed wait oversleeps by the kernel's timer slack, 50 µs by default).
// So the scheduler polls its in-flight batches, and keeps polling for a while
// after its last progress, with the lock released between polls; a poller
// spins on the completion count before it sleeps.  This keeps one host core
// busy while requests are in flight.
constexpr int64_t kSchedSpinNs = 2000000;  // scheduler: poll until 2 ms without progress
constexpr int64_t kPollSpinNs = 2000000;   // poller: spin up to 2 ms, then sleep

uint64_t out_capacity(uint64_t len) { return std::max<uint64_t>(64, len / 256); }

struct Request {
    uint64_t id = 0;
    uint32_t dict = 0;
    const uint8_t *text = nullptr;
    uint64_t len = 0;
    uint64_t tag = 0;
    int64_t arrival_ns = 0;
    uint64_t reserved = 0;  // budget bytes held from admission to release
};

// Device memory of one launch (a batch, or one plain request), freed when
// every request in it has been released.
struct Block {
    void *dev = nullptr;
    uint64_t bytes = 0;     // budget held by the block itself (workspace, tables)
    uint32_t live = 0;      // requests not yet released
};

// One batch in flight on a stream slot.
struct Inflight {
    std::vector<Request> reqs;
    std::shared_ptr<Block> block;
    glop_match_t *out = nullptr;
    uint64_t cap = 0;
    std::vector<uint64_t> slice;  // batch: first record index of each request's output slice
    int64_t launch_ns = 0;
    hipEvent_t done = nullptr;
    int slot = -1;
    bool single = false;  // one request, matched with the single-text kernels
};

// Stream slot: a stream, its completion event and pinned words.
struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    // pinned, room for max_batch_requests entries: a batch of n requests
    // uses chunk table[n] | slice_first[n] | slice_cap[n], copied in one piece
    glop_chunk_t *h_table = nullptr;
    uint64_t *h_res = nullptr;        // pinned: first[n] | count[n] | total, copied back in one piece
    bool busy = false;
};

struct Held {
    std::shared_ptr<Block> block;
    uint64_t reserved = 0;
};

}  // namespace

struct glop_server {
    glop_server_opts o{};
    int device = -1;
    std::vector<glop_handle_t> dicts;
    std::vector<uint32_t> npat;

    std::mutex mu;
    std::condition_variable cv_work;  // submit, release, stop
    std::condition_variable cv_done;  // completions
    std::vector<std::deque<Request>> pending;  // per dictionary, arrival order
    std::deque<Request> fifo;                  // plain mode: all requests in arrival order
    std::deque<Inflight> inflight;             // launch order
    std::deque<glop_completion_t> done;
    std::atomic<uint64_t> done_total{0};       // completions ever queued (read without the lock)
    std::unordered_map<uint64_t, Held> held;   // completed, not yet released
    std::vector<Slot> slots;
    hipStream_t free_stream = nullptr;
    uint64_t reserved = 0;
    uint64_t next_id = 1;
    uint64_t outstanding = 0;  // submitted, not yet completed
    bool stop = false;
    int error = GLOP_OK;
    std::string error_msg;
    std::thread worker;

    uint64_t request_need(uint64_t len) const {
        return (o.count_payload ? len : 0) + out_capacity(len) * 16;
    }

    // Budget for a batch's own memory (tables, workspace) of n requests, `bytes` in all.
    uint64_t batch_own(uint32_t dict, uint32_t n, uint64_t bytes) const {
        // Chunk table and slices, per-request results and total, counts, workspace (the layout of
        // launch_batched_locked's device block before its records).
        return align256((uint64_t)n * 32) + align256((2ull * n + 1) * 8) + align256((uint64_t)npat[dict] * 8) +
               align256(glop_batch_workspace_bytes(dicts[dict], n, bytes));
    }

    uint64_t plain_own(uint32_t dict, uint64_t len) const {
        return align256((uint64_t)npat[dict] * 8) + 256 + align256(glop_workspace_bytes(dicts[dict], len)) + 256;
    }

    void set_error(int code, const std::string &msg) {
        if (error == GLOP_OK) {
            error = code;
            error_msg = msg;
        }
    }

    // ---- scheduler (holds mu) ----

    // Finish every batch whose event has fired (streams finish out of order).
    bool reap_locked() {
        bool any = false;
        for (size_t fi = 0; fi < inflight.size();) {
            Inflight &f = inflight[fi];
            hipError_t e = hipEventQuery(f.done);
            if (e == hipErrorNotReady) {
                ++fi;
                continue;
            }
            if (e != hipSuccess) set_error(GLOP_EHIP, std::string("batch failed: ") + hipGetErrorString(e));
            const int64_t t = now_ns();
            Slot &sl = slots[f.slot];
            const uint32_t nreq = (uint32_t)f.reqs.size();
            for (uint32_t i = 0; i < nreq; ++i) {
                const Request &r = f.reqs[i];
                glop_completion_t c{};
                c.request_id = r.id;
                c.tag = r.tag;
                c.dict = r.dict;
                // Each request owns a slice of out_capacity(len) records,
                // alone or in a batch, so what it receives does not depend on
                // the requests it shares a launch with.
                uint64_t first = 0, count = 0;
                if (f.single) {
                    count = sl.h_res[0];
                } else {
                    first = f.slice[i];
                    count = sl.h_res[nreq + i];
                    if (sl.h_res[2 * nreq] == ~0ull) set_error(GLOP_EINTERNAL, "batch workspace overflow");
                }
                c.matches = count;
                c.records = std::min<uint64_t>(count, out_capacity(r.len));
                c.truncated = c.records < count ? 1u : 0u;
                c.d_records = f.out + first;
                c.arrival_ns = r.arrival_ns;
                c.launch_ns = f.launch_ns;
                c.done_ns = t;
                c.batch_requests = nreq;
                done.push_back(c);
                held[r.id] = Held{f.block, r.reserved};
            }
            outstanding -= nreq;
            sl.busy = false;
            inflight.erase(inflight.begin() + fi);
            any = true;
        }
        if (any) {
            done_total.store(done_total.load(std::memory_order_relaxed) + 1, std::memory_order_release);
            cv_done.notify_all();
        }
        return any;
    }

    int free_slot_locked() const {
        for (size_t k = 0; k < slots.size(); ++k)
            if (!slots[k].busy) return (int)k;
        return -1;
    }

    // Allocate a launch's device block on its stream.
    bool alloc_block(Slot &sl, uint64_t dev_bytes, uint64_t own, uint32_t live, std::shared_ptr<Block> &blk) {
        blk = std::make_shared<Block>();
        hipError_t e = hipMallocAsync(&blk->dev, dev_bytes, sl.stream);
        if (e != hipSuccess) {
            set_error(GLOP_ENOMEM, std::string("hipMallocAsync in the server: ") + hipGetErrorString(e));
            blk.reset();
            return false;
        }
        blk->bytes = own;
        blk->live = live;
        return true;
    }

    // Form and launch one batch if a slot is free and something fits.
    bool launch_batched_locked() {
        const int si = free_slot_locked();
        if (si < 0) return false;
        // Dictionary whose head request arrived first.
        int best = -1;
        for (size_t k = 0; k < pending.size(); ++k)
            if (!pending[k].empty() && (best < 0 || pending[k].front().arrival_ns < pending[best].front().arrival_ns ||
                                        (pending[k].front().arrival_ns == pending[best].front().arrival_ns &&
                                         pending[k].front().id < pending[best].front().id)))
                best = (int)k;
        if (best < 0) return false;
        const uint32_t dict = (uint32_t)best;
        std::deque<Request> &q = pending[dict];
        uint32_t n = 0;
        uint64_t bytes = 0, need = 0, cap = 0;
        while (n < q.size() && n < o.max_batch_requests) {
            const Request &r = q[n];
            if (n > 0 && bytes + r.len > o.max_batch_bytes) break;
            const uint64_t need2 = need + request_need(r.len);
            if (reserved + need2 + batch_own(dict, n + 1, bytes + r.len) > o.hbm_budget_bytes) break;
            need = need2;
            bytes += r.len;
            cap += out_capacity(r.len);
            ++n;
        }
        if (n == 0) return false;  // the oldest request waits for memory
        Slot &sl = slots[si];
        if (n == 1) return launch_single_locked(si, q.front(), dict, &q);
        const uint64_t own = batch_own(dict, n, bytes);
        // Device block: table, slices | first[n] count[n] total (one copy back) | counts | workspace |
        // records (one slice per request).
        const uint64_t o_table = 0, o_res = align256((uint64_t)n * 32);
        const uint64_t o_counts = o_res + align256((2ull * n + 1) * 8);
        const uint64_t o_ws = o_counts + align256((uint64_t)npat[dict] * 8);
        const uint64_t ws_bytes = glop_batch_workspace_bytes(dicts[dict], n, bytes);
        const uint64_t o_out = o_ws + align256(ws_bytes);
        const uint64_t dev_bytes = o_out + cap * 16;
        std::shared_ptr<Block> blk;
        if (!alloc_block(sl, dev_bytes, own, n, blk)) return false;
        uint8_t *b = static_cast<uint8_t *>(blk->dev);
        uint64_t *res = reinterpret_cast<uint64_t *>(b + o_res);
        Inflight f;
        f.reqs.assign(q.begin(), q.begin() + n);
        q.erase(q.begin(), q.begin() + n);
        uint64_t *h_slice_first = reinterpret_cast<uint64_t *>(sl.h_table + n), *h_slice_cap = h_slice_first + n;
        f.slice.resize(n);
        for (uint32_t i = 0, at = 0; i < n; ++i) {
            f.reqs[i].reserved = request_need(f.reqs[i].len);
            sl.h_table[i].text = f.reqs[i].len ? f.reqs[i].text : nullptr;
            sl.h_table[i].len = f.reqs[i].len;
            h_slice_first[i] = f.slice[i] = at;
            h_slice_cap[i] = out_capacity(f.reqs[i].len);
            at += h_slice_cap[i];
        }
        reserved += need + own;
        f.block = blk;
        f.out = reinterpret_cast<glop_match_t *>(b + o_out);
        f.cap = cap;
        f.slot = si;
        f.done = sl.done;
        f.launch_ns = now_ns();
        hipError_t e = hipMemcpyAsync(b + o_table, sl.h_table, (uint64_t)n * 32, hipMemcpyHostToDevice, sl.stream);
        int rc = e == hipSuccess ? GLOP_OK : GLOP_EHIP;
        if (rc == GLOP_OK)
            rc = glop_match_batch_sliced(dicts[dict], reinterpret_cast<const glop_chunk_t *>(b + o_table), n, bytes,
                                         reinterpret_cast<glop_batch_match_t *>(f.out), cap,
                                         reinterpret_cast<const uint64_t *>(b + o_table + (uint64_t)n * 16),
                                         reinterpret_cast<const uint64_t *>(b + o_table + (uint64_t)n * 24), res,
                                         res + n, reinterpret_cast<uint64_t *>(b + o_counts), res + 2 * n, b + o_ws,
                                         ws_bytes, sl.stream);
        if (rc == GLOP_OK &&
            ((e = hipMemcpyAsync(sl.h_res, res, (2ull * n + 1) * 8, hipMemcpyDeviceToHost, sl.stream)) != hipSuccess ||
             (e = hipEventRecord(sl.done, sl.stream)) != hipSuccess))
            rc = GLOP_EHIP;
        if (rc != GLOP_OK) set_error(rc, std::string("batch launch failed: ") + glop_last_error_message());
        sl.busy = true;
        inflight.push_back(std::move(f));
        return true;
    }

    // One request with the single-text kernels (glop_match_ws) on slot si;
    // `from` is the queue it is taken from (its front).
    bool launch_single_locked(int si, const Request &r0, uint32_t dict, std::deque<Request> *from) {
        const uint64_t need = request_need(r0.len), own = plain_own(dict, r0.len);
        if (reserved + need + own > o.hbm_budget_bytes) return false;
        Slot &sl = slots[si];
        const uint32_t np = npat[dict];
        const uint64_t o_counts = 0, o_total = align256((uint64_t)np * 8), o_ws = o_total + 256;
        const uint64_t ws_bytes = glop_workspace_bytes(dicts[dict], r0.len);
        const uint64_t cap = out_capacity(r0.len);
        const uint64_t o_out = o_ws + align256(ws_bytes);
        std::shared_ptr<Block> blk;
        if (!alloc_block(sl, o_out + cap * 16, own, 1, blk)) return false;
        uint8_t *b = static_cast<uint8_t *>(blk->dev);
        Inflight f;
        f.reqs.push_back(r0);
        from->pop_front();
        f.reqs[0].reserved = need;
        reserved += need + own;
        f.block = blk;
        f.out = reinterpret_cast<glop_match_t *>(b + o_out);
        f.cap = cap;
        f.slot = si;
        f.done = sl.done;
        f.single = true;
        f.launch_ns = now_ns();
        const Request &r = f.reqs[0];
        // The total goes straight to the slot's pinned word (no copy back).
        int rc = glop_match_ws(dicts[dict], r.len ? r.text : nullptr, r.len, f.out, cap,
                               reinterpret_cast<uint64_t *>(b + o_counts), sl.h_res, b + o_ws, ws_bytes, sl.stream,
                               nullptr);
        hipError_t e = hipSuccess;
        if (rc == GLOP_OK && (e = hipEventRecord(sl.done, sl.stream)) != hipSuccess) rc = GLOP_EHIP;
        if (rc != GLOP_OK) set_error(rc, std::string("launch failed: ") + glop_last_error_message());
        sl.busy = true;
        inflight.push_back(std::move(f));
        return true;
    }

    // Plain mode: every request alone, in arrival order, on one stream.
    bool launch_plain_locked() {
        if (fifo.empty()) return false;
        const int si = free_slot_locked();
        if (si < 0) return false;
        return launch_single_locked(si, fifo.front(), fifo.front().dict, &fifo);
    }

    void release_held_locked(uint64_t id) {
        auto it = held.find(id);
        if (it == held.end()) return;
        reserved -= it->second.reserved;
        std::shared_ptr<Block> blk = it->second.block;
        held.erase(it);
        if (blk && --blk->live == 0) {
            reserved -= blk->bytes;
            (void)hipFreeAsync(blk->dev, free_stream);
            blk->dev = nullptr;
        }
        cv_work.notify_all();
    }

    void run() {
        (void)hipSetDevice(device);
        std::unique_lock<std::mutex> lk(mu);
        int64_t last_progress = now_ns();
        for (;;) {
            bool progress = reap_locked();
            if (stop) {
                // Draining: records are invalid from here on, so everything
                // completed is released (its budget may be what a waiting
                // request needs).
                done.clear();
                while (!held.empty()) release_held_locked(held.begin()->first);
                if (error != GLOP_OK) {
                    // After a failed launch or allocation nothing waiting can
                    // be trusted to run: drop it.
                    for (auto &q : pending) {
                        outstanding -= q.size();
                        q.clear();
                    }
                    outstanding -= fifo.size();
                    fifo.clear();
                }
            }
            for (;;) {
                const bool launched = o.mode == GLOP_SERVE_PLAIN ? launch_plain_locked() : launch_batched_locked();
                if (!launched) break;
                progress = true;
            }
            if (stop && outstanding == 0 && inflight.empty()) break;
            const int64_t t = now_ns();
            if (progress) {
                last_progress = t;
            } else if (!inflight.empty() || t - last_progress < kSchedSpinNs) {
                // Poll again soon; submitters and pollers take the lock meanwhile.
                lk.unlock();
                std::this_thread::yield();
                lk.lock();
            } else {
                cv_work.wait_for(lk, std::chrono::milliseconds(2));
            }
        }
    }
};

namespace glop {
int set_error(int code, const std::string &msg);  // the C-ABI's last-error state
}  // namespace glop

namespace {

glop_server_t create_fail(glop_server *s, int code, const std::string &msg) {
    glop::set_error(code, msg);
    if (s) glop_server_destroy(s);
    return nullptr;
}

}  // namespace

extern "C" {

int64_t glop_now_ns(void) { return now_ns(); }

glop_server_t glop_server_create(const glop_server_opts *opts) {
    glop_server *s = new (std::nothrow) glop_server();
    if (!s) return create_fail(nullptr, GLOP_ENOMEM, "host allocation failed");
    if (opts) s->o = *opts;
    glop_server_opts &o = s->o;
    if (o.mode != GLOP_SERVE_BATCHED && o.mode != GLOP_SERVE_PLAIN)
        return create_fail(s, GLOP_EINVAL, "mode must be GLOP_SERVE_BATCHED or GLOP_SERVE_PLAIN");
    if (!o.max_inflight) o.max_inflight = 8;
    if (!o.max_batch_requests) o.max_batch_requests = 4096;
    if (!o.max_batch_bytes) o.max_batch_bytes = 1ull << 30;
    if (!o.hbm_budget_bytes) o.hbm_budget_bytes = 4ull << 30;
    if (o.mode == GLOP_SERVE_PLAIN) {
        o.max_batch_requests = 1;
        o.max_inflight = std::max<uint32_t>(o.max_inflight, 64);  // requests queued ahead on the one stream
    }
    hipError_t e = hipGetDevice(&s->device);
    if (e != hipSuccess) return create_fail(s, GLOP_ENODEV, std::string("no usable GPU: ") + hipGetErrorString(e));
    hipStream_t shared = nullptr;
    if (o.mode == GLOP_SERVE_PLAIN && (e = hipStreamCreateWithFlags(&shared, hipStreamNonBlocking)) != hipSuccess)
        return create_fail(s, GLOP_EHIP, std::string("hipStreamCreate: ") + hipGetErrorString(e));
    s->slots.resize(o.max_inflight);
    for (size_t k = 0; k < s->slots.size(); ++k) {
        Slot &sl = s->slots[k];
        if (o.mode == GLOP_SERVE_PLAIN)
            sl.stream = shared;
        else if ((e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking)) != hipSuccess)
            return create_fail(s, GLOP_EHIP, std::string("hipStreamCreate: ") + hipGetErrorString(e));
        if ((e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming)) != hipSuccess)
            return create_fail(s, GLOP_EHIP, std::string("hipEventCreate: ") + hipGetErrorString(e));
        const uint64_t n = o.max_batch_requests;
        if (hipHostMalloc((void **)&sl.h_table, n * 32, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void **)&sl.h_res, (2 * n + 1) * 8, hipHostMallocDefault) != hipSuccess)
            return create_fail(s, GLOP_ENOMEM, "pinned host allocation failed");
    }
    if ((e = hipStreamCreateWithFlags(&s->free_stream, hipStreamNonBlocking)) != hipSuccess)
        return create_fail(s, GLOP_EHIP, std::string("hipStreamCreate: ") + hipGetErrorString(e));
    s->worker = std::thread([s] { s->run(); });
    return s;
}

int glop_server_add_dict(glop_server_t s, glop_handle_t h, uint32_t *dict) {
    if (!s || !h || !dict) return GLOP_EINVAL;
    glop_info_t info{};
    int rc = glop_get_info(h, &info);
    if (rc != GLOP_OK) return rc;
    if (info.device != s->device) return GLOP_ENODEV;
    std::lock_guard<std::mutex> lk(s->mu);
    *dict = (uint32_t)s->dicts.size();
    s->dicts.push_back(h);
    s->npat.push_back(info.num_patterns);
    s->pending.emplace_back();
    return GLOP_OK;
}

int glop_server_submit(glop_server_t s, uint32_t dict, const uint8_t *d_text, uint64_t len, uint64_t tag,
                       int64_t arrival_ns, uint64_t *request_id) {
    if (!s) return GLOP_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    if (dict >= s->dicts.size() || (len > 0 && !d_text)) return GLOP_EINVAL;
    if (s->error != GLOP_OK) return s->error;
    const uint64_t own = std::max(s->plain_own(dict, len), s->batch_own(dict, 1, len));
    if (s->request_need(len) + own > s->o.hbm_budget_bytes || len > s->o.max_batch_bytes) return GLOP_EINVAL;
    Request r;
    r.id = s->next_id++;
    r.dict = dict;
    r.text = d_text;
    r.len = len;
    r.tag = tag;
    r.arrival_ns = arrival_ns >= 0 ? arrival_ns : now_ns();
    if (s->o.mode == GLOP_SERVE_PLAIN)
        s->fifo.push_back(r);
    else
        s->pending[dict].push_back(r);
    ++s->outstanding;
    if (request_id) *request_id = r.id;
    s->cv_work.notify_all();
    return GLOP_OK;
}

int glop_server_poll(glop_server_t s, glop_completion_t *out, uint32_t max, uint32_t wait_us, uint32_t *n) {
    if (!s || !n || (max > 0 && !out)) return GLOP_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->done.empty() && wait_us > 0) {
        // Spin on the completion count first (see kPollSpinNs), then sleep.
        const uint64_t seen = s->done_total.load(std::memory_order_acquire);
        const int64_t t0 = now_ns(), deadline = t0 + (int64_t)wait_us * 1000;
        lk.unlock();
        int64_t t = t0;
        while (s->done_total.load(std::memory_order_acquire) == seen && t < deadline && t - t0 < kPollSpinNs) {
            std::this_thread::yield();
            t = now_ns();
        }
        lk.lock();
        if (s->done.empty() && t < deadline)
            s->cv_done.wait_for(lk, std::chrono::nanoseconds(deadline - t), [s] { return !s->done.empty(); });
    }
    uint32_t k = 0;
    while (k < max && !s->done.empty()) {
        out[k++] = s->done.front();
        s->done.pop_front();
    }
    *n = k;
    return s->error;
}

int glop_server_release(glop_server_t s, uint64_t request_id) {
    if (!s) return GLOP_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    if (!s->held.count(request_id)) return GLOP_EINVAL;
    s->release_held_locked(request_id);
    return GLOP_OK;
}

void glop_server_destroy(glop_server_t s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv_work.notify_all();
    }
    if (s->worker.joinable()) s->worker.join();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        std::vector<uint64_t> ids;
        for (auto &kv : s->held) ids.push_back(kv.first);
        for (uint64_t id : ids) s->release_held_locked(id);
    }
    (void)hipStreamSynchronize(s->free_stream);
    hipStream_t shared = nullptr;
    for (Slot &sl : s->slots) {
        if (s->o.mode == GLOP_SERVE_PLAIN) {
            if (sl.stream) shared = sl.stream;
        } else if (sl.stream) {
            (void)hipStreamDestroy(sl.stream);
        }
        if (sl.done) (void)hipEventDestroy(sl.done);
        for (void *p : {(void *)sl.h_table, (void *)sl.h_res})
            if (p) (void)hipHostFree(p);
    }
    if (shared) (void)hipStreamDestroy(shared);
    if (s->free_stream) (void)hipStreamDestroy(s->free_stream);
    delete s;
}

int glop_server_run_trace(glop_server_t s, uint32_t n, const uint32_t *dicts, const uint8_t *const *texts,
                          const uint64_t *lens, const int64_t *at_ns, glop_match_t *copy_out,
                          const uint64_t *copy_base, const uint64_t *copy_cap, int64_t *latency_ns,
                          uint64_t *matches, uint32_t *truncated, uint32_t *batch_requests, int64_t *wall_ns) {
    if (!s || (n > 0 && (!dicts || !texts || !lens || !at_ns || !latency_ns || !matches || !truncated)) ||
        (copy_out && (!copy_base || !copy_cap)))
        return GLOP_EINVAL;
    for (uint32_t k = 0; k < n; ++k) {
        if (k && at_ns[k] < at_ns[k - 1]) return GLOP_EINVAL;
        if (dicts[k] >= s->dicts.size()) return GLOP_EINVAL;
    }
    hipStream_t copy_stream = nullptr;
    if (copy_out && hipStreamCreateWithFlags(&copy_stream, hipStreamNonBlocking) != hipSuccess) return GLOP_EHIP;
    const int64_t t0 = now_ns() + 2000000;  // first arrival 2 ms from now
    std::atomic<int> submit_rc{GLOP_OK};
    std::thread submitter([&] {
        (void)hipSetDevice(s->device);
        for (uint32_t k = 0; k < n; ++k) {
            const int64_t due = t0 + at_ns[k];
            for (;;) {
                const int64_t left = due - now_ns();
                if (left <= 0) break;
                if (left > 200000) std::this_thread::sleep_for(std::chrono::nanoseconds(left - 100000));
            }
            uint64_t id = 0;
            const int rc = glop_server_submit(s, dicts[k], texts[k], lens[k], k, due, &id);
            if (rc != GLOP_OK) {
                submit_rc = rc;
                return;
            }
        }
    });
    std::vector<glop_completion_t> buf(256);
    uint32_t got_all = 0;
    int rc = GLOP_OK;
    int64_t last = t0;
    while (got_all < n) {
        if (submit_rc.load() != GLOP_OK) {
            rc = submit_rc.load();
            break;
        }
        uint32_t got = 0;
        rc = glop_server_poll(s, buf.data(), (uint32_t)buf.size(), 1000, &got);
        if (rc != GLOP_OK) break;
        const int64_t seen = now_ns();
        for (uint32_t i = 0; i < got; ++i) {
            const glop_completion_t &c = buf[i];
            const uint64_t k = c.tag;
            latency_ns[k] = seen - c.arrival_ns;
            matches[k] = c.matches;
            truncated[k] = c.truncated;
            if (batch_requests) batch_requests[k] = c.batch_requests;
            if (copy_out) {
                const uint64_t m = std::min<uint64_t>(c.records, copy_cap[k]);
                if (m && hipMemcpyAsync(copy_out + copy_base[k], c.d_records, m * sizeof(glop_match_t),
                                        hipMemcpyDeviceToDevice, copy_stream) != hipSuccess)
                    rc = GLOP_EHIP;
            }
        }
        if (copy_out && got && hipStreamSynchronize(copy_stream) != hipSuccess) rc = GLOP_EHIP;
        for (uint32_t i = 0; i < got; ++i) (void)glop_server_release(s, buf[i].request_id);
        got_all += got;
        if (got) last = seen;
        if (rc != GLOP_OK) break;
    }
    submitter.join();
    if (copy_stream) (void)hipStreamDestroy(copy_stream);
    if (wall_ns) *wall_ns = n ? last - (t0 + at_ns[0]) : 0;
    return rc;
}

}  // extern "C"
