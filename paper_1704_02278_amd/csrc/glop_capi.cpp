// C-ABI of the matcher: argument checks, dictionary upload, workspace, errors.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "glop.h"
#include "glop_kernels.hpp"
#include "glop_trie.hpp"

struct glop_dict {
    glop::Compiled c;
    int device = -1;
    int num_cus = 0;
    void *blob = nullptr;
    uint64_t blob_bytes = 0;
    GlopDevDict dd{};
};

namespace {

thread_local int g_err = GLOP_OK;
thread_local std::string g_msg;

int fail(int code, const std::string &msg) {
    g_err = code;
    g_msg = msg;
    return code;
}

int ok() {
    g_err = GLOP_OK;
    g_msg.clear();
    return GLOP_OK;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(GLOP_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

constexpr uint64_t align256(uint64_t v) { return (v + 255) & ~255ull; }

hipError_t num_cus(int *cus) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    return hipDeviceGetAttribute(cus, hipDeviceAttributeMultiprocessorCount, dev);
}

std::mutex g_prep_mu;
bool g_prepared[64] = {};

int upload(glop_dict *h) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(GLOP_ENODEV, std::string("no usable GPU: ") + hipGetErrorString(e));
    int cus = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
    {
        std::lock_guard<std::mutex> lk(g_prep_mu);
        if (dev >= 0 && dev < 64 && !g_prepared[dev]) {
            e = glop::prepare_kernels();
            if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute");
            // The device address of the static workspace (glop_match_static),
            // looked up once per device while it is current.
            void *ws = nullptr;
            e = glop::static_scratch(dev, &ws);
            if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress of the static workspace");
            g_prepared[dev] = true;
        }
    }
    const glop::Compiled &c = h->c;
    // Where the walks read the dense rows: LDS when asked for (or, automatic,
    // when they take at most kAutoLdsTable bytes) and they fit beside the scan
    // kernel's other LDS tables for this dictionary.
    const uint64_t dense_bytes = (uint64_t)c.n_dense * c.num_classes * 4;
    const bool fits = dense_bytes <= glop::table_lds_room(c.filter, c.stride, c.bitmap_log2, c.pt_lg,
                                                          !c.pt.empty(), !c.bitmap2.empty());
    if (c.placement == GLOP_PLACE_LDS && !fits)
        return fail(GLOP_EINVAL, "placement GLOP_PLACE_LDS: the table's " + std::to_string(dense_bytes) +
                                     " bytes of dense rows do not fit in LDS beside the scan kernel's tables");
    constexpr uint64_t kAutoLdsTable = 48u << 10;
    const bool in_lds = c.placement == GLOP_PLACE_LDS || (c.placement == GLOP_PLACE_AUTO && fits &&
                                                          dense_bytes <= kAutoLdsTable && c.num_patterns > 0);
    const uint64_t o_cls = 0;
    const uint64_t o_bm = align256(o_cls + 256);
    const uint64_t o_delta = align256(o_bm + c.bitmap.size() * 4);
    const uint64_t o_nodes = align256(o_delta + dense_bytes);
    const uint64_t o_inedge = align256(o_nodes + c.nodes.size() * 8);
    const uint64_t o_term = align256(o_inedge + c.in_edge.size() * 2);
    const uint64_t o_out = align256(o_term + c.term.size() * 4);
    const uint64_t o_pbytes = align256(o_out + (c.outids.size() + 1) * 4);
    const uint64_t o_poff = align256(o_pbytes + c.pat_bytes.size());
    const uint64_t o_plen = align256(o_poff + c.pat_off.size() * 8);
    const uint64_t o_pt = align256(o_plen + c.pat_len.size() * 4);
    const uint64_t o_bm2 = align256(o_pt + c.pt.size() * 4);
    const uint64_t bytes = align256(o_bm2 + c.bitmap2.size() * 4);
    void *blob = nullptr;
    e = hipMalloc(&blob, bytes);
    if (e != hipSuccess) return fail(GLOP_ENOMEM, std::string("hipMalloc of the dictionary: ") + hipGetErrorString(e));
    uint8_t *b = static_cast<uint8_t *>(blob);
    struct Piece {
        uint64_t off;
        const void *src;
        uint64_t n;
    } pieces[] = {{o_cls, c.cls, 256},
                  {o_bm, c.bitmap.data(), c.bitmap.size() * 4},
                  {o_delta, c.delta.data(), dense_bytes},
                  {o_nodes, c.nodes.data(), c.nodes.size() * 8},
                  {o_inedge, c.in_edge.data(), c.in_edge.size() * 2},
                  {o_term, c.term.data(), c.term.size() * 4},
                  {o_out, c.outids.data(), c.outids.size() * 4},
                  {o_pbytes, c.pat_bytes.data(), c.pat_bytes.size()},
                  {o_poff, c.pat_off.data(), c.pat_off.size() * 8},
                  {o_plen, c.pat_len.data(), c.pat_len.size() * 4},
                  {o_pt, c.pt.data(), c.pt.size() * 4},
                  {o_bm2, c.bitmap2.data(), c.bitmap2.size() * 4}};
    for (const Piece &p : pieces) {
        if (!p.n) continue;
        e = hipMemcpy(b + p.off, p.src, p.n, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(blob);
            return hip_fail(e, "hipMemcpy of the dictionary");
        }
    }
    h->device = dev;
    h->num_cus = cus;
    h->blob = blob;
    h->blob_bytes = bytes;
    GlopDevDict &d = h->dd;
    d.cls = b + o_cls;
    d.bitmap = reinterpret_cast<const uint32_t *>(b + o_bm);
    d.delta = reinterpret_cast<const uint32_t *>(b + o_delta);
    d.term = reinterpret_cast<const uint32_t *>(b + o_term);
    d.outids = reinterpret_cast<const uint32_t *>(b + o_out);
    d.num_classes = c.num_classes;
    d.num_states = c.num_states;
    d.num_patterns = c.num_patterns;
    d.min_len = c.min_len;
    d.max_len = c.max_len;
    d.qgram = c.qgram;
    d.qmask = c.qmask;
    d.stride = c.stride;
    d.bitmap_log2 = c.bitmap_log2;
    d.probe_bits = c.probe_bits;
    d.tile_kib = c.tile_kib;
    d.filter = c.filter;
    d.verify_from = c.verifies() ? c.prefix_len : 0u;
    d.pat_bytes = c.verifies() ? b + o_pbytes : nullptr;
    d.pat_off = c.verifies() ? reinterpret_cast<const uint64_t *>(b + o_poff) : nullptr;
    d.pat_len = c.verifies() ? reinterpret_cast<const uint32_t *>(b + o_plen) : nullptr;
    d.pt = c.pt.empty() ? nullptr : reinterpret_cast<const uint32_t *>(b + o_pt);
    d.bitmap2 = c.bitmap2.empty() ? nullptr : reinterpret_cast<const uint32_t *>(b + o_bm2);
    d.pt_lg = c.pt_lg;
    d.pt_probes = c.pt_probes;
    d.pt_depth = c.pt_depth;
    d.pt_leaf = c.pt_leaf;
    d.n_dense = c.n_dense;
    d.nodes = c.nodes.empty() ? nullptr : reinterpret_cast<const uint64_t *>(b + o_nodes);
    d.in_edge = c.in_edge.empty() ? nullptr : reinterpret_cast<const uint16_t *>(b + o_inedge);
    d.table_lds = in_lds ? 1u : 0u;
    return GLOP_OK;
}

glop_handle_t make(const uint8_t *const *patterns, const uint32_t *lengths, uint32_t n,
                   const glop_build_opts *opts, bool device) {
    glop_dict *h = new (std::nothrow) glop_dict();
    if (!h) {
        fail(GLOP_ENOMEM, "host allocation failed");
        return nullptr;
    }
    std::string err;
    int rc = glop::compile(patterns, lengths, n, opts, h->c, err);
    if (rc != GLOP_OK) {
        delete h;
        fail(rc, err);
        return nullptr;
    }
    if (device) {
        rc = upload(h);
        if (rc != GLOP_OK) {
            delete h;
            return nullptr;
        }
    }
    ok();
    return h;
}

int check_device(const glop_dict *h) {
    if (!h->blob) return fail(GLOP_ENODEV, "handle has no device copy (built with glop_compile)");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev != h->device)
        return fail(GLOP_ENODEV, "current device " + std::to_string(dev) + " is not the handle's device " +
                                     std::to_string(h->device));
    return GLOP_OK;
}

int check_match_args(const glop_dict *h, const uint8_t *text, uint64_t len, const glop_match_t *out,
                     uint64_t max_matches, const uint64_t *counts) {
    if (!h) return fail(GLOP_EINVAL, "NULL handle");
    if (len > 0 && !text) return fail(GLOP_EINVAL, "NULL text with len > 0");
    if (max_matches > 0 && !out) return fail(GLOP_EINVAL, "NULL output with max_matches > 0");
    if (h->c.num_patterns > 0 && !counts) return fail(GLOP_EINVAL, "NULL counts with a non-empty dictionary");
    if (len > (1ull << 62)) return fail(GLOP_EINVAL, "text too long");
    return GLOP_OK;
}

}  // namespace

namespace glop {
int set_error(int code, const std::string &msg) { return fail(code, msg); }
}  // namespace glop

namespace {

// ---- Autotuning --------------------------------------------------------------

uint32_t ceil_log2_u64(uint64_t v) {
    uint32_t k = 0;
    while (k < 63 && (1ull << k) < v) ++k;
    return k;
}

std::mutex g_tune_mu;
std::map<std::string, glop_tune_result_t> g_tune_cache;
bool g_tune_file_read = false;

std::string tune_key(const glop_dict *h, uint64_t sample_len) {
    hipDeviceProp_t prop{};
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, h->device) == hipSuccess) arch = prop.gcnArchName;
    const glop::Compiled &c = h->c;
    char buf[320];
    std::snprintf(buf, sizeof buf, "%s|cu%d|n%u|min%u|max%u|states2^%u|sample2^%u", arch.c_str(), h->num_cus,
                  c.num_patterns, c.min_len, c.max_len, ceil_log2_u64(c.num_states), ceil_log2_u64(sample_len));
    return buf;
}

// Cache file lines: key TAB filter stride qgram bitmap_log2 probe_bits tile_kib prefix_len ms auto_ms
void tune_file_read_locked() {
    if (g_tune_file_read) return;
    g_tune_file_read = true;
    const char *path = std::getenv("GLOP_TUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    char line[1024];
    while (std::fgets(line, sizeof line, f)) {
        char *tab = std::strchr(line, '\t');
        if (!tab) continue;
        *tab = 0;
        glop_tune_result_t r{};
        int filter = 0;
        unsigned stride = 0, qgram = 0, lg = 0, pb = 0, tile = 0, prefix = 0, layout = 0, place = 0;
        if (std::sscanf(tab + 1, "%d %u %u %u %u %u %u %f %f %u %u", &filter, &stride, &qgram, &lg, &pb, &tile,
                        &prefix, &r.ms, &r.auto_ms, &layout, &place) < 9)
            continue;
        r.opts.layout = layout;
        r.opts.placement = place;
        r.opts.prefix_len = prefix;
        r.opts.filter = filter;
        r.opts.stride = stride;
        r.opts.qgram = qgram;
        r.opts.bitmap_log2 = lg;
        r.opts.probe_bits = pb;
        r.opts.tile_kib = tile;
        g_tune_cache[line] = r;
    }
    std::fclose(f);
}

void tune_file_append_locked(const std::string &key, const glop_tune_result_t &r) {
    const char *path = std::getenv("GLOP_TUNE_CACHE");
    if (!path || !*path) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s\t%d %u %u %u %u %u %u %.6f %.6f %u %u\n", key.c_str(), (int)r.opts.filter, r.opts.stride,
                 r.opts.qgram, r.opts.bitmap_log2, r.opts.probe_bits, r.opts.tile_kib, r.opts.prefix_len, r.ms,
                 r.auto_ms, r.opts.layout, r.opts.placement);
    std::fclose(f);
}

// Device buffers and events of one tuning run; released by the destructor.
struct TuneRun {
    glop_dict *h = nullptr;    // the engine being tuned
    glop_dict *alt = nullptr;  // the other engine (whole patterns vs truncated)
    const uint8_t *const *patterns = nullptr;
    uint32_t n = 0;
    const uint8_t *text = nullptr;
    uint64_t len = 0;
    hipStream_t s = nullptr;
    void *ws = nullptr;
    uint64_t ws_bytes = 0;
    glop_match_t *out = nullptr;
    uint64_t cap = 0;
    uint64_t *counts = nullptr;
    uint64_t *total = nullptr;
    uint32_t *bitmap = nullptr;  // largest filter bitmap (2^19 bits)
    uint32_t *bitmap2 = nullptr; // second filter (a candidate's own keys)
    hipEvent_t e0 = nullptr, e1 = nullptr;
    uint64_t expect = ~0ull;     // match count every option set must give
    uint32_t evaluated = 0;

    ~TuneRun() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        for (void *p : {ws, (void *)out, (void *)counts, (void *)total, (void *)bitmap, (void *)bitmap2})
            if (p) (void)hipFree(p);
        if (h) glop_free(h);
        if (alt) glop_free(alt);
    }

    int setup() {
        ws_bytes = glop::workspace_bytes(len, h->num_cus, glop::kMinTileKiB * 1024u);  // any candidate's tiles
        cap = std::min<uint64_t>(len / 64 + 1024, 1ull << 20);
        hipError_t e;
        if ((e = hipMalloc(&ws, ws_bytes)) != hipSuccess || (e = hipMalloc((void **)&out, cap * 16)) != hipSuccess ||
            (e = hipMalloc((void **)&counts, (uint64_t)std::max<uint32_t>(n, 1) * 8)) != hipSuccess ||
            (e = hipMalloc((void **)&total, 8)) != hipSuccess ||
            (e = hipMalloc((void **)&bitmap, (1u << 19) / 8)) != hipSuccess ||
            (e = hipMalloc((void **)&bitmap2, (1u << GLOP_FILTER2_LOG2) / 8)) != hipSuccess)
            return fail(GLOP_ENOMEM, std::string("hipMalloc while tuning: ") + hipGetErrorString(e));
        if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess)
            return hip_fail(e, "hipEventCreate");
        return GLOP_OK;
    }

    int time(glop_build_opts &o, float *ms) { return time_on(h, o, ms); }

    // Time option set o on handle hd (its free fields are resolved into o,
    // and o records hd's engine); ms = median.
    int time_on(glop_dict *hd, glop_build_opts &o, float *ms) {
        glop::Compiled f;
        f.min_len = hd->c.min_len;
        f.num_patterns = n;
        std::string err;
        int rc = glop::build_filter(patterns, n, o, f, err);
        if (rc != GLOP_OK) return fail(rc, err);
        o.filter = f.filter;
        if (f.filter == GLOP_FILTER_QGRAM) {
            o.stride = f.stride;
            o.qgram = f.qgram;
            o.bitmap_log2 = f.bitmap_log2;
            o.probe_bits = f.probe_bits;
        } else {
            o.stride = o.qgram = o.bitmap_log2 = o.probe_bits = 0;
        }
        // The tile this candidate runs on the sample (an automatic choice
        // resolved for the sample's length, which the result then fixes).
        o.tile_kib = f.call_tile_kib(len, hd->num_cus);
        o.prefix_len = hd->c.prefix_len ? hd->c.prefix_len : GLOP_PREFIX_FULL;
        o.candidates = 0;
        o.layout = hd->c.layout;
        hipError_t e = hipMemcpyAsync(bitmap, f.bitmap.data(), f.bitmap.size() * 4, hipMemcpyHostToDevice, s);
        if (e == hipSuccess && !f.bitmap2.empty())
            e = hipMemcpyAsync(bitmap2, f.bitmap2.data(), f.bitmap2.size() * 4, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "bitmap upload while tuning");
        glop::MatchLaunch a{};
        a.d = hd->dd;
        a.d.bitmap = bitmap;
        a.d.bitmap2 = f.bitmap2.empty() ? nullptr : bitmap2;
        // Rows staged in LDS must still fit beside this candidate's filter.
        if (a.d.table_lds &&
            (uint64_t)hd->c.n_dense * hd->c.num_classes * 4 >
                glop::table_lds_room(f.filter, f.stride, f.bitmap_log2, hd->c.pt_lg, !hd->c.pt.empty(),
                                     !f.bitmap2.empty()))
            a.d.table_lds = 0;
        o.placement = a.d.table_lds ? GLOP_PLACE_LDS : GLOP_PLACE_GLOBAL;
        a.d.filter = f.filter;
        a.d.qgram = f.qgram;
        a.d.qmask = f.qmask;
        a.d.stride = f.stride;
        a.d.bitmap_log2 = f.bitmap_log2;
        a.d.probe_bits = f.probe_bits;
        a.d.tile_kib = o.tile_kib;
        a.text = text;
        a.len = len;
        a.out = out;
        a.max_matches = cap;
        a.counts = counts;
        a.total = total;
        a.workspace = ws;
        a.workspace_bytes = ws_bytes;
        a.num_cus = hd->num_cus;
        constexpr int kWarm = 2, kTimed = 11;
        if (evaluated == 0) {
            // Settle the device before the first timing: launches right after
            // it idled run a few percent slow, which would handicap the
            // automatic options (timed first) against every later candidate.
            const auto t_set = std::chrono::steady_clock::now();
            while (std::chrono::steady_clock::now() - t_set < std::chrono::milliseconds(50)) {
                for (int k = 0; k < 4; ++k)
                    if ((e = glop::launch_match(a, s)) != hipSuccess) return hip_fail(e, "kernel launch while tuning");
                if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
            }
        }
        float t[kTimed];
        for (int k = 0; k < kWarm + kTimed; ++k) {
            if (k >= kWarm && (e = hipEventRecord(e0, s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
            if ((e = glop::launch_match(a, s)) != hipSuccess) return hip_fail(e, "kernel launch while tuning");
            if (k >= kWarm) {
                if ((e = hipEventRecord(e1, s)) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess ||
                    (e = hipEventElapsedTime(&t[k - kWarm], e0, e1)) != hipSuccess)
                    return hip_fail(e, "timing while tuning");
            }
        }
        uint64_t got = 0;
        if ((e = hipMemcpy(&got, total, 8, hipMemcpyDeviceToHost)) != hipSuccess)
            return hip_fail(e, "reading the match count while tuning");
        if (expect == ~0ull) expect = got;
        if (got != expect)
            return fail(GLOP_EINTERNAL, "option sets disagree on the sample: " + std::to_string(got) + " vs " +
                                            std::to_string(expect) + " matches");
        std::sort(t, t + kTimed);
        *ms = t[kTimed / 2];
        ++evaluated;
        return GLOP_OK;
    }
};

}  // namespace

extern "C" {

int glop_autotune(const uint8_t *const *patterns, const uint32_t *lengths, uint32_t n, const uint8_t *d_sample,
                  uint64_t sample_len, void *stream, glop_tune_result_t *out) {
    if (!out) return fail(GLOP_EINVAL, "NULL result");
    if (!d_sample || sample_len == 0) return fail(GLOP_EINVAL, "the sample must be at least one byte of device text");
    *out = glop_tune_result_t{};
    TuneRun run;
    run.h = make(patterns, lengths, n, nullptr, true);
    if (!run.h) return glop_last_error();
    run.patterns = patterns;
    run.n = n;
    run.text = d_sample;
    run.len = sample_len;
    run.s = static_cast<hipStream_t>(stream);
    const glop::Compiled &c = run.h->c;
    glop_build_opts cur{};
    cur.prefix_len = c.prefix_len ? c.prefix_len : GLOP_PREFIX_FULL;
    cur.filter = c.filter;
    if (c.filter == GLOP_FILTER_QGRAM) {
        cur.stride = c.stride;
        cur.qgram = c.qgram;
        cur.bitmap_log2 = c.bitmap_log2;
        cur.probe_bits = c.probe_bits;
    }
    cur.tile_kib = c.tile_kib;
    cur.layout = c.layout;
    cur.placement = run.h->dd.table_lds ? GLOP_PLACE_LDS : GLOP_PLACE_GLOBAL;
    if (n == 0) {
        out->opts = cur;
        return ok();
    }
    const std::string key = tune_key(run.h, sample_len);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_file_read_locked();
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            *out = it->second;
            out->evaluated = 0;
            out->from_cache = 1;
            return ok();
        }
    }
    int rc = run.setup();
    if (rc != GLOP_OK) return rc;
    float best = 0.f;
    cur.tile_kib = 0;  // automatic, resolved for the sample's length
    if ((rc = run.time(cur, &best)) != GLOP_OK) return rc;
    const float auto_ms = best;
    // Keep a candidate only if it is at least 3 % faster: smaller gains on a
    // sample were seen to be noise, or to reverse on the full text (a smaller
    // bitmap won 2.8 % on a quarter-size sample and lost 6 % on the text).
    // Options a dictionary cannot take (GLOP_EINVAL from the filter stage) are
    // skipped.
    constexpr float kKeep = 0.97f;
    auto consider = [&](glop_build_opts cand) -> int {
        float ms = 0.f;
        int r = run.time(cand, &ms);
        if (r == GLOP_EINVAL) return GLOP_OK;
        if (r != GLOP_OK) return r;
        if (ms < kKeep * best) {
            best = ms;
            cur = cand;
        }
        return GLOP_OK;
    };
    // Engine: whole patterns or 8-byte prefixes plus verification, each with
    // its automatic filter options.
    if (c.max_len > 8) {
        glop_build_opts eo{};
        eo.prefix_len = c.prefix_len ? GLOP_PREFIX_FULL : 8u;
        run.alt = make(patterns, lengths, n, &eo, true);
        if (!run.alt) return glop_last_error();
        glop_build_opts cand{};
        float ms = 0.f;
        if ((rc = run.time_on(run.alt, cand, &ms)) != GLOP_OK) return rc;
        if (ms < kKeep * best) {
            std::swap(run.h, run.alt);
            cur = cand;
            best = ms;
        }
    }
    // Table layout and placement of the chosen engine: the other layout, then
    // the other placement of the dense rows (LDS only where they fit).  Each is
    // a handle of its own (the device blob differs), timed with the current
    // filter options.
    auto consider_handle = [&](glop_build_opts bo) -> int {
        glop_dict *hd = make(patterns, lengths, n, &bo, true);
        if (!hd) return glop_last_error() == GLOP_EINVAL ? GLOP_OK : glop_last_error();
        glop_build_opts cand = cur;
        float ms = 0.f;
        int r = run.time_on(hd, cand, &ms);
        if (r != GLOP_OK) {
            glop_free(hd);
            return r;
        }
        if (ms < kKeep * best) {
            std::swap(run.h, hd);
            cur = cand;
            best = ms;
        }
        glop_free(hd);
        return GLOP_OK;
    };
    {
        glop_build_opts bo{};
        bo.prefix_len = cur.prefix_len;
        bo.layout = run.h->c.layout == GLOP_LAYOUT_HYBRID ? GLOP_LAYOUT_DENSE : GLOP_LAYOUT_HYBRID;
        if ((rc = consider_handle(bo)) != GLOP_OK) return rc;
        bo.layout = run.h->c.layout;
        bo.placement = run.h->dd.table_lds ? GLOP_PLACE_GLOBAL : GLOP_PLACE_LDS;
        if ((rc = consider_handle(bo)) != GLOP_OK) return rc;
    }
    const uint32_t minlen = run.h->c.min_len;
    glop_build_opts none{};
    none.prefix_len = cur.prefix_len;
    none.layout = cur.layout;
    none.placement = cur.placement;
    none.filter = GLOP_FILTER_NONE;
    none.tile_kib = 8;
    if ((rc = consider(none)) != GLOP_OK) return rc;
    if (cur.filter == GLOP_FILTER_QGRAM) {
        const glop_build_opts base = cur;
        for (uint32_t q = 1; q <= std::min<uint32_t>(4, minlen); ++q) {
            if (q == base.qgram) continue;
            glop_build_opts cand = base;
            cand.qgram = q;
            cand.stride = minlen >= q + 3 ? 4u : 1u;
            cand.bitmap_log2 = 0;
            cand.tile_kib = 8;
            if ((rc = consider(cand)) != GLOP_OK) return rc;
        }
        {
            glop_build_opts cand = cur;
            cand.stride = cur.stride == 4 ? 1u : 4u;
            cand.tile_kib = 8;
            if ((rc = consider(cand)) != GLOP_OK) return rc;
        }
        const uint32_t pb0 = cur.probe_bits;
        for (uint32_t pb = 1; pb <= 4; ++pb) {
            if (pb == pb0) continue;
            glop_build_opts cand = cur;
            cand.probe_bits = pb;
            cand.tile_kib = 0;  // 4 KiB tiles exist for one probe count per stride
            if ((rc = consider(cand)) != GLOP_OK) return rc;
        }
        const uint32_t lg0 = cur.bitmap_log2;
        for (uint32_t lg = lg0 > 15 ? lg0 - 3 : 12; lg <= std::min<uint32_t>(19, lg0 + 1); ++lg) {
            if (lg == lg0) continue;
            glop_build_opts cand = cur;
            cand.bitmap_log2 = lg;
            if ((rc = consider(cand)) != GLOP_OK) return rc;
        }
        // Bytes per lane per tile: 4 KiB tiles (64 B per lane) where they
        // exist, for the filter chosen so far.
        if (cur.qgram == 4 && ((cur.stride == 4 && cur.probe_bits == 2) || (cur.stride == 1 && cur.probe_bits == 3))) {
            glop_build_opts cand = cur;
            cand.tile_kib = cur.tile_kib == 4 ? 8u : 4u;
            if ((rc = consider(cand)) != GLOP_OK) return rc;
        }
    }
    // Where the chosen filter's automatic tile is the one that won, report it
    // as automatic, so that texts of other lengths still get their own tile.
    if (cur.filter == GLOP_FILTER_QGRAM) {
        glop_build_opts a = cur;
        a.tile_kib = 0;
        glop::Compiled f;
        f.min_len = run.h->c.min_len;
        f.num_patterns = n;
        std::string err;
        if (glop::build_filter(patterns, n, a, f, err) == GLOP_OK &&
            f.call_tile_kib(sample_len, run.h->num_cus) == cur.tile_kib)
            cur.tile_kib = 0;
    } else if (cur.tile_kib == 8) {
        cur.tile_kib = 0;  // the only tile without the filter
    }
    out->opts = cur;
    out->ms = best;
    out->auto_ms = auto_ms;
    out->evaluated = run.evaluated;
    out->from_cache = 0;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[key] = *out;
        tune_file_append_locked(key, *out);
    }
    return ok();
}

glop_handle_t glop_build(const uint8_t *const *patterns, const uint32_t *lengths, uint32_t n) {
    return make(patterns, lengths, n, nullptr, true);
}

glop_handle_t glop_build_ex(const uint8_t *const *patterns, const uint32_t *lengths, uint32_t n,
                            const glop_build_opts *opts) {
    return make(patterns, lengths, n, opts, true);
}

glop_handle_t glop_compile(const uint8_t *const *patterns, const uint32_t *lengths, uint32_t n,
                           const glop_build_opts *opts) {
    return make(patterns, lengths, n, opts, false);
}

void glop_free(glop_handle_t h) {
    if (!h) return;
    if (h->blob) (void)hipFree(h->blob);
    delete h;
}

uint64_t glop_workspace_bytes(glop_handle_t h, uint64_t len) {
    if (!h) {
        fail(GLOP_EINVAL, "NULL handle");
        return 0;
    }
    ok();
    return glop::workspace_bytes(len, h->num_cus > 0 ? h->num_cus : 1, h->c.call_tile_kib(len, h->num_cus) * 1024u);
}

int glop_match_ws(glop_handle_t h, const uint8_t *d_text, uint64_t len, glop_match_t *d_out,
                  uint64_t max_matches, uint64_t *d_counts, uint64_t *d_total, void *d_workspace,
                  uint64_t workspace_bytes, void *stream, const glop_events_t *events) {
    int rc = check_match_args(h, d_text, len, d_out, max_matches, d_counts);
    if (rc != GLOP_OK) return rc;
    rc = check_device(h);
    if (rc != GLOP_OK) return rc;
    const uint64_t need = glop::workspace_bytes(len, h->num_cus, h->c.call_tile_kib(len, h->num_cus) * 1024u);
    if (!d_workspace || (reinterpret_cast<uintptr_t>(d_workspace) & 255u) || workspace_bytes < need)
        return fail(GLOP_EINVAL, "workspace must be 256-byte aligned and at least " + std::to_string(need) +
                                     " bytes");
    glop::MatchLaunch a{};
    a.d = h->dd;
    a.d.tile_kib = h->c.call_tile_kib(len, h->num_cus);
    a.text = d_text;
    a.len = len;
    a.out = d_out;
    a.max_matches = max_matches;
    a.counts = d_counts;
    a.total = d_total;
    a.workspace = d_workspace;
    a.workspace_bytes = workspace_bytes;
    a.num_cus = h->num_cus;
    a.events = events;
    hipError_t e = glop::launch_match(a, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return ok();
}

uint64_t glop_static_max_len(glop_handle_t h) {
    if (!h) return 0;
    // Workspace bytes grow with the length; the largest length that fits.
    uint64_t lo = 0, hi = 1ull << 40;
    while (lo < hi) {
        const uint64_t mid = lo + (hi - lo + 1) / 2;
        if (glop::workspace_bytes(mid, h->num_cus, h->c.call_tile_kib(mid, h->num_cus) * 1024u) <= glop::kStaticScratchBytes) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

int glop_match_static(glop_handle_t h, const uint8_t *d_text, uint64_t len, glop_match_t *d_out,
                      uint64_t max_matches, uint64_t *d_counts, uint64_t *d_total, void *stream) {
    int rc = check_match_args(h, d_text, len, d_out, max_matches, d_counts);
    if (rc != GLOP_OK) return rc;
    rc = check_device(h);
    if (rc != GLOP_OK) return rc;
    const uint64_t need = glop::workspace_bytes(len, h->num_cus, h->c.call_tile_kib(len, h->num_cus) * 1024u);
    if (need > glop::kStaticScratchBytes)
        return fail(GLOP_ETOOLONG, "text of " + std::to_string(len) + " bytes needs " + std::to_string(need) +
                                       " bytes of workspace; the static workspace holds " +
                                       std::to_string(glop::kStaticScratchBytes) + " (at most " +
                                       std::to_string(glop_static_max_len(h)) + " bytes of text)");
    void *ws = nullptr;
    const hipError_t e = glop::static_scratch(h->device, &ws);
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress of the static workspace");
    return glop_match_ws(h, d_text, len, d_out, max_matches, d_counts, d_total, ws, glop::kStaticScratchBytes, stream,
                         nullptr);
}

int glop_match(glop_handle_t h, const uint8_t *d_text, uint64_t len, glop_match_t *d_out,
               uint64_t max_matches, uint64_t *d_counts, void *stream) {
    int rc = check_match_args(h, d_text, len, d_out, max_matches, d_counts);
    if (rc != GLOP_OK) return rc;
    rc = check_device(h);
    if (rc != GLOP_OK) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const uint64_t bytes = glop::workspace_bytes(len, h->num_cus, h->c.call_tile_kib(len, h->num_cus) * 1024u);
    void *ws = nullptr;
    hipError_t e = hipMallocAsync(&ws, bytes, s);
    if (e != hipSuccess) return fail(GLOP_ENOMEM, std::string("hipMallocAsync: ") + hipGetErrorString(e));
    rc = glop_match_ws(h, d_text, len, d_out, max_matches, d_counts, nullptr, ws, bytes, stream, nullptr);
    e = hipFreeAsync(ws, s);
    if (rc != GLOP_OK) return rc;
    if (e != hipSuccess) return hip_fail(e, "hipFreeAsync");
    return ok();
}

int glop_match_host(glop_handle_t h, const uint8_t *h_text, uint64_t len, glop_match_t *d_out,
                    uint64_t max_matches, uint64_t *d_counts, uint64_t *d_total, uint64_t chunk_bytes,
                    void *stream) {
    int rc = check_match_args(h, h_text, len, d_out, max_matches, d_counts);
    if (rc != GLOP_OK) return rc;
    rc = check_device(h);
    if (rc != GLOP_OK) return rc;
    const uint64_t chunk = chunk_bytes ? chunk_bytes : (64ull << 20);
    if (chunk < 4096) return fail(GLOP_EINVAL, "chunk_bytes must be at least 4096");
    const uint64_t halo = h->c.max_len ? h->c.max_len - 1 : 0;
    const uint64_t piece_max = std::min<uint64_t>(len, chunk + halo);
    const uint64_t npieces = len ? (len + chunk - 1) / chunk : 1;
    hipStream_t s = static_cast<hipStream_t>(stream);

    // Resources of the call, released on every path.
    struct Res {
        uint8_t *pinned[2] = {nullptr, nullptr};
        uint8_t *dev = nullptr;  // two piece buffers | workspace | two running-total words
        hipStream_t copy = nullptr;
        hipEvent_t copied[2] = {nullptr, nullptr}, consumed[2] = {nullptr, nullptr};
        ~Res() {
            for (int b = 0; b < 2; ++b) {
                if (copied[b]) (void)hipEventDestroy(copied[b]);
                if (consumed[b]) (void)hipEventDestroy(consumed[b]);
                if (pinned[b]) (void)hipHostFree(pinned[b]);
            }
            if (copy) (void)hipStreamDestroy(copy);
            if (dev) (void)hipFree(dev);
        }
    } r;
    const uint64_t buf = align256(std::max<uint64_t>(piece_max, 16));
    // Every piece runs the tile of the longest one (the workspace is sized for it).
    const uint32_t piece_tile = h->c.call_tile_kib(piece_max, h->num_cus);
    const uint64_t ws_bytes = glop::workspace_bytes(piece_max, h->num_cus, piece_tile * 1024u);
    const uint64_t o_ws = 2 * buf, o_cursor = o_ws + align256(ws_bytes);
    hipError_t e;
    if ((e = hipMalloc((void **)&r.dev, o_cursor + 256)) != hipSuccess)
        return fail(GLOP_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    for (int b = 0; b < 2; ++b) {
        if ((e = hipHostMalloc((void **)&r.pinned[b], buf, hipHostMallocDefault)) != hipSuccess)
            return fail(GLOP_ENOMEM, std::string("hipHostMalloc: ") + hipGetErrorString(e));
        if ((e = hipEventCreateWithFlags(&r.copied[b], hipEventDisableTiming)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&r.consumed[b], hipEventDisableTiming)) != hipSuccess)
            return hip_fail(e, "hipEventCreate");
    }
    if ((e = hipStreamCreateWithFlags(&r.copy, hipStreamNonBlocking)) != hipSuccess)
        return hip_fail(e, "hipStreamCreate");
    uint64_t *cursor = reinterpret_cast<uint64_t *>(r.dev + o_cursor);  // two words, used in turn
    // A text already in pinned host memory is uploaded from where it is.
    bool src_pinned = false;
    if (len) {
        hipPointerAttribute_t attr{};
        src_pinned = hipPointerGetAttributes(&attr, h_text) == hipSuccess && attr.type == hipMemoryTypeHost;
        (void)hipGetLastError();  // a pageable pointer leaves an error behind; clear it
    }
    const unsigned hw = std::thread::hardware_concurrency();
    const unsigned nthreads = std::max(1u, std::min(8u, hw ? hw : 1u));
    auto stage = [&](uint8_t *dst, const uint8_t *src, uint64_t n) {
        // Pageable to pinned, split over host threads (one pass of host memory bandwidth).
        const uint64_t per = (n + nthreads - 1) / nthreads;
        std::vector<std::thread> ts;
        for (unsigned t = 1; t < nthreads && per * t < n; ++t)
            ts.emplace_back([=] { std::memcpy(dst + per * t, src + per * t, std::min(per, n - per * t)); });
        std::memcpy(dst, src, std::min(per, n));
        for (auto &t : ts) t.join();
    };
    for (uint64_t k = 0; k < npieces; ++k) {
        const int b = (int)(k & 1);
        const uint64_t start = k * chunk;
        const uint64_t starts = len ? std::min(chunk, len - start) : 0;
        const uint64_t bytes = len ? std::min(chunk + halo, len - start) : 0;
        uint8_t *dbuf = r.dev + (uint64_t)b * buf;
        if (bytes) {
            const uint8_t *src = h_text + start;
            if (!src_pinned) {
                if (k >= 2 && (e = hipEventSynchronize(r.copied[b])) != hipSuccess) return hip_fail(e, "staging wait");
                stage(r.pinned[b], src, bytes);
                src = r.pinned[b];
            }
            if (k >= 2 && (e = hipStreamWaitEvent(r.copy, r.consumed[b], 0)) != hipSuccess)
                return hip_fail(e, "hipStreamWaitEvent");
            if ((e = hipMemcpyAsync(dbuf, src, bytes, hipMemcpyHostToDevice, r.copy)) != hipSuccess ||
                (e = hipEventRecord(r.copied[b], r.copy)) != hipSuccess ||
                (e = hipStreamWaitEvent(s, r.copied[b], 0)) != hipSuccess)
                return hip_fail(e, "piece upload");
        }
        glop::MatchLaunch a{};
        a.d = h->dd;
        a.d.tile_kib = piece_tile;
        a.text = bytes ? dbuf : nullptr;
        a.len = bytes;
        a.out = d_out;
        a.max_matches = max_matches;
        a.counts = d_counts;
        a.total = cursor + ((k + 1) & 1);
        a.workspace = r.dev + o_ws;
        a.workspace_bytes = ws_bytes;
        a.num_cus = h->num_cus;
        a.start_limit = starts;
        a.base_in = k ? cursor + (k & 1) : nullptr;
        a.offset_add = start;
        a.accumulate = k > 0;
        if ((e = glop::launch_match(a, s)) != hipSuccess) return hip_fail(e, "kernel launch");
        if ((e = hipEventRecord(r.consumed[b], s)) != hipSuccess) return hip_fail(e, "hipEventRecord");
    }
    if (d_total && (e = hipMemcpyAsync(d_total, cursor + (npieces & 1), 8, hipMemcpyDeviceToDevice, s)) != hipSuccess)
        return hip_fail(e, "total copy");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    return ok();
}

uint64_t glop_batch_workspace_bytes(glop_handle_t h, uint32_t nchunks, uint64_t max_total_bytes) {
    if (!h) {
        fail(GLOP_EINVAL, "NULL handle");
        return 0;
    }
    ok();
    return glop::batch_workspace_bytes(nchunks, max_total_bytes,
                                       h->c.batch_tile_kib(max_total_bytes, h->num_cus) * 1024u);
}

namespace {

int match_batch(glop_handle_t h, const glop_chunk_t *d_chunks, uint32_t nchunks, uint64_t max_total_bytes,
                glop_batch_match_t *d_out, uint64_t max_matches, const uint64_t *d_slice_first,
                const uint64_t *d_slice_cap, uint64_t *d_chunk_first, uint64_t *d_chunk_count, uint64_t *d_counts,
                uint64_t *d_total, void *d_workspace, uint64_t workspace_bytes, void *stream) {
    if (!h) return fail(GLOP_EINVAL, "NULL handle");
    if (nchunks == 0 || nchunks > (1u << 31)) return fail(GLOP_EINVAL, "nchunks must be 1..2^31");
    if (!d_chunks || !d_chunk_first || !d_chunk_count || !d_total)
        return fail(GLOP_EINVAL, "NULL chunk table, per-chunk output or total");
    if (max_matches > 0 && !d_out) return fail(GLOP_EINVAL, "NULL output with max_matches > 0");
    if (h->c.num_patterns > 0 && !d_counts) return fail(GLOP_EINVAL, "NULL counts with a non-empty dictionary");
    if (max_total_bytes > (1ull << 62)) return fail(GLOP_EINVAL, "max_total_bytes too large");
    int rc = check_device(h);
    if (rc != GLOP_OK) return rc;
    const uint32_t tile_kib = h->c.batch_tile_kib(max_total_bytes, h->num_cus);
    const uint64_t need = glop::batch_workspace_bytes(nchunks, max_total_bytes, tile_kib * 1024u);
    if (!d_workspace || (reinterpret_cast<uintptr_t>(d_workspace) & 255u) || workspace_bytes < need)
        return fail(GLOP_EINVAL, "workspace must be 256-byte aligned and at least " + std::to_string(need) +
                                     " bytes");
    glop::BatchLaunch a{};
    a.d = h->dd;
    a.d.tile_kib = tile_kib;
    a.chunks = d_chunks;
    a.nchunks = nchunks;
    a.max_total_bytes = max_total_bytes;
    a.out = d_out;
    a.max_matches = max_matches;
    a.chunk_first = d_chunk_first;
    a.chunk_count = d_chunk_count;
    a.counts = d_counts;
    a.total = d_total;
    a.workspace = d_workspace;
    a.num_cus = h->num_cus;
    a.slice_first = d_slice_first;
    a.slice_cap = d_slice_cap;
    hipError_t e = glop::launch_batch(a, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return ok();
}

}  // namespace

int glop_match_batch(glop_handle_t h, const glop_chunk_t *d_chunks, uint32_t nchunks, uint64_t max_total_bytes,
                     glop_batch_match_t *d_out, uint64_t max_matches, uint64_t *d_chunk_first,
                     uint64_t *d_chunk_count, uint64_t *d_counts, uint64_t *d_total, void *d_workspace,
                     uint64_t workspace_bytes, void *stream) {
    return match_batch(h, d_chunks, nchunks, max_total_bytes, d_out, max_matches, nullptr, nullptr, d_chunk_first,
                       d_chunk_count, d_counts, d_total, d_workspace, workspace_bytes, stream);
}

int glop_match_batch_sliced(glop_handle_t h, const glop_chunk_t *d_chunks, uint32_t nchunks,
                            uint64_t max_total_bytes, glop_batch_match_t *d_out, uint64_t max_matches,
                            const uint64_t *d_slice_first, const uint64_t *d_slice_cap, uint64_t *d_chunk_first,
                            uint64_t *d_chunk_count, uint64_t *d_counts, uint64_t *d_total, void *d_workspace,
                            uint64_t workspace_bytes, void *stream) {
    if (!d_slice_first || !d_slice_cap) return fail(GLOP_EINVAL, "NULL slice table");
    return match_batch(h, d_chunks, nchunks, max_total_bytes, d_out, max_matches, d_slice_first, d_slice_cap,
                       d_chunk_first, d_chunk_count, d_counts, d_total, d_workspace, workspace_bytes, stream);
}

int glop_cpu_walk(glop_handle_t h, const uint8_t *text, uint64_t len, glop_match_t *out,
                  uint64_t max_matches, uint64_t *counts, uint64_t *total, int threads) {
    if (!h) return fail(GLOP_EINVAL, "NULL handle");
    int rc = glop::cpu_walk(h->c, text, len, out, max_matches, counts, total, threads);
    if (rc != GLOP_OK) return fail(rc, "glop_cpu_walk failed");
    return ok();
}

int glop_get_info(glop_handle_t h, glop_info_t *out) {
    if (!h || !out) return fail(GLOP_EINVAL, "NULL handle or output");
    const glop::Compiled &c = h->c;
    std::memset(out, 0, sizeof(*out));
    out->num_patterns = c.num_patterns;
    out->min_len = c.min_len;
    out->max_len = c.max_len;
    out->num_classes = c.num_classes;
    out->num_states = c.num_states;
    out->table_bytes = c.device_table_bytes();
    out->layout = c.layout;
    out->placement = h->blob && h->dd.table_lds ? GLOP_PLACE_LDS : GLOP_PLACE_GLOBAL;
    out->dense_states = c.n_dense;
    out->outlist_ids = c.outids.size();
    out->filter = c.filter;
    out->stride = c.stride;
    out->qgram = c.qgram;
    out->bitmap_log2 = c.bitmap_log2;
    out->probe_bits = c.probe_bits;
    out->tile_kib = c.tile_kib;
    out->filter_keys = c.filter_keys;
    out->prefix_len = c.prefix_len;
    out->candidates = c.candidates;
    out->device_bytes = h->blob_bytes;
    out->device = h->blob ? h->device : -1;
    out->prefix_keys = c.pt_keys;
    out->prefix_slots = c.pt.empty() ? 0u : (1u << c.pt_lg);
    out->prefix_depth = c.pt_depth;
    out->filter2_log2 = c.bitmap2.empty() ? 0u : GLOP_FILTER2_LOG2;
    return ok();
}

uint32_t glop_num_patterns(glop_handle_t h) { return h ? h->c.num_patterns : 0u; }

uint32_t glop_max_len(glop_handle_t h) { return h ? h->c.max_len : 0u; }

int glop_stream_read(const uint8_t *d_data, uint64_t len, uint64_t *d_sink, void *stream) {
    if (!d_sink) return fail(GLOP_EINVAL, "NULL sink");
    if (len >= 16 && (!d_data || (reinterpret_cast<uintptr_t>(d_data) & 15u)))
        return fail(GLOP_EINVAL, "data must be a 16-byte aligned device pointer");
    int cus = 0;
    hipError_t e = num_cus(&cus);
    if (e != hipSuccess) return hip_fail(e, "device query");
    e = glop::launch_stream_read(d_data, len, d_sink, cus, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return ok();
}

int glop_last_error(void) { return g_err; }

const char *glop_last_error_message(void) { return g_msg.c_str(); }

const char *glop_strerror(int code) {
    switch (code) {
        case GLOP_OK: return "success";
        case GLOP_EINVAL: return "invalid argument";
        case GLOP_ENOMEM: return "out of memory";
        case GLOP_EHIP: return "HIP runtime error";
        case GLOP_ETOOLONG: return "pattern too long";
        case GLOP_ENODEV: return "no usable device";
        case GLOP_EINTERNAL: return "internal consistency check failed";
        default: return "unknown error";
    }
}

}  // extern "C"
