// C-ABI of the matcher: argument checks, dictionary upload, workspace, errors.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <new>
#include <string>

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
            g_prepared[dev] = true;
        }
    }
    const glop::Compiled &c = h->c;
    const uint64_t o_cls = 0;
    const uint64_t o_bm = align256(o_cls + 256);
    const uint64_t o_delta = align256(o_bm + c.bitmap.size() * 4);
    const uint64_t o_term = align256(o_delta + c.delta.size() * 4);
    const uint64_t o_out = align256(o_term + c.term.size() * 4);
    const uint64_t bytes = align256(o_out + (c.outids.size() + 1) * 4);
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
                  {o_delta, c.delta.data(), c.delta.size() * 4},
                  {o_term, c.term.data(), c.term.size() * 4},
                  {o_out, c.outids.data(), c.outids.size() * 4}};
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

extern "C" {

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
    return glop::workspace_bytes(len, h->num_cus > 0 ? h->num_cus : 1);
}

int glop_match_ws(glop_handle_t h, const uint8_t *d_text, uint64_t len, glop_match_t *d_out,
                  uint64_t max_matches, uint64_t *d_counts, uint64_t *d_total, void *d_workspace,
                  uint64_t workspace_bytes, void *stream, const glop_events_t *events) {
    int rc = check_match_args(h, d_text, len, d_out, max_matches, d_counts);
    if (rc != GLOP_OK) return rc;
    rc = check_device(h);
    if (rc != GLOP_OK) return rc;
    const uint64_t need = glop::workspace_bytes(len, h->num_cus);
    if (!d_workspace || (reinterpret_cast<uintptr_t>(d_workspace) & 255u) || workspace_bytes < need)
        return fail(GLOP_EINVAL, "workspace must be 256-byte aligned and at least " + std::to_string(need) +
                                     " bytes");
    glop::MatchLaunch a{};
    a.d = h->dd;
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

int glop_match(glop_handle_t h, const uint8_t *d_text, uint64_t len, glop_match_t *d_out,
               uint64_t max_matches, uint64_t *d_counts, void *stream) {
    int rc = check_match_args(h, d_text, len, d_out, max_matches, d_counts);
    if (rc != GLOP_OK) return rc;
    rc = check_device(h);
    if (rc != GLOP_OK) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const uint64_t bytes = glop::workspace_bytes(len, h->num_cus);
    void *ws = nullptr;
    hipError_t e = hipMallocAsync(&ws, bytes, s);
    if (e != hipSuccess) return fail(GLOP_ENOMEM, std::string("hipMallocAsync: ") + hipGetErrorString(e));
    rc = glop_match_ws(h, d_text, len, d_out, max_matches, d_counts, nullptr, ws, bytes, stream, nullptr);
    e = hipFreeAsync(ws, s);
    if (rc != GLOP_OK) return rc;
    if (e != hipSuccess) return hip_fail(e, "hipFreeAsync");
    return ok();
}

uint64_t glop_batch_workspace_bytes(glop_handle_t h, uint32_t nchunks, uint64_t max_total_bytes) {
    if (!h) {
        fail(GLOP_EINVAL, "NULL handle");
        return 0;
    }
    ok();
    return glop::batch_workspace_bytes(nchunks, max_total_bytes);
}

int glop_match_batch(glop_handle_t h, const glop_chunk_t *d_chunks, uint32_t nchunks, uint64_t max_total_bytes,
                     glop_batch_match_t *d_out, uint64_t max_matches, uint64_t *d_chunk_first,
                     uint64_t *d_chunk_count, uint64_t *d_counts, uint64_t *d_total, void *d_workspace,
                     uint64_t workspace_bytes, void *stream) {
    if (!h) return fail(GLOP_EINVAL, "NULL handle");
    if (nchunks == 0 || nchunks > (1u << 31)) return fail(GLOP_EINVAL, "nchunks must be 1..2^31");
    if (!d_chunks || !d_chunk_first || !d_chunk_count || !d_total)
        return fail(GLOP_EINVAL, "NULL chunk table, per-chunk output or total");
    if (max_matches > 0 && !d_out) return fail(GLOP_EINVAL, "NULL output with max_matches > 0");
    if (h->c.num_patterns > 0 && !d_counts) return fail(GLOP_EINVAL, "NULL counts with a non-empty dictionary");
    if (max_total_bytes > (1ull << 62)) return fail(GLOP_EINVAL, "max_total_bytes too large");
    int rc = check_device(h);
    if (rc != GLOP_OK) return rc;
    const uint64_t need = glop::batch_workspace_bytes(nchunks, max_total_bytes);
    if (!d_workspace || (reinterpret_cast<uintptr_t>(d_workspace) & 255u) || workspace_bytes < need)
        return fail(GLOP_EINVAL, "workspace must be 256-byte aligned and at least " + std::to_string(need) +
                                     " bytes");
    glop::BatchLaunch a{};
    a.d = h->dd;
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
    hipError_t e = glop::launch_batch(a, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return ok();
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
    out->table_bytes = (uint64_t)c.delta.size() * 4;
    out->outlist_ids = c.outids.size();
    out->filter = c.filter;
    out->stride = c.stride;
    out->qgram = c.qgram;
    out->bitmap_log2 = c.bitmap_log2;
    out->probe_bits = c.probe_bits;
    out->tile_kib = c.tile_kib;
    out->filter_keys = c.filter_keys;
    out->device_bytes = h->blob_bytes;
    out->device = h->blob ? h->device : -1;
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
        default: return "unknown error";
    }
}

}  // extern "C"
