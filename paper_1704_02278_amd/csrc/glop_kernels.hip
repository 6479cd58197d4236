// Dispatch of the matching kernels: picks the Kernels<> variant for a
// dictionary and enqueues a single-text match or a batch.
#include "glop_kernels_impl.hpp"

#include <mutex>

namespace glop {
namespace detail {

GLOP_DECLARE_VARIANT(1, 0, 1, 0, 8)
GLOP_DECLARE_VARIANT(1, 1, 1, 0, 8)
GLOP_DECLARE_VARIANT(1, 1, 1, 1, 8)
GLOP_DECLARE_VARIANT(1, 1, 2, 0, 8)
GLOP_DECLARE_VARIANT(1, 1, 2, 1, 8)
GLOP_DECLARE_VARIANT(4, 1, 1, 0, 8)
GLOP_DECLARE_VARIANT(4, 1, 1, 1, 8)
GLOP_DECLARE_VARIANT(4, 1, 2, 0, 8)
GLOP_DECLARE_VARIANT(4, 1, 2, 1, 8)
GLOP_DECLARE_VARIANT(1, 1, 4, 1, 8)
GLOP_DECLARE_VARIANT(1, 1, 3, 0, 8)
GLOP_DECLARE_VARIANT(1, 1, 3, 1, 8)
GLOP_DECLARE_VARIANT(4, 1, 3, 0, 8)
GLOP_DECLARE_VARIANT(4, 1, 3, 1, 8)
GLOP_DECLARE_VARIANT(4, 1, 2, 1, 4)
GLOP_DECLARE_VARIANT(1, 1, 3, 1, 4)

namespace {

// The Kernels<> variant that serves dictionary d.
const VariantFns &variant_for(const GlopDevDict &d) {
    // 4 KiB tiles exist for the two default filters (the build refuses others).
    if (d.tile_kib == 4)
        return d.stride == 4 ? GLOP_VARIANT_ID(4, 1, 2, 1, 4)() : GLOP_VARIANT_ID(1, 1, 3, 1, 4)();
    if (d.filter != GLOP_FILTER_QGRAM) return GLOP_VARIANT_ID(1, 0, 1, 0, 8)();
    const bool q4 = d.qgram == 4, k2 = d.probe_bits == 2;
    if (d.probe_bits == 4) return GLOP_VARIANT_ID(1, 1, 4, 1, 8)();  // stride 1, 4-byte q-grams (checked at build)
    if (d.probe_bits == 3) {
        if (d.stride == 4) return q4 ? GLOP_VARIANT_ID(4, 1, 3, 1, 8)() : GLOP_VARIANT_ID(4, 1, 3, 0, 8)();
        return q4 ? GLOP_VARIANT_ID(1, 1, 3, 1, 8)() : GLOP_VARIANT_ID(1, 1, 3, 0, 8)();
    }
    if (d.stride == 4) {
        if (k2) return q4 ? GLOP_VARIANT_ID(4, 1, 2, 1, 8)() : GLOP_VARIANT_ID(4, 1, 2, 0, 8)();
        return q4 ? GLOP_VARIANT_ID(4, 1, 1, 1, 8)() : GLOP_VARIANT_ID(4, 1, 1, 0, 8)();
    }
    if (k2) return q4 ? GLOP_VARIANT_ID(1, 1, 2, 1, 8)() : GLOP_VARIANT_ID(1, 1, 2, 0, 8)();
    return q4 ? GLOP_VARIANT_ID(1, 1, 1, 1, 8)() : GLOP_VARIANT_ID(1, 1, 1, 0, 8)();
}

// Read stream with the scan kernel's load shape and nothing else: workgroup b
// takes the 8 KiB tiles [b * tpi, (b + 1) * tpi), wave w every 16th of them
// from the w-th, a lane 16 bytes of each 1 KiB round with non-temporal loads,
// and a tile's loads go out as soon as the one before it is consumed.
__global__ __launch_bounds__(kBlock) void glop_stream_read_kernel(const uint8_t *p, uint64_t n16, uint64_t tpi,
                                                                 uint64_t *sink) {
    constexpr uint64_t kTile16 = 8 * kWave;  // 16-byte units per 8 KiB tile
    const uint64_t ntiles = (n16 + kTile16 - 1) / kTile16;
    const uint64_t tb = (uint64_t)blockIdx.x * tpi;
    const uint64_t te = min(ntiles, tb + tpi);
    const uint64_t lane = lane_id();
    uint4 v[8];
    auto load = [&](uint64_t t) {
        const uint64_t base = t * kTile16 + lane;
        if ((t + 1) * kTile16 <= n16) {
#pragma unroll
            for (int k = 0; k < 8; ++k) v[k] = load_stream16(p + (base + (uint64_t)k * kWave) * 16);
        } else {
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const uint64_t i = base + (uint64_t)k * kWave;
                v[k] = i < n16 ? *reinterpret_cast<const uint4 *>(p + i * 16) : make_uint4(0u, 0u, 0u, 0u);
            }
        }
    };
    uint32_t acc = 0;
    uint64_t t = tb + wave_id();
    if (t < te) load(t);
    for (; t < te; t += kWaves) {
#pragma unroll
        for (int k = 0; k < 8; ++k) acc ^= v[k].x ^ v[k].y ^ v[k].z ^ v[k].w;
        if (t + kWaves < te) load(t + kWaves);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc ^= __shfl_xor(acc, o);
    if (lane_id() == 0) atomicXor(reinterpret_cast<unsigned int *>(sink), acc);
}

ScanParams base_params(const GlopDevDict &d, uint64_t *counts) {
    ScanParams P{};
    P.d = d;
    P.bm_bytes = d.filter == GLOP_FILTER_QGRAM ? (1u << d.bitmap_log2) / 8 : 0u;
    // The prefix table is used when it fits in LDS beside the rest of the scan
    // kernel's layout (stride-4 layout for the stride-4 filter, else stride 1).
    const uint32_t pt_bytes = d.pt ? (16u << d.pt_lg) : 0u;
    const uint32_t pt_cap = d.filter == GLOP_FILTER_QGRAM && d.stride == 4 ? pt_lds_cap<4>() : pt_lds_cap<1>();
    P.pt_lds_bytes = pt_bytes <= pt_cap ? pt_bytes : 0u;
    // The second filter takes the prefix table's place when that is not
    // staged (the two never fit together; it is built for stride 1 only).
    P.f2_lds_bytes = d.bitmap2 && !P.pt_lds_bytes && d.filter == GLOP_FILTER_QGRAM && d.stride == 1
                         ? (1u << GLOP_FILTER2_LOG2) / 8
                         : 0u;
    P.tab_lds_bytes = d.table_lds ? d.n_dense * d.num_classes * 4u : 0u;
    P.counts = counts;
    return P;
}

}  // namespace
}  // namespace detail

using namespace detail;

// Workspace for callers that cannot allocate: one array per device, held from
// the library's load until the process ends.  In host code `scratch` names a
// host-side stand-in, never the device memory: every use goes through the
// device address that hipGetSymbolAddress returns, looked up once per device.
static __device__ __align__(256) uint8_t scratch[kStaticScratchBytes];

hipError_t static_scratch(int device, void **ptr) {
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));  // the current device's copy
        if (e != hipSuccess) return e;
        addr[device] = p;
    }
    *ptr = addr[device];
    return hipSuccess;
}

uint64_t workspace_bytes(uint64_t len, int num_cus, uint32_t tile_bytes) {
    return geometry(len, num_cus, tile_bytes, 15).bytes;
}

uint64_t table_lds_room(int32_t filter, uint32_t stride, uint32_t bitmap_log2, uint32_t pt_lg, bool has_pt,
                        bool has_f2) {
    GlopDevDict d{};
    d.filter = filter;
    d.stride = stride;
    d.bitmap_log2 = bitmap_log2;
    d.pt_lg = pt_lg;
    d.pt = has_pt ? reinterpret_cast<const uint32_t *>(16) : nullptr;  // presence only, never read
    d.bitmap2 = has_f2 ? reinterpret_cast<const uint32_t *>(16) : nullptr;
    const ScanParams P = base_params(d, nullptr);
    // The single-text layout is the larger of the two (more tiles per item).
    const uint64_t used = filter == GLOP_FILTER_QGRAM && stride == 4
                              ? dyn_lds<4, false>(P.bm_bytes, P.pt_lds_bytes, P.f2_lds_bytes)
                              : dyn_lds<1, false>(P.bm_bytes, P.pt_lds_bytes, P.f2_lds_bytes);
    return used < kScanLdsLimit ? kScanLdsLimit - used : 0;
}

uint64_t batch_workspace_bytes(uint32_t nchunks, uint64_t max_total_bytes, uint32_t tile_bytes) {
    return batch_geometry(nchunks, max_total_bytes, tile_bytes).bytes;
}

hipError_t prepare_kernels() {
    const VariantFns *all[] = {&GLOP_VARIANT_ID(1, 0, 1, 0, 8)(),  &GLOP_VARIANT_ID(1, 1, 1, 0, 8)(),
                               &GLOP_VARIANT_ID(1, 1, 1, 1, 8)(),  &GLOP_VARIANT_ID(1, 1, 2, 0, 8)(),
                               &GLOP_VARIANT_ID(1, 1, 2, 1, 8)(),  &GLOP_VARIANT_ID(4, 1, 1, 0, 8)(),
                               &GLOP_VARIANT_ID(4, 1, 1, 1, 8)(),  &GLOP_VARIANT_ID(4, 1, 2, 0, 8)(),
                               &GLOP_VARIANT_ID(4, 1, 2, 1, 8)(),  &GLOP_VARIANT_ID(1, 1, 3, 0, 8)(),
                               &GLOP_VARIANT_ID(1, 1, 3, 1, 8)(),   &GLOP_VARIANT_ID(4, 1, 3, 0, 8)(),
                               &GLOP_VARIANT_ID(4, 1, 3, 1, 8)(),   &GLOP_VARIANT_ID(1, 1, 4, 1, 8)(),
                               &GLOP_VARIANT_ID(4, 1, 2, 1, 4)(),   &GLOP_VARIANT_ID(1, 1, 3, 1, 4)()};
    for (const VariantFns *v : all) {
        const hipError_t e = v->set_lds_limit();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_match(const MatchLaunch &a, hipStream_t stream) {
    const GlopDevDict &d = a.d;
    if (d.num_patterns == 0 || a.len < d.min_len) {
        if (a.events && a.events->scan_begin) (void)hipEventRecord((hipEvent_t)a.events->scan_begin, stream);
        const uint32_t n = d.num_patterns;
        const uint32_t blocks = n ? (n + 255) / 256 : 1;
        hipLaunchKernelGGL(glop_zero_kernel<0>, dim3(blocks > 1024 ? 1024 : blocks), dim3(256), 0, stream, a.counts, n,
                           a.total, a.base_in, a.accumulate ? 0u : 1u);
        hipError_t e = hipGetLastError();
        if (a.events && a.events->scan_end) (void)hipEventRecord((hipEvent_t)a.events->scan_end, stream);
        if (a.events && a.events->emit_end) (void)hipEventRecord((hipEvent_t)a.events->emit_end, stream);
        return e;
    }
    const uint32_t tile = d.tile_kib * 1024u;
    ScanParams P = base_params(d, a.counts);
    P.one = make_span(a.text, a.len, d.min_len);
    const Geometry g = geometry(a.len, a.num_cus, tile, P.one.head);
    if (g.bytes > a.workspace_bytes) return hipErrorInvalidValue;
    if (a.start_limit && a.start_limit < a.len && P.one.head + a.start_limit < P.one.valid_end)
        P.one.valid_end = P.one.head + a.start_limit;
    P.zero_counts = a.accumulate ? 0u : 1u;
    P.ntiles = g.ntiles;
    P.tiles_per_item = g.tiles_per_item;
    uint8_t *ws = static_cast<uint8_t *>(a.workspace);
    P.tile_rec = reinterpret_cast<uint64_t *>(ws + g.off_rec);
    P.tile_nm = reinterpret_cast<uint32_t *>(ws + g.off_nm);
    P.staging = reinterpret_cast<uint64_t *>(ws + g.off_stage);
    P.itemsum = reinterpret_cast<uint64_t *>(ws + g.off_item);
    const EmitParams E{a.out, a.max_matches, a.total, nullptr, a.base_in, a.offset_add, nullptr, nullptr};
    return variant_for(d).one(P, E, g.grid, stream, a.events);
}

hipError_t launch_batch(const BatchLaunch &a, hipStream_t stream) {
    // a.d.tile_kib is the batch's tile (the caller sized the workspace for it).
    const GlopDevDict &d = a.d;
    const BatchGeometry g = batch_geometry(a.nchunks, a.max_total_bytes, d.tile_kib * 1024u);
    ScanParams P = base_params(d, a.counts);
    P.chunks = a.chunks;
    P.nchunks = a.nchunks;
    P.tile_cap = g.tile_cap;
    P.item_cap = g.item_cap;
    // The prep kernel sizes the work items once it knows the tile count
    // (kMetaPer); this is only their upper bound.
    P.tiles_per_item = kMaxBatchTilesPerItem;
    uint8_t *ws = static_cast<uint8_t *>(a.workspace);
    P.tile_rec = reinterpret_cast<uint64_t *>(ws + g.off_rec);
    P.tile_nm = reinterpret_cast<uint32_t *>(ws + g.off_nm);
    P.staging = reinterpret_cast<uint64_t *>(ws + g.off_stage);
    P.tile_desc = reinterpret_cast<TileDesc *>(ws + g.off_desc);
    P.tile_start = reinterpret_cast<uint64_t *>(ws + g.off_start);
    P.itemsum = reinterpret_cast<uint64_t *>(ws + g.off_item);
    P.meta = reinterpret_cast<uint64_t *>(ws + g.off_meta);
    const EmitParams E{reinterpret_cast<glop_match_t *>(a.out), a.max_matches, nullptr, a.chunk_first, nullptr, 0,
                       a.slice_first, a.slice_cap};
    return variant_for(d).batch(P, E, a.chunk_count, a.total, a.num_cus, stream);
}

hipError_t launch_stream_read(const uint8_t *data, uint64_t len, uint64_t *sink, int num_cus, hipStream_t stream) {
    // The single-text scan's item split.
    const uint64_t n16 = len / 16, ntiles = (n16 + 8 * kWave - 1) / (8 * kWave);
    if (ntiles == 0) return hipSuccess;
    const uint64_t cus = (uint64_t)(num_cus > 0 ? num_cus : 1);
    const uint64_t tpi = single_tiles_per_item(ntiles, cus);
    const uint32_t grid = (uint32_t)((ntiles + tpi - 1) / tpi);
    hipLaunchKernelGGL(glop_stream_read_kernel, dim3(grid), dim3(kBlock), 0, stream, data, n16, tpi, sink);
    return hipGetLastError();
}

}  // namespace glop
