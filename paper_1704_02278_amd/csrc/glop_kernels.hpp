// Host-visible interface of the matching kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "glop.h"
#include "glop_layout.hpp"

namespace glop {

struct MatchLaunch {
    GlopDevDict d;
    const uint8_t *text;
    uint64_t len;
    glop_match_t *out;
    uint64_t max_matches;
    uint64_t *counts;
    uint64_t *total;  // may be null
    void *workspace;
    uint64_t workspace_bytes;
    int num_cus;
    const glop_events_t *events;  // may be null
    // A text matched in consecutive pieces (each piece one call on one stream):
    uint64_t start_limit;         // only starts below this offset of the piece (0 = all)
    const uint64_t *base_in;      // device word: records of earlier pieces (null = 0); not `total`
    uint64_t offset_add;          // the piece's offset in the whole text
    bool accumulate;              // add to the counts instead of clearing them first
};

struct BatchLaunch {
    GlopDevDict d;
    const glop_chunk_t *chunks;
    uint32_t nchunks;
    uint64_t max_total_bytes;
    glop_batch_match_t *out;
    uint64_t max_matches;
    uint64_t *chunk_first;
    uint64_t *chunk_count;
    uint64_t *counts;
    uint64_t *total;
    void *workspace;
    int num_cus;
    const uint64_t *slice_first;  // optional per-chunk output slices (both or neither)
    const uint64_t *slice_cap;
};

// Device workspace needed for a text of `len` bytes (any alignment).
uint64_t workspace_bytes(uint64_t len, int num_cus, uint32_t tile_bytes);

// The library's own workspace for callers that cannot allocate: a static
// device array of kStaticScratchBytes per device.  static_scratch() gives its
// address on `device`, which must be the current device (looked up on the
// first call, then cached).
constexpr uint64_t kStaticScratchBytes = 32ull << 20;
// The smallest tile a dictionary can use (tile_kib 4): the tuner sizes its
// workspace for it.
constexpr uint32_t kMinTileKiB = 4;
constexpr int kMaxDevices = 64;
hipError_t static_scratch(int device, void **ptr);

// Device workspace needed for a batch of nchunks chunks, max_total_bytes in all.
uint64_t batch_workspace_bytes(uint32_t nchunks, uint64_t max_total_bytes, uint32_t tile_bytes);

// Enqueue a batch on `stream`.
hipError_t launch_batch(const BatchLaunch &a, hipStream_t stream);

// Enqueue the whole match on `stream`.
hipError_t launch_match(const MatchLaunch &a, hipStream_t stream);

// One-time per-device kernel attribute setup (dynamic LDS above 64 KiB).
hipError_t prepare_kernels();

// LDS bytes the scan kernel has left, after its other tables, for a copy of
// the dense transition rows, for a dictionary with these filter and prefix
// table settings (pt_lg = log2 of the prefix table's slots when has_pt).
uint64_t table_lds_room(int32_t filter, uint32_t stride, uint32_t bitmap_log2, uint32_t pt_lg, bool has_pt,
                        bool has_f2);

// Read floor(len / 16) * 16 bytes once (16-byte aligned data) and fold them
// into *sink: the HBM read-stream ceiling the scan kernel is compared with.
hipError_t launch_stream_read(const uint8_t *data, uint64_t len, uint64_t *sink, int num_cus, hipStream_t stream);

}  // namespace glop
