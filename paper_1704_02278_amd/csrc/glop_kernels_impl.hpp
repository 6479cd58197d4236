// Matching kernels: shared device code and the Kernels<> launch template.
// Each variant translation unit instantiates a disjoint set of Kernels<>;
// glop_kernels.hip holds the dispatch.
#pragma once
// Matching kernels for gfx950 (CDNA4, wave64).
//
// Every byte offset of the text starts a walk of the failureless trie
// (Section 5).  The work is split in two kernels:
//
// scan  -- streams the text once from HBM.  Waves claim 4 or 8 KiB tiles; a lane
//          holds 16 consecutive bytes per 1 KiB round (one coalesced 16-byte
//          load).  With the q-gram filter, the lane first probes an LDS Bloom
//          filter that summarises the trie's first q levels: an offset whose
//          q-gram misses the filter cannot start any pattern and needs no walk.
//          At stride 4 only aligned 4-byte words are probed; a word that hits
//          stands for the four offsets whose patterns must contain it.  This is
//          the prefix-filter stage of Sections 2 and 5, made exact because
//          every surviving offset is then walked through the full trie.
//          Survivors are appended in order to a per-wave LDS ring and walked
//          64 at a time, one per lane, so walks run with full waves instead of
//          the few divergent lanes Section 5 describes.  A tile's next loads
//          are issued as soon as its filter bits are known, before its walks.  A walk reads bytes
//          past its tile as needed (the overlap of at least the longest
//          pattern minus one byte that Section 4 requires between chunks).
//          Each tile's matched starts (offset, deepest terminal state) are
//          staged in workspace; the tile's record count is written out.
//          At stride 4 the walks are deferred: hit words go to a
//          workgroup-wide LDS list that all waves walk together, 16 words (64
//          offsets) per wave at a time, once the work item's tiles have
//          streamed, so no wave's stream stalls on walk latency.
// emit  -- turns the per-tile record counts into output positions (sum over
//          earlier work items, then a block scan over the tiles) and writes the
//          (offset, id) records in order, plus the per-pattern counts.  A tile
//          with more matched starts than the staging slots is rescanned here
//          and written directly.
//
// One text is split statically: workgroup g owns work item g (a run of up to
// 1024 tiles).  A batch of chunks is first laid out as one list of tiles (each
// chunk starts a new tile; a prep kernel scans the chunk table and maps every
// tile to its chunk), and the scan workgroups stay resident and take work
// items from a device ticket until none is left.
//
// No workgroup ever waits for another, so the kernels are safe to run beside
// any other work on the device.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "glop_kernels.hpp"

namespace glop {
namespace detail {

constexpr int kWave = 64;
constexpr int kWaves = 16;                  // waves per workgroup
constexpr int kBlock = kWave * kWaves;      // 1024 threads
constexpr int kRoundBytes = kWave * 16;     // 1 KiB: 16 bytes per lane
constexpr uint32_t kMinTileBytes = 4 * kRoundBytes;  // the smallest tile (tile_kib 4)
constexpr uint32_t kStageCap = 16;          // staged matched starts per tile
// Per-wave LDS rings (u16 entries) for tiles walked at once.  Stride 1 queues
// offsets half a round at a time: at most 63 left over plus 512.  Stride 4
// queues hit words: at most 15 left over plus 256 from one round plus the word
// after the tile.
constexpr uint32_t kRing1 = 1024;
constexpr uint32_t kRing4 = 512;
// Deferred hit list (both strides): entry = tile index in the item << 15 |
// position in the tile (stride 4: a hit word's, stride 1: a surviving
// offset's); unwritten slots hold kHitFree.
constexpr uint32_t kHitCap = 8192;
constexpr uint32_t kHitFree = 0xFFFFFFFFu;
constexpr uint32_t kPosBits = 15;
// Tiles per work item at most (per-tile result counters live in LDS: 12 KiB).
// Every item ends in a phase without HBM reads (the deferred walks, the tile
// results), so long items pay it less often; a batch's items, handed out
// from a ticket, stay at 512 tiles or less (with longer ones the last items
// left CUs idle), and at least one tile per wave.
constexpr uint32_t kMaxTilesPerItem = 1024;
constexpr uint32_t kMaxBatchTilesPerItem = 1024;
constexpr uint32_t kMinBatchTilesPerItem = 16;

// A single text's split: the fewest rounds of one item per CU whose items stay
// within kMaxTilesPerItem, items of equal size (so no round runs a few
// stragglers alone).
__host__ __device__ constexpr uint64_t single_tiles_per_item(uint64_t ntiles, uint64_t cus) {
    const uint64_t rounds = ntiles ? (ntiles + cus * kMaxTilesPerItem - 1) / (cus * kMaxTilesPerItem) : 1;
    const uint64_t items = cus * rounds;
    return ntiles ? (ntiles + items - 1) / items : 1;
}

// Batch metadata words in the workspace.
enum {
    kMetaTiles = 0, kMetaItems = 1, kMetaTicket = 2, kMetaOverflow = 3, kMetaTotal = 4, kMetaError = 5, kMetaPer = 6,
    kMetaWords = 8
};

// A listed hit word is written right after its space is reserved; a walker
// waits for it at most this many short sleeps (about 0.1 s) before giving up
// and failing the call, so no wave can wait forever.
constexpr uint32_t kSpinLimit = 1u << 22;
// Record total of a work item that failed; the emit kernel then reports the
// call's total as UINT64_MAX.
constexpr uint64_t kItemFailed = ~0ull;

template <int STRIDE>
constexpr uint32_t ring_cap() { return STRIDE == 4 ? kRing4 : kRing1; }

// Largest prefix table the scan kernel stages in LDS (what the rest of its
// layout leaves of the 160 KiB).  A larger one is not used: a hashed lookup in
// global memory costs about what the first steps through the transition
// table's hot root rows cost (measured slower on a 20,000-pattern dictionary).
template <int STRIDE>
constexpr uint32_t pt_lds_cap() { return STRIDE == 4 ? 32768u : 16384u; }
// The second filter (stride 1) uses the prefix table's room.
static_assert((1u << GLOP_FILTER2_LOG2) / 8 <= pt_lds_cap<1>(), "second filter exceeds its LDS room");

// Tile counters a work item holds in LDS (a batch's prep kernel sizes its
// items within the same bound: fewer item ends per workgroup measured faster
// than items of at most 512 tiles).
template <bool BATCH>
constexpr uint32_t item_tiles_cap() { return BATCH ? kMaxBatchTilesPerItem : kMaxTilesPerItem; }

// Dynamic LDS the scan kernels may use (of the workgroup's 160 KiB).
constexpr uint32_t kScanLdsLimit = 160u * 1024u - 1024u;

// The scan kernel's shared words (in dynamic LDS, after its tables).
struct ScanShared {
    uint32_t hl_count, item_failed, tile_next, hl_walked;
    uint64_t item_sh;
    uint64_t red[16];
};
constexpr uint32_t kScanSharedBytes = (sizeof(ScanShared) + 15u) & ~15u;

// Dynamic LDS: bitmap | byte classes | per-wave rings | hit list (stride 4) |
// per-tile matched-start counts | per-tile record counts | prefix table or
// second filter (scan kernel, when staged; never both) | dense transition
// rows (scan kernel, when placed in LDS).
template <int STRIDE, bool BATCH>
struct LdsLayout {
    uint32_t bm_bytes;
    uint32_t pt_bytes = 0;
    uint32_t f2_bytes = 0;
    uint32_t tab_bytes = 0;
    __host__ __device__ constexpr uint32_t cls_off() const { return bm_bytes; }
    __host__ __device__ constexpr uint32_t ring_off() const { return bm_bytes + 256; }
    __host__ __device__ constexpr uint32_t hits_off() const { return ring_off() + kWaves * ring_cap<STRIDE>() * 2; }
    __host__ __device__ constexpr uint32_t nm_off() const { return hits_off() + kHitCap * 4; }
    __host__ __device__ constexpr uint32_t rec_off() const { return nm_off() + item_tiles_cap<BATCH>() * 4; }
    __host__ __device__ constexpr uint32_t pt_off() const { return rec_off() + item_tiles_cap<BATCH>() * 8; }
    __host__ __device__ constexpr uint32_t f2_off() const { return pt_off() + pt_bytes; }
    __host__ __device__ constexpr uint32_t tab_off() const { return f2_off() + f2_bytes; }
    // The scan kernel's few shared words come last, so that its LDS tables
    // start at address 0 (a table address is then its index, with no base
    // to add).
    __host__ __device__ constexpr uint32_t sh_off() const { return (tab_off() + tab_bytes + 15u) & ~15u; }
    __host__ __device__ constexpr uint32_t bytes() const { return sh_off() + kScanSharedBytes; }
};

// A text as the kernels see it: coordinates x count bytes from abase, the
// text's first byte rounded down to 16 bytes.
struct Span {
    const uint8_t *abase;
    uint64_t head;       // coordinate of the first text byte (0..15)
    uint64_t span_end;   // head + len
    uint64_t valid_end;  // starts x with head <= x < valid_end leave room for the shortest pattern
};

__host__ __device__ __forceinline__ Span make_span(const uint8_t *text, uint64_t len, uint32_t min_len) {
    Span s;
    s.head = reinterpret_cast<uintptr_t>(text) & 15u;
    s.abase = text - s.head;
    s.span_end = s.head + len;
    s.valid_end = len >= min_len ? s.head + len - min_len + 1 : 0;
    return s;
}

// A batch tile's chunk, written by the map kernel so that one 32-byte read
// gives tile_info everything it needs.
struct __align__(32) TileDesc {
    const uint8_t *text;  // the chunk's first byte
    uint64_t len;         // the chunk's bytes
    uint64_t k;           // the tile's index within the chunk
    uint32_t chunk;
    uint32_t pad;
};
static_assert(sizeof(TileDesc) == 32, "TileDesc is read as eight words");

struct ScanParams {
    GlopDevDict d;
    Span one;                    // single text
    uint64_t ntiles;             // single text: tiles
    const glop_chunk_t *chunks;  // batch: chunk table
    uint32_t nchunks;
    uint64_t *tile_start;        // batch: first tile of each chunk, nchunks + 1
    TileDesc *tile_desc;         // batch: chunk of each tile
    uint64_t *meta;              // batch: kMeta* words
    uint64_t tile_cap;           // batch: tiles the workspace holds
    uint64_t item_cap;           // batch: work items the workspace holds
    uint64_t tiles_per_item;
    uint32_t bm_bytes;           // bitmap bytes staged in LDS (0 without filter)
    uint32_t pt_lds_bytes;       // prefix table bytes the scan kernel stages in LDS (0: the walks start at the root)
    uint32_t f2_lds_bytes;       // second filter bytes the scan kernel stages in LDS (0: none)
    uint32_t tab_lds_bytes;      // dense transition rows the scan kernel stages in LDS (0: read from memory)
    uint64_t *tile_rec;          // records per tile
    uint32_t *tile_nm;           // matched starts per tile
    uint64_t *staging;           // kStageCap per tile: stage_entry() words
    uint64_t *itemsum;           // records per work item
    uint64_t *counts;            // per-pattern counts
    uint32_t zero_counts;        // single text: the scan kernel clears the counts first
};

struct EmitParams {
    glop_match_t *out;       // (offset, id, chunk) records; glop_batch_match_t has this layout
    uint64_t max_matches;
    uint64_t *total;         // single text (may be null): records before this call plus its own
    uint64_t *chunk_first;   // batch
    const uint64_t *base_in; // single text: device word with the records before this call, or null (0)
    uint64_t offset_add;     // single text: added to every record's offset
    // Batch, optional: chunk c's j-th record goes to out[slice_first[c] + j]
    // for j < slice_cap[c] (a fixed slice per chunk) instead of to its
    // position in the batch's concatenated order.
    const uint64_t *slice_first;
    const uint64_t *slice_cap;
};

// Write one record: `pos` is its position in the concatenated order, `first`
// that of its chunk's first record (used with per-chunk slices only).  In a
// batch, m.reserved holds the chunk (the glop_batch_match_t layout).
template <bool BATCH>
__device__ __forceinline__ void put_record(const EmitParams &E, uint64_t pos, uint64_t first, const glop_match_t &m) {
    if (BATCH && E.slice_first) {
        const uint64_t j = pos - first;
        if (j < E.slice_cap[m.reserved]) {
            const uint64_t q = E.slice_first[m.reserved] + j;
            if (q < E.max_matches) E.out[q] = m;
        }
    } else if (pos < E.max_matches) {
        E.out[pos] = m;
    }
}

// The lane's index, opaque to the optimiser: values derived from it are
// computed where they are used, not hoisted out of the kernel's loops and held
// in registers for its whole length (that pushed the stride-1 kernels past
// their register budget into scratch).
__device__ __forceinline__ uint32_t lane_id() {
    uint32_t l = threadIdx.x & (kWave - 1);
    __asm__ volatile("" : "+v"(l));
    return l;
}

// Wave index in the workgroup, known to the compiler as wave-uniform (so the
// tile indices and addresses derived from it live in scalar registers).
__device__ __forceinline__ uint32_t wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x / kWave); }

__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << lane_id()) - 1ull; }

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Exclusive scan over the wave; `total` = sum.
__device__ __forceinline__ uint32_t wave_excl_scan_u32(uint32_t v, uint32_t &total) {
    const uint32_t lane = lane_id();
    uint32_t incl = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        uint32_t y = __shfl_up(incl, o);
        if (lane >= (uint32_t)o) incl += y;
    }
    total = __shfl(incl, kWave - 1);
    return incl - v;
}

// Exclusive prefix over the wave of small counts c < 2^BITS, and the total.
template <int BITS>
__device__ __forceinline__ uint32_t wave_prefix_small(uint32_t c, uint32_t &total) {
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (int b = 0; b < BITS; ++b) {
        const uint64_t bal = __ballot((c >> b) & 1u);
        pre += (uint32_t)__popcll(bal & lanemask_lt()) << b;
        tot += (uint32_t)__popcll(bal) << b;
    }
    total = tot;
    return pre;
}

// Workgroup barrier that first waits until this wave's own LDS operations,
// atomics included, have completed, so that every wave reads their results
// after it.  The compiler's barrier alone leaves out that wait on some paths
// (where a loop that ends in an LDS atomic add exits straight into the
// barrier): a per-tile record count read after it then missed the last add of
// another wave's walk batch now and then, and the call reported too few
// matches.  lgkmcnt(0), vmcnt and expcnt unconstrained: 0xC07F in the gfx9
// s_waitcnt encoding.
__device__ __forceinline__ void wg_barrier() {
    __builtin_amdgcn_s_waitcnt(0xC07F);
    __syncthreads();
}

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Exclusive scan over the block (1024 threads); `total` = block sum.
__device__ __forceinline__ uint64_t block_excl_scan_u64(uint64_t v, uint64_t *sh, uint64_t &total) {
    const uint32_t lane = lane_id(), wave = wave_id();
    uint64_t incl = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        uint64_t y = __shfl_up(incl, o);
        if (lane >= (uint32_t)o) incl += y;
    }
    if (lane == kWave - 1) sh[wave] = incl;
    wg_barrier();
    if (wave == 0) {
        const uint64_t w = lane < kWaves ? sh[lane] : 0ull;
        uint64_t wi = w;
#pragma unroll
        for (int o = 1; o < kWaves; o <<= 1) {
            uint64_t y = __shfl_up(wi, o);
            if (lane >= (uint32_t)o) wi += y;
        }
        if (lane < kWaves) sh[lane] = wi - w;
        if (lane == kWaves - 1) sh[kWaves] = wi;
    }
    wg_barrier();
    const uint64_t excl = sh[wave] + incl - v;
    total = sh[kWaves];
    wg_barrier();
    return excl;
}

// Sum over the block (1024 threads), returned to every thread.
__device__ __forceinline__ uint64_t block_sum_u64(uint64_t v, uint64_t *sh) {
    const uint32_t lane = lane_id(), wave = wave_id();
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane == 0) sh[wave] = v;
    wg_barrier();
    uint64_t s = 0;
    for (int w = 0; w < kWaves; ++w) s += sh[w];
    wg_barrier();
    return s;
}

// Zero the bytes of little-endian word w (coordinates x .. x+3) outside [lo, hi).
__device__ __forceinline__ uint32_t keep_bytes(uint32_t w, int64_t x, int64_t lo, int64_t hi) {
    int64_t a = lo - x, b = hi - x;  // keep byte k iff a <= k < b
    a = a < 0 ? 0 : (a > 4 ? 4 : a);
    b = b < 0 ? 0 : (b > 4 ? 4 : b);
    if (b <= a) return 0u;
    const uint32_t hi_mask = b == 4 ? 0xFFFFFFFFu : ((1u << (8 * b)) - 1u);
    const uint32_t lo_mask = a == 0 ? 0u : ((1u << (8 * a)) - 1u);
    return w & hi_mask & ~lo_mask;
}

// 16 bytes at an aligned address; NT marks the load non-temporal (the text is
// streamed once, so its lines are the first the caches may give up).
template <bool NT = true>
__device__ __forceinline__ uint4 load_stream16(const uint8_t *p) {
    if constexpr (NT) {
        typedef unsigned v4u __attribute__((ext_vector_type(4)));
        const v4u v = __builtin_nontemporal_load(reinterpret_cast<const v4u *>(p));
        return make_uint4(v.x, v.y, v.z, v.w);
    } else {
        return *reinterpret_cast<const uint4 *>(p);
    }
}

// 16 text bytes at aligned coordinate x; bytes outside the text read as 0.
// An aligned 16-byte block holding at least one text byte lies in the same
// page as that byte, so it is read whole and the outside bytes are masked;
// a block holding none is not read.
__device__ __forceinline__ uint4 load16(const Span &s, uint64_t x) {
    if (x + 16 <= s.head || x >= s.span_end) return make_uint4(0u, 0u, 0u, 0u);
    uint4 v = *reinterpret_cast<const uint4 *>(s.abase + x);
    if (x >= s.head && x + 16 <= s.span_end) return v;
    const int64_t lo = (int64_t)s.head, hi = (int64_t)s.span_end, xi = (int64_t)x;
    v.x = keep_bytes(v.x, xi, lo, hi);
    v.y = keep_bytes(v.y, xi + 4, lo, hi);
    v.z = keep_bytes(v.z, xi + 8, lo, hi);
    v.w = keep_bytes(v.w, xi + 12, lo, hi);
    return v;
}

// 4 text bytes at aligned coordinate x (multiple of 4); outside reads as 0
// (same rule as load16).
__device__ __forceinline__ uint32_t load4(const Span &s, uint64_t x) {
    if (x + 4 <= s.head || x >= s.span_end) return 0u;
    const uint32_t w = *reinterpret_cast<const uint32_t *>(s.abase + x);
    return keep_bytes(w, (int64_t)x, (int64_t)s.head, (int64_t)s.span_end);
}

// Bloom probe: 1 if every probe bit of q-gram g is set.  K = 1 or 2 bits at
// independent positions; K = 3: two bits in one word (blocked).
template <int K, bool Q4>
__device__ __forceinline__ uint32_t probe(const uint32_t *bm, uint32_t g, uint32_t qmask, uint32_t sh) {
    if (!Q4) g &= qmask;
    if (K == 3) {
        const uint32_t h = glop_hash1(g);
        // Both bits set, written as "no bit of the pair missing" so the two
        // one-bit masks feed a single three-input logic op.
        return (~bm[h >> (sh + 5u)] & glop_block_bits(g)) == 0u ? 1u : 0u;
    }
    const uint32_t s1 = glop_hash1(g) >> sh;
    uint32_t hit = bm[s1 >> 5] >> (s1 & 31);
    if (K == 2) {
        const uint32_t s2 = glop_hash2(g) >> sh;
        hit &= bm[s2 >> 5] >> (s2 & 31);
    }
    return hit & 1u;
}

// The same probe, accumulated: the probe's bit (both bits for K = 2 or 3, one
// into each accumulator) enters at the top of a1/a2 as their contents move
// down one place (v_alignbit).  After 16 probes, bit 16 + u of a1 & a2 is
// probe u's result.  A shift takes its amount modulo 32, so the tested bit
// needs no mask and no compare.  For K = 3, `g1` holds the key's second byte
// in its low byte: at stride 1 with q = 4 that is the next offset's key,
// already in a register, so the blocked probe costs a hash, two instructions
// of address, the read, and two shift + align pairs.
template <int K, bool Q4>
__device__ __forceinline__ void probe_acc(const uint32_t *bm, uint32_t g, uint32_t g1, uint32_t qmask, uint32_t sh,
                                          uint32_t &a1, uint32_t &a2) {
    if (!Q4) g &= qmask;
    if (K == 3) {
        if (!Q4) g1 = g >> 8;  // the masked key's second byte (0 when q = 1)
        const uint32_t h = glop_hash1(g);
        const uint32_t w = bm[h >> (sh + 5u)];
        a1 = __builtin_amdgcn_alignbit(w >> (g & 31u), a1, 1u);
        a2 = __builtin_amdgcn_alignbit(w >> (g1 & 31u), a2, 1u);
        return;
    }
    const uint32_t s1 = glop_hash1(g) >> sh;
    a1 = __builtin_amdgcn_alignbit(bm[s1 >> 5] >> (s1 & 31u), a1, 1u);
    if (K == 2) {
        const uint32_t s2 = glop_hash2(g) >> sh;
        a2 = __builtin_amdgcn_alignbit(bm[s2 >> 5] >> (s2 & 31u), a2, 1u);
    }
}

// Offsets x .. x+15 that may start a pattern: head <= x+u < valid_end.
__device__ __forceinline__ uint32_t valid_mask16(const Span &s, uint64_t x) {
    int64_t lo = (int64_t)s.head - (int64_t)x;
    int64_t hi = (int64_t)s.valid_end - (int64_t)x;
    lo = lo < 0 ? 0 : (lo > 16 ? 16 : lo);
    hi = hi < 0 ? 0 : (hi > 16 ? 16 : hi);
    if (hi <= lo) return 0u;
    return ((1u << hi) - 1u) & ~((1u << lo) - 1u);
}

// 8 text bytes at coordinate z (z >= head; the caller masks bytes past the
// text).  Built from aligned 8-byte blocks; the second block is read only if
// it holds a text byte, so both lie in pages the text occupies.
__device__ __forceinline__ uint64_t text_u64(const Span &s, uint64_t z) {
    const uint64_t a = z & ~7ull;
    const uint32_t sh = (uint32_t)(z & 7u) * 8u;
    const uint64_t lo = *reinterpret_cast<const uint64_t *>(s.abase + a);
    if (!sh) return lo;
    const uint64_t hi = a + 8 < s.span_end ? *reinterpret_cast<const uint64_t *>(s.abase + a + 8) : 0ull;
    return (lo >> sh) | (hi << (64u - sh));
}

// What a walk reads from LDS: the byte classes, the prefix table (null when
// the dictionary has none, when it is too large for LDS, and in the emit
// kernel's rare rescans) and a copy of the dense transition rows (null: the
// rows are read from device memory).
struct WalkTabs {
    const uint8_t *cls;
    const uint4 *pt;
    const uint32_t *delta = nullptr;
};

// One transition from state st on class c: the next state | GLOP_TERM_BIT, or
// 0 (no edge).  Dense rows come from LDS when staged there, else from device
// memory; deeper states of the hybrid layout from their nodes.
__device__ __forceinline__ uint32_t next_state(const GlopDevDict &d, const WalkTabs &tabs, uint32_t st, uint32_t c) {
    if (st < d.n_dense) {
        const uint64_t idx = (uint64_t)st * d.num_classes + c;
        return tabs.delta ? tabs.delta[idx] : d.delta[idx];
    }
    return glop_node_step(d.nodes, d.in_edge, d.n_dense, st, c);
}

// The prefix table's entry for a key (0: no pattern begins so); one 16-byte
// read per slot.
__device__ __forceinline__ uint32_t prefix_entry(const GlopDevDict &d, const uint4 *pt, uint32_t lo, uint32_t hi) {
    const uint32_t mask = (1u << d.pt_lg) - 1u;
    const uint32_t home = glop_pt_slot(lo, hi, d.pt_lg);
    for (uint32_t i = 0; i <= d.pt_probes; ++i) {
        const uint4 e = pt[(home + i) & mask];
        if (e.z == 0u) return 0u;  // an empty slot ends the key's run
        if (e.x == lo && e.y == hi) return e.z;
    }
    return 0u;
}

// The failureless walk from coordinate x (Section 5): follow goto edges while
// they exist; return the deepest terminal state passed (0 = none).  Text bytes
// come 8 at a time from aligned loads; the walk may run past its tile up to
// the end of its text.
__device__ __forceinline__ uint32_t walk(const GlopDevDict &d, const Span &s, const WalkTabs &tabs, uint64_t x) {
    uint32_t st = 0, last = 0;
    if (tabs.pt) {
        // The first D steps in one lookup.  Every pattern is at least D bytes
        // long and every start leaves room for the shortest, so the D bytes
        // are text, and no pattern ends above depth D.
        const uint64_t w = text_u64(s, x);
        const uint32_t e = prefix_entry(d, tabs.pt, (uint32_t)w, d.pt_depth == 8 ? (uint32_t)(w >> 32) : 0u);
        if (e == 0u) return 0u;
        st = e & GLOP_STATE_MASK;
        if (e & GLOP_TERM_BIT) last = st;
        if (d.pt_leaf) return last;
        x += d.pt_depth;
    }
    uint64_t win = 0;
    uint32_t have = 0;
    while (x < s.span_end) {
        if (have == 0) {
            const uint64_t xa = x & ~7ull;
            if (xa >= s.head && xa + 8 <= s.span_end) {
                win = *reinterpret_cast<const uint64_t *>(s.abase + xa);
            } else {
                win = 0;
                for (int k = 0; k < 8; ++k) {
                    const uint64_t y = xa + k;
                    if (y >= s.head && y < s.span_end) win |= (uint64_t)s.abase[y] << (8 * k);
                }
            }
            win >>= 8 * (x - xa);
            have = 8 - (uint32_t)(x - xa);
        }
        const uint32_t c = tabs.cls[win & 0xFFu];
        win >>= 8;
        --have;
        const uint32_t e = next_state(d, tabs, st, c);
        if (e == 0) break;
        st = e & GLOP_STATE_MASK;
        if (e & GLOP_TERM_BIT) last = st;
        ++x;
    }
    return last;
}

// Verify stage of a truncated trie (Sections 2 and 5 complete a truncated
// match by comparing the rest of the pattern): listed pattern id matches at
// coordinate x only if its bytes [verify_from, len) follow in the text.  The
// comparison runs 8 bytes at a time from the 8-byte boundary at or below
// verify_from (patterns are stored 8-byte aligned), four words per step with
// every load issued before the compares.
__device__ __forceinline__ bool verified(const GlopDevDict &d, const Span &s, uint64_t x, uint32_t id) {
    const uint32_t len = d.pat_len[id];
    if (len <= d.verify_from) return true;
    if (x + len > s.span_end) return false;
    const uint64_t *p = reinterpret_cast<const uint64_t *>(d.pat_bytes + d.pat_off[id]);
    for (uint32_t k = d.verify_from & ~7u; k < len; k += 32) {
        uint64_t t[4], q[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t b = k + 8u * u;
            t[u] = b < len ? text_u64(s, x + b) : 0ull;
            q[u] = b < len ? p[b / 8] : 0ull;
        }
        uint64_t diff = 0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t b = k + 8u * u;
            if (b < len) {
                const uint32_t r = len - b;
                const uint64_t m = r >= 8 ? ~0ull : ((1ull << (8 * r)) - 1ull);
                diff |= (t[u] ^ q[u]) & m;
            }
        }
        if (diff) return false;
    }
    return true;
}

// Records at coordinate x of a walk whose deepest terminal is st: the listed
// patterns that match (all of them without a verify stage, those whose rest
// follows in the text with one), and which of the first 16 do (`pass`, bit k
// for the k-th; complete when the list has at most 16 entries).
struct StateRecords {
    uint32_t n;       // records: listed patterns that match here
    uint32_t first;   // the state's output list: outids[first .. first + listed)
    uint32_t listed;
    uint32_t pass;    // bit k: listed pattern k matches (k < 16)
};

__device__ __forceinline__ StateRecords state_records(const GlopDevDict &d, const Span &s, uint64_t x, uint32_t st) {
    const uint2 tl = *reinterpret_cast<const uint2 *>(d.term + 2 * st);  // (first, count), one load
    StateRecords r{tl.y, tl.x, tl.y, 0u};
    if (!d.verify_from) {
        r.pass = tl.y <= 16 ? (1u << tl.y) - 1u : 0u;
        return r;
    }
    r.n = 0;
    for (uint32_t k = 0; k < tl.y; ++k) {
        const bool ok = verified(d, s, x, d.outids[tl.x + k]);
        r.n += ok ? 1u : 0u;
        if (ok && k < 16) r.pass |= 1u << k;
    }
    return r;
}

// A staged matched start, ordered by its offset in the tile (top 15 bits):
// offset << 49 | list-form << 48 | pass mask << 32 | low word.  With at most
// 16 listed patterns (list form) the low word is the output list's first
// index and the mask names the records, so the emit kernel reads neither the
// state's list bounds nor, after a verify stage, a single pattern byte again;
// otherwise the low word is the deepest terminal state.
__device__ __forceinline__ uint64_t stage_entry(uint32_t off, uint32_t st, const StateRecords &r) {
    const bool list = r.listed <= 16;
    return ((uint64_t)off << 49) | ((uint64_t)(list ? 1u : 0u) << 48) | ((uint64_t)(r.pass & 0xFFFFu) << 32) |
           (list ? r.first : st);
}

// Where tile t lies: its text (or chunk), its first coordinate, and whether
// every byte it loads is inside that text.
struct TileInfo {
    Span s;
    uint64_t x0;
    uint32_t chunk;
    uint32_t interior;  // 1: every byte the tile loads is inside its text
};

template <int TILE>
__device__ __forceinline__ TileInfo tile_info_of(const Span &s, uint64_t k, uint32_t chunk) {
    TileInfo ti;
    ti.s = s;
    ti.chunk = chunk;
    ti.x0 = k * (uint64_t)TILE;
    ti.interior = (ti.x0 >= ti.s.head && ti.x0 + TILE + 4 <= ti.s.span_end) ? 1u : 0u;
    return ti;
}

template <bool BATCH, int TILE>
__device__ __forceinline__ TileInfo tile_info(const ScanParams &P, uint64_t t) {
    if (BATCH) {
        const TileDesc dsc = P.tile_desc[t];
        return tile_info_of<TILE>(make_span(dsc.text, dsc.len, P.d.min_len), dsc.k, dsc.chunk);
    }
    return tile_info_of<TILE>(P.one, t, 0u);
}

// A batch tile's descriptor as a vector load, lane j < 8 holding its word j.
// It stays in flight through the current tile's probes: a scalar load would
// be drained by their first LDS wait, which waits on scalar loads too.
__device__ __forceinline__ uint32_t tile_desc_lanes(const ScanParams &P, uint64_t t) {
    return reinterpret_cast<const uint32_t *>(P.tile_desc + t)[lane_id() & 7u];
}

template <int TILE>
__device__ __forceinline__ TileInfo tile_info_lanes(const ScanParams &P, uint32_t v) {
    uint32_t w[7];
#pragma unroll
    for (int j = 0; j < 7; ++j) w[j] = (uint32_t)__builtin_amdgcn_readlane((int)v, j);
    const uint8_t *text = reinterpret_cast<const uint8_t *>(((uint64_t)w[1] << 32) | w[0]);
    const uint64_t len = ((uint64_t)w[3] << 32) | w[2], k = ((uint64_t)w[5] << 32) | w[4];
    return tile_info_of<TILE>(make_span(text, len, P.d.min_len), k, w[6]);
}

// A wave's tile in registers: 16 bytes per lane per round, plus the first
// word after the tile (for the probes of the tile's last offsets).
template <int R>
struct TileRegs {
    uint4 v[R];
    uint32_t extra;
};

// A tile's bytes into registers.  NT: non-temporal loads, for the stride-4
// filter, whose walks rarely re-read the text; the stride-1 walks re-read
// their windows right after the load and want them kept in L2.
template <int R, bool FILTER, bool NT = false>
__device__ __forceinline__ void load_tile(const TileInfo &ti, TileRegs<R> &r) {
    const uint64_t x = ti.x0 + lane_id() * 16u;
    if (ti.interior) {
        const uint8_t *p = ti.s.abase + x;
#pragma unroll
        for (int k = 0; k < R; ++k) r.v[k] = load_stream16<NT>(p + k * kRoundBytes);
        r.extra = FILTER ? *reinterpret_cast<const uint32_t *>(ti.s.abase + ti.x0 + R * kRoundBytes) : 0u;
    } else {
#pragma unroll
        for (int k = 0; k < R; ++k) r.v[k] = load16(ti.s, x + (uint64_t)k * kRoundBytes);
        r.extra = FILTER ? load4(ti.s, ti.x0 + R * kRoundBytes) : 0u;
    }
}

// Sink of the scan kernel: stage matched starts of the tile, count records;
// the tile's totals go to the item's LDS counters.
struct StageSink {
    uint32_t *nm_l;    // per-tile matched starts (LDS), indexed by t - tb
    uint64_t *rec_l;   // per-tile records (LDS)
    uint64_t tb;
    uint32_t nm = 0;   // matched starts so far (wave-uniform)
    uint64_t rec = 0;  // records so far (wave-uniform)

    __device__ __forceinline__ StageSink(uint32_t *nm_, uint64_t *rec_, uint64_t tb_)
        : nm_l(nm_), rec_l(rec_), tb(tb_) {}

    __device__ __forceinline__ void batch(const ScanParams &P, uint64_t t, const TileInfo &ti, uint32_t off,
                                          uint32_t last) {
        StateRecords sr{0u, 0u, 0u, 0u};
        if (last) sr = state_records(P.d, ti.s, ti.x0 + off, last);
        const uint32_t cnt = sr.n;
        const bool m = cnt != 0;
        const uint64_t bal = __ballot(m);
        if (bal == 0) return;
        const uint32_t pos = nm + (uint32_t)__popcll(bal & lanemask_lt());
        if (m && pos < kStageCap) P.staging[t * kStageCap + pos] = stage_entry(off, last, sr);
        nm += (uint32_t)__popcll(bal);
        rec += wave_sum_u32(cnt);
    }
    __device__ __forceinline__ void finish(uint64_t t) {
        if (lane_id() == 0) {
            nm_l[t - tb] = nm;
            rec_l[t - tb] = rec;
        }
    }
};

// Per-pattern counts of the emit kernel, gathered per workgroup first: a small
// LDS table keyed by pattern id (open addressing, a few probes, claimed by
// compare-and-swap) takes the increments, and each work item's distinct ids
// then go to the global counts with one atomic add each.  Short patterns that
// occur all over a log text would otherwise put thousands of same-address
// atomics on a few L2 lines.  An id that finds no slot adds to the global
// count directly.  A count stays below 2^32: an item holds at most
// kMaxTilesPerItem * 8 KiB offsets and a pattern occurs once per offset.
struct CountTable {
    static constexpr uint32_t kLog2 = 11;
    static constexpr uint32_t kSlots = 1u << kLog2;
    static constexpr int kProbes = 8;
    uint32_t *key;   // id + 1, 0 = free
    uint32_t *val;
    uint64_t *counts;

    __device__ __forceinline__ void add(uint32_t id) const {
        const uint32_t want = id + 1u;
        uint32_t s = (id * 0x9E3779B1u) >> (32u - kLog2);
        for (int p = 0; p < kProbes; ++p) {
            uint32_t k = __hip_atomic_load(&key[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (k == 0u) {
                k = atomicCAS(&key[s], 0u, want);
                if (k == 0u) k = want;
            }
            if (k == want) {
                atomicAdd(&val[s], 1u);
                return;
            }
            s = (s + 1u) & (kSlots - 1u);
        }
        atomicAdd(reinterpret_cast<unsigned long long *>(counts + id), 1ull);
    }
    // Clear every slot (the whole workgroup; a barrier must follow).
    __device__ __forceinline__ void clear() const {
        for (uint32_t k = threadIdx.x; k < kSlots; k += kBlock) {
            key[k] = 0u;
            val[k] = 0u;
        }
    }
    // Add the gathered counts to the global ones and clear the table (the
    // whole workgroup, between barriers).
    __device__ __forceinline__ void flush() const {
        for (uint32_t k = threadIdx.x; k < kSlots; k += kBlock) {
            const uint32_t id1 = key[k];
            if (id1) {
                atomicAdd(reinterpret_cast<unsigned long long *>(counts + (id1 - 1u)), (unsigned long long)val[k]);
                key[k] = 0u;
                val[k] = 0u;
            }
        }
    }
};

// Sink of the emit kernel's rescan: write the records directly, in order.
template <bool BATCH>
struct DirectSink {
    const EmitParams *E;
    const CountTable *ct;
    uint64_t base;         // output position of the tile's first record
    uint64_t chunk_first;  // output position of its chunk's first record (batch)
    uint64_t cursor = 0;   // records written so far in the tile

    __device__ __forceinline__ DirectSink(const EmitParams *e, const CountTable *c, uint64_t b, uint64_t f)
        : E(e), ct(c), base(b), chunk_first(f) {}

    __device__ __forceinline__ void batch(const ScanParams &P, uint64_t, const TileInfo &ti, uint32_t off,
                                          uint32_t last) {
        const uint64_t x = ti.x0 + off;
        const uint32_t cnt = last ? state_records(P.d, ti.s, x, last).n : 0u;
        const bool m = cnt != 0;
        if (__ballot(m) == 0) return;
        uint32_t tot;
        const uint32_t excl = wave_excl_scan_u32(cnt, tot);
        if (m) {
            const uint64_t i = x - ti.s.head + E->offset_add;
            const uint32_t first = P.d.term[2 * last], listed = P.d.term[2 * last + 1];
            uint32_t j = 0;
            for (uint32_t k = 0; k < listed; ++k) {
                const uint32_t id = P.d.outids[first + k];
                if (P.d.verify_from && !verified(P.d, ti.s, x, id)) continue;
                const uint64_t pos = base + cursor + excl + j++;
                put_record<BATCH>(*E, pos, chunk_first, glop_match_t{i, id, ti.chunk});
                ct->add(id);
            }
        }
        cursor += tot;
    }
    __device__ __forceinline__ void finish(uint64_t) {}
};

// ---- stride 4: one probe per aligned word ---------------------------------
//
// Offset x needs the word at roundup4(x) to hit (every pattern is at least
// q + 3 bytes, so that word lies inside any occurrence starting at x, at
// pattern position t = roundup4(x) - x in 0..3).  Bit 4k+w of the lane's
// result is the word at x0 + k*1024 + lane*16 + 4w; `extra` is the word after
// the tile (it serves the tile's last three offsets).
template <int R>
using HitBits = typename std::conditional<(4 * R > 32), uint64_t, uint32_t>::type;

template <int R, int K, bool Q4>
__device__ __forceinline__ void tile_hits4(const GlopDevDict &d, const TileRegs<R> &r, const uint32_t *bm,
                                           HitBits<R> &pbits, uint32_t &extra_bit) {
    const uint32_t qmask = d.qmask, sh = 32u - d.bitmap_log2;
    if constexpr (4 * R == 32) {
        // Exactly 32 probes: accumulated as in tile_masks1, probe i ends at bit i.
        uint32_t a1 = 0, a2 = K == 1 ? ~0u : 0u;
#pragma unroll
        for (int k = 0; k < R; ++k) {
            probe_acc<K, Q4>(bm, r.v[k].x, r.v[k].x >> 8, qmask, sh, a1, a2);
            probe_acc<K, Q4>(bm, r.v[k].y, r.v[k].y >> 8, qmask, sh, a1, a2);
            probe_acc<K, Q4>(bm, r.v[k].z, r.v[k].z >> 8, qmask, sh, a1, a2);
            probe_acc<K, Q4>(bm, r.v[k].w, r.v[k].w >> 8, qmask, sh, a1, a2);
            __asm__ volatile("" : "+v"(a1), "+v"(a2));
            __builtin_amdgcn_sched_barrier(0);
        }
        pbits = (HitBits<R>)(a1 & a2);
        extra_bit = probe<K, Q4>(bm, r.extra, qmask, sh);
        return;
    }
    HitBits<R> b = 0;
#pragma unroll
    for (int k = 0; k < R; ++k) {
        b |= (HitBits<R>)probe<K, Q4>(bm, r.v[k].x, qmask, sh) << (4 * k);
        b |= (HitBits<R>)probe<K, Q4>(bm, r.v[k].y, qmask, sh) << (4 * k + 1);
        b |= (HitBits<R>)probe<K, Q4>(bm, r.v[k].z, qmask, sh) << (4 * k + 2);
        b |= (HitBits<R>)probe<K, Q4>(bm, r.v[k].w, qmask, sh) << (4 * k + 3);
        // Finish each round's probes in place: left alone, the compiler defers
        // the bit tests and spills every hash and word.
        __asm__ volatile("" : "+v"(b));
        __builtin_amdgcn_sched_barrier(0);
    }
    pbits = b;
    extra_bit = probe<K, Q4>(bm, r.extra, qmask, sh);
}

template <class B>
__device__ __forceinline__ uint32_t popcount(B b) {
    return sizeof(B) == 8 ? (uint32_t)__popcll((uint64_t)b) : (uint32_t)__popc((uint32_t)b);
}

// Walk the four offsets of each of n queued hit words: lanes 4h..4h+3 take hit
// h's offsets p-3, p-2, p-1, p, so a batch of 16 hits is in offset order.
template <int TILE, class Sink>
__device__ __forceinline__ void walk_hit_batch(const ScanParams &P, uint64_t t, const TileInfo &ti,
                                               const WalkTabs &tabs, const uint16_t *queue, uint32_t qhead,
                                               uint32_t n, Sink &sink) {
    const uint32_t lane = lane_id();
    const uint32_t h = lane >> 2;
    bool act = h < n;
    const int32_t p = act ? (int32_t)queue[(qhead + h) & (kRing4 - 1)] : 0;
    const int32_t off = p - 3 + (int32_t)(lane & 3);
    const uint64_t x = ti.x0 + (int64_t)off;
    act = act && off >= 0 && off < TILE && x >= ti.s.head && x < ti.s.valid_end;
    const uint32_t last = act ? walk(P.d, ti.s, tabs, x) : 0u;
    sink.batch(P, t, ti, act ? (uint32_t)off : 0u, last);
}

// Walk a tile's hit words right away (per-wave ring).
template <int R, class Sink>
__device__ __forceinline__ void walk_hits4(const ScanParams &P, uint64_t t, const TileInfo &ti, HitBits<R> pbits,
                                           uint32_t extra_bit, const WalkTabs &tabs, uint16_t *queue, Sink &sink) {
    constexpr int TILE = R * kRoundBytes;
    const uint32_t lane = lane_id();
    if (__ballot(pbits != 0) != 0 || extra_bit) {
        uint32_t qhead = 0, qtail = 0;  // wave-uniform ring indices
#pragma unroll
        for (int k = 0; k < R; ++k) {
            uint32_t bits = (uint32_t)(pbits >> (4 * k)) & 0xFu;
            if (__ballot(bits != 0) == 0) continue;
            uint32_t tot;
            uint32_t pos = qtail + wave_prefix_small<3>((uint32_t)__popc(bits), tot);
            const uint32_t base = (uint32_t)k * kRoundBytes + lane * 16u;
            while (bits) {
                const uint32_t w = (uint32_t)__builtin_ctz(bits);
                bits &= bits - 1u;
                queue[(pos++) & (kRing4 - 1)] = (uint16_t)(base + 4u * w);
            }
            qtail += tot;
            wave_lds_sync();
            for (; qtail - qhead >= 16u; qhead += 16u) walk_hit_batch<TILE>(P, t, ti, tabs, queue, qhead, 16u, sink);
        }
        if (extra_bit) {
            if (lane == 0) queue[qtail & (kRing4 - 1)] = (uint16_t)TILE;
            qtail += 1;
            wave_lds_sync();
        }
        for (; qtail != qhead;) {
            const uint32_t n = min(16u, qtail - qhead);
            walk_hit_batch<TILE>(P, t, ti, tabs, queue, qhead, n, sink);
            qhead += n;
        }
    }
    sink.finish(t);
    __builtin_amdgcn_wave_barrier();
}

// Workgroup hit list of the current work item (stride 4).
struct HitList {
    uint32_t *hits;   // kHitCap entries (LDS)
    uint32_t *count;  // entries reserved, all of which get written (LDS)
};

// Record tile t's hit words in the list; false if they do not fit (then the
// tile must be walked right away).  Space is reserved with compare-and-swap so
// `count` never exceeds what will be written.
template <int R>
__device__ __forceinline__ bool list_hits(const HitList &L, uint32_t t_rel, HitBits<R> pbits, uint32_t extra_bit) {
    const uint32_t lane = lane_id();
    uint32_t tot;
    const uint32_t pre = wave_prefix_small<7>(popcount(pbits), tot);
    const uint32_t n = tot + extra_bit;
    uint32_t base = 0, ok = 0;
    if (lane == 0) {
        uint32_t c = __hip_atomic_load(L.count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        while (c + n <= kHitCap) {
            const uint32_t prev = atomicCAS(L.count, c, c + n);
            if (prev == c) {
                base = c;
                ok = 1;
                break;
            }
            c = prev;
        }
    }
    ok = __builtin_amdgcn_readfirstlane(ok);
    base = __builtin_amdgcn_readfirstlane(base);
    if (!ok) return false;
    const uint32_t tag = t_rel << kPosBits;
    uint32_t pos = base + pre;
    HitBits<R> b = pbits;
    while (b) {
        const uint32_t i = (uint32_t)(sizeof(b) == 8 ? __builtin_ctzll((uint64_t)b) : __builtin_ctz((uint32_t)b));
        b &= b - 1;
        __hip_atomic_store(&L.hits[pos++], tag | ((i >> 2) * kRoundBytes + lane * 16u + 4u * (i & 3u)),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    if (extra_bit && lane == 0)
        __hip_atomic_store(&L.hits[base + tot], tag | (uint32_t)(R * kRoundBytes), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
    return true;
}

// Walk n listed hit words from index `first` (n <= 16).  Matched starts claim
// their tile's staging slots with LDS atomics, so a tile's slots are in no
// particular order (the emit kernel sorts them).
// PER = starts per entry: 4 for a stride-4 hit word (lanes 4h..4h+3 take its
// four candidate starts), 1 for a stride-1 offset (a lane per entry).
template <bool BATCH, int TILE, int PER>
__device__ __forceinline__ void walk_listed(const ScanParams &P, const HitList &L, uint32_t first, uint32_t n,
                                            uint64_t tb, const WalkTabs &tabs, uint32_t *nm_l, uint64_t *rec_l,
                                            uint32_t *failed) {
    const uint32_t lane = lane_id();
    const uint32_t h = PER == 4 ? lane >> 2 : lane;
    bool act = h < n;
    uint32_t ent = 0;
    if (act) {
        // Every reserved entry is written right after its reservation; the
        // wait is bounded all the same.
        for (uint32_t spin = 0;; ++spin) {
            ent = __hip_atomic_load(&L.hits[first + h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (ent != kHitFree) break;
            if (spin == kSpinLimit) {
                atomicOr(failed, 1u);
                act = false;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    const uint32_t t_rel = ent >> kPosBits;
    const int32_t off = PER == 4 ? (int32_t)(ent & ((1u << kPosBits) - 1u)) - 3 + (int32_t)(lane & 3)
                                 : (int32_t)(ent & ((1u << kPosBits) - 1u));
    const uint64_t t = tb + t_rel;
    uint32_t last = 0;
    StateRecords sr{0u, 0u, 0u, 0u};
    if (act) {
        const TileInfo ti = tile_info<BATCH, TILE>(P, t);
        const uint64_t x = ti.x0 + (int64_t)off;
        if (off >= 0 && off < TILE && x >= ti.s.head && x < ti.s.valid_end) {
            last = walk(P.d, ti.s, tabs, x);
            if (last) sr = state_records(P.d, ti.s, x, last);
        }
    }
    if (sr.n) {
        const uint32_t slot = atomicAdd(&nm_l[t_rel], 1u);
        if (slot < kStageCap) P.staging[t * kStageCap + slot] = stage_entry((uint32_t)off, last, sr);
        atomicAdd(reinterpret_cast<unsigned long long *>(&rec_l[t_rel]), (unsigned long long)sr.n);
    }
}

// Record every offset of tile t that survived the filters (bit u of round k's
// mask is offset k*1024 + lane*16 + u) in the list; false if they do not all
// fit (then the tile must be walked right away).  Reserved as in list_hits.
template <int R>
__device__ __forceinline__ bool list_offsets1(const HitList &L, uint32_t t_rel, const uint32_t (&m)[R / 2]) {
    const uint32_t lane = lane_id();
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < R / 2; ++k) c += (uint32_t)__popc(m[k]);
    uint32_t tot;
    const uint32_t pre = wave_prefix_small<8>(c, tot);  // c <= 16 * R = 128
    if (tot == 0) return true;
    uint32_t base = 0, ok = 0;
    if (lane == 0) {
        uint32_t cur = __hip_atomic_load(L.count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        while (cur + tot <= kHitCap) {
            const uint32_t prev = atomicCAS(L.count, cur, cur + tot);
            if (prev == cur) {
                base = cur;
                ok = 1;
                break;
            }
            cur = prev;
        }
    }
    if (!__builtin_amdgcn_readfirstlane(ok)) return false;
    uint32_t pos = __builtin_amdgcn_readfirstlane(base) + pre;
    const uint32_t tag = t_rel << kPosBits;
#pragma unroll
    for (int k = 0; k < R; ++k) {
        uint32_t mask = (m[k / 2] >> (16 * (k % 2))) & 0xFFFFu;
        const uint32_t at = (uint32_t)k * kRoundBytes + lane * 16u;
        while (mask) {
            const uint32_t u = (uint32_t)__builtin_ctz(mask);
            mask &= mask - 1u;
            __hip_atomic_store(&L.hits[pos++], tag | (at + u), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    }
    return true;
}

// ---- stride 1: one probe per offset (or none: walk every offset) ----------
//
// Bit u of round k's 16-bit mask (word k/2, half k%2) marks offset
// x0 + k*1024 + lane*16 + u as not ruled out.

// The second filter's five bits for key g (double hashing: the top bits of h,
// k, h + k, h + 2k and h + 3k); bit 0 of the result is 1 if all five are set.
__device__ __forceinline__ uint32_t filter2_bits(const uint32_t *bm2, uint32_t g) {
    const uint32_t h = glop_hash2(g), k = glop_f2_mix(h), hk = h + k, h2 = hk + k, h3 = h2 + k;
    constexpr uint32_t sh2 = 32u - GLOP_FILTER2_LOG2;
    return (bm2[h >> (sh2 + 5u)] >> ((h >> sh2) & 31u)) & (bm2[k >> (sh2 + 5u)] >> ((k >> sh2) & 31u)) &
           (bm2[hk >> (sh2 + 5u)] >> ((hk >> sh2) & 31u)) & (bm2[h2 >> (sh2 + 5u)] >> ((h2 >> sh2) & 31u)) &
           (bm2[h3 >> (sh2 + 5u)] >> ((h3 >> sh2) & 31u));
}

// Per-wave staging of the second filter (stride 1), in the wave's LDS ring,
// which is otherwise used only after the tile's masks are known: a ring of
// (key, offset in tile) pairs waiting for the second filter, and one word per
// lane and round pair collecting the bits the second filter rejects.
struct Stage2 {
    static constexpr uint32_t kEntries = 128;  // at most 63 waiting + 64 added at once
    uint2 *ent;    // kEntries
    uint32_t *rej; // kWave * 4 words: lane L, rounds 2j and 2j+1 -> rej[L * 4 + j]
};
static_assert(Stage2::kEntries * 8 + kWave * 4 * 4 <= kRing1 * 2, "second-filter staging exceeds the wave's ring");

// The second filter on n staged entries from `head` (n <= 64, one per lane):
// a rejected offset's bit is set in its owner lane's reject word.
template <bool Q4>
__device__ __forceinline__ void filter2_batch(const Stage2 &st, const uint32_t *bm2, uint32_t qmask, uint32_t head,
                                              uint32_t n) {
    const uint32_t lane = lane_id();
    if (lane < n) {
        const uint2 e = st.ent[(head + lane) & (Stage2::kEntries - 1)];
        const uint32_t g = Q4 ? e.x : e.x & qmask;
        if ((filter2_bits(bm2, g) & 1u) == 0u) {
            const uint32_t off = e.y;  // k * 1024 + owner * 16 + u
            const uint32_t owner = (off >> 4) & (kWave - 1), k = off >> 10;
            atomicOr(&st.rej[owner * 4 + (k >> 1)], 1u << ((k & 1u) * 16u + (off & 15u)));
        }
    }
}

template <int R, bool FILTER, int K, bool Q4>
__device__ __forceinline__ void tile_masks1(const GlopDevDict &d, const TileInfo &ti, const TileRegs<R> &r,
                                            const uint32_t *bm, uint32_t bm_addr, const uint32_t *bm2,
                                            uint32_t (&m)[R / 2], const Stage2 *st = nullptr) {
    static_assert(R / 2 <= 4, "reject words hold four round pairs");
    const uint32_t lane = lane_id();
    const uint32_t qmask = d.qmask, sh = 32u - d.bitmap_log2;
    const bool full = ti.x0 >= ti.s.head && ti.x0 + R * kRoundBytes <= ti.s.valid_end;
    // Second filter, for the few offsets the first one lets through: their
    // keys wait in the staging ring and are checked 64 at a time, one per
    // lane, instead of each lane looping over its own survivors while the
    // wave waits for the lane with the most.
    const bool f2 = FILTER && bm2 != nullptr && st != nullptr;
    uint32_t head = 0, tail = 0;  // wave-uniform ring indices
    if (f2) {
        reinterpret_cast<uint4 *>(st->rej)[lane] = make_uint4(0u, 0u, 0u, 0u);
        wave_lds_sync();
    }
#pragma unroll
    for (int k = 0; k < R / 2; ++k) m[k] = 0;
#pragma unroll
    for (int k = 0; k < R; ++k) {
        uint32_t mask = 0xFFFFu;
        if (FILTER) {
            // Bytes 16..19 of the lane are the next lane's first word; for the
            // last lane, the next round's lane 0 (read wave-wide, before any
            // divergence) or the word after the tile.
            const uint32_t next0 = (k + 1 < R) ? __builtin_amdgcn_readfirstlane(r.v[(k + 1) % R].x) : r.extra;
            uint32_t nx = __shfl_down(r.v[k].x, 1);
            if (lane == kWave - 1) nx = next0;
            const uint32_t w[5] = {r.v[k].x, r.v[k].y, r.v[k].z, r.v[k].w, nx};
            uint32_t a1 = 0, a2 = K == 1 ? ~0u : 0u;
            // Key of offset u (u = 16 is the next lane's first word).
            auto key = [&](int u) -> uint32_t {
                return (u & 3) ? __builtin_amdgcn_alignbyte(w[(u >> 2) + 1], w[u >> 2], u & 3) : w[u >> 2];
            };
            if constexpr (K == 4) {
                // Paired probes (glop_layout.hpp): offsets u and u + 2 in the
                // two 16-bit halves.  The word at u holds the low halves of
                // both keys and the first bytes' shift amounts, the word at
                // u + 2 the high halves, the word at u + 1 the second bytes'
                // shift amounts.  Pair (u, u + 2) sets bits u and u + 16 of
                // a1, and bit 16 + u lands on offset u + 2 below.
                typedef unsigned short us2 __attribute__((ext_vector_type(2)));
                const us2 hA = {(unsigned short)GLOP_HASH16_A, (unsigned short)GLOP_HASH16_A};
                const us2 hB = {(unsigned short)GLOP_HASH16_B, (unsigned short)GLOP_HASH16_B};
                // A block's byte address is the masked hash plus the filter's
                // LDS address bm_addr: 0 in the scan kernel, whose tables start
                // at LDS address 0 (the build checks that it has no static
                // LDS), so there the sum is the masked hash itself.
                typedef __attribute__((address_space(3))) const unsigned short lds_u16;
#pragma unroll
                for (int v = 0; v < 8; ++v) {
                    const int u = (v & 1) + 4 * (v >> 1);  // 0, 1, 4, 5, 8, 9, 12, 13
                    const uint32_t xu = key(u), xu1 = key(u + 1), xu2 = key(u + 2);
                    const us2 h = __builtin_bit_cast(us2, xu) * hA + __builtin_bit_cast(us2, xu2) * hB;
                    const uint32_t hh = __builtin_bit_cast(uint32_t, h);
                    const us2 wb = {*(lds_u16 *)(size_t)(bm_addr + (hh & 0xFFFEu)),
                                    *(lds_u16 *)(size_t)(bm_addr + ((hh >> 16) & 0xFFFEu))};
                    // Each half shifted by the low four bits of its own byte
                    // (v_pk_lshrrev_b16 reads only those, so the keys need no
                    // mask; written out because C shifts by 16 or more are
                    // undefined).
                    uint32_t s1, s2;
                    const uint32_t wr = __builtin_bit_cast(uint32_t, wb);
                    __asm__("v_pk_lshrrev_b16 %0, %1, %2" : "=v"(s1) : "v"(xu), "v"(wr));
                    __asm__("v_pk_lshrrev_b16 %0, %1, %2" : "=v"(s2) : "v"(xu1), "v"(wr));
                    a1 = ((s1 & s2 & 0x00010001u) << u) | a1;
                    if ((v & 1) == 1) {
                        __asm__ volatile("" : "+v"(a1));
                        __builtin_amdgcn_sched_barrier(0);
                    }
                }
                mask = (a1 | (a1 >> 14)) & 0xFFFFu;
            } else {
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    probe_acc<K, Q4>(bm, key(u), key(u + 1), qmask, sh, a1, a2);
                    if ((u & 3) == 3) {
                        // Finish these probes here (see tile_hits4).
                        __asm__ volatile("" : "+v"(a1), "+v"(a2));
                        __builtin_amdgcn_sched_barrier(0);
                    }
                }
                mask = (a1 & a2) >> 16;
            }
            if (!full) mask &= valid_mask16(ti.s, ti.x0 + (uint64_t)k * kRoundBytes + lane * 16u);
            if (f2) {
                // Stage each lane's first survivor of the round; 64 waiting
                // entries are checked at once.  A lane's further survivors
                // in the round (about one lane-round in 170 has one) skip
                // the second filter: it only removes offsets, so an offset
                // it does not see is walked, which gives the same result.
                // One pass per round instead of one per survivor of the lane
                // with the most.
                const uint64_t bal = __ballot(mask != 0u);
                if (bal != 0) {
                    if (mask) {
                        const uint32_t u = (uint32_t)__builtin_ctz(mask);
                        // Word pair (w[a], w[a+1]), a = u / 4, picked in two steps.
                        const bool up = (u & 8u) != 0, odd = (u & 4u) != 0;
                        const uint32_t p0 = up ? w[2] : w[0], p1 = up ? w[3] : w[1], p2 = up ? w[4] : w[2];
                        // (v_alignbyte reads only the low two bits of its shift.)
                        const uint32_t g = __builtin_amdgcn_alignbyte(odd ? p2 : p1, odd ? p1 : p0, u);
                        const uint32_t pos =
                            tail + __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                             __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
                        st->ent[pos & (Stage2::kEntries - 1)] = make_uint2(g, (uint32_t)k * kRoundBytes + lane * 16u + u);
                    }
                    tail += (uint32_t)__popcll(bal);
                    if (tail - head >= (uint32_t)kWave) {
                        wave_lds_sync();
                        filter2_batch<Q4>(*st, bm2, qmask, head, kWave);
                        head += kWave;
                    }
                }
            }
        } else if (!full) {
            mask &= valid_mask16(ti.s, ti.x0 + (uint64_t)k * kRoundBytes + lane * 16u);
        }
        m[k / 2] |= mask << (16 * (k % 2));
        // Keep rounds apart: interleaving all probes of the tile costs more
        // registers than the wave has.
        __builtin_amdgcn_sched_barrier(0);
    }
    if (f2) {
        if (tail != head) {
            wave_lds_sync();
            filter2_batch<Q4>(*st, bm2, qmask, head, tail - head);
        }
        wave_lds_sync();
        const uint4 rj = reinterpret_cast<const uint4 *>(st->rej)[lane];
        const uint32_t rw[4] = {rj.x, rj.y, rj.z, rj.w};
#pragma unroll
        for (int k = 0; k < R / 2; ++k) m[k] &= ~rw[k];
        wave_lds_sync();  // the ring is free again (reads done before anyone writes it)
    }
}

template <int R, class Sink>
__device__ __forceinline__ void walk_offsets1(const ScanParams &P, uint64_t t, const TileInfo &ti,
                                              const uint32_t (&m)[R / 2], const WalkTabs &tabs, uint16_t *queue,
                                              Sink &sink) {
    const uint32_t lane = lane_id();
    uint32_t qhead = 0, qtail = 0;  // wave-uniform ring indices
    // Half a round at a time, lanes 0-31 and then lanes 32-63, so the queue
    // holds offsets in ascending order (the emit kernel's rescan writes its
    // records in queue order) and a half adds at most 512.
#pragma unroll
    for (int k = 0; k < 2 * R; ++k) {
        uint32_t mask = (lane >> 5) == (uint32_t)(k % 2) ? (m[k / 4] >> (16 * ((k / 2) % 2))) & 0xFFFFu : 0u;
        if (__ballot(mask != 0) == 0) continue;
        uint32_t tot;
        uint32_t pos = qtail + wave_prefix_small<5>((uint32_t)__popc(mask), tot);
        const uint32_t base = (uint32_t)(k / 2) * kRoundBytes + lane * 16u;
        while (mask) {
            const uint32_t u = (uint32_t)__builtin_ctz(mask);
            mask &= mask - 1u;
            queue[(pos++) & (kRing1 - 1)] = (uint16_t)(base + u);
        }
        qtail += tot;
        wave_lds_sync();
        for (; qtail - qhead >= (uint32_t)kWave; qhead += kWave) {
            const uint32_t off = queue[(qhead + lane) & (kRing1 - 1)];
            const uint32_t last = walk(P.d, ti.s, tabs, ti.x0 + off);
            sink.batch(P, t, ti, off, last);
        }
    }
    if (qtail != qhead) {
        const uint32_t n = qtail - qhead;
        const bool act = lane < n;
        const uint32_t off = act ? queue[(qhead + lane) & (kRing1 - 1)] : 0u;
        const uint32_t last = act ? walk(P.d, ti.s, tabs, ti.x0 + off) : 0u;
        sink.batch(P, t, ti, off, last);
    }
    sink.finish(t);
    __builtin_amdgcn_wave_barrier();
}

// Filter then walk one tile already in registers, walks right away.
template <int STRIDE, bool FILTER, int K, bool Q4, int R, class Sink>
__device__ __forceinline__ void scan_loaded_tile(const ScanParams &P, uint64_t t, const TileInfo &ti,
                                                 const TileRegs<R> &r, const uint32_t *bm, const WalkTabs &tabs,
                                                 uint16_t *queue, Sink &sink) {
    if constexpr (STRIDE == 4) {
        HitBits<R> pbits;
        uint32_t xb;
        tile_hits4<R, K, Q4>(P.d, r, bm, pbits, xb);
        walk_hits4<R>(P, t, ti, pbits, xb, tabs, queue, sink);
    } else {
        uint32_t m[R / 2];
        typedef __attribute__((address_space(3))) const uint32_t lds_u32;
        tile_masks1<R, FILTER, K, Q4>(P.d, ti, r, bm, (uint32_t)(size_t)(lds_u32 *)bm, nullptr, m);
        walk_offsets1<R>(P, t, ti, m, tabs, queue, sink);
    }
}

// Copy the bitmap and byte classes into LDS.
template <bool FILTER>
__device__ __forceinline__ void stage_tables(const ScanParams &P, uint32_t *bm, uint8_t *cls) {
    if (FILTER) {
        const uint4 *src = reinterpret_cast<const uint4 *>(P.d.bitmap);
        uint4 *dst = reinterpret_cast<uint4 *>(bm);
        for (uint32_t k = threadIdx.x; k < P.bm_bytes / 16; k += kBlock) dst[k] = src[k];
    }
    if (threadIdx.x < 64)
        reinterpret_cast<uint32_t *>(cls)[threadIdx.x] = reinterpret_cast<const uint32_t *>(P.d.cls)[threadIdx.x];
}

// A batch's counts come from device memory; they are clamped to what the
// workspace holds so that no loop can run past it.
template <bool BATCH>
__device__ __forceinline__ uint64_t total_tiles(const ScanParams &P) {
    return BATCH ? min(P.meta[kMetaTiles], P.tile_cap) : P.ntiles;
}

template <bool BATCH>
__device__ __forceinline__ uint64_t total_items(const ScanParams &P) {
    return BATCH ? min(P.meta[kMetaItems], P.item_cap) : (uint64_t)gridDim.x;
}

// Tiles per work item: the launch's for one text; a batch's, chosen by its
// prep kernel once the tile count is known (clamped so that no loop can run
// past the LDS arrays it indexes).
template <bool BATCH>
__device__ __forceinline__ uint64_t item_tiles(const ScanParams &P) {
    return BATCH ? min(max(P.meta[kMetaPer], 1ull), (unsigned long long)kMaxBatchTilesPerItem) : P.tiles_per_item;
}

// Clear a work item's LDS tile counters (and hit list at stride 4).
template <bool DEFER, bool BATCH>
__device__ __forceinline__ void reset_item_lds(uint32_t *nm_l, uint64_t *rec_l, uint32_t *hits) {
    for (uint32_t k = threadIdx.x; k < item_tiles_cap<BATCH>(); k += kBlock) {
        nm_l[k] = 0;
        rec_l[k] = 0;
    }
    if (DEFER)
        for (uint32_t k = threadIdx.x; k < kHitCap; k += kBlock) hits[k] = kHitFree;
}

template <int STRIDE, bool FILTER, int K, bool Q4, int R, bool BATCH>
__global__ __launch_bounds__(kBlock) void glop_scan_kernel(ScanParams P) {
    constexpr int TILE = R * kRoundBytes;
    constexpr bool kDefer = FILTER;  // deferred walks through the workgroup list (every filtered variant)
    extern __shared__ __align__(16) uint8_t lds[];
    const LdsLayout<STRIDE, BATCH> Lo{P.bm_bytes, P.pt_lds_bytes, P.f2_lds_bytes, P.tab_lds_bytes};
    ScanShared &sh = *reinterpret_cast<ScanShared *>(lds + Lo.sh_off());
    uint32_t &hl_count = sh.hl_count, &item_failed = sh.item_failed, &tile_next = sh.tile_next,
             &hl_walked = sh.hl_walked;
    uint64_t &item_sh = sh.item_sh;
    uint64_t *red = sh.red;
    static_assert(sizeof(ScanShared::red) == kWaves * sizeof(uint64_t), "one reduction word per wave");
    uint32_t *bm = reinterpret_cast<uint32_t *>(lds);
    uint8_t *cls = lds + Lo.cls_off();
    const uint32_t wave = wave_id();
    uint16_t *queue = reinterpret_cast<uint16_t *>(lds + Lo.ring_off()) + wave * ring_cap<STRIDE>();
    uint32_t *nm_l = reinterpret_cast<uint32_t *>(lds + Lo.nm_off());
    uint64_t *rec_l = reinterpret_cast<uint64_t *>(lds + Lo.rec_off());
    const HitList HL{reinterpret_cast<uint32_t *>(lds + Lo.hits_off()), &hl_count};

    // One text: the emit kernel adds into the counts after this kernel ends.
    // (A batch's prep kernel zeroes them.)
    if (!BATCH && P.zero_counts)
        for (uint64_t k = (uint64_t)blockIdx.x * kBlock + threadIdx.x; k < P.d.num_patterns;
             k += (uint64_t)gridDim.x * kBlock)
            P.counts[k] = 0;
    stage_tables<FILTER>(P, bm, cls);
    const uint4 *pt = nullptr;
    if (P.pt_lds_bytes) {
        const uint4 *src = reinterpret_cast<const uint4 *>(P.d.pt);
        uint4 *dst = reinterpret_cast<uint4 *>(lds + Lo.pt_off());
        for (uint32_t k = threadIdx.x; k < P.pt_lds_bytes / 16; k += kBlock) dst[k] = src[k];
        pt = reinterpret_cast<const uint4 *>(lds + Lo.pt_off());
    }
    const uint32_t *bm2 = nullptr;
    if constexpr (STRIDE == 1) {  // the second filter exists for stride 1 only
        if (P.f2_lds_bytes) {
            const uint4 *src = reinterpret_cast<const uint4 *>(P.d.bitmap2);
            uint4 *dst = reinterpret_cast<uint4 *>(lds + Lo.f2_off());
            for (uint32_t k = threadIdx.x; k < P.f2_lds_bytes / 16; k += kBlock) dst[k] = src[k];
            bm2 = reinterpret_cast<const uint32_t *>(lds + Lo.f2_off());
        }
    }
    const uint32_t *tab = nullptr;
    if (P.tab_lds_bytes) {
        const uint4 *src = reinterpret_cast<const uint4 *>(P.d.delta);
        uint4 *dst = reinterpret_cast<uint4 *>(lds + Lo.tab_off());
        for (uint32_t k = threadIdx.x; k < P.tab_lds_bytes / 16; k += kBlock) dst[k] = src[k];
        uint32_t *dst4 = reinterpret_cast<uint32_t *>(lds + Lo.tab_off());
        for (uint32_t k = (P.tab_lds_bytes / 16) * 4 + threadIdx.x; k < P.tab_lds_bytes / 4; k += kBlock)
            dst4[k] = P.d.delta[k];
        tab = dst4;
    }
    const WalkTabs tabs{cls, pt, tab};

    const uint64_t nt = total_tiles<BATCH>(P), tpi = item_tiles<BATCH>(P);
    // First work item: a device ticket for a batch, the block index otherwise.
    // Later items are taken at the end of each round, before its closing
    // barrier: every thread-0 step sits between two barriers of the same
    // round, so the compiler cannot route thread 0 around the loop on its own
    // (a wave whose lanes split across rounds would pass the barrier without
    // its lane 0 and never see the next ticket).
    if (threadIdx.x == 0) {
        item_sh = BATCH ? atomicAdd(reinterpret_cast<unsigned long long *>(&P.meta[kMetaTicket]), 1ull)
                        : (uint64_t)blockIdx.x;
        item_failed = 0;
        tile_next = 0;
        if (kDefer) hl_count = hl_walked = 0;
    }
    reset_item_lds<kDefer, BATCH>(nm_l, rec_l, HL.hits);
    // A wave takes the item's next tile from an LDS counter whenever it starts
    // one, so all 16 waves keep loads in flight until the item's last tile (a
    // fixed share per wave left some waves idle for a fifth of the item while
    // others were still streaming).
    auto claim = [&]() -> uint32_t {
        uint32_t c = 0;
        if (lane_id() == 0) c = atomicAdd(&tile_next, 1u);
        return __builtin_amdgcn_readfirstlane(c);
    };
    for (;;) {
        wg_barrier();
        const uint64_t item = item_sh;
        if (item >= total_items<BATCH>(P)) break;
        const uint64_t tb = item * tpi;
        const uint64_t te = min(nt, tb + tpi);

        // Pipelined: once a tile's filter bits are known its bytes are dead,
        // so the next tile's loads go out before anything else.
        const uint32_t ntile = (uint32_t)(te - tb);
        TileRegs<R> r;
        TileInfo cur{};
        uint32_t c = claim();
        if (c < ntile) {
            cur = tile_info<BATCH, TILE>(P, tb + c);
            load_tile<R, FILTER, STRIDE == 4>(cur, r);
        }
        while (c < ntile) {
            const uint64_t t = tb + c;
            const uint32_t cn = claim();
            const bool has_next = cn < ntile;
            TileInfo nxt = cur;
            uint32_t next_desc = 0;  // batch: read once this tile's probes are done
            if (has_next) {
                if constexpr (BATCH) next_desc = tile_desc_lanes(P, tb + cn);
                else nxt = tile_info<BATCH, TILE>(P, tb + cn);
            }
            auto load_next = [&](auto nt_loads) {
                if (!has_next) return;
                if constexpr (BATCH) nxt = tile_info_lanes<TILE>(P, next_desc);
                load_tile<R, FILTER, decltype(nt_loads)::value>(nxt, r);
            };
            StageSink sink(nm_l, rec_l, tb);
            if constexpr (STRIDE == 4) {
                HitBits<R> pbits;
                uint32_t xb;
                tile_hits4<R, K, Q4>(P.d, r, bm, pbits, xb);
                load_next(std::true_type{});
                if (__ballot(pbits != 0) != 0 || xb) {
                    if (!list_hits<R>(HL, (uint32_t)(t - tb), pbits, xb))
                        walk_hits4<R>(P, t, cur, pbits, xb, tabs, queue, sink);
                }
            } else {
                uint32_t m[R / 2];
                const Stage2 st2{reinterpret_cast<uint2 *>(queue),
                                 reinterpret_cast<uint32_t *>(queue) + 2 * Stage2::kEntries};
                tile_masks1<R, FILTER, K, Q4>(P.d, cur, r, bm, 0u, bm2, m, &st2);  // bm: LDS address 0
                load_next(std::false_type{});
                // Survivors wait in the workgroup list, so walks run in full
                // batches of 64 instead of one short batch per tile.  Here the
                // probes keep the vector units busy, so a wave that finds 64
                // entries nobody has taken walks them now, hidden behind the
                // other waves' probes, rather than in the item's last phase.
                if (!kDefer || !list_offsets1<R>(HL, (uint32_t)(t - tb), m)) {
                    walk_offsets1<R>(P, t, cur, m, tabs, queue, sink);
                } else {
                    uint32_t first = 0, ok = 0;
                    if (lane_id() == 0) {
                        uint32_t w = __hip_atomic_load(&hl_walked, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                        const uint32_t have = __hip_atomic_load(&hl_count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                        while (w + 64u <= have) {
                            const uint32_t prev = atomicCAS(&hl_walked, w, w + 64u);
                            if (prev == w) {
                                first = w;
                                ok = 1;
                                break;
                            }
                            w = prev;
                        }
                    }
                    if (__builtin_amdgcn_readfirstlane(ok))
                        walk_listed<BATCH, TILE, 1>(P, HL, __builtin_amdgcn_readfirstlane(first), 64u, tb, tabs,
                                                    nm_l, rec_l, &item_failed);
                }
            }
            cur = nxt;
            c = cn;
        }
        if (kDefer) {
            // The rest of the list (stride 1: past what waves took while
            // streaming), shared by all waves.
            wg_barrier();
            const uint32_t n = hl_count, w0 = STRIDE == 1 ? hl_walked : 0u;
            constexpr uint32_t kPer = STRIDE == 4 ? 16u : 64u;  // entries per walk batch
            for (uint32_t f = w0 + wave * kPer; f < n; f += kWaves * kPer)
                walk_listed<BATCH, TILE, STRIDE == 4 ? 4 : 1>(P, HL, f, min(kPer, n - f), tb, tabs, nm_l, rec_l,
                                                              &item_failed);
        }
        wg_barrier();
        // The item's tile results, coalesced, and its total.
        uint64_t part = 0;
        for (uint64_t k = tb + threadIdx.x; k < te; k += kBlock) {
            const uint64_t rc = rec_l[k - tb];
            P.tile_rec[k] = rc;
            P.tile_nm[k] = nm_l[k - tb];
            part += rc;
        }
        part = block_sum_u64(part, red);
        if (threadIdx.x == 0) {
            P.itemsum[item] = item_failed ? kItemFailed : part;
            item_sh = BATCH ? atomicAdd(reinterpret_cast<unsigned long long *>(&P.meta[kMetaTicket]), 1ull) : ~0ull;
            item_failed = 0;
            tile_next = 0;
            if (kDefer) hl_count = hl_walked = 0;
        }
        reset_item_lds<kDefer, BATCH>(nm_l, rec_l, HL.hits);
    }
}

template <int STRIDE, bool FILTER, int K, bool Q4, int R, bool BATCH>
__global__ __launch_bounds__(kBlock) void glop_emit_kernel(ScanParams P, EmitParams E) {
    constexpr int TILE = R * kRoundBytes;
    extern __shared__ __align__(16) uint8_t lds[];
    __shared__ uint64_t scan_sh[kWaves + 1];
    __shared__ uint64_t red[kWaves];
    __shared__ uint32_t n_over, any_over, any_failed;
    __shared__ uint64_t over_tile[kBlock];
    __shared__ uint64_t over_base[kBlock];
    // Batch with per-chunk slices: output position of each tile of the item
    // (read for the tiles that start a chunk), and of the first record of the
    // chunk that began before the item.
    __shared__ uint64_t tile_first[BATCH ? kMaxBatchTilesPerItem : 1];
    __shared__ uint64_t carry_first;
    __shared__ uint32_t count_key[CountTable::kSlots];
    __shared__ uint32_t count_val[CountTable::kSlots];
    const CountTable ct{count_key, count_val, P.counts};
    const LdsLayout<STRIDE, BATCH> Lo{P.bm_bytes};
    uint32_t *bm = reinterpret_cast<uint32_t *>(lds);
    uint8_t *cls = lds + Lo.cls_off();
    const WalkTabs tabs{cls, nullptr};
    const uint32_t wave = wave_id();
    uint16_t *queue = reinterpret_cast<uint16_t *>(lds + Lo.ring_off()) + wave * ring_cap<STRIDE>();
    const uint64_t nt = total_tiles<BATCH>(P), items = total_items<BATCH>(P), tpi = item_tiles<BATCH>(P);
    bool staged = false, has_last = false;
    uint64_t last_total = 0;
    // Records written by earlier calls into the same output (a text matched
    // in consecutive pieces); read before any workgroup can write the total.
    const uint64_t call_base = (!BATCH && E.base_in) ? *E.base_in : 0ull;
    if (threadIdx.x == 0) {
        any_failed = call_base == kItemFailed ? 1u : 0u;  // an earlier piece failed
        any_over = 0;
    }
    ct.clear();
    wg_barrier();

    // Thread-0 steps inside the loop sit between barriers of the same item
    // (see the scan kernel); the call's total is written after the loop.
    for (uint64_t item = blockIdx.x; item < items; item += gridDim.x) {
        const uint64_t tb = item * tpi;
        const uint64_t te = min(nt, tb + tpi);
        // Records of all earlier items, and whether any tile here overflowed.
        // A failed item (kItemFailed) fails the whole call.
        uint64_t part = 0;
        uint32_t bad = 0;
        const uint64_t upto = item == items - 1 ? items : item;  // the last item also checks itself
        for (uint64_t g = threadIdx.x; g < upto; g += kBlock) {
            const uint64_t v = P.itemsum[g];
            bad |= v == kItemFailed;
            if (g < item) part += v;
        }
        if (bad) atomicOr(&any_failed, 1u);
        uint32_t over = 0;
        for (uint64_t t = tb + threadIdx.x; t < te; t += kBlock) over |= P.tile_nm[t] > kStageCap;
        if (over) atomicOr(&any_over, 1u);
        // The first block of tile record counts, read beside the sums above.
        const uint64_t rec0 = tb + threadIdx.x < te ? P.tile_rec[tb + threadIdx.x] : 0ull;
        uint64_t base = call_base + block_sum_u64(part, red);  // its barriers publish any_over
        const bool sliced = BATCH && E.slice_first != nullptr;
        if (sliced) {
            // The chunk holding the item's first tile may have begun in an
            // earlier item i0: its first record follows the records of items
            // before i0 and of i0's tiles before the chunk's first tile.
            const uint64_t t0 = tb - P.tile_desc[tb].k;
            const uint64_t i0 = t0 / tpi;
            uint64_t before = 0;
            if (t0 < tb) {
                for (uint64_t g = threadIdx.x; g < i0; g += kBlock) before += P.itemsum[g];
                for (uint64_t t = i0 * tpi + threadIdx.x; t < t0; t += kBlock) before += P.tile_rec[t];
            }
            before = block_sum_u64(before, red);
            if (threadIdx.x == 0) carry_first = before;  // read after the scan's barriers below
        }
        if (any_over && !staged) {
            stage_tables<FILTER>(P, bm, cls);
            staged = true;
            wg_barrier();
        }

        for (uint64_t c0 = tb; c0 < te; c0 += kBlock) {
            const uint64_t t = c0 + threadIdx.x;
            const bool in = t < te;
            const uint64_t rec = c0 == tb ? rec0 : (in ? P.tile_rec[t] : 0ull);
            uint64_t chunk_total;
            const uint64_t tile_base = base + block_excl_scan_u64(rec, scan_sh, chunk_total);
            if (sliced && in) tile_first[t - tb] = tile_base;  // batch items fit one pass (<= kBlock tiles)
            if (threadIdx.x == 0) n_over = 0;
            wg_barrier();
            // Output position of the first record of the chunk that tile t lies in.
            auto chunk_first_pos = [&](uint32_t chunk) -> uint64_t {
                if (!sliced) return 0;
                const uint64_t t0 = P.tile_start[chunk];
                return t0 >= tb ? tile_first[t0 - tb] : carry_first;
            };
            if (in) {
                const TileInfo ti = tile_info<BATCH, TILE>(P, t);
                if (BATCH && ti.x0 == 0) E.chunk_first[ti.chunk] = tile_base;  // the chunk's first tile
                const uint32_t nm = rec > 0 ? P.tile_nm[t] : 0u;
                if (nm > kStageCap) {
                    const uint32_t slot = atomicAdd(&n_over, 1u);
                    over_tile[slot] = t;
                    over_base[slot] = tile_base;
                } else if (nm > 0) {
                    // Staged starts, in ascending offset (slots may be
                    // unordered; offsets are distinct, so the smallest entry
                    // above the last one written is the next).
                    const uint64_t cf = chunk_first_pos(ti.chunk);
                    uint64_t pos = tile_base;
                    uint64_t prev = 0;
                    for (uint32_t e = 0; e < nm; ++e) {
                        uint64_t ent = ~0ull;
                        for (uint32_t j = 0; j < nm; ++j) {
                            const uint64_t c = P.staging[t * kStageCap + j];
                            if ((e == 0 || c > prev) && c < ent) ent = c;
                        }
                        prev = ent;
                        const uint32_t low = (uint32_t)ent;
                        const uint64_t x = ti.x0 + (ent >> 49);
                        const uint64_t i = x - ti.s.head + E.offset_add;
                        if ((ent >> 48) & 1u) {
                            // List form: the mask names the records, in list order.
                            uint32_t bits = (uint32_t)(ent >> 32) & 0xFFFFu;
                            while (bits) {
                                const uint32_t k = (uint32_t)__builtin_ctz(bits);
                                bits &= bits - 1u;
                                const uint32_t id = P.d.outids[low + k];
                                put_record<BATCH>(E, pos, cf, glop_match_t{i, id, ti.chunk});
                                ct.add(id);
                                ++pos;
                            }
                        } else {
                            const uint32_t first = P.d.term[2 * low], cnt = P.d.term[2 * low + 1];
                            for (uint32_t k = 0; k < cnt; ++k) {
                                const uint32_t id = P.d.outids[first + k];
                                if (P.d.verify_from && !verified(P.d, ti.s, x, id)) continue;
                                put_record<BATCH>(E, pos, cf, glop_match_t{i, id, ti.chunk});
                                ct.add(id);
                                ++pos;
                            }
                        }
                    }
                }
            }
            wg_barrier();
            for (uint32_t o = wave; o < n_over; o += kWaves) {
                const uint64_t ot = over_tile[o];
                const TileInfo ti = tile_info<BATCH, TILE>(P, ot);
                DirectSink<BATCH> sink(&E, &ct, over_base[o], chunk_first_pos(ti.chunk));
                // Two rounds at a time, in order, through one sink: a rare
                // path that keeps a quarter of the tile in registers (the whole
                // tile would push the kernel past its register budget).
                constexpr int kSub = 2;
                for (int s = 0; s < R / kSub; ++s) {
                    TileInfo sub = ti;
                    sub.x0 = ti.x0 + (uint64_t)s * kSub * kRoundBytes;
                    sub.interior =
                        (sub.x0 >= sub.s.head && sub.x0 + kSub * kRoundBytes + 4 <= sub.s.span_end) ? 1u : 0u;
                    TileRegs<kSub> r;
                    load_tile<kSub, FILTER>(sub, r);
                    scan_loaded_tile<STRIDE, FILTER, K, Q4, kSub>(P, ot, sub, r, bm, tabs, queue, sink);
                }
            }
            wg_barrier();
            base += chunk_total;
        }
        if (item == items - 1) {
            has_last = true;
            last_total = base;
        }
        if (threadIdx.x == 0) any_over = 0;  // every read of it preceded the last barrier
        ct.flush();  // every add of the item preceded the last barrier
        wg_barrier();
    }
    if (has_last && threadIdx.x == 0) {
        if (E.total) *E.total = any_failed ? ~0ull : last_total;
        if (BATCH) {
            P.meta[kMetaTotal] = last_total;
            if (any_failed) P.meta[kMetaError] = 1;
        }
    }
}

// A call with nothing to match: clear the counts (unless they accumulate over
// consecutive pieces) and carry the running record total.
template <int = 0>
__global__ void glop_zero_kernel(uint64_t *counts, uint32_t n, uint64_t *total, const uint64_t *base_in,
                                 uint32_t zero_counts) {
    if (zero_counts)
        for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) counts[k] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0 && total) *total = base_in ? *base_in : 0ull;
}

// Batch prep (one workgroup): tiles per chunk -> first tile of each chunk,
// total tiles and work items, a zero ticket, zero counts.  Every chunk gets at
// least one tile, so each has a first tile to report its output position.
template <int TILE>
__global__ __launch_bounds__(kBlock) void glop_batch_prep_kernel(ScanParams P, uint32_t wgs) {
    __shared__ uint64_t sh[kWaves + 1];
    uint64_t running = 0;
    for (uint64_t c0 = 0; c0 < P.nchunks; c0 += kBlock) {
        const uint64_t c = c0 + threadIdx.x;
        uint64_t nt = 0;
        if (c < P.nchunks) {
            const glop_chunk_t ch = P.chunks[c];
            const uint64_t span = (reinterpret_cast<uintptr_t>(ch.text) & 15u) + ch.len;
            nt = span ? (span + TILE - 1) / TILE : 1;
        }
        uint64_t tot;
        const uint64_t ex = block_excl_scan_u64(nt, sh, tot);
        if (c < P.nchunks) P.tile_start[c] = running + ex;
        running += tot;
    }
    if (threadIdx.x == 0) {
        P.tile_start[P.nchunks] = running;
        const bool overflow = running > P.tile_cap;
        P.meta[kMetaTiles] = overflow ? 0 : running;
        // Items of equal size in the fewest whole rounds of one item per
        // workgroup (as for one text): each item end costs its workgroup a
        // walk and write-out phase, and a last round with fewer items than
        // workgroups leaves CUs idle.  At least kMinBatchTilesPerItem tiles,
        // so the items fit the workspace's item capacity.
        const uint64_t w = wgs ? wgs : 1;
        const uint64_t rounds = running ? (running + w * kMaxBatchTilesPerItem - 1) / (w * kMaxBatchTilesPerItem) : 1;
        uint64_t per = running ? (running + w * rounds - 1) / (w * rounds) : 1;
        per = per < kMinBatchTilesPerItem ? kMinBatchTilesPerItem : per;
        P.meta[kMetaPer] = per;
        P.meta[kMetaItems] = overflow ? 0 : (running + per - 1) / per;
        P.meta[kMetaTicket] = 0;
        P.meta[kMetaOverflow] = overflow ? 1 : 0;
        P.meta[kMetaTotal] = 0;
        P.meta[kMetaError] = 0;
    }
    for (uint32_t k = threadIdx.x; k < P.d.num_patterns; k += kBlock) P.counts[k] = 0;
}

// Batch: every tile's descriptor, chunk by chunk (a workgroup takes a chunk
// and its threads its tiles).
template <int = 0>
__global__ void glop_batch_map_kernel(ScanParams P) {
    const uint64_t nt = min(P.meta[kMetaTiles], P.tile_cap);
    for (uint32_t c = blockIdx.x; c < P.nchunks; c += gridDim.x) {
        const uint64_t t0 = P.tile_start[c], t1 = min(P.tile_start[c + 1], nt);
        const glop_chunk_t ch = P.chunks[c];
        for (uint64_t t = t0 + threadIdx.x; t < t1; t += blockDim.x) {
            TileDesc dsc;
            dsc.text = ch.text;
            dsc.len = ch.len;
            dsc.k = t - t0;
            dsc.chunk = c;
            dsc.pad = 0;
            P.tile_desc[t] = dsc;
        }
    }
}

// Batch: occurrences per chunk, the total, and the overflow verdict.
template <int = 0>
__global__ void glop_batch_finish_kernel(ScanParams P, uint64_t *chunk_first, uint64_t *chunk_count,
                                         uint64_t *total) {
    const bool overflow = P.meta[kMetaOverflow] != 0 || P.meta[kMetaError] != 0;
    const uint64_t tot = P.meta[kMetaTotal];
    for (uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; c < P.nchunks;
         c += (uint64_t)gridDim.x * blockDim.x) {
        if (overflow) {
            chunk_first[c] = 0;
            chunk_count[c] = 0;
        } else {
            const uint64_t next = c + 1 < P.nchunks ? chunk_first[c + 1] : tot;
            chunk_count[c] = next - chunk_first[c];
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *total = overflow ? ~0ull : tot;
}

constexpr uint64_t align256(uint64_t v) { return (v + 255) & ~255ull; }

struct Geometry {
    uint64_t ntiles, tiles_per_item;
    uint32_t grid;
    uint64_t off_rec, off_nm, off_stage, off_item, bytes;
};

// One text: tiles of `tile` bytes, at most kMaxTilesPerItem per workgroup.
// Tile coordinates start at the text's first byte rounded down to 16 bytes,
// `head` bytes before it.  The exact head matters: an aligned 4 GiB text is
// 2^19 tiles, two rounds of full items on 256 CUs, where one more tile would
// need a third round.  Every region grows with the number of tiles (the item
// sums are sized for whole rounds: the item count itself is not monotone, 257
// tiles make 129 items of 2 and 256 tiles 256 items of 1), so a workspace
// sized with the smallest tile and head 15 holds every launch of that length.
inline Geometry geometry(uint64_t len, int num_cus, uint32_t tile, uint64_t head) {
    Geometry g{};
    g.ntiles = (head + len + tile - 1) / tile;
    const uint64_t wgs = (uint64_t)(num_cus > 0 ? num_cus : 1);
    g.tiles_per_item = single_tiles_per_item(g.ntiles, wgs);
    g.grid = (uint32_t)(g.ntiles ? (g.ntiles + g.tiles_per_item - 1) / g.tiles_per_item : 0);
    const uint64_t rounds = g.ntiles ? (g.ntiles + wgs * kMaxTilesPerItem - 1) / (wgs * kMaxTilesPerItem) : 1;
    g.off_rec = 0;
    g.off_nm = align256(g.off_rec + g.ntiles * 8);
    g.off_stage = align256(g.off_nm + g.ntiles * 4);
    g.off_item = align256(g.off_stage + g.ntiles * kStageCap * 8);
    g.bytes = align256(g.off_item + wgs * rounds * 8);
    return g;
}

struct BatchGeometry {
    uint64_t tile_cap, item_cap;
    uint64_t off_rec, off_nm, off_stage, off_desc, off_start, off_item, off_meta, bytes;
};

// A batch: sized for the smallest tile, so it holds either tile size.
inline BatchGeometry batch_geometry(uint32_t nchunks, uint64_t max_total_bytes, uint32_t tile_bytes) {
    BatchGeometry g{};
    g.tile_cap = (max_total_bytes + 16ull * nchunks) / tile_bytes + nchunks + 1;
    g.item_cap = (g.tile_cap + kMinBatchTilesPerItem - 1) / kMinBatchTilesPerItem;
    g.off_rec = 0;
    g.off_nm = align256(g.off_rec + g.tile_cap * 8);
    g.off_stage = align256(g.off_nm + g.tile_cap * 4);
    g.off_desc = align256(g.off_stage + g.tile_cap * kStageCap * 8);
    g.off_start = align256(g.off_desc + g.tile_cap * sizeof(TileDesc));
    g.off_item = align256(g.off_start + ((uint64_t)nchunks + 1) * 8);
    g.off_meta = align256(g.off_item + g.item_cap * 8);
    g.bytes = align256(g.off_meta + kMetaWords * 8);
    return g;
}

template <int STRIDE, bool BATCH>
constexpr size_t dyn_lds(uint32_t bm_bytes, uint32_t pt_bytes, uint32_t f2_bytes = 0, uint32_t tab_bytes = 0) {
    return LdsLayout<STRIDE, BATCH>{bm_bytes, pt_bytes, f2_bytes, tab_bytes}.bytes();
}

// The emit kernel uses the bitmap, the byte classes and the per-wave rings of
// the layout (for its rare rescans), nothing after them.
template <int STRIDE, bool BATCH>
constexpr size_t emit_dyn_lds(uint32_t bm_bytes) {
    return LdsLayout<STRIDE, BATCH>{bm_bytes}.hits_off();
}

template <int STRIDE, bool FILTER, int K, bool Q4, int R>
struct Kernels {
    static hipError_t set_lds_limit() {
        // The scan kernels may stage a prefix table or second filter and the
        // dense rows (a launch checks its own size); the emit kernels never do.
        constexpr uint32_t bm = (1u << 19) / 8;
        static_assert(dyn_lds<STRIDE, false>(bm, pt_lds_cap<STRIDE>()) <= kScanLdsLimit, "scan layout exceeds LDS");
        const int bytes[4] = {(int)kScanLdsLimit, (int)kScanLdsLimit, (int)emit_dyn_lds<STRIDE, false>(bm),
                              (int)emit_dyn_lds<STRIDE, true>(bm)};
        const void *fns[] = {reinterpret_cast<const void *>(&glop_scan_kernel<STRIDE, FILTER, K, Q4, R, false>),
                             reinterpret_cast<const void *>(&glop_scan_kernel<STRIDE, FILTER, K, Q4, R, true>),
                             reinterpret_cast<const void *>(&glop_emit_kernel<STRIDE, FILTER, K, Q4, R, false>),
                             reinterpret_cast<const void *>(&glop_emit_kernel<STRIDE, FILTER, K, Q4, R, true>)};
        for (int k = 0; k < 4; ++k) {
            hipError_t e = hipFuncSetAttribute(fns[k], hipFuncAttributeMaxDynamicSharedMemorySize, bytes[k]);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }

    static hipError_t one(const ScanParams &P, const EmitParams &E, uint32_t grid, hipStream_t s,
                          const glop_events_t *ev) {
        const size_t lds = dyn_lds<STRIDE, false>(P.bm_bytes, P.pt_lds_bytes, P.f2_lds_bytes, P.tab_lds_bytes);
        if (lds > kScanLdsLimit) return hipErrorInvalidValue;
        const size_t emit_lds = emit_dyn_lds<STRIDE, false>(P.bm_bytes);
        hipError_t e;
        if (ev && ev->scan_begin && (e = hipEventRecord((hipEvent_t)ev->scan_begin, s)) != hipSuccess) return e;
        hipLaunchKernelGGL((glop_scan_kernel<STRIDE, FILTER, K, Q4, R, false>), dim3(grid), dim3(kBlock), lds, s, P);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (ev && ev->scan_end && (e = hipEventRecord((hipEvent_t)ev->scan_end, s)) != hipSuccess) return e;
        hipLaunchKernelGGL((glop_emit_kernel<STRIDE, FILTER, K, Q4, R, false>), dim3(grid), dim3(kBlock), emit_lds, s,
                           P, E);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (ev && ev->emit_end) e = hipEventRecord((hipEvent_t)ev->emit_end, s);
        return e;
    }

    static hipError_t batch(const ScanParams &P, const EmitParams &E, uint64_t *chunk_count, uint64_t *total,
                            int num_cus, hipStream_t s) {
        const size_t lds = dyn_lds<STRIDE, true>(P.bm_bytes, P.pt_lds_bytes, P.f2_lds_bytes, P.tab_lds_bytes);
        if (lds > kScanLdsLimit) return hipErrorInvalidValue;
        const size_t emit_lds = emit_dyn_lds<STRIDE, true>(P.bm_bytes);
        // Persistent workgroups: one per CU, fewer if the batch has fewer items.
        uint64_t wg = (uint64_t)(num_cus > 0 ? num_cus : 1);
        const uint64_t items = (P.tile_cap + kMinBatchTilesPerItem - 1) / kMinBatchTilesPerItem;
        if (items < wg) wg = items ? items : 1;
        const uint32_t cus = (uint32_t)wg;
        hipLaunchKernelGGL((glop_batch_prep_kernel<R * kRoundBytes>), dim3(1), dim3(kBlock), 0, s, P, cus);
        hipError_t e;
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(glop_batch_map_kernel<0>, dim3(4 * cus), dim3(256), 0, s, P);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL((glop_scan_kernel<STRIDE, FILTER, K, Q4, R, true>), dim3(cus), dim3(kBlock), lds, s, P);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL((glop_emit_kernel<STRIDE, FILTER, K, Q4, R, true>), dim3(cus), dim3(kBlock), emit_lds, s, P,
                           E);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        const uint32_t fb = (P.nchunks + 255) / 256 > 1024 ? 1024u : (uint32_t)((P.nchunks + 255) / 256);
        hipLaunchKernelGGL(glop_batch_finish_kernel<0>, dim3(fb ? fb : 1), dim3(256), 0, s, P, E.chunk_first,
                           chunk_count, total);
        return hipGetLastError();
    }
};


// Launch entry points of one Kernels<> variant.  Each variant translation unit
// defines the tables of its variants; the dispatch only declares them, so it
// never instantiates a kernel itself.
struct VariantFns {
    hipError_t (*one)(const ScanParams &, const EmitParams &, uint32_t, hipStream_t, const glop_events_t *);
    hipError_t (*batch)(const ScanParams &, const EmitParams &, uint64_t *, uint64_t *, int, hipStream_t);
    hipError_t (*set_lds_limit)();
};

#define GLOP_VARIANT_ID(S, F, K, Q, R) glop_variant_##S##_##F##_##K##_##Q##_##R
#define GLOP_DECLARE_VARIANT(S, F, K, Q, R) const VariantFns &GLOP_VARIANT_ID(S, F, K, Q, R)();
#define GLOP_DEFINE_VARIANT(S, F, K, Q, R)                                                         \
    const VariantFns &GLOP_VARIANT_ID(S, F, K, Q, R)() {                                            \
        static const VariantFns v = {&Kernels<S, (F != 0), K, (Q != 0), R>::one,                    \
                                     &Kernels<S, (F != 0), K, (Q != 0), R>::batch,                  \
                                     &Kernels<S, (F != 0), K, (Q != 0), R>::set_lds_limit};         \
        return v;                                                                                   \
    }

}  // namespace detail
}  // namespace glop
